"""Approximate minimum / maximum wave speeds.

Oracle (test infrastructure only; see the package docstring).

5-moment: Baradaran's approximation (Appendix B, eq. ws-max-baradaran-orig).
14-moment: the paper's proposed approximation (Section 5.1, eq. 14mom-approx-ws-equations;
Appendix B.2, eq. 14mom-approx-ws-equations-appendix), for the sweep direction d:
dimensionless state (P*_dd, q*_d, transverse |q*_t|, sigma), lambda*_min by reversing q*_d,
inflation by k, re-dimensionalisation by sqrt(p/rho) and the bulk velocity u_d.  The other
directions use the same formulas with the direction's own components (Section 5.1).

Readings (the paper is silent or the formulas leave their domain):
  * sigma_w = min(sigma_bar, 1) inside the wave speeds: the 14-moment realizability bound is
    only sufficient, so sigma_bar may exceed 1 and sqrt(3 - 3 sigma) would be imaginary.
  * P*_dd is clamped at 0 and every square-root argument at 0.
  * zeta + sqrt(X) is evaluated as (X - zeta^2) / (sqrt(X) - zeta) when zeta < 0, with
    X - zeta^2 formed term by term (no cancellation); when X <= 0 the root is zeta itself.
"""
import numpy as np

from .closure import sigma14_star, sigma5_star


def _hyperbola(zeta, rest):
    """zeta + sqrt(max(0, zeta^2 + rest)) without cancellation."""
    X = zeta * zeta + rest
    sX = np.sqrt(np.maximum(X, 0.0))
    with np.errstate(divide='ignore', invalid='ignore'):
        neg = rest / (sX - zeta)
    out = np.where(zeta >= 0.0, zeta + sX, neg)
    return np.where(X <= 0.0, zeta, out)


def _B_Y_E_C(sw, Pdd):
    C = np.sqrt(np.maximum((3.0 - 3.0 * sw) * Pdd, 0.0))
    E = 0.8 * C
    rs = np.sqrt(sw)
    B = 5.0 - 4.0 * rs + np.sqrt(np.maximum(10.0 - 16.0 * rs + 6.0 * sw, 0.0))
    Y = B + E * E - 2.0 * E * np.sqrt(B)
    return B, Y, E, C


def lam_max_star14(Pdd, qd, qt, sigma_bar):
    """Dimensionless maximum wave speed of the 14-moment system (bulk frame)."""
    sw = np.minimum(sigma_bar, 1.0)
    Pdd = np.maximum(Pdd, 0.0)
    alpha = 0.6 * Pdd**2 - 0.38 * Pdd + 0.35
    zeta = qd + np.sqrt(qt * qt) * alpha
    a = 1.4 * np.power(Pdd, 1.1) * np.exp(-Pdd**2)
    b = 0.9 * Pdd * np.exp(-0.5 * np.power(Pdd, 1.4))
    B, Y, E, C = _B_Y_E_C(sw, Pdd)
    rest = -0.8 * zeta * sw * C + 4.0 * sw * sw * Y + qt * qt / 10.0
    return (a * sw + b) / (2.0 * sw) * _hyperbola(zeta, rest) + E


def lam_max_star5(qs, sigma_bar):
    """Baradaran's dimensionless maximum wave speed of the 5-moment system."""
    sw = np.minimum(sigma_bar, 1.0)
    B, Y, E, C = _B_Y_E_C(sw, 1.0)
    rest = -0.8 * qs * sw * C + 4.0 * sw * sw * Y
    return _hyperbola(qs, rest) / (2.0 * sw) + E


def wavespeeds14(W, sigma_lim, d, k=1.0):
    """(lambda_min, lambda_max) along axis d in {0,1,2} for 14-moment primitive states W.
    sigma_bar is that of the same state (the closure's limited mapping parameter)."""
    W = np.asarray(W, dtype=np.float64)
    rho = W[0]
    u = W[1:4]
    Pm = np.stack([[W[4], W[5], W[6]], [W[5], W[7], W[8]], [W[6], W[8], W[9]]])
    q = W[10:13]
    R = W[13]
    p = (Pm[0, 0] + Pm[1, 1] + Pm[2, 2]) / 3.0
    c = np.sqrt(p / rho)
    Ps = np.moveaxis(np.moveaxis(Pm / p, 0, -1), 0, -1)  # (...,3,3); symmetric
    qs = np.moveaxis(q / (rho * c**3), 0, -1)
    Rs = R / (rho * c**4)
    sb = np.maximum(sigma14_star(Ps, qs, Rs), sigma_lim)
    t = [a for a in range(3) if a != d]
    qt = np.sqrt(qs[..., t[0]]**2 + qs[..., t[1]]**2)
    Pdd = Ps[..., d, d]
    lmax = u[d] + k * lam_max_star14(Pdd, qs[..., d], qt, sb) * c
    lmin = u[d] - k * lam_max_star14(Pdd, -qs[..., d], qt, sb) * c
    return lmin, lmax


def wavespeeds5(W, sigma_lim, k=1.0):
    rho, u, P, q, r = np.asarray(W, dtype=np.float64)
    c = np.sqrt(P / rho)
    qs = q / (rho * c**3)
    rs = r / (rho * c**4)
    sb = np.maximum(sigma5_star(qs, rs), sigma_lim)
    lmax = u + k * lam_max_star5(qs, sb) * c
    lmin = u - k * lam_max_star5(-qs, sb) * c
    return lmin, lmax

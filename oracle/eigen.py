"""Characteristic speeds of the closed moment systems from their flux Jacobians.

Oracle (test infrastructure only; see the package docstring).

The closed 5-moment system and the 14-moment system along a direction d read
dU/dt + dF_d(U)/dx_d = 0, with F_d closed by the interpolative closure (Section 2.3 and
Appendix A).  Their characteristic speeds are the eigenvalues of the flux Jacobian
A = dF_d/dU.  The paper fits its approximate wave speeds (Section 5.1, Appendix B) to the
extreme eigenvalues, computed numerically (Appendix B); this module does the same, as a
diagnostic of the fits: A by central differences of U -> W -> closure -> F_d (one conserved
component perturbed at a time, by h times that component's natural scale rho c^n, where n
is the component's velocity order), then ``numpy.linalg.eigvals``.

The system is hyperbolic where every eigenvalue is real; the imaginary parts are returned
so that a caller can check that.
"""
import numpy as np

from .closure import closure5, closure14
from .fluxes import flux5, flux14
from .moments import cons_to_prim5, cons_to_prim14, prim_to_cons5, prim_to_cons14, pressure14

# velocity order of each conserved component: rho; rho u_i; E_ij; F_i; G
_ORDER14 = np.array([0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 4])
_ORDER5 = np.array([0, 1, 2, 3, 4])


def closed_flux14(U, d, sigma_lim):
    """F_d of conserved 14-moment states U (14, ...)."""
    W = cons_to_prim14(U)
    Q, Rt, S, _ = closure14(W, sigma_lim)
    return flux14(W, Q, Rt, S, d)


def closed_flux5(U, sigma_lim):
    W = cons_to_prim5(U)
    s, _ = closure5(W, sigma_lim)
    return flux5(W, s)


def _jacobian(flux, U, scales, h):
    """Central-difference Jacobian of flux at the states U (n, N): returns (N, n, n)."""
    n, N = U.shape
    A = np.empty((N, n, n))
    for j in range(n):
        dU = np.zeros_like(U)
        dU[j] = h * scales[j]
        Fp = flux(U + dU)
        Fm = flux(U - dU)
        A[:, :, j] = ((Fp - Fm) / (2.0 * h * scales[j])).T
    return A


def jacobian14(W, d, sigma_lim, h=1e-5):
    """dF_d/dU of 14-moment primitive states W (14, N); (N, 14, 14)."""
    W = np.asarray(W, dtype=np.float64).reshape(14, -1)
    U = prim_to_cons14(W)
    rho = W[0]
    c = np.sqrt(pressure14(W) / rho)
    scales = rho[None, :] * c[None, :] ** _ORDER14[:, None]
    return _jacobian(lambda V: closed_flux14(V, d, sigma_lim), U, scales, h)


def jacobian5(W, sigma_lim, h=1e-5):
    """dF/dU of 5-moment primitive states W (5, N); (N, 5, 5)."""
    W = np.asarray(W, dtype=np.float64).reshape(5, -1)
    U = prim_to_cons5(W)
    rho = W[0]
    c = np.sqrt(W[2] / rho)
    scales = rho[None, :] * c[None, :] ** _ORDER5[:, None]
    return _jacobian(lambda V: closed_flux5(V, sigma_lim), U, scales, h)


def _extremes(A):
    ev = np.linalg.eigvals(A)
    return ev.real.min(axis=-1), ev.real.max(axis=-1), np.abs(ev.imag).max(axis=-1), ev


def eigen_speeds14(W, d, sigma_lim, h=1e-5):
    """(lambda_min, lambda_max, max |imaginary part|, all eigenvalues) of the 14-moment flux
    Jacobian along d at each state of W (14, N)."""
    return _extremes(jacobian14(W, d, sigma_lim, h))


def eigen_speeds5(W, sigma_lim, h=1e-5):
    """(lambda_min, lambda_max, max |imaginary part|, all eigenvalues) of the 5-moment flux
    Jacobian at each state of W (5, N)."""
    return _extremes(jacobian5(W, sigma_lim, h))


def state5_from_star(qs, sigma, rho=1.0, u=0.0, P=1.0):
    """5-moment primitive states with given dimensionless heat flux q* and mapping parameter
    sigma: r* follows from the sigma mapping's quadratic 2 sigma^2 - (3 - r*) sigma - q*^2 = 0
    (eq. sigma-mapping-5mom)."""
    qs = np.asarray(qs, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    rs = 3.0 - (2.0 * sigma**2 - qs**2) / sigma
    c = np.sqrt(P / rho)
    z = np.zeros(np.broadcast(qs, sigma).shape)
    return np.stack([rho + z, u + z, P + z, qs * rho * c**3 + z, rs * rho * c**4 + z], 0)


def state14_from_star(Pxx, qx, qy, sigma, rho=1.0, p=1.0):
    """14-moment primitive states in the reduced variables of Appendix B.2: at rest, P* =
    diag(P*_xx, (3 - P*_xx)/2, (3 - P*_xx)/2), q* = (q*_x, q*_y, 0), and R* from the sigma
    mapping's quadratic 2 t2 sigma^2 - A sigma - D = 0 with A = 2 t2 + t1^2 - R*, t1 = 3,
    t2 = tr P*^2, D = q*.P*^-1.q* (eq. sigma-mapping-14mom)."""
    Pxx, qx, qy, sigma = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64)
                                               for a in (Pxx, qx, qy, sigma)])
    Pt = 0.5 * (3.0 - Pxx)
    t2 = Pxx**2 + 2.0 * Pt**2
    D = qx**2 / Pxx + qy**2 / Pt
    A = (2.0 * t2 * sigma**2 - D) / sigma
    Rs = 2.0 * t2 + 9.0 - A
    c = np.sqrt(p / rho)
    z = np.zeros_like(Pxx)
    s3, s4 = rho * c**3, rho * c**4
    return np.stack([rho + z, z, z, z, p * Pxx, z, z, p * Pt, z, p * Pt,
                     qx * s3, qy * s3, z, Rs * s4], 0)

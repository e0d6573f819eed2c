"""Interpolative maximum-entropy closure with sigma limiting.

Oracle (test infrastructure only; see the package docstring).

5-moment: parabolic mapping (eq. sigma-mapping-5mom) and closing moment
(eq. closure-1D1V-s-approx, with the square-root exponent the paper adopts).
14-moment: parabolic mapping (eq. sigma-mapping-14mom) and closing moments Q_ijk, R_ijkk,
S_ijjkk (eqs. closure-14mom-Qijk-approx, -Rijkk-approx, -Sijjkk-approx, with the auxiliary
tensors B, K, W printed right after them).

Both are evaluated in the dimensionless variables of eq. dimensionless-variables
(rho* = 1, scaling by rho and sqrt(p/rho)) and re-dimensionalised afterwards, as Section 3.3
recommends.  sigma_bar = max(sigma, sigma_lim) replaces sigma everywhere in the closing
formulas (Section 2.3 and Appendix A); the stored state is never modified.

Reading (the paper is silent): the square-root form of sigma cancels catastrophically when
its bracket A is negative, i.e. close to the Junk subspace.  For A < 0 the algebraically
identical rationalised form  sigma = 2 D / (sqrt(X) - A)  (14-moment; 2 q*^2/(sqrt(X) - A) for
5 moments) is used.  The 50-digit check in tests compares both forms to the printed one.
"""
import numpy as np

from .moments import split14


def _sigma_from_quadratic(A, X, num_small, denom_big):
    """Positive root of the mapping quadratic, cancellation-free.
    A >= 0: (A + sqrt X) / denom_big;  A < 0: num_small / (sqrt X - A)."""
    sX = np.sqrt(X)
    with np.errstate(divide='ignore', invalid='ignore'):
        s_pos = (A + sX) / denom_big
        s_neg = num_small / (sX - A)
    return np.where(A >= 0.0, s_pos, s_neg)


def sigma5_star(qs, rs):
    """eq. sigma-mapping-5mom in dimensionless variables q*, r*."""
    A = 3.0 - rs
    X = A * A + 8.0 * qs * qs
    return _sigma_from_quadratic(A, X, 2.0 * qs * qs, 4.0)


def closure5(W, sigma_lim):
    """Closing moment s of the 5-moment system.

    W = [rho, u, P, q, r] on axis 0.  Returns (s, sigma) with sigma the unlimited mapping
    parameter.  Dimensionless: c = sqrt(P/rho), q* = q/(rho c^3), r* = r/(rho c^4);
    s* = q*^3/sigma_bar^2 + (10 - 8 sigma_bar^(1/2)) q*; s = s* rho c^5.
    """
    rho, u, P, q, r = np.asarray(W, dtype=np.float64)
    c = np.sqrt(P / rho)
    qs = q / (rho * c**3)
    rs = r / (rho * c**4)
    sig = sigma5_star(qs, rs)
    sb = np.maximum(sig, sigma_lim)
    ss = qs**3 / sb**2 + (10.0 - 8.0 * np.sqrt(sb)) * qs
    return ss * rho * c**5, sig


def _tr(M):
    return np.einsum('...ii->...', M)


def nondim14(W):
    """Dimensionless 14-moment state (eq. dimensionless-variables, rho* = 1):
    returns (rho, u, p, c, P*, q*, R*)."""
    rho, u, P, q, R = split14(W)
    p = _tr(P) / 3.0
    c = np.sqrt(p / rho)
    Ps = P / p[..., None, None]
    qs = q / (rho * c**3)[..., None]
    Rs = R / (rho * c**4)
    return rho, u, p, c, Ps, qs, Rs


def sigma14_star(Ps, qs, Rs):
    """eq. sigma-mapping-14mom with rho* = 1:
    sigma = [2 tr(P^2) + (tr P)^2 - R + sqrt((...)^2 + 8 tr(P^2) q.P^-1.q)] / (4 tr(P^2))."""
    P2 = Ps @ Ps
    t1 = _tr(Ps)
    t2 = _tr(P2)
    Pinv = np.linalg.inv(Ps)
    D = np.einsum('...k,...kl,...l->...', qs, Pinv, qs)
    A = 2.0 * t2 + t1 * t1 - Rs
    X = A * A + 8.0 * t2 * D
    return _sigma_from_quadratic(A, X, 2.0 * D, 4.0 * t2)


def closure14_star(Ps, qs, Rs, sigma_lim):
    """Dimensionless closing moments Q*_ijk (3,3,3), R*_ijkk (3,3), S*_ijjkk (3) and sigma.

    Direct transcription of the closure tensors with rho* = 1:
      B_lm   = 2 P_lm (P^2)_aa + 4 (P^3)_lm
      K_ijkm = [2 P_il (P^2)_jk + 2 P_kl (P^2)_ij + 2 P_jl (P^2)_ik] B^-1_lm
      Q_ijk  = K_ijkm q_m
      R_ijkk = Q_ijl P^-1_lm q_m / sigma_bar + 2 (1 - sigma_bar) (P^2)_ij + P_ij P_kk
      W_im   = [2 P_il P_aa^3 + 12 P_il (P^3)_aa + 14 (P^2)_aa (P^2)_il + 20 P_aa (P^3)_il
                + 20 (P^4)_il - 2 (P^2)_aa P_bb P_il - 6 P_aa^2 (P^2)_il] B^-1_lm
      S_i    = P^-1_kn P^-1_lm q_n q_m Q_ikl / sigma_bar^2 + 2 sigma_bar^(1/2) P_jj q_i
               + (1 - sigma_bar^(1/2)) W_im q_m
    """
    sig = sigma14_star(Ps, qs, Rs)
    sb = np.maximum(sig, sigma_lim)
    P2 = Ps @ Ps
    P3 = P2 @ Ps
    P4 = P2 @ P2
    t1 = _tr(Ps)
    t2 = _tr(P2)
    t3 = _tr(P3)
    Pinv = np.linalg.inv(Ps)
    B = 2.0 * Ps * t2[..., None, None] + 4.0 * P3
    Binv = np.linalg.inv(B)
    K = (2.0 * np.einsum('...il,...jk,...lm->...ijkm', Ps, P2, Binv)
         + 2.0 * np.einsum('...kl,...ij,...lm->...ijkm', Ps, P2, Binv)
         + 2.0 * np.einsum('...jl,...ik,...lm->...ijkm', Ps, P2, Binv))
    Q = np.einsum('...ijkm,...m->...ijk', K, qs)
    Rt = (np.einsum('...ijl,...lm,...m->...ij', Q, Pinv, qs) / sb[..., None, None]
          + 2.0 * (1.0 - sb)[..., None, None] * P2 + Ps * t1[..., None, None])
    e = lambda s: s[..., None, None]  # noqa: E731
    Mbr = (2.0 * Ps * e(t1**3) + 12.0 * Ps * e(t3) + 14.0 * e(t2) * P2 + 20.0 * e(t1) * P3
           + 20.0 * P4 - 2.0 * e(t2 * t1) * Ps - 6.0 * e(t1**2) * P2)
    Wm = Mbr @ Binv
    S = (np.einsum('...kn,...lm,...n,...m,...ikl->...i', Pinv, Pinv, qs, qs, Q) / (sb**2)[..., None]
         + 2.0 * (np.sqrt(sb) * t1)[..., None] * qs
         + (1.0 - np.sqrt(sb))[..., None] * np.einsum('...im,...m->...i', Wm, qs))
    return Q, Rt, S, sig


def closure14(W, sigma_lim):
    """Dimensional closing moments of a 14-moment primitive state W (axis 0 = components).
    Returns (Q (...,3,3,3), R_ijkk (...,3,3), S (...,3), sigma)."""
    rho, u, p, c, Ps, qs, Rs = nondim14(W)
    Qs, Rts, Ss, sig = closure14_star(Ps, qs, Rs, sigma_lim)
    s3 = rho * c**3
    s4 = rho * c**4
    s5 = rho * c**5
    return (Qs * s3[..., None, None, None], Rts * s4[..., None, None],
            Ss * s5[..., None], sig)

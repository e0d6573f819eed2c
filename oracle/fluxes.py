"""Physical fluxes, BGK sources, collision time and the HLL / Rusanov interface fluxes.

Oracle (test infrastructure only; see the package docstring).

Physical fluxes are the divergence arguments of the moment equations: eq.
ch-theory-5mom-sys-eqs (5 moments) and the 14-moment equations of Section 2.4, written for a
general direction index k with the closing moments Q_ijk, R_ikjj and S_kiijj supplied by the
closure.  BGK sources: right-hand sides of the same equations (C_1, C_i, C_ij, C_ijj,
C_iijj), evaluated with a local collision time.  Interface fluxes: Section 3.1 (HLL and the
Rusanov / local Lax-Friedrichs flux).
"""
import numpy as np

from .moments import split14, join14, mat_to_sym, prim_to_cons14, prim_to_cons5
from .closure import closure14, closure5


def flux14(W, Q, Rt, S, k):
    """Flux along direction k of the 14 conserved moments (Section 2.4), primitive state W,
    closing moments Q (...,3,3,3), Rt = R_ikjj (...,3,3), S = S_kiijj (...,3)."""
    rho, u, P, q, R = split14(W)
    uk = u[..., k]
    uu = np.einsum('...i,...i->...', u, u)
    trP = np.einsum('...jj->...', P)
    Pk = P[..., :, k]                                   # P_ik
    uPk = np.einsum('...j,...j->...', u, Pk)            # u_j P_jk
    Pu = np.einsum('...ij,...j->...i', P, u)            # u_j P_ij
    uPu = np.einsum('...i,...i->...', u, Pu)
    uq = np.einsum('...i,...i->...', u, q)
    Qk = Q[..., :, :, k]                                # Q_ijk
    uQk = np.einsum('...j,...ij->...i', u, Qk)          # u_j Q_ijk
    uuQk = np.einsum('...i,...i->...', u, uQk)          # u_i u_j Q_ijk
    Rk = Rt[..., :, k]                                  # R_ikjj
    uRk = np.einsum('...i,...i->...', u, Rk)
    e = lambda a: a[..., None]                           # noqa: E731
    f_rho = rho * uk
    f_mom = e(rho * uk) * u + Pk
    f_E = (e(e(rho * uk)) * np.einsum('...i,...j->...ij', u, u)
           + np.einsum('...i,...j->...ij', u, Pk) + np.einsum('...j,...i->...ij', u, Pk)
           + e(e(uk)) * P + Qk)
    f_F = (e(rho * uk * uu) * u + e(uk * trP) * u + 2.0 * e(uPk) * u + 2.0 * e(uk) * Pu
           + e(uu) * Pk + u * e(q[..., k]) + e(uk) * q + 2.0 * uQk + Rk)
    f_G = (rho * uk * uu * uu + 2.0 * uk * uu * trP + 4.0 * uu * uPk + 4.0 * uk * uPu
           + 2.0 * uu * q[..., k] + 4.0 * uk * uq + 4.0 * uuQk + 4.0 * uRk
           + uk * R + S[..., k])
    return np.concatenate([f_rho[None], np.moveaxis(f_mom, -1, 0), mat_to_sym(f_E),
                           np.moveaxis(f_F, -1, 0), f_G[None]], 0)


def flux5(W, s):
    """eq. ch-theory-5mom-sys-eqs divergence terms."""
    rho, u, P, q, r = np.asarray(W, dtype=np.float64)
    return np.stack([rho * u,
                     rho * u**2 + P,
                     rho * u**3 + 3.0 * u * P + q,
                     rho * u**4 + 6.0 * u**2 * P + 4.0 * u * q + r,
                     rho * u**5 + 10.0 * u**3 * P + 10.0 * u**2 * q + 5.0 * u * r + s], 0)


def tau_local(rho, T, tau_ref, rho_ref, T_ref):
    """Collision time tau = (n sigma v_th)^-1 with v_th ~ sqrt(T) (Section 4), scaled from a
    reference state: tau = tau_ref (rho_ref/rho) sqrt(T_ref/T)."""
    return tau_ref * (rho_ref / rho) * np.sqrt(T_ref / T)


def source14(W, tau):
    """BGK relaxation sources of the 14-moment system (Section 2.4):
    C_1 = C_i = 0, C_ij = -(P_ij - p d_ij)/tau, C_ijj = -(2 u_j P_ij + q_i - 2 u_i p)/tau,
    C_iijj = -[(4 u_i u_j P_ij + 4 u_i q_i + R) - (4 |u|^2 p + 15 p^2/rho)]/tau."""
    rho, u, P, q, R = split14(W)
    p = np.einsum('...ii->...', P) / 3.0
    Pu = np.einsum('...ij,...j->...i', P, u)
    uPu = np.einsum('...i,...i->...', u, Pu)
    uq = np.einsum('...i,...i->...', u, q)
    uu = np.einsum('...i,...i->...', u, u)
    z = np.zeros_like(rho)
    tau = np.asarray(tau, dtype=np.float64) + z
    CE = -(P - p[..., None, None] * np.eye(3)) / tau[..., None, None]
    CF = -(2.0 * Pu + q - 2.0 * u * p[..., None]) / tau[..., None]
    CG = -((4.0 * uPu + 4.0 * uq + R) - (4.0 * uu * p + 15.0 * p * p / rho)) / tau
    return np.concatenate([z[None], z[None], z[None], z[None], mat_to_sym(CE),
                           np.moveaxis(CF, -1, 0), CG[None]], 0)


def source5(W, tau):
    """eq. ch-theory-5mom-sys-eqs right-hand sides: [0, 0, 0, -q/tau, -(4uq + r - 3P^2/rho)/tau]."""
    rho, u, P, q, r = np.asarray(W, dtype=np.float64)
    z = np.zeros_like(rho)
    return np.stack([z, z, z, -q / tau, -(4.0 * u * q + r - 3.0 * P * P / rho) / tau], 0)


def state_flux14(W, k, sigma_lim):
    """(U, F_k, sigma) of 14-moment primitive states, closing moments from the closure."""
    Q, Rt, S, sig = closure14(W, sigma_lim)
    return prim_to_cons14(W), flux14(W, Q, Rt, S, k), sig


def state_flux5(W, sigma_lim):
    s, sig = closure5(W, sigma_lim)
    return prim_to_cons5(W), flux5(W, s), sig


def hll(FL, FR, UL, UR, SL, SR):
    """HLL flux: F_L if S_L >= 0, F_R if S_R <= 0, else
    (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L)."""
    with np.errstate(divide='ignore', invalid='ignore'):
        mid = (SR * FL - SL * FR + SL * SR * (UR - UL)) / (SR - SL)
    return np.where(SL >= 0.0, FL, np.where(SR <= 0.0, FR, mid))


def rusanov(FL, FR, UL, UR, amax):
    """Local Lax-Friedrichs: 0.5 (F_L + F_R) - 0.5 a* (U_R - U_L)."""
    return 0.5 * (FL + FR) - 0.5 * amax * (UR - UL)


def davis_speeds(lminL, lmaxL, lminR, lmaxR):
    """Reading: HLL signal speeds are the extremes over both reconstructed face states."""
    return np.minimum(lminL, lminR), np.maximum(lmaxL, lmaxR)


# keep join14 importable from here for the problem set-ups
__all__ = ['flux14', 'flux5', 'tau_local', 'source14', 'source5', 'state_flux14',
           'state_flux5', 'hll', 'rusanov', 'davis_speeds', 'join14']

"""Primitive <-> conserved maps of the 5- and 14-moment systems.

Oracle (test infrastructure only; see the package docstring).

Component order
  14-moment primitives  W = [rho, u_x, u_y, u_z, P_xx, P_xy, P_xz, P_yy, P_yz, P_zz, q_x, q_y, q_z, R]
  14-moment conserved   U = [rho, rho u_i (3), E_ij = rho u_i u_j + P_ij (6, same order as P),
                             F_i (3), G]
  5-moment primitives   W = [rho, u, P, q, r]
  5-moment conserved    U = [rho, rho u, rho u^2 + P, rho u^3 + 3uP + q, rho u^4 + 6u^2P + 4uq + r]

The conserved quantities are the time-derivative arguments of the moment equations:
Section 2.3 (system of five balance laws, eq. ch-theory-5mom-sys-eqs) and Section 2.4 (the
14-moment equations, with q_i = Q_ijj and R = R_iijj).  Arrays carry the components on
axis 0; any trailing shape is a batch of cells.
"""
import numpy as np

NV5 = 5
NV14 = 14

# (i, j) index of each stored symmetric-tensor component, in storage order
SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def sym_to_mat(c6):
    """6 stored components (axis 0) -> (..., 3, 3) symmetric matrix."""
    xx, xy, xz, yy, yz, zz = c6
    return np.stack([np.stack([xx, xy, xz], -1),
                     np.stack([xy, yy, yz], -1),
                     np.stack([xz, yz, zz], -1)], -2)


def mat_to_sym(M):
    """(..., 3, 3) symmetric matrix -> 6 stored components on axis 0."""
    return np.stack([M[..., i, j] for (i, j) in SYM], 0)


def split14(W):
    """Unpack 14 primitives into rho (...), u (...,3), P (...,3,3), q (...,3), R (...)."""
    W = np.asarray(W, dtype=np.float64)
    rho = W[0]
    u = np.moveaxis(W[1:4], 0, -1)
    P = sym_to_mat(W[4:10])
    q = np.moveaxis(W[10:13], 0, -1)
    R = W[13]
    return rho, u, P, q, R


def join14(rho, u, P, q, R):
    return np.concatenate([rho[None], np.moveaxis(u, -1, 0), mat_to_sym(P),
                           np.moveaxis(q, -1, 0), R[None]], 0)


def prim_to_cons14(W):
    """Conserved 14-moment vector from primitives: the time-derivative terms of the
    14-moment equations (Section 2.4), with Q_ijj = q_i and R_iijj = R."""
    rho, u, P, q, R = split14(W)
    uu = np.einsum('...i,...i->...', u, u)
    trP = np.einsum('...ii->...', P)
    Pu = np.einsum('...ij,...j->...i', P, u)
    uPu = np.einsum('...i,...i->...', u, Pu)
    uq = np.einsum('...i,...i->...', u, q)
    E = rho[..., None, None] * np.einsum('...i,...j->...ij', u, u) + P
    F = (rho * uu)[..., None] * u + trP[..., None] * u + 2.0 * Pu + q
    G = rho * uu * uu + 2.0 * uu * trP + 4.0 * uPu + 4.0 * uq + R
    return np.concatenate([rho[None], np.moveaxis(rho[..., None] * u, -1, 0),
                           mat_to_sym(E), np.moveaxis(F, -1, 0), G[None]], 0)


def cons_to_prim14(U):
    """Inverse of prim_to_cons14: u, then P, then q, then R (each uses the previous)."""
    U = np.asarray(U, dtype=np.float64)
    rho = U[0]
    u = np.moveaxis(U[1:4], 0, -1) / rho[..., None]
    E = sym_to_mat(U[4:10])
    P = E - rho[..., None, None] * np.einsum('...i,...j->...ij', u, u)
    uu = np.einsum('...i,...i->...', u, u)
    trP = np.einsum('...ii->...', P)
    Pu = np.einsum('...ij,...j->...i', P, u)
    F = np.moveaxis(U[10:13], 0, -1)
    q = F - (rho * uu)[..., None] * u - trP[..., None] * u - 2.0 * Pu
    uPu = np.einsum('...i,...i->...', u, Pu)
    uq = np.einsum('...i,...i->...', u, q)
    R = U[13] - rho * uu * uu - 2.0 * uu * trP - 4.0 * uPu - 4.0 * uq
    return join14(rho, u, P, q, R)


def prim_to_cons5(W):
    """Conserved 5-moment vector: time-derivative terms of eq. ch-theory-5mom-sys-eqs."""
    rho, u, P, q, r = np.asarray(W, dtype=np.float64)
    return np.stack([rho,
                     rho * u,
                     rho * u**2 + P,
                     rho * u**3 + 3.0 * u * P + q,
                     rho * u**4 + 6.0 * u**2 * P + 4.0 * u * q + r], 0)


def cons_to_prim5(U):
    U = np.asarray(U, dtype=np.float64)
    rho = U[0]
    u = U[1] / rho
    P = U[2] - rho * u**2
    q = U[3] - rho * u**3 - 3.0 * u * P
    r = U[4] - rho * u**4 - 6.0 * u**2 * P - 4.0 * u * q
    return np.stack([rho, u, P, q, r], 0)


def maxwellian_prim14(rho, u, p):
    """Equilibrium primitives: P = p I, q = 0, R = 15 p^2 / rho (Section 2.2)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    z = np.zeros_like(rho)
    ux, uy, uz = (u[..., 0], u[..., 1], u[..., 2])
    return np.stack([rho, ux, uy, uz, p, z, z, p, z, p, z, z, z, 15.0 * p * p / rho], 0)


def maxwellian_prim5(rho, u, P):
    """1D1V equilibrium: q = 0, r = 3 P^2 / rho (Section 2.3)."""
    rho = np.asarray(rho, dtype=np.float64)
    z = np.zeros_like(rho)
    return np.stack([rho, u + z, P + z, z, 3.0 * P * P / rho], 0)


def pressure14(W):
    """Hydrostatic pressure p = P_ii / 3."""
    W = np.asarray(W, dtype=np.float64)
    return (W[4] + W[7] + W[9]) / 3.0

"""Reference gradients of the 14-moment finite-volume step: the oracle's step transcribed
into PyTorch (CPU, float64) and differentiated by reverse-mode automatic differentiation.

Oracle (test infrastructure only; see the package docstring).  Nothing here comes from the
HIP path: every function below is the oracle function of the same name (moments, closure,
wavespeeds, fluxes, scheme), written with torch operations instead of NumPy so that autograd
can differentiate it.  The forward values equal the NumPy oracle's up to summation order
(pinned in tests/test_adjoint_ref.py, together with the gradients against the oracle's
central differences).

What is differentiated (the discrete adjoint of the explicit step, dt frozen to a given
list): J(U_0, M_jet, rho_jet, tau_ref) for a linear functional J = sum(w U_n).  The
parameters enter through the jet ghost states (M_jet, rho_jet) and the BGK source (tau_ref).

At non-smooth points the derivative of the branch the forward evaluation took is used:
  * sigma_bar = max(sigma, sigma_lim), sigma_w = min(sigma_bar, 1), P*_dd = max(P*_dd, 0):
    the strict comparison picks the first operand (a tie gives the constant, no derivative);
  * square roots of clamped arguments have no derivative where the argument is <= 0;
  * the common limiter's minimum over variables is a running minimum in component order
    starting at 1 that only a strictly smaller factor replaces (ties keep the earlier
    variable; a factor of exactly 1 carries no derivative); minmod's min(|a|, |b|) takes |b|
    at a tie; a neutral variable's factor 1 is a constant;
  * HLL's three cases, Rusanov's max of speeds and the positivity fallback follow the
    forward's choice.
frozen_limiter=True treats the common limiter factor of every cell as a constant (the
derivative of the scheme with its limiter frozen at the forward trajectory's values).
"""
import math

import torch
from torch.utils.checkpoint import checkpoint

F64 = torch.float64
SYM = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
NEUTRAL_EPS = 1e-10


# ----------------------------------------------------------------------------- helpers
class _SafeSqrt(torch.autograd.Function):
    """sqrt(max(x, 0)); the derivative is 1 / (2 sqrt x) where x > 0 and 0 elsewhere."""

    @staticmethod
    def forward(ctx, x):
        y = torch.sqrt(torch.clamp(x, min=0.0))
        ctx.save_for_backward(x, y)
        return y

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        pos = x > 0.0
        return torch.where(pos, g * 0.5 / torch.where(pos, y, torch.ones_like(y)),
                           torch.zeros_like(g))


def ssqrt(x):
    return _SafeSqrt.apply(x)


def tmax(a, b):
    """max with the first operand on strict '>' (the second at a tie)."""
    a, b = torch.broadcast_tensors(torch.as_tensor(a, dtype=F64), torch.as_tensor(b, dtype=F64))
    return torch.where(a > b, a, b)


def tmin(a, b):
    """min with the first operand on strict '<' (the second at a tie)."""
    a, b = torch.broadcast_tensors(torch.as_tensor(a, dtype=F64), torch.as_tensor(b, dtype=F64))
    return torch.where(a < b, a, b)


def safe_div(num, den, use):
    """num / den where `use`, 0 elsewhere, without non-finite values in either branch."""
    return torch.where(use, num / torch.where(use, den, torch.ones_like(den)),
                       torch.zeros_like(num))


def tr(M):
    return torch.einsum('...ii->...', M)


# ----------------------------------------------------------------------------- moments
def sym_to_mat(c6):
    xx, xy, xz, yy, yz, zz = c6
    return torch.stack([torch.stack([xx, xy, xz], -1),
                        torch.stack([xy, yy, yz], -1),
                        torch.stack([xz, yz, zz], -1)], -2)


def mat_to_sym(M):
    return torch.stack([M[..., i, j] for (i, j) in SYM], 0)


def split14(W):
    rho = W[0]
    u = torch.movedim(W[1:4], 0, -1)
    P = sym_to_mat(W[4:10])
    q = torch.movedim(W[10:13], 0, -1)
    R = W[13]
    return rho, u, P, q, R


def join14(rho, u, P, q, R):
    return torch.cat([rho[None], torch.movedim(u, -1, 0), mat_to_sym(P),
                      torch.movedim(q, -1, 0), R[None]], 0)


def prim_to_cons14(W):
    rho, u, P, q, R = split14(W)
    uu = torch.einsum('...i,...i->...', u, u)
    trP = tr(P)
    Pu = torch.einsum('...ij,...j->...i', P, u)
    uPu = torch.einsum('...i,...i->...', u, Pu)
    uq = torch.einsum('...i,...i->...', u, q)
    E = rho[..., None, None] * torch.einsum('...i,...j->...ij', u, u) + P
    F = (rho * uu)[..., None] * u + trP[..., None] * u + 2.0 * Pu + q
    G = rho * uu * uu + 2.0 * uu * trP + 4.0 * uPu + 4.0 * uq + R
    return torch.cat([rho[None], torch.movedim(rho[..., None] * u, -1, 0), mat_to_sym(E),
                      torch.movedim(F, -1, 0), G[None]], 0)


def cons_to_prim14(U):
    rho = U[0]
    u = torch.movedim(U[1:4], 0, -1) / rho[..., None]
    E = sym_to_mat(U[4:10])
    P = E - rho[..., None, None] * torch.einsum('...i,...j->...ij', u, u)
    uu = torch.einsum('...i,...i->...', u, u)
    trP = tr(P)
    Pu = torch.einsum('...ij,...j->...i', P, u)
    F = torch.movedim(U[10:13], 0, -1)
    q = F - (rho * uu)[..., None] * u - trP[..., None] * u - 2.0 * Pu
    uPu = torch.einsum('...i,...i->...', u, Pu)
    uq = torch.einsum('...i,...i->...', u, q)
    R = U[13] - rho * uu * uu - 2.0 * uu * trP - 4.0 * uPu - 4.0 * uq
    return join14(rho, u, P, q, R)


def maxwellian_prim14(rho, u, p):
    z = torch.zeros_like(rho)
    return torch.stack([rho, u[0], u[1], u[2], p, z, z, p, z, p, z, z, z, 15.0 * p * p / rho], 0)


# ----------------------------------------------------------------------------- closure
def sigma_from_quadratic(A, X, num_small, denom_big):
    sX = ssqrt(X)
    pos = A >= 0.0
    s_pos = (A + sX) / denom_big
    s_neg = safe_div(num_small, sX - A, ~pos)
    return torch.where(pos, s_pos, s_neg)


def nondim14(W):
    rho, u, P, q, R = split14(W)
    p = tr(P) / 3.0
    c = torch.sqrt(p / rho)
    Ps = P / p[..., None, None]
    qs = q / (rho * c**3)[..., None]
    Rs = R / (rho * c**4)
    return rho, u, p, c, Ps, qs, Rs


def sigma14_star(Ps, qs, Rs):
    P2 = Ps @ Ps
    t1 = tr(Ps)
    t2 = tr(P2)
    Pinv = torch.linalg.inv(Ps)
    D = torch.einsum('...k,...kl,...l->...', qs, Pinv, qs)
    A = 2.0 * t2 + t1 * t1 - Rs
    X = A * A + 8.0 * t2 * D
    return sigma_from_quadratic(A, X, 2.0 * D, 4.0 * t2)


def closure14_star(Ps, qs, Rs, sigma_lim):
    sig = sigma14_star(Ps, qs, Rs)
    sb = tmax(sig, sigma_lim)
    P2 = Ps @ Ps
    P3 = P2 @ Ps
    P4 = P2 @ P2
    t1 = tr(Ps)
    t2 = tr(P2)
    t3 = tr(P3)
    Pinv = torch.linalg.inv(Ps)
    B = 2.0 * Ps * t2[..., None, None] + 4.0 * P3
    Binv = torch.linalg.inv(B)
    K = (2.0 * torch.einsum('...il,...jk,...lm->...ijkm', Ps, P2, Binv)
         + 2.0 * torch.einsum('...kl,...ij,...lm->...ijkm', Ps, P2, Binv)
         + 2.0 * torch.einsum('...jl,...ik,...lm->...ijkm', Ps, P2, Binv))
    Q = torch.einsum('...ijkm,...m->...ijk', K, qs)
    Rt = (torch.einsum('...ijl,...lm,...m->...ij', Q, Pinv, qs) / sb[..., None, None]
          + 2.0 * (1.0 - sb)[..., None, None] * P2 + Ps * t1[..., None, None])

    def e(s):
        return s[..., None, None]

    Mbr = (2.0 * Ps * e(t1**3) + 12.0 * Ps * e(t3) + 14.0 * e(t2) * P2 + 20.0 * e(t1) * P3
           + 20.0 * P4 - 2.0 * e(t2 * t1) * Ps - 6.0 * e(t1**2) * P2)
    Wm = Mbr @ Binv
    S = (torch.einsum('...kn,...lm,...n,...m,...ikl->...i', Pinv, Pinv, qs, qs, Q) / (sb**2)[..., None]
         + 2.0 * (torch.sqrt(sb) * t1)[..., None] * qs
         + (1.0 - torch.sqrt(sb))[..., None] * torch.einsum('...im,...m->...i', Wm, qs))
    return Q, Rt, S, sig


def closure14(W, sigma_lim):
    rho, u, p, c, Ps, qs, Rs = nondim14(W)
    Qs, Rts, Ss, sig = closure14_star(Ps, qs, Rs, sigma_lim)
    s3 = rho * c**3
    s4 = rho * c**4
    s5 = rho * c**5
    return (Qs * s3[..., None, None, None], Rts * s4[..., None, None], Ss * s5[..., None], sig)


# ----------------------------------------------------------------------------- wave speeds
def hyperbola(zeta, rest):
    """zeta + sqrt(max(0, zeta^2 + rest)) without cancellation."""
    X = zeta * zeta + rest
    sX = ssqrt(X)
    nonneg = zeta >= 0.0
    out = torch.where(nonneg, zeta + sX, safe_div(rest, sX - zeta, ~nonneg))
    return torch.where(X <= 0.0, zeta, out)


def B_Y_E_C(sw, Pdd):
    C = ssqrt((3.0 - 3.0 * sw) * Pdd)
    E = 0.8 * C
    rs = torch.sqrt(sw)
    B = 5.0 - 4.0 * rs + ssqrt(10.0 - 16.0 * rs + 6.0 * sw)
    Y = B + E * E - 2.0 * E * torch.sqrt(B)
    return B, Y, E, C


def _pow_pos(x, a):
    """x^a for x >= 0 with x^a = 0 (and no derivative) at x = 0."""
    pos = x > 0.0
    return torch.where(pos, torch.pow(torch.where(pos, x, torch.ones_like(x)), a),
                       torch.zeros_like(x))


def lam_max_star14(Pdd, qd, qt, sigma_bar):
    sw = tmin(sigma_bar, 1.0)
    Pdd = tmax(Pdd, 0.0)
    alpha = 0.6 * Pdd**2 - 0.38 * Pdd + 0.35
    zeta = qd + ssqrt(qt * qt) * alpha
    a = 1.4 * _pow_pos(Pdd, 1.1) * torch.exp(-Pdd**2)
    b = 0.9 * Pdd * torch.exp(-0.5 * _pow_pos(Pdd, 1.4))
    B, Y, E, C = B_Y_E_C(sw, Pdd)
    rest = -0.8 * zeta * sw * C + 4.0 * sw * sw * Y + qt * qt / 10.0
    return (a * sw + b) / (2.0 * sw) * hyperbola(zeta, rest) + E


def wavespeeds14(W, sigma_lim, d, k=1.0):
    rho = W[0]
    u = W[1:4]
    Pm = [[W[4], W[5], W[6]], [W[5], W[7], W[8]], [W[6], W[8], W[9]]]
    q = W[10:13]
    R = W[13]
    p = (Pm[0][0] + Pm[1][1] + Pm[2][2]) / 3.0
    c = torch.sqrt(p / rho)
    Ps = torch.stack([torch.stack([Pm[i][j] / p for j in range(3)], -1) for i in range(3)], -2)
    qs = torch.movedim(q / (rho * c**3), 0, -1)
    Rs = R / (rho * c**4)
    sb = tmax(sigma14_star(Ps, qs, Rs), sigma_lim)
    t = [a for a in range(3) if a != d]
    qt = ssqrt(qs[..., t[0]]**2 + qs[..., t[1]]**2)
    Pdd = Ps[..., d, d]
    lmax = u[d] + k * lam_max_star14(Pdd, qs[..., d], qt, sb) * c
    lmin = u[d] - k * lam_max_star14(Pdd, -qs[..., d], qt, sb) * c
    return lmin, lmax


# ----------------------------------------------------------------------------- fluxes
def flux14(W, Q, Rt, S, k):
    rho, u, P, q, R = split14(W)
    uk = u[..., k]
    uu = torch.einsum('...i,...i->...', u, u)
    trP = tr(P)
    Pk = P[..., :, k]
    uPk = torch.einsum('...j,...j->...', u, Pk)
    Pu = torch.einsum('...ij,...j->...i', P, u)
    uPu = torch.einsum('...i,...i->...', u, Pu)
    uq = torch.einsum('...i,...i->...', u, q)
    Qk = Q[..., :, :, k]
    uQk = torch.einsum('...j,...ij->...i', u, Qk)
    uuQk = torch.einsum('...i,...i->...', u, uQk)
    Rk = Rt[..., :, k]
    uRk = torch.einsum('...i,...i->...', u, Rk)

    def e(a):
        return a[..., None]

    f_rho = rho * uk
    f_mom = e(rho * uk) * u + Pk
    f_E = (e(e(rho * uk)) * torch.einsum('...i,...j->...ij', u, u)
           + torch.einsum('...i,...j->...ij', u, Pk) + torch.einsum('...j,...i->...ij', u, Pk)
           + e(e(uk)) * P + Qk)
    f_F = (e(rho * uk * uu) * u + e(uk * trP) * u + 2.0 * e(uPk) * u + 2.0 * e(uk) * Pu
           + e(uu) * Pk + u * e(q[..., k]) + e(uk) * q + 2.0 * uQk + Rk)
    f_G = (rho * uk * uu * uu + 2.0 * uk * uu * trP + 4.0 * uu * uPk + 4.0 * uk * uPu
           + 2.0 * uu * q[..., k] + 4.0 * uk * uq + 4.0 * uuQk + 4.0 * uRk
           + uk * R + S[..., k])
    return torch.cat([f_rho[None], torch.movedim(f_mom, -1, 0), mat_to_sym(f_E),
                      torch.movedim(f_F, -1, 0), f_G[None]], 0)


def tau_local(rho, T, tau_ref, rho_ref, T_ref):
    return tau_ref * (rho_ref / rho) * torch.sqrt(T_ref / T)


def source14(W, tau):
    rho, u, P, q, R = split14(W)
    p = tr(P) / 3.0
    Pu = torch.einsum('...ij,...j->...i', P, u)
    uPu = torch.einsum('...i,...i->...', u, Pu)
    uq = torch.einsum('...i,...i->...', u, q)
    uu = torch.einsum('...i,...i->...', u, u)
    z = torch.zeros_like(rho)
    tau = tau + z
    eye = torch.eye(3, dtype=F64)
    CE = -(P - p[..., None, None] * eye) / tau[..., None, None]
    CF = -(2.0 * Pu + q - 2.0 * u * p[..., None]) / tau[..., None]
    CG = -((4.0 * uPu + 4.0 * uq + R) - (4.0 * uu * p + 15.0 * p * p / rho)) / tau
    return torch.cat([z[None], z[None], z[None], z[None], mat_to_sym(CE),
                      torch.movedim(CF, -1, 0), CG[None]], 0)


def hll(FL, FR, UL, UR, SL, SR):
    mid_used = ~(SL >= 0.0) & ~(SR <= 0.0)
    den = torch.where(mid_used, SR - SL, torch.ones_like(SR))
    mid = (SR * FL - SL * FR + SL * SR * (UR - UL)) / den
    return torch.where(SL >= 0.0, FL, torch.where(SR <= 0.0, FR, mid))


def rusanov(FL, FR, UL, UR, amax):
    return 0.5 * (FL + FR) - 0.5 * amax * (UR - UL)


# ----------------------------------------------------------------------------- scheme
class Setup:
    """The subset of the oracle's Setup the 14-moment reference needs (same names and
    defaults); jet_mach and jet_rho may be 0-d tensors that require gradients."""

    def __init__(self, dim=2, nx=16, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                 bc=('transmissive',) * 4, jets=(), jet_mach=3.0, jet_rho=1.0, jet_T=1.0,
                 tau_mode='local', rho_ref=1.0, T_ref=1.0, order=2, limiter='minmod', flux='hll',
                 integrator='ssprk2', sigma_lim=1e-4, k_ws=1.0, positivity_fallback=True,
                 frozen_limiter=False, **ignored):
        self.dim, self.nx, self.ny = dim, nx, ny
        self.x0, self.x1, self.y0, self.y1 = x0, x1, y0, y1
        self.bc = tuple(bc)
        self.jets = [tuple(j) for j in jets]
        self.jet_mach, self.jet_rho, self.jet_T = jet_mach, jet_rho, jet_T
        self.tau_mode, self.rho_ref, self.T_ref = tau_mode, rho_ref, T_ref
        self.order, self.limiter, self.flux, self.integrator = order, limiter, flux, integrator
        self.sigma_lim, self.k_ws = sigma_lim, k_ws
        self.positivity_fallback = positivity_fallback
        self.frozen_limiter = frozen_limiter

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny


def jet_prim(s, angle_deg):
    a = math.radians(angle_deg)
    mach = torch.as_tensor(s.jet_mach, dtype=F64)
    rho = torch.as_tensor(s.jet_rho, dtype=F64)
    speed = mach * math.sqrt(5.0 / 3.0 * s.jet_T)
    p = rho * s.jet_T
    return maxwellian_prim14(rho, torch.stack([speed * math.cos(a), speed * math.sin(a),
                                               torch.zeros_like(speed)]), p)


def odd_components(d):
    Po = [4 + m for m, (i, j) in enumerate(SYM) if (i == d) != (j == d)]
    return [1 + d] + Po + [10 + d]


def pad_axis(W, g, axis, lo, hi, s, wall_centres=None):
    """g ghost layers on both ends of array axis `axis` (component axis 0)."""
    n = W.shape[axis]
    d = 0 if axis == W.dim() - 1 else 1
    parts = []
    for side, kind in (('lo', lo), ('hi', hi)):
        ghost_idx = list(range(-g, 0)) if side == 'lo' else list(range(n, n + g))
        if kind == 'transmissive' or kind == 'jet':
            ix = [min(max(i, 0), n - 1) for i in ghost_idx]
            gh = W.index_select(axis, torch.tensor(ix))
        elif kind == 'periodic':
            gh = W.index_select(axis, torch.tensor([i % n for i in ghost_idx]))
        elif kind == 'reflective':
            ix = [-i - 1 if side == 'lo' else 2 * n - 1 - i for i in ghost_idx]
            gh = W.index_select(axis, torch.tensor(ix))
            sign = torch.ones(W.shape[0], dtype=F64)
            sign[odd_components(d)] = -1.0
            gh = gh * sign.reshape((-1,) + (1,) * (W.dim() - 1))
        else:
            raise ValueError(kind)
        if kind == 'jet':
            wall = 2 * d + (0 if side == 'lo' else 1)
            for jet in s.jets:
                centre, w, ang = jet[:3]
                if (jet[3] if len(jet) > 3 else 0) != wall:
                    continue
                Wj = jet_prim(s, ang)
                band = torch.as_tensor((wall_centres >= centre - 0.5 * w) &
                                       (wall_centres <= centre + 0.5 * w))
                if d == 0:      # x wall: ghosts (nv, ny, g), band over rows
                    m = band[None, :, None]
                    gh = torch.where(m, Wj[:, None, None], gh)
                else:           # y wall: ghosts (nv, g, nx), band over columns
                    m = band[None, None, :]
                    gh = torch.where(m, Wj[:, None, None], gh)
        parts.append(gh)
    return torch.cat([parts[0], W, parts[1]], axis)


def ghosted_prims(U, s, g):
    W = cons_to_prim14(U)
    if s.dim == 1:
        return pad_axis(W, g, 1, s.bc[0], s.bc[1], s)
    import numpy as np
    yc = s.y0 + (np.arange(s.ny) + 0.5) * s.dy
    xc = s.x0 + (np.arange(-g, s.nx + g) + 0.5) * s.dx
    Wx = pad_axis(W, g, 2, s.bc[0], s.bc[1], s, wall_centres=yc)
    return pad_axis(Wx, g, 1, s.bc[2], s.bc[3], s, wall_centres=xc)


def variable_scales(Wc):
    rho = torch.abs(Wc[0])
    p = torch.abs(Wc[4] + Wc[7] + Wc[9]) / 3.0
    c = torch.sqrt(p / rho)
    return torch.stack([rho, c, c, c, p, p, p, p, p, p, rho * c**3, rho * c**3, rho * c**3,
                        rho * c**4], 0)


def common_limiter(a, b, kind, scale):
    """phi = the most stringent per-variable factor (running minimum in component order,
    starting at 1, replaced only by a strictly smaller factor)."""
    neutral = (torch.abs(a) + torch.abs(b)) <= NEUTRAL_EPS * scale
    opposite = (a * b) <= 0.0
    if kind == 'minmod':
        aa, ab = torch.abs(a), torch.abs(b)
        val = safe_div(2.0 * tmin(aa, ab), aa + ab, ~neutral & ~opposite)
    elif kind == 'vanalbada':
        val = safe_div(2.0 * a * b, a * a + b * b, ~neutral & ~opposite)
    else:
        raise ValueError(kind)
    phi_v = torch.where(neutral, torch.ones_like(a), torch.where(opposite, torch.zeros_like(a), val))
    phi = torch.ones_like(a[0])
    for v in range(a.shape[0]):
        phi = torch.where(phi_v[v] < phi, phi_v[v], phi)
    return phi


def admissible(W):
    Pxx, Pxy, Pxz, Pyy, Pyz, Pzz = W[4:10]
    m2 = Pxx * Pyy - Pxy * Pxy
    m3 = (Pxx * (Pyy * Pzz - Pyz * Pyz) - Pxy * (Pxy * Pzz - Pyz * Pxz)
          + Pxz * (Pxy * Pyz - Pyy * Pxz))
    return (W[0] > 0.0) & (Pxx > 0.0) & (m2 > 0.0) & (m3 > 0.0)


def face_states(Wg, axis, g, s):
    n = Wg.shape[axis] - 2 * g

    def sl(a, b):
        return Wg.narrow(axis, a, b - a)

    if s.order == 1:
        return sl(g - 1, g + n), sl(g, g + n + 1)
    Wc = sl(g - 1, g + n + 1)
    a = Wc - sl(g - 2, g + n)
    b = sl(g, g + n + 2) - Wc
    with torch.no_grad():
        scale = variable_scales(Wc)
    phi = common_limiter(a, b, s.limiter, scale)
    if s.frozen_limiter:
        phi = phi.detach()
    slope = phi[None] * (a + b) / 2.0
    Wp = Wc + slope / 2.0
    Wm = Wc - slope / 2.0
    if s.positivity_fallback:
        with torch.no_grad():
            bad = ~(admissible(Wp) & admissible(Wm))
        Wp = torch.where(bad[None], Wc, Wp)
        Wm = torch.where(bad[None], Wc, Wm)
    return Wp.narrow(axis, 0, n + 1), Wm.narrow(axis, 1, n + 1)


def state_terms(W, d, s):
    Q, Rt, S, _ = closure14(W, s.sigma_lim)
    lmin, lmax = wavespeeds14(W, s.sigma_lim, d, s.k_ws)
    return prim_to_cons14(W), flux14(W, Q, Rt, S, d), lmin, lmax


def interface_flux(WL, WR, d, s):
    UL, FL, lminL, lmaxL = state_terms(WL, d, s)
    UR, FR, lminR, lmaxR = state_terms(WR, d, s)
    if s.flux == 'hll':
        return hll(FL, FR, UL, UR, tmin(lminL, lminR), tmax(lmaxL, lmaxR))
    if s.flux == 'rusanov':
        amax = tmax(tmax(torch.abs(lminL), torch.abs(lmaxL)), tmax(torch.abs(lminR), torch.abs(lmaxR)))
        return rusanov(FL, FR, UL, UR, amax)
    raise ValueError(s.flux)


def bgk_source(W, s, tau_ref):
    rho = W[0]
    T = (W[4] + W[7] + W[9]) / 3.0 / rho
    if s.tau_mode == 'local':
        tau = tau_local(rho, T, tau_ref, s.rho_ref, s.T_ref)
    else:
        tau = tau_ref + torch.zeros_like(rho)
    return source14(W, tau)


def residual(U, s, tau_ref):
    g = 1 if s.order == 1 else 2
    Wg = ghosted_prims(U, s, g)
    if s.dim == 1:
        WL, WR = face_states(Wg, 1, g, s)
        Fx = interface_flux(WL, WR, 0, s)
        W = Wg[:, g:-g]
        L = -(Fx[:, 1:] - Fx[:, :-1]) / s.dx
    else:
        WLx, WRx = face_states(Wg[:, g:g + s.ny, :], 2, g, s)
        WLy, WRy = face_states(Wg[:, :, g:g + s.nx], 1, g, s)
        Fx = interface_flux(WLx, WRx, 0, s)
        Fy = interface_flux(WLy, WRy, 1, s)
        W = Wg[:, g:g + s.ny, g:g + s.nx]
        L = -(Fx[:, :, 1:] - Fx[:, :, :-1]) / s.dx - (Fy[:, 1:, :] - Fy[:, :-1, :]) / s.dy
    t_ref = float(torch.as_tensor(tau_ref).detach())
    collisional = t_ref > 0.0 and math.isfinite(t_ref)
    if collisional:
        L = L + bgk_source(W, s, tau_ref)
    return L


def step(U, dt, s, tau_ref):
    L0 = residual(U, s, tau_ref)
    if s.integrator == 'fe':
        return U + dt * L0
    if s.integrator == 'ssprk2':
        Us = U + dt * L0
        return 0.5 * U + 0.5 * (Us + dt * residual(Us, s, tau_ref))
    if s.integrator == 'midpoint':
        Us = U + (0.5 * dt) * L0
        return U + dt * residual(Us, s, tau_ref)
    raise ValueError(s.integrator)


def run(U0, s, tau_ref, dts, checkpoint_steps=True):
    """March the fixed time steps `dts` from U0 (conserved, float64 tensor).  With
    checkpoint_steps, each step's graph is recomputed in the backward pass instead of kept
    (memory of one step instead of all)."""
    U = U0
    for dt in dts:
        if checkpoint_steps and torch.is_grad_enabled():
            U = checkpoint(lambda V, h=float(dt): step(V, h, s, tau_ref), U, use_reentrant=False)
        else:
            U = step(U, float(dt), s, tau_ref)
    return U


def gradients(U0, w, dts, tau_ref, frozen_limiter=False, **setup):
    """J = sum(w U_n) after the fixed steps `dts` and its gradients with respect to
    (jet Mach, jet density, tau_ref) and U0.  U0, w: NumPy arrays [14][ny][nx] (or [14][nx]).
    Returns (J, [dJ/dM, dJ/drho_jet, dJ/dtau_ref], dJ/dU0 as a NumPy array)."""
    import numpy as np
    mach = torch.tensor(float(setup.pop('jet_mach', 3.0)), dtype=F64, requires_grad=True)
    rho = torch.tensor(float(setup.pop('jet_rho', 1.0)), dtype=F64, requires_grad=True)
    tau = torch.tensor(float(tau_ref), dtype=F64, requires_grad=True)
    s = Setup(jet_mach=mach, jet_rho=rho, frozen_limiter=frozen_limiter, **setup)
    U = torch.tensor(np.asarray(U0, dtype=np.float64), requires_grad=True)
    Un = run(U, s, tau, dts)
    J = (torch.tensor(np.asarray(w, dtype=np.float64)) * Un).sum()
    gm, gr, gt, gU = torch.autograd.grad(J, (mach, rho, tau, U), allow_unused=True)
    z = torch.zeros((), dtype=F64)
    g = [float(x if x is not None else z) for x in (gm, gr, gt)]
    return float(J.detach()), g, gU.numpy()


def forward(U0, dts, tau_ref, **setup):
    """U_n after the fixed steps `dts` (NumPy in, NumPy out), without gradients."""
    import numpy as np
    s = Setup(**setup)
    with torch.no_grad():
        return run(torch.tensor(np.asarray(U0, dtype=np.float64)), s,
                   torch.tensor(float(tau_ref), dtype=F64), dts).numpy()

"""Cell-centred finite-volume scheme: ghost cells, MUSCL reconstruction with one common
limiter, interface fluxes, BGK source, CFL time step and the explicit integrators.

Oracle (test infrastructure only; see the package docstring).

Paper passages followed
  * Section 3 opening: cell-centred finite volumes, explicit forward Euler or midpoint
    (2nd-order Runge-Kutta) time marching, explicit collision source.
  * Section 3.1: HLL and Rusanov interface fluxes with the approximate wave speeds.
  * Section 3.2: linear (MUSCL) reconstruction of the PRIMITIVE variables, with the same,
    most stringent limiter value used for all of them (van Albada in the paper; minmod is
    the workload's choice).
  * Section 6 set-up: jet states imposed in ghost cells; the other sides let gas escape.
  * Section 4.3: the CFL condition with the maximum wave speed sets the time step.

Readings (silent points; each also listed in the design notes)
  * common limiter: phi_v = 2 min(|a|,|b|)/(|a|+|b|) (minmod) or 2ab/(a^2+b^2) (van Albada)
    relative to the central slope (a+b)/2; phi_v = 0 when ab <= 0; phi = min_v phi_v;
    slope = phi (a+b)/2.  A variable with |a| + |b| <= 1e-10 x its natural scale (rho, c,
    p, rho c^3, rho c^4 of the cell) is neutral (phi_v = 1): the paper limits every variable
    when a discontinuity appears in any one of them, and round-off in a nominally constant
    variable is no discontinuity (without this, second order collapses to first order).
  * positivity fallback: a cell whose reconstructed face states along a direction have
    rho <= 0 or a non-SPD pressure tensor is reconstructed at first order along it.
  * HLL signal speeds: min / max over both reconstructed face states (Davis).
  * SSP-RK2 (Heun) is the workload's integrator; forward Euler and midpoint are flags.
  * dt from the cell-centre states of U^n: 1D dt = CFL dx / max Lambda,
    2D dt = CFL / max(Lambda_x/dx + Lambda_y/dy), Lambda_d = max(|lambda_min|, |lambda_max|),
    clipped to t_end - t; the same dt serves both stages.
  * collision time local to the cell centre, tau = tau_ref (rho_ref/rho) sqrt(T_ref/T),
    T = p/rho; tau_ref <= 0 switches the source off (collisionless).
  * ghost cells are filled in primitive variables: transmissive copies the edge cell,
    periodic wraps, reflective mirrors and negates the components odd in the normal
    direction, jet inflow writes the jet Maxwellian into the ghost cells of the boundary
    rows (x walls) or columns (y walls) whose centre lies in a jet on that wall and is
    transmissive elsewhere (Section 6: jets centred on the walls, L/7 wide).
  * point-implicit source (forward Euler only; Section 4.3 names it for stiff collisions):
    transport by forward Euler, then the BGK source alone by backward Euler.
"""
from dataclasses import dataclass, field
import math

import numpy as np

from . import moments as mo
from .closure import closure5, closure14
from .wavespeeds import wavespeeds5, wavespeeds14, lam_max_star14, lam_max_star5
from .fluxes import (flux5, flux14, source5, source14, tau_local, hll, rusanov,
                     davis_speeds)


@dataclass
class Setup:
    system: int = 14                  # 5 or 14
    dim: int = 1                      # 1 or 2
    nx: int = 100
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    bc: tuple = ('transmissive',) * 4  # XLO, XHI, YLO, YHI
    # [(centre along the wall, width, angle_deg[, wall]), ...]; wall 0 x-low (default),
    # 1 x-high, 2 y-low, 3 y-high
    jets: list = field(default_factory=list)
    jet_mach: float = 3.0
    jet_rho: float = 1.0
    jet_T: float = 1.0
    tau_mode: str = 'local'           # 'local' | 'const'
    rho_ref: float = 1.0
    T_ref: float = 1.0
    order: int = 2
    limiter: str = 'minmod'           # 'minmod' | 'vanalbada'
    flux: str = 'hll'                 # 'hll' | 'rusanov'
    integrator: str = 'ssprk2'        # 'fe' | 'ssprk2' | 'midpoint'
    cfl: float = 0.5
    sigma_lim: float = 1e-4
    k_ws: float = 1.0
    positivity_fallback: bool = True
    source_implicit: bool = False     # forward Euler with a backward-Euler BGK source

    @property
    def nv(self):
        return 5 if self.system == 5 else 14

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny


# ----------------------------------------------------------------------------- states
def cons_to_prim(U, s):
    return mo.cons_to_prim5(U) if s.system == 5 else mo.cons_to_prim14(U)


def prim_to_cons(W, s):
    return mo.prim_to_cons5(W) if s.system == 5 else mo.prim_to_cons14(W)


def jet_prim(s, angle_deg):
    """Jet Maxwellian: rho_j, T_j, |u| = M sqrt(gamma T_j) with gamma = 5/3 (a 3V monatomic
    gas; Section 6 quotes M = 5 at 300 K argon as 1613 m/s), direction angle_deg in x-y."""
    a = math.radians(angle_deg)
    speed = s.jet_mach * math.sqrt(5.0 / 3.0 * s.jet_T)
    p = s.jet_rho * s.jet_T
    return mo.maxwellian_prim14(np.float64(s.jet_rho),
                                np.array([speed * math.cos(a), speed * math.sin(a), 0.0]),
                                np.float64(p))


def _odd_components(system, d):
    """Components of W that change sign under reflection of axis d."""
    if system == 5:
        return [1, 3]
    uo = [1 + d]
    Po = [4 + m for m, (i, j) in enumerate(mo.SYM) if (i == d) != (j == d)]
    qo = [10 + d]
    return uo + Po + qo


def pad_axis(W, g, axis, lo, hi, s, wall_centres=None):
    """Add g ghost layers along array axis `axis` (component axis is 0).  wall_centres: the
    coordinates, along the wall, of the cells of the other array axis (for jet inflow)."""
    n = W.shape[axis]
    d = 0 if axis == W.ndim - 1 else 1          # physical direction: last axis is x
    idx = np.arange(-g, n + g)

    def take(ix):
        return np.take(W, ix, axis=axis)

    out = take(np.clip(idx, 0, n - 1))          # transmissive everywhere first
    sl_lo = [slice(None)] * W.ndim
    sl_hi = [slice(None)] * W.ndim
    sl_lo[axis] = slice(0, g)
    sl_hi[axis] = slice(n + g, n + 2 * g)
    for side, kind, sl in (('lo', lo, sl_lo), ('hi', hi, sl_hi)):
        ghost_idx = idx[:g] if side == 'lo' else idx[n + g:]
        if kind == 'transmissive':
            continue
        if kind == 'periodic':
            out[tuple(sl)] = take(ghost_idx % n)
        elif kind == 'reflective':
            mirror = -ghost_idx - 1 if side == 'lo' else 2 * n - 1 - ghost_idx
            gh = take(mirror).copy()
            for c in _odd_components(s.system, d):
                gh[c] = -gh[c]
            out[tuple(sl)] = gh
        elif kind == 'jet':
            wall = 2 * d + (0 if side == 'lo' else 1)
            gh = out[tuple(sl)].copy()       # (nv, ny, g) on the x walls, (nv, g, nx) on y
            for jet in s.jets:
                centre, w, ang = jet[:3]
                if (jet[3] if len(jet) > 3 else 0) != wall:
                    continue
                Wj = jet_prim(s, ang)
                band = (wall_centres >= centre - 0.5 * w) & (wall_centres <= centre + 0.5 * w)
                if d == 0:
                    gh[:, band, :] = Wj[:, None, None]
                else:
                    gh[:, :, band] = Wj[:, None, None]
            out[tuple(sl)] = gh
        else:
            raise ValueError(kind)
    return out


def ghosted_prims(U, s, g):
    """Primitive field with g ghost layers on every physical side."""
    W = cons_to_prim(U, s)
    if s.dim == 1:
        return pad_axis(W, g, 1, s.bc[0], s.bc[1], s)
    yc = s.y0 + (np.arange(s.ny) + 0.5) * s.dy
    xc = s.x0 + (np.arange(-g, s.nx + g) + 0.5) * s.dx     # columns of the x-padded field
    Wx = pad_axis(W, g, 2, s.bc[0], s.bc[1], s, wall_centres=yc)
    return pad_axis(Wx, g, 1, s.bc[2], s.bc[3], s, wall_centres=xc)


# ----------------------------------------------------------------------------- MUSCL
NEUTRAL_EPS = 1e-10


def variable_scales(Wc, system):
    """Natural scale of each primitive at a cell: rho, c = sqrt(p/rho) for velocities,
    p for pressures, rho c^3 for heat fluxes, rho c^4 for the fourth moment."""
    rho = np.abs(Wc[0])
    if system == 5:
        p = np.abs(Wc[2])
        c = np.sqrt(p / rho)
        return np.stack([rho, c, p, rho * c**3, rho * c**4], 0)
    p = np.abs(Wc[4] + Wc[7] + Wc[9]) / 3.0
    c = np.sqrt(p / rho)
    return np.stack([rho, c, c, c, p, p, p, p, p, p, rho * c**3, rho * c**3, rho * c**3,
                     rho * c**4], 0)


def limiter_phi(a, b, kind, scale=None):
    """Per-variable limiter factor relative to the central slope (a + b)/2.  A variable
    whose jumps are both below NEUTRAL_EPS times its scale is neutral (factor 1): round-off
    in a nominally constant variable is not a discontinuity."""
    with np.errstate(divide='ignore', invalid='ignore'):
        if kind == 'minmod':
            val = 2.0 * np.minimum(np.abs(a), np.abs(b)) / (np.abs(a) + np.abs(b))
        elif kind == 'vanalbada':
            val = 2.0 * a * b / (a * a + b * b)
        else:
            raise ValueError(kind)
    phi = np.where(a * b <= 0.0, 0.0, val)
    if scale is None:
        return np.where((a == 0.0) & (b == 0.0), 1.0, phi)
    return np.where(np.abs(a) + np.abs(b) <= NEUTRAL_EPS * scale, 1.0, phi)


def _admissible(W, s):
    """rho > 0 and SPD pressure (leading principal minors > 0)."""
    if s.system == 5:
        return (W[0] > 0.0) & (W[2] > 0.0)
    Pxx, Pxy, Pxz, Pyy, Pyz, Pzz = W[4:10]
    m1 = Pxx
    m2 = Pxx * Pyy - Pxy * Pxy
    m3 = (Pxx * (Pyy * Pzz - Pyz * Pyz) - Pxy * (Pxy * Pzz - Pyz * Pxz)
          + Pxz * (Pxy * Pyz - Pyy * Pxz))
    return (W[0] > 0.0) & (m1 > 0.0) & (m2 > 0.0) & (m3 > 0.0)


def face_states(Wg, axis, g, s):
    """Left/right states at the n+1 interior faces along `axis` of a ghosted field.

    Returns (WL, WR, n_fallback).  Face f sits between cells g-1+f and g+f of Wg.
    """
    n = Wg.shape[axis] - 2 * g

    def sl(a, b):
        t = [slice(None)] * Wg.ndim
        t[axis] = slice(a, b)
        return tuple(t)

    if s.order == 1:
        return Wg[sl(g - 1, g + n)], Wg[sl(g, g + n + 1)], 0
    # cells g-1 .. g+n (n+2 cells) need slopes
    Wc = Wg[sl(g - 1, g + n + 1)]
    a = Wc - Wg[sl(g - 2, g + n)]
    b = Wg[sl(g, g + n + 2)] - Wc
    phi = limiter_phi(a, b, s.limiter, variable_scales(Wc, s.system)).min(axis=0)
    slope = phi[None] * (a + b) / 2.0
    Wp = Wc + slope / 2.0          # state at the cell's upper face
    Wm = Wc - slope / 2.0          # state at the cell's lower face
    nfb = 0
    if s.positivity_fallback:
        bad = ~(_admissible(Wp, s) & _admissible(Wm, s))
        nfb = int(bad.sum())
        if nfb:
            Wp = np.where(bad[None], Wc, Wp)
            Wm = np.where(bad[None], Wc, Wm)
    # face f: left state = upper state of cell f (index f in Wc), right = lower of cell f+1
    WL = np.take(Wp, np.arange(0, n + 1), axis=axis)
    WR = np.take(Wm, np.arange(1, n + 2), axis=axis)
    return WL, WR, nfb


# ----------------------------------------------------------------------------- fluxes
def _state_terms(W, d, s):
    """(U, F_d, lambda_min, lambda_max) of primitive states along direction d."""
    if s.system == 5:
        sc, _ = closure5(W, s.sigma_lim)
        lmin, lmax = wavespeeds5(W, s.sigma_lim, s.k_ws)
        return mo.prim_to_cons5(W), flux5(W, sc), lmin, lmax
    Q, Rt, S, _ = closure14(W, s.sigma_lim)
    lmin, lmax = wavespeeds14(W, s.sigma_lim, d, s.k_ws)
    return mo.prim_to_cons14(W), flux14(W, Q, Rt, S, d), lmin, lmax


def interface_flux(WL, WR, d, s):
    UL, FL, lminL, lmaxL = _state_terms(WL, d, s)
    UR, FR, lminR, lmaxR = _state_terms(WR, d, s)
    if s.flux == 'hll':
        SL, SR = davis_speeds(lminL, lmaxL, lminR, lmaxR)
        return hll(FL, FR, UL, UR, SL, SR)
    if s.flux == 'rusanov':
        amax = np.maximum(np.maximum(np.abs(lminL), np.abs(lmaxL)),
                          np.maximum(np.abs(lminR), np.abs(lmaxR)))
        return rusanov(FL, FR, UL, UR, amax)
    raise ValueError(s.flux)


def bgk_source(W, s, tau_ref):
    if not (tau_ref > 0.0) or math.isinf(tau_ref):
        return np.zeros_like(W)
    rho = W[0]
    if s.system == 5:
        T = W[2] / rho
    else:
        T = mo.pressure14(W) / rho
    if s.tau_mode == 'local':
        tau = tau_local(rho, T, tau_ref, s.rho_ref, s.T_ref)
    else:
        tau = tau_ref + np.zeros_like(rho)
    return source5(W, tau) if s.system == 5 else source14(W, tau)


def residual(U, s, tau_ref, stats=None):
    """L(U) = -(F_{i+1/2} - F_{i-1/2})/dx - (G_{j+1/2} - G_{j-1/2})/dy + C(W_i)."""
    g = 1 if s.order == 1 else 2
    Wg = ghosted_prims(U, s, g)
    if s.dim == 1:
        WL, WR, nfb = face_states(Wg, 1, g, s)
        Fx = interface_flux(WL, WR, 0, s)
        W = Wg[:, g:-g]
        L = -(Fx[:, 1:] - Fx[:, :-1]) / s.dx
    else:
        rows = slice(g, g + s.ny)
        cols = slice(g, g + s.nx)
        WLx, WRx, nfx = face_states(Wg[:, rows, :], 2, g, s)
        WLy, WRy, nfy = face_states(Wg[:, :, cols], 1, g, s)
        nfb = nfx + nfy
        Fx = interface_flux(WLx, WRx, 0, s)
        Fy = interface_flux(WLy, WRy, 1, s)
        W = Wg[:, rows, cols]
        L = -(Fx[:, :, 1:] - Fx[:, :, :-1]) / s.dx - (Fy[:, 1:, :] - Fy[:, :-1, :]) / s.dy
    L = L + bgk_source(W, s, tau_ref)
    if stats is not None:
        stats['n_fallback'] = stats.get('n_fallback', 0) + nfb
    return L


# ----------------------------------------------------------------------------- time step
def cell_lambda(U, s, d):
    """Lambda_d = max(|lambda_min|, |lambda_max|) at the cell centres."""
    W = cons_to_prim(U, s)
    if s.system == 5:
        lmin, lmax = wavespeeds5(W, s.sigma_lim, s.k_ws)
    else:
        lmin, lmax = wavespeeds14(W, s.sigma_lim, d, s.k_ws)
    return np.maximum(np.abs(lmin), np.abs(lmax))


def cfl_dt(U, s):
    if s.dim == 1:
        return s.cfl * s.dx / cell_lambda(U, s, 0).max()
    return s.cfl / (cell_lambda(U, s, 0) / s.dx + cell_lambda(U, s, 1) / s.dy).max()


class OracleFailure(RuntimeError):
    """A failed step: `step` is its 1-based index, `reason` 'nonfinite' or 'unrealizable'."""

    def __init__(self, msg, step=0, reason=''):
        super().__init__(msg)
        self.step = step
        self.reason = reason


def check_state(U, s, step):
    """Failure on a non-finite value, rho <= 0 or a non-SPD pressure at a cell centre of a
    stage's new state (reading: checked per stage, since the next stage evaluates the
    closure of the intermediate state)."""
    if not np.all(np.isfinite(U)):
        raise OracleFailure(f'non-finite state in step {step}', step, 'nonfinite')
    W = cons_to_prim(U, s)
    if not np.all(_admissible(W, s)):
        raise OracleFailure(f'unrealizable state (rho <= 0 or P not SPD) in step {step}', step,
                            'unrealizable')


def relax_backward_euler(Ut, h_dt, s, tau_ref):
    """Backward-Euler step of the BGK source alone, U = Ut + h_dt C(U).  The source relaxes
    the non-conserved moments towards the local Maxwellian and keeps rho, rho u and the
    energy (Sections 2.3-2.4), so the Maxwellian U_eq and the collision time of U are those
    of Ut, and C(U) = (U_eq - U) / tau makes the implicit equation linear:
    U = (Ut + (h_dt / tau) U_eq) / (1 + h_dt / tau)."""
    if not (tau_ref > 0.0) or math.isinf(tau_ref):
        return Ut
    W = cons_to_prim(Ut, s)
    rho = W[0]
    if s.system == 5:
        T = W[2] / rho
        Weq = mo.maxwellian_prim5(rho, W[1], W[2])
    else:
        p = mo.pressure14(W)
        T = p / rho
        Weq = mo.maxwellian_prim14(rho, np.moveaxis(W[1:4], 0, -1), p)
    tau = tau_local(rho, T, tau_ref, s.rho_ref, s.T_ref) if s.tau_mode == 'local' \
        else tau_ref + np.zeros_like(rho)
    h = h_dt / tau
    return (Ut + h * prim_to_cons(Weq, s)) / (1.0 + h)


def step(U, dt, s, tau_ref, stats=None, check=None):
    """One full time step with the configured integrator (ghosts refilled per stage).
    `check`, if given, is called with every stage's new state (the intermediate state of a
    two-stage integrator and the step's result): the closure of an intermediate state is
    evaluated by the next stage, so an unrealizable one is a failure of the step."""
    chk = check if check is not None else (lambda V: None)
    if s.source_implicit:
        if s.integrator != 'fe':
            raise ValueError('the implicit source is defined for forward Euler')
        out = relax_backward_euler(U + dt * residual(U, s, 0.0, stats), dt, s, tau_ref)
        chk(out)
        return out
    L0 = residual(U, s, tau_ref, stats)
    if s.integrator == 'fe':
        out = U + dt * L0
    elif s.integrator == 'ssprk2':
        Us = U + dt * L0
        chk(Us)
        out = 0.5 * U + 0.5 * (Us + dt * residual(Us, s, tau_ref, stats))
    elif s.integrator == 'midpoint':
        Us = U + (0.5 * dt) * L0
        chk(Us)
        out = U + dt * residual(Us, s, tau_ref, stats)
    else:
        raise ValueError(s.integrator)
    chk(out)
    return out


def run(U, s, tau_ref, nsteps=None, t_end=None, dt=None, t0=0.0, record=None,
        check=True):
    """March nsteps steps (or until t_end).  dt=None uses the CFL step clipped to t_end.
    Returns (U, t, steps).  `record` (list) receives each step's dt."""
    t = t0
    n = 0
    while True:
        if nsteps is not None and n >= nsteps:
            break
        if t_end is not None and t >= t_end * (1.0 - 1e-14):
            break
        h = cfl_dt(U, s) if dt is None else dt
        if t_end is not None:
            h = min(h, t_end - t)
        U = step(U, h, s, tau_ref,
                 check=(lambda V, k=n + 1: check_state(V, s, k)) if check else None)
        t += h
        n += 1
        if record is not None:
            record.append(h)
    return U, t, n


__all__ = ['Setup', 'OracleFailure', 'residual', 'step', 'run', 'cfl_dt', 'cell_lambda',
           'face_states', 'limiter_phi', 'ghosted_prims', 'jet_prim', 'interface_flux',
           'bgk_source', 'lam_max_star14', 'lam_max_star5']

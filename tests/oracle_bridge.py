"""Test helpers: map solver keyword settings to the oracle's Setup, run both sides on the
same seeded inputs, compare per moment.  Test infrastructure only."""
import contextlib
import dataclasses

import numpy as np

from oracle import scheme as sc, moments as mo

SOLVER_TO_SETUP = ('system', 'dim', 'nx', 'ny', 'x0', 'x1', 'y0', 'y1', 'jet_mach', 'jet_rho',
                   'jet_T', 'tau_mode', 'rho_ref', 'T_ref', 'order', 'limiter', 'flux',
                   'integrator', 'cfl', 'sigma_lim', 'k_ws', 'positivity_fallback',
                   'source_implicit')
WALLS = {'xlo': 0, 'xhi': 1, 'ylo': 2, 'yhi': 3}


def to_setup(kw):
    s = sc.Setup()
    for k in SOLVER_TO_SETUP:
        if k in kw:
            setattr(s, k, kw[k])
    if 'bc' in kw:
        s.bc = tuple(kw['bc'])
    if 'jets' in kw:
        s.jets = [tuple(j[:3]) + ((WALLS.get(j[3], j[3]),) if len(j) > 3 else ()) for j in kw['jets']]
    return s


def prim_to_cons(W, system):
    return mo.prim_to_cons5(W) if system == 5 else mo.prim_to_cons14(W)


def field_rel_err(a, b):
    """Per-moment error max_i |a - b| / max_i |b| (field-relative, so moments that vanish
    in part of the field, such as q or P_xy, are compared on the field's own scale)."""
    a = np.asarray(a, dtype=float).reshape(b.shape[0], -1)
    b = np.asarray(b, dtype=float).reshape(b.shape[0], -1)
    out = np.zeros(b.shape[0])
    for v in range(b.shape[0]):
        d = np.abs(a[v] - b[v]).max()
        out[v] = 0.0 if d == 0.0 else d / max(np.abs(b[v]).max(), 1e-300)
    return out


def oracle_run(kw, W0, nsteps=None, dt=0.0, tau_ref=0.0, t_end=0.0):
    s = to_setup(kw)
    U0 = prim_to_cons(np.asarray(W0, dtype=float), s.system)
    if s.dim == 1:
        U0 = U0.reshape(U0.shape[0], -1)
    U, t, n = sc.run(U0, s, tau_ref, nsteps=nsteps, dt=dt if dt > 0 else None,
                     t_end=t_end if t_end > 0 else None)
    return U, t, n


def oracle_cell_step(W, i, j, kw, dt, tau_ref, r=4, patch=None):
    """One full oracle step for the single cell (i, j) of a large 2D field, computed on the
    (2r+1)^2 patch around it: with two stages of a 2-cell stencil nothing beyond r = 4
    cells away reaches the centre, so the patch's own ghost cells never matter unless the
    patch side is a real domain side (where the real boundary condition is kept).  `patch`,
    if given, replaces W on the (2r+1)^2 patch (clipped to the field)."""
    s = to_setup(kw)
    ny, nx = W.shape[1:]
    dx, dy = s.dx, s.dy
    i0, i1 = max(0, i - r), min(nx, i + r + 1)
    j0, j1 = max(0, j - r), min(ny, j + r + 1)
    bc = list(s.bc)
    if i0 > 0:
        bc[0] = 'transmissive'
    if i1 < nx:
        bc[1] = 'transmissive'
    if j0 > 0:
        bc[2] = 'transmissive'
    if j1 < ny:
        bc[3] = 'transmissive'
    sp = dataclasses.replace(s, nx=i1 - i0, ny=j1 - j0, x0=s.x0 + i0 * dx, x1=s.x0 + i1 * dx,
                             y0=s.y0 + j0 * dy, y1=s.y0 + j1 * dy, bc=tuple(bc))
    U = mo.prim_to_cons14(W[:, j0:j1, i0:i1] if patch is None else patch)
    U1 = sc.step(U, dt, sp, tau_ref)
    return U1[:, j - j0, i - i0]


ULP = 2.220446049250313e-16              # one unit in the last place, relative (2^-52)
PERTURB = 4 * ULP                         # input perturbation: 4 ulp relative
# Bar factor over the larger of the two spreads below.  Each spread is the maximum over a few
# random draws of how far a correct FP64 computation can move; an independent implementation
# is one more such draw, so it stays within the observed maximum up to sampling (factor 2).
SPREAD_FACTOR = 2.0

# Every stage function of the oracle whose inputs and outputs an implementation with another
# operation order (FMA contraction, reciprocal multiplies, Newton-Raphson division and square
# root, another algebraic form of the closure) rounds differently.
_ROUNDED = ((mo, ('cons_to_prim14', 'cons_to_prim5', 'prim_to_cons14', 'prim_to_cons5')),
            (sc, ('closure14', 'closure5', 'wavespeeds14', 'wavespeeds5', 'flux14', 'flux5',
                  'source14', 'source5', 'hll', 'rusanov', 'limiter_phi', 'residual',
                  'relax_backward_euler')))


@contextlib.contextmanager
def rounded_intermediates(rng, rel=ULP):
    """Within the block, every stage function listed in _ROUNDED takes each float64 array
    argument and returns each float64 array result with one random +-rel relative rounding
    per value (random signs): the oracle's arithmetic itself is untouched.  Rounding the
    inputs models operands that a cancelling sum (primitive recovery, the sigma bracket A,
    the flux terms) rounds at the scale of its largest term; rounding the outputs models the
    function's own result rounding."""
    # random factors 1 +- rel, drawn once; each rounding takes a window at a random offset
    table = np.where(rng.random(1 << 21) < 0.5, 1.0 - rel, 1.0 + rel)

    def rnd(x):
        if isinstance(x, np.ndarray) and x.dtype == np.float64 and x.size:
            if x.size > table.size // 2:
                return x * np.where(rng.random(x.shape) < 0.5, 1.0 - rel, 1.0 + rel)
            o = int(rng.integers(0, table.size - x.size))
            return x * table[o:o + x.size].reshape(x.shape)
        if isinstance(x, tuple):
            return tuple(rnd(y) for y in x)
        return x

    def wrap(f):
        def g(*a, **k):
            return rnd(f(*(rnd(x) for x in a), **k))
        return g

    saved = []
    try:
        for mod, names in _ROUNDED:
            for name in names:
                f = getattr(mod, name)
                saved.append((mod, name, f))
                setattr(mod, name, wrap(f))
        yield
    finally:
        for mod, name, f in reversed(saved):
            setattr(mod, name, f)


def oracle_spreads(fn, U0, trials=3, seed=0, perturb=PERTURB, rel=ULP, reduce=None):
    """The two spreads of an oracle computation fn(U0) -> array (computed by the oracle
    alone): (input spread, intermediate spread) = the largest change of each output value
    (a) when U0 is perturbed by +-perturb relative (random signs per value), and (b) when every
    stage function rounds its inputs and outputs by +-rel (rounded_intermediates), over
    `trials` runs each.  `reduce` maps a difference array to what is compared (default:
    its absolute value)."""
    base = fn(U0)
    red = reduce if reduce is not None else np.abs
    rng = np.random.default_rng(seed)
    s_in = np.zeros_like(red(base - base))
    s_mid = np.zeros_like(s_in)
    for _ in range(trials):
        Up = U0 * (1.0 + rng.choice([-1.0, 1.0], U0.shape) * perturb)
        s_in = np.maximum(s_in, red(fn(Up) - base))
    for _ in range(trials):
        with rounded_intermediates(rng, rel):
            out = fn(U0)
        s_mid = np.maximum(s_mid, red(out - base))
    return base, s_in, s_mid


def oracle_with_spread(kw, W0, nsteps=None, dt=0.0, tau_ref=0.0, t_end=0.0, trials=3, seed=0,
                       check=True, parts=False):
    """The oracle's result and its own spread: the larger, per output value, of its change
    under +-4 ulp input perturbations and under 1-ulp rounding of every intermediate
    (oracle_spreads).  The spread measures the conditioning of the step on this input; any
    FP64 implementation that rounds differently (FMA contraction, other libm, other operation
    order) can differ from the oracle by about this much.  parts=True also returns the two
    spreads separately."""
    s = to_setup(kw)
    U0 = prim_to_cons(np.asarray(W0, dtype=float), s.system)
    if s.dim == 1:
        U0 = U0.reshape(U0.shape[0], -1)
    kwr = dict(nsteps=nsteps, dt=dt if dt > 0 else None, t_end=t_end if t_end > 0 else None,
               check=check)
    _, t, n = sc.run(U0, s, tau_ref, **kwr)
    base, s_in, s_mid = oracle_spreads(lambda U: sc.run(U, s, tau_ref, **kwr)[0], U0,
                                       trials=trials, seed=seed)
    spread = np.maximum(s_in, s_mid)
    if parts:
        return base, spread, t, n, (s_in, s_mid)
    return base, spread, t, n


def within_spread(gpu, base, spread, rel_floor=1e-12, factor=SPREAD_FACTOR):
    """Per cell and moment: |gpu - oracle| <= rel_floor * max|oracle_v| + factor * spread.
    Returns (ok, worst excess ratio, per-moment field-relative error)."""
    g = np.asarray(gpu, dtype=float).reshape(base.shape[0], -1)
    b = base.reshape(base.shape[0], -1)
    sp = spread.reshape(base.shape[0], -1)
    scale = np.maximum(np.abs(b).max(1, keepdims=True), 1e-300)
    d = np.abs(g - b)
    bound = rel_floor * scale + factor * sp
    ratio = np.where(d == 0.0, 0.0, d / np.maximum(bound, 1e-300))
    err = np.where(d.max(1) == 0.0, 0.0, d.max(1) / scale[:, 0])
    return bool(ratio.max() <= 1.0), float(ratio.max()), err


def oracle_cells_1d(W, cells, kw, nsteps, dt, tau_ref, trials=3, seed=0):
    """Oracle values after `nsteps` fixed-dt steps at selected cells of a long 1D field, each
    computed on the patch [i - 4 nsteps, i + 4 nsteps] (the dependency cone of SSP-RK2 with
    a two-cell stencil per stage); a patch side inside the domain gets transmissive ghosts,
    which never reach the centre.  Also returns the spread (oracle_spreads, larger of the
    input and intermediate spreads) of each value."""
    s = to_setup(kw)
    nx = W.shape[-1]
    r = 4 * nsteps
    vals, spreads = [], []
    for k, i in enumerate(cells):
        i0, i1 = max(0, i - r), min(nx, i + r + 1)
        bc = list(s.bc)
        if i0 > 0:
            bc[0] = 'transmissive'
        if i1 < nx:
            bc[1] = 'transmissive'
        if bc[0] == 'periodic' or bc[1] == 'periodic':
            raise ValueError('periodic fields are not patchable')
        sp = dataclasses.replace(s, nx=i1 - i0, x0=s.x0 + i0 * s.dx, x1=s.x0 + i1 * s.dx,
                                 bc=tuple(bc))
        U = prim_to_cons(W[:, i0:i1], s.system)
        base, s_in, s_mid = oracle_spreads(
            lambda Ux: sc.run(Ux, sp, tau_ref, nsteps=nsteps, dt=dt, check=False)[0][:, i - i0],
            U, trials=trials, seed=seed + k)
        vals.append(base)
        spreads.append(np.maximum(s_in, s_mid))
    return np.array(vals).T, np.array(spreads).T


def oracle_with_l1_spread(kw, W0, t_end, tau_ref, trials=3, seed=0, perturb=PERTURB, nsteps=None,
                          intermediate=True):
    """Long runs: the oracle's result at t_end, its L1 spread per moment (the largest
    ||changed - base||_1 under +-perturb input perturbations and, if `intermediate`, under
    1-ulp rounding of every intermediate) and the largest change of the step count under the
    same changes."""
    s = to_setup(kw)
    U0 = prim_to_cons(np.asarray(W0, dtype=float), s.system)
    if s.dim == 1:
        U0 = U0.reshape(U0.shape[0], -1)
    kwr = dict(t_end=t_end if t_end and t_end > 0 else None, nsteps=nsteps)
    base, t, n = sc.run(U0, s, tau_ref, **kwr)
    rng = np.random.default_rng(seed)
    spread = np.zeros(base.shape[0])
    nspread = 0

    def take(out, nk):
        nonlocal spread, nspread
        spread = np.maximum(spread, np.abs(out - base).reshape(base.shape[0], -1).sum(1))
        nspread = max(nspread, abs(nk - n))

    for _ in range(trials):
        Up = U0 * (1.0 + rng.choice([-1.0, 1.0], U0.shape) * perturb)
        out, _, nk = sc.run(Up, s, tau_ref, **kwr)
        take(out, nk)
    if intermediate:
        for _ in range(trials):
            with rounded_intermediates(rng):
                out, _, nk = sc.run(U0, s, tau_ref, **kwr)
            take(out, nk)
    return base, spread, t, n, nspread


def oracle_with_flux_rounding_spread(kw, W0, tau_ref, nsteps, trials=2, seed=0, rel=2.0 ** -24):
    """The oracle's L1 change per moment when every closure (closing moments), physical flux
    component and wave speed it evaluates carries one random relative rounding of size rel
    (2^-24: one FP32 rounding), with the oracle's arithmetic otherwise untouched: how far a
    correct computation whose per-face closure, flux and wave-speed evaluations are rounded to
    single precision can move.  Returns (base, spread)."""
    s = to_setup(kw)
    U0 = prim_to_cons(np.asarray(W0, dtype=float), s.system)
    if s.dim == 1:
        U0 = U0.reshape(U0.shape[0], -1)
    base, _, _ = sc.run(U0, s, tau_ref, nsteps=nsteps)
    rng = np.random.default_rng(seed)
    names = (('flux14', 'wavespeeds14', 'closure14') if s.system == 14
             else ('flux5', 'wavespeeds5', 'closure5'))
    orig = {k: getattr(sc, k) for k in names}

    def rnd(a):
        a = np.asarray(a, dtype=float)
        return a * (1.0 + rng.choice([-1.0, 1.0], a.shape) * rel)

    def flux(*a, **k):
        return rnd(orig[names[0]](*a, **k))

    def speeds(*a, **k):
        lmin, lmax = orig[names[1]](*a, **k)
        return rnd(lmin), rnd(lmax)

    def closure(*a, **k):
        out = orig[names[2]](*a, **k)
        # the closing values; the last item (sigma) is not a flux input
        return tuple(rnd(x) for x in out[:-1]) + (out[-1],)

    spread = np.zeros(base.shape[0])
    try:
        setattr(sc, names[0], flux)
        setattr(sc, names[1], speeds)
        setattr(sc, names[2], closure)
        for _ in range(trials):
            out, _, _ = sc.run(U0, s, tau_ref, nsteps=nsteps)
            spread = np.maximum(spread, np.abs(out - base).reshape(base.shape[0], -1).sum(1))
    finally:
        for k, f in orig.items():
            setattr(sc, k, f)
    return base, spread


# ---------------------------------------------------------------- adjoint references
def oracle_objective(kw, U0, weights, nsteps, dt, tau_ref, mach=None, rho=None):
    """J = sum(weights * U_n) after nsteps oracle steps of fixed dt from the conserved U0
    (a linear functional of the final state; dt frozen as in the discrete adjoint)."""
    s = to_setup(kw)
    if mach is not None:
        s.jet_mach = mach
    if rho is not None:
        s.jet_rho = rho
    U = np.array(U0, dtype=float)
    if s.dim == 1:
        U = U.reshape(U.shape[0], -1)
    Un, _, n = sc.run(U, s, tau_ref, nsteps=nsteps, dt=dt)
    assert n == nsteps
    return float((np.asarray(weights).reshape(Un.shape) * Un).sum())


def central_difference(f, x, h):
    """(f(x + h) - f(x - h)) / 2h at step h and at 2h; the difference of the two estimates
    the truncation error of the first (3x its size, with smooth f)."""
    d1 = (f(x + h) - f(x - h)) / (2 * h)
    d2 = (f(x + 2 * h) - f(x - 2 * h)) / (4 * h)
    return d1, d2

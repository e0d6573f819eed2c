"""Pins of the reference-gradient transcription (oracle/adjoint_ref.py, PyTorch CPU autograd
of the oracle's 14-moment step), CPU only.

* Its forward steps equal the NumPy oracle's up to summation order.
* Its exact gradients (jet Mach, jet density, tau_ref, U0 along a direction) equal central
  differences of the NumPy oracle within the differences' own error.
* Its frozen-limiter gradients equal central differences of the NumPy oracle run with every
  common limiter factor replayed from the unperturbed run (the limiter held fixed).
"""
import numpy as np
import pytest

from oracle import adjoint_ref as ar, moments as mo, scheme as sc
from paper_2401_15233_amd import inputs as I
import oracle_bridge as ob

EPS = 2.220446049250313e-16
JETS = dict(system=14, dim=2, order=2, integrator='ssprk2', flux='hll', cfl=0.4,
            limiter='minmod', bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
            jets=[(0.35, 0.1, 30.0), (0.65, 0.1, -30.0)], jet_mach=3.0, jet_rho=1.0, jet_T=1.0)
TAU_JET = I.kn_to_tau_ref(0.1, L_ref=0.1)
VARIANT = dict(system=14, dim=2, order=2, integrator='midpoint', flux='rusanov', limiter='vanalbada',
               bc=('periodic', 'periodic', 'reflective', 'reflective'), jets=[], tau_mode='const')


def field_rel(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return float((np.abs(a - b).max(1) / np.maximum(np.abs(b).max(1), 1e-300)).max())


@pytest.mark.parametrize('case', ['jets', 'variant', 'sod1d'])
def test_forward_equals_numpy_oracle(case):
    if case == 'jets':
        kw = dict(JETS, nx=18, ny=16)
        U0 = mo.prim_to_cons14(I.crossed_jets_developed(18, 16, seed=5))
    elif case == 'variant':
        kw = dict(VARIANT, nx=14, ny=12)
        U0 = mo.prim_to_cons14(I.random_smooth_field14(14, 12, seed=3))
    else:
        kw = dict(system=14, dim=1, nx=50, order=2, integrator='fe', flux='hll', limiter='minmod',
                  bc=('transmissive',) * 4)
        U0 = mo.prim_to_cons14(I.sod_prims(14, 50))
    s = ob.to_setup(kw)
    dt = 0.8 * sc.cfl_dt(U0, s)
    Uo = sc.run(U0, s, TAU_JET, nsteps=4, dt=dt)[0]
    Ut = ar.forward(U0, [dt] * 4, TAU_JET, **kw)
    assert field_rel(Ut, Uo) < 1e-13


def check_grad(name, g, d1, d2, J, h, scale):
    bar = 2 * abs(d1 - d2) + 1e3 * EPS * (abs(J) + scale) / h + 1e-9 * abs(d1)
    print(f'   {name}: autograd {g:+.12e} FD {d1:+.12e} (2h {d2:+.12e})', flush=True)
    assert abs(g - d1) <= bar, (name, g, d1, d2)


class ReplayedLimiter:
    """Run the NumPy oracle with every common limiter factor taken from a recorded run."""

    def __init__(self):
        self.rec = []
        self.k = None
        self.orig = sc.limiter_phi

    def __enter__(self):
        def phi(a, b, kind, scale=None):
            out = self.orig(a, b, kind, scale)
            if self.k is None:
                self.rec.append(out.min(axis=0))
                return out
            p = self.rec[self.k]
            self.k += 1
            return np.broadcast_to(p[None], out.shape)
        sc.limiter_phi = phi
        return self

    def replay(self):
        self.k = 0

    def __exit__(self, *exc):
        sc.limiter_phi = self.orig


@pytest.mark.parametrize('frozen', [False, True])
def test_gradients_equal_oracle_central_differences(frozen):
    n, nsteps = 14, 4
    kw = dict(JETS, nx=n, ny=n)
    U0 = mo.prim_to_cons14(I.crossed_jets_developed(n, n, seed=5))
    Ubg = mo.prim_to_cons14(I.crossed_jets_initial(n, n))
    s = ob.to_setup(kw)
    dt = 0.8 * sc.cfl_dt(U0, s)
    w = np.random.default_rng(7).standard_normal(U0.shape) / (n * n)
    J, g, gU = ar.gradients(U0, w, [dt] * nsteps, TAU_JET, frozen_limiter=frozen, **kw)
    rng = np.random.default_rng(8)
    v = (U0 - Ubg) * rng.uniform(-1, 1, (n, n))[None]      # beams only: the background stays uniform
    with ReplayedLimiter() as rl:
        Jo = ob.oracle_objective(kw, U0, w, nsteps, dt, TAU_JET)
        if frozen:
            rl.replay()

        def J_of(mach=None, rho=None, tau=TAU_JET, dU=0.0):
            if frozen:
                rl.replay()
            return ob.oracle_objective(kw, U0 + dU, w, nsteps, dt, tau, mach=mach, rho=rho)

        scale = float(np.abs(w).sum())
        assert abs(J - Jo) <= 1e-12 * scale
        for name, k, f, p0 in (('dJ/dM', 0, lambda x: J_of(mach=x), 3.0),
                               ('dJ/drho_jet', 1, lambda x: J_of(rho=x), 1.0),
                               ('dJ/dtau_ref', 2, lambda x: J_of(tau=x), TAU_JET)):
            h = 1e-6 * p0
            d1, d2 = ob.central_difference(f, p0, h)
            check_grad(name, g[k], d1, d2, J, h, scale)
        d1, d2 = ob.central_difference(lambda e: J_of(dU=e * v), 0.0, 1e-6)
        check_grad('dJ/dU0 . v', float((gU * v).sum()), d1, d2, J, 1e-6, scale)


def test_frozen_limiter_gradient_differs_from_exact_one():
    """Control for the replay pin: the limiter's derivative matters on this field."""
    n, nsteps = 14, 4
    kw = dict(JETS, nx=n, ny=n)
    U0 = mo.prim_to_cons14(I.crossed_jets_developed(n, n, seed=5))
    dt = 0.8 * sc.cfl_dt(U0, ob.to_setup(kw))
    w = np.random.default_rng(7).standard_normal(U0.shape) / (n * n)
    _, ge, _ = ar.gradients(U0, w, [dt] * nsteps, TAU_JET, **kw)
    _, gf, _ = ar.gradients(U0, w, [dt] * nsteps, TAU_JET, frozen_limiter=True, **kw)
    assert abs(ge[0] - gf[0]) > 1e-6 * abs(ge[0])


def test_sod_tube_gradients_equal_oracle_central_differences():
    nx, nsteps = 40, 6
    kw = dict(system=14, dim=1, nx=nx, order=2, integrator='ssprk2', flux='hll', limiter='minmod',
              bc=('transmissive',) * 4)
    U0 = mo.prim_to_cons14(I.sod_prims(14, nx))
    tau = I.kn_to_tau_ref(0.01)
    dt = 0.9 * sc.cfl_dt(U0, ob.to_setup(kw))
    w = np.random.default_rng(9).standard_normal(U0.shape) / nx
    J, g, gU = ar.gradients(U0, w, [dt] * nsteps, tau, **kw)
    scale = float(np.abs(w).sum())
    f = lambda t: ob.oracle_objective(kw, U0, w, nsteps, dt, t)       # noqa: E731
    h = 1e-6 * tau
    d1, d2 = ob.central_difference(f, tau, h)
    check_grad('dJ/dtau_ref', g[2], d1, d2, J, h, scale)
    v = U0 * np.where(np.arange(nx) < nx // 2, 0.7, -0.4)[None, :]
    d1, d2 = ob.central_difference(lambda e: ob.oracle_objective(kw, U0 + e * v, w, nsteps, dt, tau),
                                   0.0, 1e-6)
    check_grad('dJ/dU0 . v', float((gU * v).sum()), d1, d2, J, 1e-6, scale)
    assert g[0] == 0.0 and g[1] == 0.0

"""The paper's own crossed-jets geometry and the point-implicit BGK source, GPU against the
oracle.

* Geometry (Section 6): unit square, M = 5 jets of width L/7 centred on the left and bottom
  walls and pointing to the centre (at a right angle), background at 1e-5 of the jet density,
  second order with van Albada, forward Euler, CFL 0.5, collisionless.
* Jets on the bottom wall are the x <-> y mirror image of jets on the left wall.
* Point-implicit source (forward Euler transport, then the BGK source by backward Euler;
  Section 4.3 names it for stiff collisions, Kn below about 1e-4): Sod tubes in the stiff
  range (dt / tau ~ 7 and ~ 700, where the explicit source diverges) and the closed-form
  homogeneous relaxation.
"""
import math

import numpy as np
import pytest

from paper_2401_15233_amd import inputs as I
from oracle import moments as mo
import oracle_bridge as ob
from test_gpu_parity import compare, gpu_run

pytestmark = pytest.mark.gpu

PJ = I.PAPER_JETS
PAPER = dict(system=14, dim=2, order=2, integrator='fe', flux='hll', cfl=0.5, limiter='vanalbada',
             bc=('jet', 'transmissive', 'jet', 'transmissive'), jets=list(PJ['jets']),
             jet_mach=PJ['mach'], jet_rho=PJ['rho'], jet_T=PJ['T'])


@pytest.mark.parametrize('nx,ny,steps', [(40, 40, 30), (37, 46, 20)])
def test_paper_jets_against_oracle(gpu_lib, nx, ny, steps):
    """Collisionless, CFL steps from rest: several tiles and ragged edges in both directions."""
    kw = dict(PAPER, nx=nx, ny=ny)
    Ug, info, base, t, n = compare(f'paper jets {nx}x{ny} {steps} steps', gpu_lib, kw,
                                   I.paper_jets_initial(nx, ny), steps)
    # the CFL steps follow the state, whose rounding spread here is ~1e-10
    assert info['steps'] == steps and abs(info['t'] - t) <= 1e-9 * t
    # both jets have entered: density raised near each inlet centre
    W = mo.cons_to_prim14(Ug)
    assert W[0, ny // 2, 1] > 0.1 and W[0, 1, nx // 2] > 0.1


def test_paper_jets_with_collisions_and_minmod(gpu_lib):
    kw = dict(PAPER, nx=32, ny=30, limiter='minmod')
    compare('paper jets Kn = 1 minmod', gpu_lib, kw, I.paper_jets_initial(32, 30), 25,
            tau_ref=I.kn_to_tau_ref(1.0, L_ref=1.0 / 7.0))


def _swap_xy(F):
    perm = [0, 2, 1, 3, 7, 5, 8, 4, 6, 9, 11, 10, 12, 13]
    return np.swapaxes(F[perm], 1, 2)


def test_bottom_wall_jet_mirrors_left_wall_jet(gpu_lib):
    """One jet on the bottom wall at 90 degrees against the mirrored problem with the jet on
    the left wall at 0 degrees, fixed dt, 20 steps: equal up to the order of the x and y flux
    differences in the update (rounding)."""
    nx, ny = 33, 47
    kw_b = dict(PAPER, nx=nx, ny=ny, bc=('transmissive', 'transmissive', 'jet', 'transmissive'),
                jets=[(0.4, 0.2, 90.0, 'ylo')])
    kw_l = dict(PAPER, nx=ny, ny=nx, bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
                jets=[(0.4, 0.2, 0.0, 'xlo')])
    W0 = I.random_smooth_field14(nx, ny, seed=12)
    dt = 2e-4
    Ub, _ = gpu_run(gpu_lib, kw_b, W0, 20, dt=dt, tau_ref=0.01)
    Ul, _ = gpu_run(gpu_lib, kw_l, _swap_xy(W0), 20, dt=dt, tau_ref=0.01)
    err = ob.field_rel_err(_swap_xy(Ul), Ub)
    print(f'bottom vs mirrored left jet: field-relative difference max {err.max():.2e}', flush=True)
    assert err.max() < 1e-12
    # the jet matters: without it the field differs
    Ut, _ = gpu_run(gpu_lib, dict(kw_b, bc=('transmissive',) * 4, jets=[]), W0, 20, dt=dt, tau_ref=0.01)
    assert ob.field_rel_err(Ut, Ub).max() > 1e-3


SOD14_FE = dict(system=14, dim=1, nx=300, order=2, integrator='fe', flux='hll', cfl=0.5,
                limiter='minmod', bc=('transmissive',) * 4, source_implicit=True)
SOD5_FE = dict(system=5, dim=1, nx=1000, order=1, integrator='fe', flux='hll', cfl=0.5,
               bc=('transmissive',) * 4, source_implicit=True)


@pytest.mark.parametrize('kn', [1e-4, 1e-6])
def test_implicit_source_sod14_stiff(gpu_lib, kn):
    tau = I.kn_to_tau_ref(kn)
    Ug, info, base, t, n = compare(f'sod14 FE implicit source Kn={kn}', gpu_lib, SOD14_FE,
                                   I.sod_prims(14, 300), 40, tau_ref=tau)
    print(f'   dt / tau_ref = {info["dt_last"] / tau:.1f}', flush=True)
    assert info['dt_last'] / tau > 5      # the explicit forward-Euler source needs dt / tau < 2


def test_implicit_source_sod5_full_run(gpu_lib):
    """The 5-moment Sod tube at Kn = 1e-5 to t = 0.2 with the point-implicit source: near the
    Euler limit the trajectory is smooth, so the full run is compared pointwise."""
    kn = 1e-5
    tau = I.kn_to_tau_ref(kn)
    Ug, info, base, t, n = compare('sod5 FE implicit source Kn=1e-5 to t = 0.2', gpu_lib, SOD5_FE,
                                   I.sod_prims(5, 1000), None, tau_ref=tau, t_end=0.2, trials=2)
    assert abs(info['t'] - 0.2) < 1e-14 and info['steps'] == n


def test_implicit_source_homogeneous_relaxation(gpu_lib):
    """Uniform non-equilibrium state, periodic: U_n = U_M + (U_0 - U_M) (1 + dt/tau)^-n at
    dt/tau = 5, where the explicit source would diverge."""
    nx, ny = 24, 20
    W0 = I.random_states14(1, seed=19)
    W = np.broadcast_to(W0[:, :, None], (14, ny, nx)).copy()
    p = mo.pressure14(W0)[0]
    UM = mo.prim_to_cons14(mo.maxwellian_prim14(W0[0], W0[1:4].T, np.array([p])))[:, 0]
    T = p / W0[0, 0]
    tau_ref = 0.05
    tau = tau_ref / W0[0, 0] * math.sqrt(1.0 / T)
    z = 5.0
    kw = dict(system=14, dim=2, nx=nx, ny=ny, order=2, integrator='fe', cfl=0.5,
              bc=('periodic',) * 4, source_implicit=True)
    Ug, info = gpu_run(gpu_lib, kw, W, 7, dt=z * tau, tau_ref=tau_ref)
    U0 = mo.prim_to_cons14(W)
    expect = UM[:, None, None] + (1.0 + z) ** -7 * (U0 - UM[:, None, None])
    err = np.max(np.abs(Ug - expect)) / np.max(np.abs(expect))
    print(f'homogeneous implicit relaxation: max relative error {err:.2e}', flush=True)
    assert err < 1e-13


def test_implicit_source_is_rejected_by_the_adjoint(gpu_lib):
    s = gpu_lib.MaxEntSolver(**dict(SOD14_FE, nx=64))
    try:
        s.init_state(I.sod_prims(14, 64))
        with pytest.raises(gpu_lib.MaxentError):
            s.record(4, 10)
    finally:
        s.close()

"""Read-backs and counters of the C-ABI on the device, against the oracle on the same
states: the closing moments (MAXENT_CLOSING), the count of sigma-limited cells, and the FP32
precision setting (every face-state evaluation in single precision, no FP64 re-evaluation),
whose L1 error against the FP64 oracle is stated per moment."""
import numpy as np
import pytest

from oracle import closure as cl, moments as mo
from paper_2401_15233_amd import inputs as I
import oracle_bridge as ob
from test_gpu_parity import JETS, TAU_JET, SOD14, gpu_run

pytestmark = pytest.mark.gpu

Q_ORDER = ((0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2),
           (1, 2, 2), (2, 2, 2))
R_ORDER = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def oracle_closing14(W, sigma_lim):
    Q, Rt, S, _ = cl.closure14(W, sigma_lim)
    return np.concatenate([np.stack([Q[..., i, j, k] for (i, j, k) in Q_ORDER], 0),
                           np.stack([Rt[..., i, j] for (i, j) in R_ORDER], 0),
                           np.moveaxis(S, -1, 0)], 0)


@pytest.mark.parametrize('field', ['random states', 'developed jets'])
def test_closing_moments_readback_14(gpu_lib, field):
    """The 19 closing moments of every cell, computed on the device from its state, against
    the oracle's closure (the printed tensor form) evaluated on the device's own primitive
    read-back: per moment, |gpu - oracle| <= 1e-12 max|oracle| + 2 x the oracle's change under
    +-4 ulp perturbations of W."""
    if field == 'random states':
        W0 = I.random_states14(400, seed=44)
        kw = dict(SOD14, nx=400)
    else:
        W0 = I.crossed_jets_developed(48, 40, seed=2)
        kw = dict(JETS, nx=48, ny=40)
    s = gpu_lib.MaxEntSolver(**kw)
    s.init_state(W0)
    Wg = s.get('primitive').cpu().numpy().reshape(14, -1)
    Cg = s.get('closing').cpu().numpy().reshape(19, -1)
    s.close()
    base, s_in, _ = ob.oracle_spreads(lambda W: oracle_closing14(W, 1e-4), Wg, trials=3, seed=1)
    scale = np.maximum(np.abs(base).max(1, keepdims=True), 1e-300)
    d = np.abs(Cg - base)
    ratio = np.where(d == 0, 0.0, d / (1e-12 * scale + 2 * s_in))
    print(f'closing moments ({field}): field-relative error max {(d / scale).max():.2e}, '
          f'bound use {ratio.max():.2f}', flush=True)
    assert ratio.max() <= 1.0
    # the contractions the closure must satisfy: Q_ijj = q_i, R_iijj = R (sigma >= sigma_lim)
    qx = Cg[0] + Cg[3] + Cg[5]
    assert np.max(np.abs(qx - Wg[10])) <= 1e-10 * np.abs(Wg[10]).max() + 1e-12 * np.abs(Cg[0]).max()


def test_closing_moment_readback_5(gpu_lib):
    W0 = I.random_states5(300, seed=45)
    kw = dict(system=5, dim=1, nx=300, order=1, integrator='fe', cfl=0.5)
    s = gpu_lib.MaxEntSolver(**kw)
    s.init_state(W0)
    Wg = s.get('primitive').cpu().numpy()[:, 0, :]
    sg = s.get('closing').cpu().numpy()[0]
    s.close()
    base, s_in, _ = ob.oracle_spreads(lambda W: cl.closure5(W, 1e-4)[0], Wg, trials=3, seed=2)
    d = np.abs(sg - base)
    assert np.all(d <= 1e-12 * np.abs(base).max() + 2 * s_in)


def test_sigma_limited_count(gpu_lib):
    """maxent_get_info counts the cells whose unlimited sigma lies below sigma_lim: every
    cell of a uniform Maxwellian background, and on a developed jets field the same cells as
    the oracle's sigma mapping (cells within rounding of the threshold excepted)."""
    n = 40
    kw = dict(JETS, nx=n, ny=n)
    s = gpu_lib.MaxEntSolver(**kw)
    s.init_state(I.crossed_jets_initial(n, n))
    assert s.info()['n_sigma_limited'] == n * n
    assert s.step(1, tau_ref=TAU_JET)['n_sigma_limited'] == -1
    W0 = I.crossed_jets_developed(n, n, seed=7)
    s.init_state(W0)
    got = s.info()['n_sigma_limited']
    Wg = s.get('primitive').cpu().numpy()
    s.close()
    sig = cl.sigma14_star(*cl.nondim14(Wg)[4:])
    expect = int((sig < 1e-4).sum())
    near = int((np.abs(sig - 1e-4) < 1e-12).sum())
    print(f'sigma-limited cells: gpu {got}, oracle {expect} (within rounding of sigma_lim: {near})',
          flush=True)
    assert 0 < expect < n * n
    assert abs(got - expect) <= near


@pytest.mark.parametrize('field', ['from_rest', 'developed'])
def test_fp32_jets_l1_error_against_fp64_oracle(gpu_lib, field):
    """FP32 face evaluation (no FP64 re-evaluation): finite, conservative at the FP64 level,
    no FP64 work counted, and its L1 error per moment stated against the FP64 oracle beside
    the mixed setting's (which re-evaluates near-Junk and near-boundary states in FP64)."""
    nx, ny = 70, 50
    W0 = I.crossed_jets_developed(nx, ny, seed=2) if field == 'developed' else I.crossed_jets_initial(nx, ny)
    n = 4 if field == 'developed' else 15
    kw = dict(JETS, nx=nx, ny=ny)
    U32, info = gpu_run(gpu_lib, dict(kw, precision='fp32'), W0, n, tau_ref=TAU_JET)
    Umx, _ = gpu_run(gpu_lib, dict(kw, precision='mixed'), W0, n, tau_ref=TAU_JET)
    base, _, _ = ob.oracle_run(kw, W0, nsteps=n, tau_ref=TAU_JET)
    b1 = np.maximum(np.abs(base).reshape(14, -1).sum(1), 1e-300)
    e32 = np.abs(U32 - base).reshape(14, -1).sum(1) / b1
    emx = np.abs(Umx - base).reshape(14, -1).sum(1) / b1
    fmt = lambda a: '[' + ' '.join(f'{x:.1e}' for x in a) + ']'       # noqa: E731
    print(f'fp32 jets {field} {n} steps: L1 relative error per moment {fmt(e32)}; mixed {fmt(emx)}',
          flush=True)
    assert np.all(np.isfinite(U32))
    assert info['n_face_states'] > 0 and info['n_fp64_states'] == 0 and info['fp64_fraction'] == 0.0
    assert np.max(e32) < 1e-2
    live = e32 > 0
    assert np.max(emx[live]) <= 1.5 * np.max(e32[live])


def test_fp32_periodic_conservation_fp64_level(gpu_lib):
    n = 64
    kw = dict(JETS, nx=n, ny=n, bc=('periodic',) * 4, jets=[], precision='fp32')
    W0 = I.random_smooth_field14(n, n, seed=12)
    U0 = mo.prim_to_cons14(W0)
    Ug, info = gpu_run(gpu_lib, kw, W0, 5, tau_ref=0.02)
    for comp in ([0], [1], [2], [3], [4, 7, 9]):
        assert abs(U0[comp].sum() - Ug[comp].sum()) < 1e-12 * np.abs(U0[comp]).sum(), comp


def test_fp32_is_rejected_by_the_adjoint(gpu_lib):
    s = gpu_lib.MaxEntSolver(**dict(JETS, nx=16, ny=16, precision='fp32'))
    try:
        s.init_state(I.crossed_jets_initial(16, 16))
        with pytest.raises(gpu_lib.MaxentError):
            s.record(2, 4)
    finally:
        s.close()

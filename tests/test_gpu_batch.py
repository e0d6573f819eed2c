"""Batched 1D tubes (maxent_create_batch / maxent_step_batch) through the C-ABI.

The batched kernel runs the single-instance 1D kernel's per-cell arithmetic (same device
functions, same update), so each batched instance must equal the same instance run alone
bit for bit, whatever launch shape the autotuner picks; the single-instance path is itself
checked against the oracle (test_gpu_parity.py), and a few small instances are checked
against the oracle directly here."""
import numpy as np
import pytest

from paper_2401_15233_amd import inputs as I
import oracle_bridge as ob

pytestmark = pytest.mark.gpu

NUM = dict(order=2, integrator='ssprk2', flux='hll', limiter='minmod', cfl=0.5)


def small_batch(seed=5, n=7):
    rng = np.random.default_rng(seed)
    sizes = [100, 60, 61, 252, 500, 124, 1000][:n]   # tile edges: 60, 124 and 252 cells
    out = []
    for k in range(n):
        out.append(dict(n=sizes[k], p_ratio=float(rng.uniform(2, 100)), rho_ratio=float(rng.uniform(2, 20)),
                        kn=float(np.exp(rng.uniform(np.log(1e-3), np.log(10)))), t_end=0.01 + 0.01 * k))
    for d in out:
        d['tau_ref'] = I.kn_to_tau_ref(d['kn'])
    return out


def run_batch(S, insts, precision='fp64', launch=None, autotune=False, reduced=True):
    b = S.MaxEntBatch(insts, precision=precision, **NUM)
    b.set_reduced(reduced)
    b.init_state(I.batch_sod_prims(insts))
    assert b.info()['reduced'] == (2 if reduced else 0)
    tuned = None
    if autotune:
        tuned = b.autotune(trial_steps=3)
    if launch:
        b.set_launch(*launch)
    info = b.step(chunk=16)
    U = b.get('conserved').cpu().numpy()
    parts = [p.copy() for p in b.split(U)]
    b.close()
    return parts, info, tuned


def run_single(S, d, precision='fp64', reduced=True):
    s = S.MaxEntSolver(system=14, dim=1, nx=d['n'], precision=precision, **NUM)
    s.set_reduced(reduced)
    s.init_state(I.batch_sod_prims([d]))
    info = s.step(10 ** 6, tau_ref=d['tau_ref'], t_end=d['t_end'])
    U = s.get('conserved').cpu().numpy()[:, 0, :]
    s.close()
    return U, info


@pytest.mark.parametrize('reduced', [True, False])
@pytest.mark.parametrize('precision', ['fp64', 'mixed'])
def test_batch_equals_instances_run_alone_bitwise(gpu_lib, precision, reduced):
    """Shock tubes from Maxwellians at rest are axially symmetric: the axial kernel (seven
    moments) runs by default, the full 14-moment kernel with the reduced mode off; each batched
    tube equals the same tube run alone with the same kernel, bit for bit."""
    insts = small_batch()
    parts, info, _ = run_batch(gpu_lib, insts, precision, reduced=reduced)
    assert info['n_active'] == 0
    for d, Ub, pi in zip(insts, parts, info['instances']):
        Us, si = run_single(gpu_lib, d, precision, reduced=reduced)
        assert pi['steps'] == si['steps'] and pi['t'] == si['t']
        assert np.array_equal(Ub, Us), d


@pytest.mark.parametrize('launch', [(64, 1, 2), (64, 2, 4), (64, 4, 8), (128, 1, 4), (128, 2, 8),
                                    (256, 1, 8), (64, 1, 16), (64, 2, 1)])
def test_batch_launch_shapes_do_not_change_results(gpu_lib, launch):
    """(threads, cells per thread, workgroups per CU): tiles of 60 to 252 cells, work-list
    ranges of one to many tiles per workgroup."""
    insts = small_batch(seed=8)
    ref, _, _ = run_batch(gpu_lib, insts, launch=(64, 1, 4))
    got, _, _ = run_batch(gpu_lib, insts, launch=launch)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_batch_autotune_keeps_state_and_results(gpu_lib):
    insts = small_batch(seed=9)
    ref, _, _ = run_batch(gpu_lib, insts, launch=(64, 1, 4))
    got, info, tuned = run_batch(gpu_lib, insts, autotune=True)
    print('autotuned launch', tuned, flush=True)
    assert tuned['threads'] in (64, 128, 256) and tuned['cells_per_thread'] in (1, 2, 4)
    assert tuned['threads'] * tuned['cells_per_thread'] <= 256 and tuned['cell_updates_per_s'] > 0
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_batch_small_instances_against_oracle(gpu_lib):
    insts = [dict(n=80, p_ratio=10.0, rho_ratio=8.0, kn=0.01, t_end=0.02),
             dict(n=131, p_ratio=50.0, rho_ratio=3.0, kn=1.0, t_end=0.015),
             dict(n=64, p_ratio=2.5, rho_ratio=15.0, kn=1e-3, t_end=0.03)]
    for d in insts:
        d['tau_ref'] = I.kn_to_tau_ref(d['kn'])
    parts, info, _ = run_batch(gpu_lib, insts)
    for d, Ub in zip(insts, parts):
        kw = dict(system=14, dim=1, nx=d['n'], **NUM)
        base, spread, t, n, nspread = ob.oracle_with_l1_spread(kw, I.batch_sod_prims([d]), d['t_end'],
                                                               d['tau_ref'])
        d1 = np.abs(Ub - base).sum(1)
        b1 = np.maximum(np.abs(base).sum(1), 1e-300)
        print(f"instance n={d['n']}: L1 relative error {np.array2string(d1 / b1, precision=1)}", flush=True)
        assert np.all(d1 <= 1e-12 * b1 + ob.SPREAD_FACTOR * spread)


def test_batch_collisionless_instance_and_status(gpu_lib):
    insts = small_batch(seed=3, n=3)
    insts[1]['tau_ref'] = 0.0
    parts, info, _ = run_batch(gpu_lib, insts)
    assert info['status'] == 'OK' and info['fail_code'] == 0
    assert all(abs(p['t'] - d['t_end']) < 1e-14 for p, d in zip(info['instances'], insts))


@pytest.mark.parametrize('bad', [(64, 3, 4), (256, 2, 4), (128, 4, 4), (32, 1, 4), (64, 1, 0), (64, 1, 33)])
def test_batch_rejects_unsupported_launch_shapes(gpu_lib, bad):
    b = gpu_lib.MaxEntBatch(small_batch(n=2), **NUM)
    try:
        with pytest.raises(gpu_lib.MaxentError):
            b.set_launch(*bad)
        assert b.launch() == (64, 1, 4)   # unchanged by the rejected calls
    finally:
        b.close()


def test_batch_queue_order_and_one_tile_instances(gpu_lib):
    """Instances of one tile or less (4 to 60 cells) between long ones, given in increasing
    order of work so that the queue reverses them: results equal each instance run alone."""
    rng = np.random.default_rng(21)
    sizes = [4, 7, 60, 61, 200, 700]
    insts = [dict(n=n, p_ratio=float(rng.uniform(2, 50)), rho_ratio=float(rng.uniform(2, 10)), kn=0.01,
                  t_end=0.004 * (k + 1)) for k, n in enumerate(sizes)]
    for d in insts:
        d['tau_ref'] = I.kn_to_tau_ref(d['kn'])
    parts, info, _ = run_batch(gpu_lib, insts, launch=(128, 2, 2))
    assert info['n_active'] == 0
    for d, Ub, pi in zip(insts, parts, info['instances']):
        Us, si = run_single(gpu_lib, d)
        assert pi['steps'] == si['steps'] and pi['t'] == si['t']
        assert np.array_equal(Ub, Us), d


@pytest.mark.parametrize('precision', ['fp64', 'mixed'])
def test_full_size_batch_sampled_tubes(gpu_lib, precision):
    """The batched workload at full size in the benchmark's launch configuration (512 tubes,
    4.29 M cells, autotuned shape, wave speeds x 1.2): after 300 steps of the whole batch,
    sampled tubes (the smallest, the largest, the strongest pressure ratio, a seeded one) equal
    the same tubes run alone bit for bit, and the smallest one matches the oracle."""
    insts = I.batch_instances()
    for d in insts:
        d['tau_ref'] = I.kn_to_tau_ref(d['kn'])
        d['t_end'] = 0.15
    num = dict(order=2, integrator='ssprk2', flux='hll', limiter='minmod', cfl=0.5, k_ws=1.2)
    b = gpu_lib.MaxEntBatch(insts, precision=precision, **num)
    b.init_state(I.batch_sod_prims(insts))
    tuned = b.autotune(trial_steps=3)
    b.init_state(I.batch_sod_prims(insts))
    info = b.step(max_steps=300, chunk=100)
    parts = b.split(b.get('conserved').cpu().numpy())
    b.close()
    print(f'{precision}: launch {tuned}, longest {info["max_steps"]} steps', flush=True)
    sizes = [d['n'] for d in insts]
    picks = {int(np.argmin(sizes)), int(np.argmax(sizes)),
             int(np.argmax([d['p_ratio'] for d in insts])), int(np.random.default_rng(4).integers(512))}
    for k in sorted(picks):
        d = insts[k]
        steps = info['instances'][k]['steps']
        s = gpu_lib.MaxEntSolver(system=14, dim=1, nx=d['n'], precision=precision, **num)
        s.init_state(I.batch_sod_prims([d]))
        si = s.step(steps, tau_ref=d['tau_ref'], t_end=d['t_end'])
        Us = s.get('conserved').cpu().numpy()[:, 0, :]
        s.close()
        assert si['steps'] == steps and si['t'] == info['instances'][k]['t']
        assert np.array_equal(parts[k], Us), (k, d['n'])
    if precision == 'fp64':
        k = int(np.argmin(sizes))
        d = insts[k]
        kw = dict(system=14, dim=1, nx=d['n'], bc=('transmissive',) * 4, **num)
        steps = info['instances'][k]['steps']
        # 300 steps through a shock with minmod: a +-4 ulp input change already moves single
        # cells by ~1e-2 of the field (limiter branches flip), so the oracle's own pointwise
        # spread is not a stable bar here; the L1 norm per moment is, as for the other long runs
        base, spread, t, n, nspread = ob.oracle_with_l1_spread(kw, I.batch_sod_prims([d]), d['t_end'],
                                                               d['tau_ref'], nsteps=steps)
        d1 = np.abs(parts[k] - base).sum(1)
        b1 = np.maximum(np.abs(base).sum(1), 1e-300)
        print(f'smallest tube ({d["n"]} cells, {steps} steps) vs oracle: L1 relative error '
              f'{np.array2string(d1 / b1, precision=1)}, oracle L1 spread '
              f'{np.array2string(spread / b1, precision=1)}', flush=True)
        assert np.all(d1 <= 1e-12 * b1 + ob.SPREAD_FACTOR * spread)
        assert n == steps and abs(t - info['instances'][k]['t']) <= 1e-9 * t

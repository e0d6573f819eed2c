"""Limits and degenerate calls on the device: an allocation beyond the card's memory reports
NOMEM and leaves a usable library behind; a zero-step call is a no-op; the smallest grids
(4 cells per axis, less than one tile) step like the oracle; a failing first stage is
reported in the same step, for the same reason, as by the oracle."""
import numpy as np
import pytest

from paper_2401_15233_amd import inputs as I
from oracle import scheme as sc
import oracle_bridge as ob
from test_gpu_parity import compare, gpu_run

pytestmark = pytest.mark.gpu


def test_allocation_beyond_memory_is_nomem(gpu_lib):
    # more than 2^31 cells: rejected before any allocation
    with pytest.raises(gpu_lib.MaxentError) as err:
        gpu_lib.MaxEntSolver(system=14, dim=2, nx=60000, ny=60000)
    assert err.value.status == 'INVAL'
    # 1.6e9 cells: two state arrays of 179 GB each do not fit the card together
    with pytest.raises(gpu_lib.MaxentError) as err:
        gpu_lib.MaxEntSolver(system=14, dim=2, nx=40000, ny=40000)
    assert err.value.status == 'NOMEM'
    # the library still works afterwards
    s = gpu_lib.MaxEntSolver(system=14, dim=1, nx=16)
    s.init_state(I.sod_prims(14, 16))
    assert s.step(2, tau_ref=0.01)['steps'] == 2
    s.close()


def test_zero_steps_is_a_no_op(gpu_lib):
    s = gpu_lib.MaxEntSolver(system=14, dim=1, nx=64)
    s.init_state(I.sod_prims(14, 64))
    U0 = s.get('conserved').cpu().numpy()
    info = s.step(0, tau_ref=0.01)
    assert info['steps'] == 0 and info['t'] == 0.0
    assert np.array_equal(s.get('conserved').cpu().numpy(), U0)
    s.close()


@pytest.mark.parametrize('kw,W0', [
    (dict(system=5, dim=1, nx=4, order=1, integrator='fe', flux='hll', cfl=0.5,
          bc=('transmissive',) * 4), I.sod_prims(5, 4)),
    (dict(system=14, dim=1, nx=4, order=2, integrator='ssprk2', flux='hll', cfl=0.5,
          limiter='minmod', bc=('periodic', 'periodic', 'transmissive', 'transmissive')),
     I.sod_prims(14, 4)),
    # CFL 0.2 (at 0.4 the first stage fails: test_stage_failure_reported_like_the_oracle)
    (dict(system=14, dim=2, nx=4, ny=4, order=2, integrator='ssprk2', flux='rusanov', cfl=0.2,
          limiter='vanalbada', bc=('reflective', 'transmissive', 'periodic', 'periodic')),
     I.random_smooth_field14(4, 4, seed=3)),
])
def test_smallest_grids_against_oracle(gpu_lib, kw, W0):
    compare(f"{kw['system']}-moment {kw['dim']}D {kw['nx']} cells", gpu_lib, kw, W0, 5,
            tau_ref=0.02)


def test_stage_failure_reported_like_the_oracle(gpu_lib):
    """At CFL 0.4 the first SSP-RK2 stage of this coarse random field has a cell whose P is
    not positive definite.  Both sides check every stage's new state (the second stage would
    evaluate the closure of the intermediate state), so both report an unrealizable state in
    step 1, although the averaged second stage happens to be admissible again."""
    kw = dict(system=14, dim=2, nx=4, ny=4, order=2, integrator='ssprk2', flux='rusanov', cfl=0.4,
              limiter='vanalbada', bc=('reflective', 'transmissive', 'periodic', 'periodic'))
    W0 = I.random_smooth_field14(4, 4, seed=3)
    with pytest.raises(sc.OracleFailure) as e:
        ob.oracle_run(kw, W0, nsteps=5, tau_ref=0.02)
    _, info = gpu_run(gpu_lib, kw, W0, 5, tau_ref=0.02, check=False)
    print(f'oracle: {e.value}; gpu: {info["status"]} in step {info["fail_step"]}', flush=True)
    assert e.value.step == 1 and e.value.reason == 'unrealizable'
    assert info['status'] == 'UNREALIZABLE' and info['fail_step'] == 1

"""The planar 14-moment system (csrc/mx_planar.hpp: the ten moments of a state even in the
z velocity) equals the full 14-moment system (csrc/mx_physics.hpp, csrc/mx_scheme.hpp) on
planar-symmetric states, function by function, to rounding, and the full system's z-odd
outputs vanish exactly there (which is why the planar kernel may leave them out).

tests/planar_host.cpp runs both on the host (the same templated code the kernels use) over
seeded planar states: in-plane Maxwellians, beam mixtures and mirrored particle sets with
random scales and boosts, and cells of the developed crossed-jets field.  Host-only build: no
GPU needed.  The full system is itself checked against the oracle on the GPU.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_2401_15233_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, 'paper_2401_15233_amd', 'csrc')
SRC = os.path.join(ROOT, 'tests', 'planar_host.cpp')

# rounding of a few dozen operations on values of similar size; the flux and closure
# expressions are the same sums with the vanishing terms left out, so agreement is at the
# level of a few ulp of the largest term
TOL = {'default': 1e-13}


def _hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.fixture(scope='module')
def results(tmp_path_factory):
    cc = _hipcc()
    if cc is None:
        pytest.skip('hipcc not available')
    d = tmp_path_factory.mktemp('planarhost')
    exe = str(d / 'planarcheck')
    cmd = [cc, '-O1', '-std=c++17', '-x', 'c++', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include',
           f'-I{CSRC}', SRC, '-o', exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    W = [inputs.random_planar_states14(400, seed=5)]
    Wj = inputs.crossed_jets_developed(48, 48, seed=2)
    W.append(Wj.reshape(14, -1)[:, ::13])
    W = np.concatenate(W, axis=1).T.copy()
    assert np.all(W[:, [3, 6, 8, 12]] == 0.0)
    path = str(d / 'states.bin')
    with open(path, 'wb') as f:
        f.write(struct.pack('i', W.shape[0]))
        f.write(W.astype(np.float64).tobytes())
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        name, rel, zodd, cnt = line.split()
        out[name] = (float(rel), float(zodd), int(cnt))
    return out


CHECKS = ['cons_to_prim', 'prim_to_cons', 'closure_x', 'closure_y', 'flux_x', 'flux_y',
          'wavespeeds_x', 'wavespeeds_y', 'source', 'equilibrium', 'cell_rate2d', 'hll_x', 'hll_y',
          'rusanov_x', 'rusanov_y', 'face_state']


@pytest.mark.parametrize('name', CHECKS)
def test_planar_equals_full_system(results, name):
    rel, zodd, cnt = results[name]
    print(f'{name}: max relative difference {rel:.2e}, largest z-odd output {zodd:.1e} ({cnt} cases)')
    assert cnt > 0
    assert rel <= TOL['default'], name
    assert zodd == 0.0, name


def test_limiter_factor_is_identical(results):
    """The z-odd variables have no jumps, so they are neutral in the common limiter: the
    factor is the same arithmetic on the same carried variables, bit for bit."""
    rel, _, cnt = results['limiter_factor']
    assert cnt > 0 and rel == 0.0


def test_admissibility_agrees(results):
    mismatch, _, cnt = results['admissible_mismatch']
    assert cnt > 0 and mismatch == 0

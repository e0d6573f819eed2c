"""The host checks of the library's templated pointwise code (tests/adjoint_host.cpp,
tests/planar_host.cpp, tests/tangent_host.cpp) rebuilt with AddressSanitizer and
UndefinedBehaviorSanitizer and run on the inputs of their own tests: no out-of-bounds access,
use of uninitialised stack memory through a bad index, signed overflow or other undefined
behaviour in the closure, wave speeds, fluxes, reconstruction, boundary handling and their
reverse and tangent code, and the plain builds' accuracy bars still met.  Host code only: the
sanitizer flags go to the host compilation; no GPU code is built.  CPU only."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_2401_15233_amd import inputs
from oracle import moments as mo
import tangent_tools as tt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, 'paper_2401_15233_amd', 'csrc')
SAN = ['-Xarch_host', '-fsanitize=address', '-Xarch_host', '-fsanitize=undefined',
       '-Xarch_host', '-fno-sanitize-recover=undefined', '-fno-omit-frame-pointer', '-g']
ENV = dict(os.environ, ASAN_OPTIONS='abort_on_error=0:halt_on_error=1',
           UBSAN_OPTIONS='print_stacktrace=1:halt_on_error=1')


def _hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    return None


def _build(src, out):
    cc = _hipcc()
    if cc is None:
        pytest.skip('hipcc not available')
    cmd = [cc, '-O1', '-std=c++17', '-x', 'c++', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include',
           f'-I{CSRC}', *SAN, os.path.join(ROOT, 'tests', src), '-o', out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _clean(r):
    assert r.returncode == 0, r.stderr[-4000:]
    assert 'AddressSanitizer' not in r.stderr and 'runtime error' not in r.stderr, r.stderr[-4000:]


def _write_states(path, W):
    with open(path, 'wb') as f:
        f.write(struct.pack('i', W.shape[0]))
        f.write(np.ascontiguousarray(W, dtype=np.float64).tobytes())


def test_adjoint_host_check_under_sanitizers(tmp_path):
    exe = _build('adjoint_host.cpp', str(tmp_path / 'adjcheck'))
    W = [inputs.random_states14(96, seed=11),
         inputs.crossed_jets_developed(48, 48, seed=2).reshape(14, -1)[:, ::97]]
    path = str(tmp_path / 'states.bin')
    _write_states(path, np.concatenate(W, axis=1).T)
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=600, env=ENV)
    _clean(r)
    out = {l.split()[0]: l.split()[1:] for l in r.stdout.splitlines()}
    for name in ('cons_to_prim', 'face_terms_x', 'face_terms_y', 'face_flux_hll', 'recon_minmod'):
        assert float(out[name][0]) <= 1e-13, name


@pytest.mark.parametrize('which', ['planar', 'axial'])
def test_reduced_system_host_check_under_sanitizers(tmp_path, which):
    exe = _build('planar_host.cpp', str(tmp_path / 'planarcheck'))
    if which == 'planar':
        W = [inputs.random_planar_states14(200, seed=5),
             inputs.crossed_jets_developed(48, 48, seed=2).reshape(14, -1)[:, ::13]]
    else:
        W = [inputs.random_axial_states14(200, seed=6), inputs.sod_prims(14, 200).reshape(14, -1)[:, ::3]]
    path = str(tmp_path / f'{which}.bin')
    _write_states(path, np.concatenate(W, axis=1).T)
    r = subprocess.run([exe, which, path], capture_output=True, text=True, timeout=600, env=ENV)
    _clean(r)
    for line in r.stdout.splitlines():
        name, rel, zodd, cnt = line.split()
        if name != 'admissible_mismatch':
            assert float(rel) <= 1e-13 and float(zodd) == 0.0, (which, name)


def test_tangent_host_under_sanitizers(tmp_path, monkeypatch):
    exe = _build('tangent_host.cpp', str(tmp_path / 'tangent_host'))
    n = 10
    U0 = mo.prim_to_cons14(inputs.crossed_jets_developed(n, n, seed=5))
    rng = np.random.default_rng(3)
    w = rng.standard_normal(U0.shape) / (n * n)
    v = rng.standard_normal(U0.shape) * 1e-3
    monkeypatch.setenv('ASAN_OPTIONS', ENV['ASAN_OPTIONS'])
    monkeypatch.setenv('UBSAN_OPTIONS', ENV['UBSAN_OPTIONS'])
    for seed in ('mach', 'U0'):
        J, dJ = tt.tangent(exe, U0, w, [2e-4, 2e-4], seed, tau=1e-3, v=v)
        assert np.isfinite(J) and np.isfinite(dJ)

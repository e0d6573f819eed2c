"""The hand-written reverse-mode pieces (csrc/mx_adjoint.hpp) are exact transposes of the
forward code's derivatives.

tests/adjoint_host.cpp instantiates the templated forward physics with a dual-number type
(forward mode, exact derivatives of the same code) and checks, for every reverse function,
ybar . (J xdot) == (J^T ybar) . xdot to rounding on seeded random states: primitive recovery,
conserved map, closure + wave speeds + flux of a face state along x and y, the BGK source
(local and constant tau, and its tau_ref derivative), the HLL and Rusanov interface fluxes in
all three HLL cases, and the limited reconstruction (minmod and van Albada, neutral
variables, positivity fallback).  The dual type is checked against central differences.
Host-only build: no GPU needed.
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
SRC = os.path.join(ROOT, 'tests', 'adjoint_host.cpp')


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
    d = tmp_path_factory.mktemp('adjhost')
    exe = str(d / 'adjcheck')
    cmd = [cc, '-O1', '-std=c++17', '-x', 'c++', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include',
           f'-I{CSRC}', SRC, '-o', exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # states: every family of the seeded generator, plus developed crossed-jet cells
    W = [inputs.random_states14(96, seed=11)]
    Wj = inputs.crossed_jets_developed(48, 48, seed=2)
    W.append(Wj.reshape(14, -1)[:, ::97])
    W = np.concatenate(W, axis=1).T.copy()
    path = str(d / 'states.bin')
    with open(path, 'wb') as f:
        f.write(struct.pack('i', W.shape[0]))
        f.write(W.astype(np.float64).tobytes())
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = {}
    for line in r.stdout.splitlines():
        parts = line.split()
        if parts[0] == 'hll_branches':
            out['hll_branches'] = [int(x) for x in parts[1:]]
        else:
            out[parts[0]] = (float(parts[1]), int(parts[2]))
    return out


@pytest.mark.parametrize('name', ['cons_to_prim', 'prim_to_cons', 'face_terms_x', 'face_terms_y',
                                  'source_local', 'source_const', 'source_tau_ref', 'face_flux_hll',
                                  'face_flux_rusanov', 'recon_minmod', 'recon_vanalbada'])
def test_reverse_is_transpose_of_forward_derivative(results, name):
    err, n = results[name]
    assert n > 50
    assert err <= 1e-13, (name, err)


def test_reverse_limiter_selects_the_forward_factor(results):
    err, n = results['limiter_phi_equal']
    assert n > 100 and err == 0.0


def test_dual_numbers_match_central_differences(results):
    err, n = results['dual_vs_fd']
    assert n > 100 and err <= 1e-6


def test_interface_reverse_split_over_two_threads(results):
    """interface_side_vjp (each face state's share, from the pair's wave speeds and the flux
    adjoint's products with both sides' U and F) equals interface_vjp's outputs for that side,
    in every HLL case, for Rusanov, and with every min / max tied: the U and F adjoints bit for
    bit, the wave-speed adjoints (sums over the components taken in another order) to within
    1e-14 of the absolute sums they are formed from."""
    err, n = results['interface_side_split']
    assert n > 10000 and err == 0.0
    err, n = results['interface_side_speeds']
    assert n > 1000 and err <= 1e-14, err


def test_every_hll_case_is_exercised(results):
    assert min(results['hll_branches']) > 0

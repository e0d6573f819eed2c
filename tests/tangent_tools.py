"""Build and run tests/tangent_host.cpp (host tangent-linear reference of the crossed-jets
scheme, dual numbers through the library's templated pointwise code).  Test helper."""
import os
import shutil
import struct
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, 'paper_2401_15233_amd', 'csrc')
SRC = os.path.join(ROOT, 'tests', 'tangent_host.cpp')
SEEDS = {'mach': 0, 'rho': 1, 'tau': 2, 'U0': 3}


def hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    return None


def build(outdir):
    exe = os.path.join(outdir, 'tangent_host')
    cmd = [hipcc(), '-O2', '-std=c++17', '-x', 'c++', '-D__HIP_PLATFORM_AMD__', '-I/opt/rocm/include',
           f'-I{CSRC}', SRC, '-o', exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-4000:])
    return exe


CROSSED_JETS = ((0.35, 0.1, 30.0, 0), (0.65, 0.1, -30.0, 0))
WALLS = {'xlo': 0, 'xhi': 1, 'ylo': 2, 'yhi': 3}


def tangent(exe, U0, w, dts, seed, mach=3.0, rho=1.0, T=1.0, tau=0.0, v=None, frozen=False,
            integrator='ssprk2', limiter='minmod', jets=CROSSED_JETS):
    """(J, dJ) along `seed` ('mach', 'rho', 'tau' or 'U0' with direction v).  jets: (centre,
    width, angle, wall) per jet, wall 0..3 or its name."""
    nv, ny, nx = U0.shape
    if v is None:
        v = np.zeros_like(U0)
    with tempfile.NamedTemporaryFile(suffix='.bin', delete=False) as f:
        f.write(struct.pack('5i', nx, ny, len(dts), SEEDS[seed], int(bool(frozen))))
        f.write(struct.pack('4d', mach, rho, T, tau))
        f.write(struct.pack('3i', {'fe': 0, 'ssprk2': 1}[integrator],
                            {'minmod': 0, 'vanalbada': 1}[limiter], len(jets)))
        for j in jets:
            wall = j[3] if len(j) > 3 else 0
            f.write(struct.pack('4d', j[0], j[1], j[2], float(WALLS.get(wall, wall))))
        f.write(np.asarray(dts, dtype=np.float64).tobytes())
        for a in (U0, v, w):
            f.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        path = f.name
    try:
        r = subprocess.run([exe, path], capture_output=True, text=True, timeout=600)
    finally:
        os.unlink(path)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    J, dJ = (float(x) for x in r.stdout.split())
    return J, dJ

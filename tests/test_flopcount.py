"""The algorithmic operation counts bench.py uses for the roofline are what the library's
own device code performs (counted by paper_2401_15233_amd/csrc/flopcount.cpp on the host)."""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_flop_constants_match_the_counter(tmp_path):
    hipcc = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(hipcc):
        pytest.skip('hipcc not available')
    csrc = os.path.join(ROOT, 'paper_2401_15233_amd', 'csrc')
    exe = str(tmp_path / 'flopcount')
    subprocess.run([hipcc, '-x', 'hip', '--offload-arch=gfx950', '-O1', '-std=c++17', f'-I{csrc}',
                    os.path.join(csrc, 'flopcount.cpp'), '-o', exe], check=True,
                   stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    out = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    import bench
    assert bench.FLOPS_PER_CELL_STAGE == {1: out['flops_stage1'], 2: out['flops_stage2']}
    assert bench.PLANAR_FLOPS_PER_CELL_STAGE == {1: out['planar_flops_stage1'],
                                                 2: out['planar_flops_stage2']}
    # the planar kernel carries 10 of the 14 moments (the z-odd four vanish by symmetry)
    assert bench.PLANAR_BYTES_PER_CELL_STAGE == {k: v * 10 / 14 for k, v in bench.BYTES_PER_CELL_STAGE.items()}

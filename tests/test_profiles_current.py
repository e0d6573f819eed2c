"""The committed rocprofv3 summaries describe the kernels in the tree: the stage kernel's HBM
traffic and VALU-busy summaries carry the hash of the kernel sources they were measured on,
and bench.py reports them (roofline.traffic, roofline.valu_busy) only while that hash matches.
A kernel change without a new profile would silently turn both into null.  CPU only."""
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hash_in(path):
    m = re.search(r'^kernel_source_hash:\s*(\S+)', open(os.path.join(ROOT, path)).read(), re.M)
    return m.group(1) if m else None


def test_stage_kernel_profiles_match_the_sources():
    h = bench.kernel_source_hash()
    for path in (bench.TRAFFIC_PROFILE, bench.VALU_PROFILE,
                 'profiles/stage_kernel_jets2048_fp64_stalls.txt'):
        assert _hash_in(path) == h, path
    traffic = bench.measured_traffic()
    busy = bench.measured_valu_busy()
    assert traffic is not None and busy is not None
    # the measured bytes cover at least the planar kernel's own state passes, and the busy
    # fraction is a fraction
    cells = 2048 * 2048
    own = cells * 0.5 * (bench.PLANAR_BYTES_PER_CELL_STAGE[1] + bench.PLANAR_BYTES_PER_CELL_STAGE[2])
    assert traffic >= own
    assert 0.0 < busy <= 1.0


def test_profiles_are_short_text_summaries_with_their_commands():
    d = os.path.join(ROOT, 'profiles')
    for name in os.listdir(d):
        path = os.path.join(d, name)
        assert name.endswith(('.txt', '.md')), name
        assert os.path.getsize(path) < 64 * 1024, name
        text = open(path).read()
        assert 'rocprofv3' in text and 'command' in text, name

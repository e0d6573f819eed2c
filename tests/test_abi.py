"""The C-ABI library loads, exports every symbol include/maxent.h declares, and validates
arguments before touching a device (no compute calls here: no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2401_15233_amd import solver as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'maxent.h')


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
    return sorted(set(re.findall(r'\b(maxent_[a-z_]+)\s*\(', text)))


@pytest.fixture(scope='module')
def lib():
    if not os.path.exists(S.LIB_PATH):
        pytest.fail('libmaxent.so is not built (run python -m paper_2401_15233_amd.build)')
    return S.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(S.EXPORTED) <= set(names)


def test_abi_version(lib):
    assert lib.maxent_abi_version() == 4


def test_struct_layouts_match_header():
    """ctypes mirrors of the header structs have the C layout (size and field offsets)."""
    assert ctypes.sizeof(S.Problem) == 4 * 4 + 4 * 8 + 4 * 4 + 4 + 4 + 12 * 8 + 3 * 8 + 8 + 2 * 8 + 4 * 4
    assert S.Problem.x0.offset == 16 and S.Problem.n_jets.offset == 64
    assert S.Problem.jet_wall.offset == 216
    assert ctypes.sizeof(S.Numerics) == 5 * 4 + 4 + 3 * 8 + 4 + 4
    assert S.Numerics.source_implicit.offset == 52
    assert ctypes.sizeof(S.Info) == 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8 + 8 + 8 + 4 + 4
    assert S.Info.n_sigma_limited.offset == 56 and S.Info.fp64_fraction.offset == 64
    assert S.Info.reduced.offset == 72


def test_struct_layout_matches_the_c_compiler(tmp_path):
    """sizeof / offsetof of the header's structs, printed by a C program built with the host
    compiler, equal the ctypes mirrors'."""
    import shutil
    import subprocess
    cc = shutil.which('gcc') or shutil.which('cc')
    if cc is None:
        pytest.skip('no host C compiler')
    structs = {'maxent_problem': S.Problem, 'maxent_numerics': S.Numerics, 'maxent_info': S.Info,
               'maxent_instance': S.Instance, 'maxent_batch_info': S.BatchInfo,
               'maxent_instance_info': S.InstanceInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / 'layout.c'
    src.write_text('\n'.join(lines) + '\n')
    exe = tmp_path / 'layout'
    subprocess.run([cc, '-std=c99', str(src), '-o', str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split('\n')
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, 'size')] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


@pytest.mark.parametrize('bad', [
    dict(system=7), dict(system=5, dim=2, ny=8), dict(nx=2), dict(dim=1, ny=4),
    dict(bc=('periodic', 'transmissive', 'transmissive', 'transmissive')),
    dict(dim=2, ny=8, bc=('transmissive', 'jet', 'transmissive', 'transmissive')),
    dict(bc=('jet', 'transmissive', 'transmissive', 'transmissive')),
    dict(dim=2, ny=8, bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
         jets=[(0.5, 0.2, 0.0, 'ylo')]),                      # the jet's wall is not JET
    dict(dim=2, ny=8, bc=('jet', 'transmissive', 'jet', 'transmissive'),
         jets=[(0.5, 0.2, 0.0, 'xlo')]),                      # a JET side without a jet
    dict(dim=2, ny=8, bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
         jets=[(0.5, 0.2, 0.0, 7)]),                          # no such wall
    dict(x1=-1.0)])
def test_create_rejects_bad_problem(lib, bad):
    kw = dict(system=14, dim=1, nx=16, ny=1)
    kw.update(bad)
    p = S.make_problem(**kw)
    n = S.make_numerics()
    h = ctypes.c_void_p()
    rc = lib.maxent_create(ctypes.byref(p), ctypes.byref(n), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert len(lib.maxent_last_error(None)) > 0


@pytest.mark.parametrize('bad', [dict(order=3), dict(cfl=0.0), dict(cfl=1.5), dict(sigma_lim=0.0),
                                 dict(k_ws=0.5), dict(source_implicit=True),
                                 dict(source_implicit=True, integrator='midpoint')])
def test_create_rejects_bad_numerics(lib, bad):
    p = S.make_problem(system=14, dim=1, nx=16)
    n = S.make_numerics(**bad)
    h = ctypes.c_void_p()
    assert lib.maxent_create(ctypes.byref(p), ctypes.byref(n), None, ctypes.byref(h)) == -1


def test_null_handle_calls_are_rejected(lib):
    info = S.Info()
    assert lib.maxent_step(None, 1, 0.0, 0.0, 0.0, ctypes.byref(info)) == -1
    assert lib.maxent_init_state(None, 0, None, 0, 0.0) == -1
    assert lib.maxent_get_moments(None, 0, None, 0) == -1
    assert lib.maxent_num_vars(None) == 0
    lib.maxent_destroy(None)


@pytest.mark.parametrize('bad', [dict(system=5), dict(order=1), dict(integrator='fe'),
                                 dict(n=3), dict(x1=-1.0), dict(t_end=0.0)])
def test_create_batch_rejects_bad_arguments(lib, bad):
    prob_kw = {'system': bad.get('system', 14)}
    num_kw = {k: v for k, v in bad.items() if k in ('order', 'integrator')}
    p = S.make_problem(**prob_kw)
    n = S.make_numerics(**num_kw)
    inst = (S.Instance * 2)()
    for k in range(2):
        inst[k].x0, inst[k].x1 = 0.0, bad.get('x1', 1.0)
        inst[k].tau_ref, inst[k].t_end = 0.01, bad.get('t_end', 0.1)
        inst[k].n_cells = bad.get('n', 64)
    h = ctypes.c_void_p()
    assert lib.maxent_create_batch(ctypes.byref(p), ctypes.byref(n), 2, inst, None, ctypes.byref(h)) == -1
    assert not h.value


def test_batch_rejects_fp32_precision(lib):
    """FP32 face evaluation is a single-solver setting; the batch takes FP64 or MIXED."""
    p = S.make_problem(system=14, dim=1, nx=16)
    n = S.make_numerics(precision='fp32')
    inst = (S.Instance * 1)()
    inst[0].x0, inst[0].x1, inst[0].tau_ref, inst[0].t_end, inst[0].n_cells = 0.0, 1.0, 0.01, 0.1, 16
    h = ctypes.c_void_p()
    assert lib.maxent_create_batch(ctypes.byref(p), ctypes.byref(n), 1, inst, None, ctypes.byref(h)) == -1
    assert b'FP64 or MIXED' in lib.maxent_last_error(None)

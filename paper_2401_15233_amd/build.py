"""Build the gfx950 shared library ``libmaxent.so`` in-tree with hipcc.

Usage: ``python -m paper_2401_15233_amd.build`` (or ``build()`` from Python).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'libmaxent.so')
SOURCES = ['mx_api.hip', 'mx_kernels.hip', 'mx_batch.hip', 'mx_adjoint.hip']
ARCH = os.environ.get('MAXENT_OFFLOAD_ARCH', 'gfx950')


def hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError('hipcc not found (set HIPCC)')


def flags():
    return ['-O3', f'--offload-arch={ARCH}', '-std=c++17', '-fPIC',
            # packed FP32 instructions are disabled for all device code of this library
            '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
            '-munsafe-fp-atomics', '-Wno-unused-command-line-argument',
            # single-precision division and square root of the mixed-precision path need
            # not be correctly rounded (about 1 ulp is enough there)
            '-fno-hip-fp32-correctly-rounded-divide-sqrt',
            f'-I{os.path.join(ROOT, "include")}', f'-I{CSRC}']


# Per-source additions.  The adjoint kernels are compiled without signed zeros, NaN or
# infinity: their planar runs read the four z-odd moments as the constant 0, and only under
# these assumptions may the compiler drop x * 0 and x + 0 (the adjoint runs only on recorded
# runs that stayed finite, and a signed zero changes no later value there).
SOURCE_FLAGS = {'mx_adjoint.hip': ['-fno-signed-zeros', '-ffinite-math-only']}


def build(verbose=False, extra=()):
    """Compile every source into LIB.  Always recompiles."""
    cc = hipcc()
    objs = []
    build_dir = os.path.join(ROOT, '_build')
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src.replace('.hip', '.o'))
        cmd = [cc, *flags(), *SOURCE_FLAGS.get(src, []), *extra, '-c', os.path.join(CSRC, src), '-o', obj]
        if verbose:
            print(' '.join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
    for p, src in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors='replace'))
            raise RuntimeError(f'hipcc failed on {src}')
        if verbose and out:
            sys.stderr.write(out.decode(errors='replace'))
    tmp = LIB + '.tmp'
    cmd = [cc, f'--offload-arch={ARCH}', '-shared', '-fPIC', '-o', tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    build(verbose='-v' in sys.argv)
    print(LIB)

"""Python binding of ``libmaxent.so`` (the C-ABI in include/maxent.h).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch provides device buffers and the current HIP stream.  There is no CPU fallback:
if the library is not built or cannot be loaded, every entry point raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libmaxent.so')

MAXENT_OK = 0
STATUS = {-1: 'INVAL', -2: 'NOMEM', -3: 'DEVICE', -4: 'NONFINITE', -5: 'UNREALIZABLE',
          -6: 'STATE'}
BC = {'transmissive': 0, 'periodic': 1, 'reflective': 2, 'jet': 3}
WALL = {'xlo': 0, 'xhi': 1, 'ylo': 2, 'yhi': 3}
LIMITER = {'minmod': 0, 'vanalbada': 1}
FLUX = {'hll': 0, 'rusanov': 1}
INTEGRATOR = {'fe': 0, 'ssprk2': 1, 'midpoint': 2}
TAU_MODE = {'local': 0, 'const': 1}
REPR = {'primitive': 0, 'conserved': 1, 'sigma': 2, 'closing': 3}
PRECISION = {'fp64': 0, 'fp32': 1, 'mixed': 2}
CLOSING_COMPONENTS_14 = 19
ADJOINT_MODE = {'exact': 0, 'frozen_limiter': 1}

EXPORTED = ('maxent_create', 'maxent_init_state', 'maxent_step', 'maxent_get_moments',
            'maxent_num_vars', 'maxent_get_info', 'maxent_destroy', 'maxent_last_error',
            'maxent_abi_version', 'maxent_set_profiling', 'maxent_get_profile',
            'maxent_create_batch', 'maxent_step_batch', 'maxent_set_batch_launch',
            'maxent_get_batch_launch', 'maxent_autotune_batch', 'maxent_record',
            'maxent_set_inflow', 'maxent_step_adjoint', 'maxent_tape_info',
            'maxent_set_adjoint_mode', 'maxent_step_noalloc', 'maxent_set_reduced')


class MaxentError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f'{STATUS.get(code, code)}: {msg}')
        self.code = code
        self.status = STATUS.get(code, str(code))


class Problem(ctypes.Structure):
    _fields_ = [('system', ctypes.c_int), ('dim', ctypes.c_int), ('nx', ctypes.c_int),
                ('ny', ctypes.c_int), ('x0', ctypes.c_double), ('x1', ctypes.c_double),
                ('y0', ctypes.c_double), ('y1', ctypes.c_double), ('bc', ctypes.c_int * 4),
                ('n_jets', ctypes.c_int), ('jet_yc', ctypes.c_double * 4),
                ('jet_width', ctypes.c_double * 4), ('jet_angle_deg', ctypes.c_double * 4),
                ('jet_mach', ctypes.c_double), ('jet_rho', ctypes.c_double),
                ('jet_T', ctypes.c_double), ('tau_mode', ctypes.c_int),
                ('rho_ref', ctypes.c_double), ('T_ref', ctypes.c_double),
                ('jet_wall', ctypes.c_int * 4)]


class Numerics(ctypes.Structure):
    _fields_ = [('precision', ctypes.c_int), ('order', ctypes.c_int), ('limiter', ctypes.c_int),
                ('flux', ctypes.c_int), ('integrator', ctypes.c_int), ('cfl', ctypes.c_double),
                ('sigma_lim', ctypes.c_double), ('k_ws', ctypes.c_double),
                ('positivity_fallback', ctypes.c_int), ('source_implicit', ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [('t', ctypes.c_double), ('dt_last', ctypes.c_double),
                ('steps', ctypes.c_longlong), ('n_fallback', ctypes.c_longlong),
                ('fail_step', ctypes.c_int), ('fail_code', ctypes.c_int),
                ('n_fp64_states', ctypes.c_longlong), ('n_face_states', ctypes.c_longlong),
                ('n_sigma_limited', ctypes.c_longlong), ('fp64_fraction', ctypes.c_double),
                ('reduced', ctypes.c_int), ('reserved', ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [('x0', ctypes.c_double), ('x1', ctypes.c_double), ('tau_ref', ctypes.c_double),
                ('t_end', ctypes.c_double), ('n_cells', ctypes.c_int), ('pad', ctypes.c_int)]


class InstanceInfo(ctypes.Structure):
    _fields_ = [('t', ctypes.c_double), ('dt_last', ctypes.c_double), ('steps', ctypes.c_longlong),
                ('fail_step', ctypes.c_int), ('fail_code', ctypes.c_int)]


class BatchInfo(ctypes.Structure):
    _fields_ = [('max_steps', ctypes.c_longlong), ('cell_updates', ctypes.c_longlong),
                ('n_active', ctypes.c_longlong), ('n_fallback', ctypes.c_longlong),
                ('n_fp64_states', ctypes.c_longlong), ('n_face_states', ctypes.c_longlong),
                ('fail_step', ctypes.c_int), ('fail_code', ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path=LIB_PATH):
    """Load the HIP library (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f'{path} is not built; run `python -m paper_2401_15233_amd.build`')
    # PyTorch-ROCm ships its own HIP runtime under the same soname as the system one: load
    # torch first so that the library binds to that runtime.  Loading the library first would
    # put a second HIP runtime into the process, and device discovery then fails.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.maxent_create.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Numerics), vp,
                                ctypes.POINTER(vp)]
    L.maxent_init_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_double]
    L.maxent_step.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.POINTER(Info)]
    L.maxent_get_moments.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    L.maxent_num_vars.argtypes = [vp]
    L.maxent_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.maxent_destroy.argtypes = [vp]
    L.maxent_destroy.restype = None
    L.maxent_last_error.argtypes = [vp]
    L.maxent_last_error.restype = ctypes.c_char_p
    L.maxent_abi_version.argtypes = []
    L.maxent_set_profiling.argtypes = [vp, ctypes.c_int]
    L.maxent_create_batch.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Numerics), ctypes.c_int,
                                      ctypes.POINTER(Instance), vp, ctypes.POINTER(vp)]
    L.maxent_step_batch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(BatchInfo),
                                    ctypes.POINTER(InstanceInfo)]
    L.maxent_set_batch_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    pint = ctypes.POINTER(ctypes.c_int)
    L.maxent_get_batch_launch.argtypes = [vp, pint, pint, pint]
    L.maxent_autotune_batch.argtypes = [vp, ctypes.c_int, pint, pint, pint, ctypes.POINTER(ctypes.c_double)]
    L.maxent_get_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_longlong)]
    L.maxent_record.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.maxent_set_inflow.argtypes = [vp, ctypes.c_double, ctypes.c_double]
    L.maxent_tape_info.argtypes = [vp, ctypes.POINTER(ctypes.c_longlong), vp]
    L.maxent_set_adjoint_mode.argtypes = [vp, ctypes.c_int]
    L.maxent_set_reduced.argtypes = [vp, ctypes.c_int]
    L.maxent_step_adjoint.argtypes = [vp, vp, ctypes.c_int, vp, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_double)]
    L.maxent_step_noalloc.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Numerics), vp,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, vp, ctypes.POINTER(Info)]
    _lib = L
    return L


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError('no HIP device visible to torch')
    return torch


def make_problem(system=14, dim=1, nx=100, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                 bc=('transmissive',) * 4, jets=(), jet_mach=3.0, jet_rho=1.0, jet_T=1.0,
                 tau_mode='local', rho_ref=1.0, T_ref=1.0):
    p = Problem()
    p.system, p.dim, p.nx, p.ny = system, dim, nx, ny
    p.x0, p.x1, p.y0, p.y1 = x0, x1, y0, y1
    for k, b in enumerate(bc):
        p.bc[k] = BC[b] if isinstance(b, str) else int(b)
    p.n_jets = len(jets)
    for k, jet in enumerate(jets):
        # (centre along the wall, width, angle in degrees[, wall]); wall 0 x-low (default),
        # 1 x-high, 2 y-low, 3 y-high, or its name
        p.jet_yc[k], p.jet_width[k], p.jet_angle_deg[k] = jet[:3]
        w = jet[3] if len(jet) > 3 else 0
        p.jet_wall[k] = WALL[w] if isinstance(w, str) else int(w)
    p.jet_mach, p.jet_rho, p.jet_T = jet_mach, jet_rho, jet_T
    p.tau_mode = TAU_MODE[tau_mode] if isinstance(tau_mode, str) else int(tau_mode)
    p.rho_ref, p.T_ref = rho_ref, T_ref
    return p


def make_numerics(precision='fp64', order=2, limiter='minmod', flux='hll', integrator='ssprk2',
                  cfl=0.5, sigma_lim=1e-4, k_ws=1.0, positivity_fallback=True, source_implicit=False):
    n = Numerics()
    n.precision = PRECISION[precision]
    n.order = order
    n.limiter = LIMITER[limiter]
    n.flux = FLUX[flux]
    n.integrator = INTEGRATOR[integrator]
    n.cfl, n.sigma_lim, n.k_ws = cfl, sigma_lim, k_ws
    n.positivity_fallback = int(bool(positivity_fallback))
    n.source_implicit = int(bool(source_implicit))
    return n


_PROBLEM_KEYS = ('system', 'dim', 'nx', 'ny', 'x0', 'x1', 'y0', 'y1', 'bc', 'jets', 'jet_mach',
                 'jet_rho', 'jet_T', 'tau_mode', 'rho_ref', 'T_ref')


class MaxEntSolver:
    """One solver instance on the current HIP device and stream.

    init_state(W) -> step(n, dt, tau_ref, t_end) -> get('primitive' | 'conserved' | 'sigma').
    Fields are [nv][ny][nx] float64 (torch CUDA tensors or NumPy arrays on input; torch CUDA
    tensors on output)."""

    # bumped by every call that changes the state or the recorded tape, so that a reverse
    # pass can tell whether the tape is still the one it was taken for
    generation = 0

    def __init__(self, stream=None, **kw):
        self._lib = load_library()
        torch = _torch()
        pk = {k: v for k, v in kw.items() if k in _PROBLEM_KEYS}
        nk = {k: v for k, v in kw.items() if k not in _PROBLEM_KEYS}
        self.problem = make_problem(**pk)
        self.numerics = make_numerics(**nk)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = ctypes.c_void_p()
        rc = self._lib.maxent_create(ctypes.byref(self.problem), ctypes.byref(self.numerics),
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != MAXENT_OK:
            raise MaxentError(rc, self._lib.maxent_last_error(None).decode())
        self._h = h
        self.nv = self._lib.maxent_num_vars(h)
        self.shape = (self.nv, self.problem.ny, self.problem.nx)

    def _check(self, rc):
        if rc != MAXENT_OK:
            raise MaxentError(rc, self._lib.maxent_last_error(self._h).decode())

    def close(self):
        self.generation += 1
        if getattr(self, '_h', None):
            self._lib.maxent_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_state(self, field, repr='primitive', t0=0.0):
        torch = _torch()
        self.generation += 1
        if isinstance(field, np.ndarray):
            a = np.ascontiguousarray(field, dtype=np.float64)
            if a.size != int(np.prod(self.shape)):
                raise ValueError(f'field has {a.size} values, expected shape {self.shape}')
            rc = self._lib.maxent_init_state(self._h, REPR[repr], a.ctypes.data_as(ctypes.c_void_p),
                                             0, float(t0))
        else:
            a = field.to(dtype=torch.float64).contiguous()
            if a.numel() != int(np.prod(self.shape)) or not a.is_cuda:
                raise ValueError(f'field must be a CUDA tensor with shape {self.shape}')
            rc = self._lib.maxent_init_state(self._h, REPR[repr], ctypes.c_void_p(a.data_ptr()), 1,
                                             float(t0))
        self._check(rc)

    def step(self, n, dt=0.0, tau_ref=0.0, t_end=0.0, check=True):
        self.generation += 1
        info = Info()
        rc = self._lib.maxent_step(self._h, int(n), float(dt), float(tau_ref), float(t_end),
                                   ctypes.byref(info))
        if check:
            self._check(rc)
        d = info.as_dict()
        d['status'] = STATUS.get(rc, 'OK') if rc else 'OK'
        return d

    def set_profiling(self, enable=True):
        self._check(self._lib.maxent_set_profiling(self._h, int(bool(enable))))

    def profile(self):
        """(total milliseconds, launches) of the stage kernels since profiling was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        self._check(self._lib.maxent_get_profile(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def info(self):
        info = Info()
        self._check(self._lib.maxent_get_info(self._h, ctypes.byref(info)))
        return info.as_dict()

    def get(self, repr='primitive', out=None):
        """'primitive' | 'conserved' ([nv][ny][nx]), 'sigma' ([ny][nx]), 'closing' (closing
        moments: [19][ny][nx] for 14 moments, [ny][nx] for 5)."""
        torch = _torch()
        if repr == 'sigma' or (repr == 'closing' and self.nv == 5):
            shape = self.shape[1:]
        elif repr == 'closing':
            shape = (CLOSING_COMPONENTS_14,) + self.shape[1:]
        else:
            shape = self.shape
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device='cuda')
        self._check(self._lib.maxent_get_moments(self._h, REPR[repr], ctypes.c_void_p(out.data_ptr()), 1))
        return out


    # ---------------------------------------------------------------- discrete adjoint
    def record(self, checkpoint_every, max_steps):
        """Start a tape at the current state (checkpoint_every = 0 ends it)."""
        self.generation += 1
        self._check(self._lib.maxent_record(self._h, int(checkpoint_every), int(max_steps)))

    def set_inflow(self, mach, rho):
        self.generation += 1
        self._check(self._lib.maxent_set_inflow(self._h, float(mach), float(rho)))
        self.problem.jet_mach, self.problem.jet_rho = float(mach), float(rho)

    def set_adjoint_mode(self, mode):
        """'exact' (default) or 'frozen_limiter'."""
        self._check(self._lib.maxent_set_adjoint_mode(self._h, ADJOINT_MODE[mode]))

    def set_reduced(self, enable):
        """Symmetric 14-moment states (2D planar, 1D axial) run the reduced stage kernels
        (True, the default) or always the full 14-moment kernels (False)."""
        self._check(self._lib.maxent_set_reduced(self._h, 1 if enable else 0))

    def tape(self):
        """Time steps of the recorded steps (NumPy array)."""
        n = ctypes.c_longlong()
        self._check(self._lib.maxent_tape_info(self._h, ctypes.byref(n), None))
        dt = np.zeros(max(n.value, 1))
        self._check(self._lib.maxent_tape_info(self._h, ctypes.byref(n), dt.ctypes.data_as(ctypes.c_void_p)))
        return dt[:n.value]

    def adjoint(self, dJ_dU, want_dU0=True):
        """Reverse the tape: returns (dJ/dU0 as a CUDA tensor or None, [dJ/dM, dJ/drho_jet,
        dJ/dtau_ref]).  dJ_dU: conserved-shaped CUDA tensor or NumPy array."""
        torch = _torch()
        g = (ctypes.c_double * 3)()
        out = torch.empty(self.shape, dtype=torch.float64, device='cuda') if want_dU0 else None
        optr = ctypes.c_void_p(out.data_ptr()) if want_dU0 else None
        if isinstance(dJ_dU, np.ndarray):
            a = np.ascontiguousarray(dJ_dU, dtype=np.float64)
            if a.size != int(np.prod(self.shape)):
                raise ValueError(f'dJ_dU must have shape {self.shape}')
            rc = self._lib.maxent_step_adjoint(self._h, a.ctypes.data_as(ctypes.c_void_p), 0, optr, 1, g)
        else:
            a = dJ_dU.to(dtype=torch.float64).contiguous()
            if a.numel() != int(np.prod(self.shape)) or not a.is_cuda:
                raise ValueError(f'dJ_dU must be a CUDA tensor with shape {self.shape}')
            rc = self._lib.maxent_step_adjoint(self._h, ctypes.c_void_p(a.data_ptr()), 1, optr, 1, g)
        self._check(rc)
        return out, [g[0], g[1], g[2]]


class MaxEntBatch(MaxEntSolver):
    """Many independent 1D 14-moment tubes advanced together (maxent_create_batch).

    instances: list of dicts with n (cells), tau_ref, t_end and optionally x0, x1.  The field
    of init_state / get is the concatenation [14][sum n]."""

    def __init__(self, instances, stream=None, **kw):
        self._lib = load_library()
        torch = _torch()
        pk = {k: v for k, v in kw.items() if k in _PROBLEM_KEYS}
        nk = {k: v for k, v in kw.items() if k not in _PROBLEM_KEYS}
        pk.setdefault('system', 14)
        self.problem = make_problem(**pk)
        self.numerics = make_numerics(**nk)
        arr = (Instance * len(instances))()
        for k, d in enumerate(instances):
            arr[k].x0 = d.get('x0', 0.0)
            arr[k].x1 = d.get('x1', 1.0)
            arr[k].tau_ref = d.get('tau_ref', 0.0)
            arr[k].t_end = d['t_end']
            arr[k].n_cells = int(d['n'])
        self.n_inst = len(instances)
        self.sizes = [int(d['n']) for d in instances]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = ctypes.c_void_p()
        rc = self._lib.maxent_create_batch(ctypes.byref(self.problem), ctypes.byref(self.numerics),
                                           self.n_inst, arr, ctypes.c_void_p(stream.cuda_stream),
                                           ctypes.byref(h))
        if rc != MAXENT_OK:
            raise MaxentError(rc, self._lib.maxent_last_error(None).decode())
        self._h = h
        self.nv = 14
        self.shape = (14, 1, int(self.offsets[-1]))

    def step(self, max_steps=10 ** 9, chunk=100, check=True):
        info = BatchInfo()
        per = (InstanceInfo * self.n_inst)()
        rc = self._lib.maxent_step_batch(self._h, int(max_steps), int(chunk), ctypes.byref(info), per)
        if check:
            self._check(rc)
        d = info.as_dict()
        d['status'] = STATUS.get(rc, 'OK') if rc else 'OK'
        d['instances'] = [{k: getattr(per[i], k) for k, _ in InstanceInfo._fields_}
                          for i in range(self.n_inst)]
        return d

    def set_launch(self, threads, cells_per_thread, wg_per_cu):
        self._check(self._lib.maxent_set_batch_launch(self._h, int(threads), int(cells_per_thread),
                                                      int(wg_per_cu)))

    def launch(self):
        a, c, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.maxent_get_batch_launch(self._h, ctypes.byref(a), ctypes.byref(c),
                                                      ctypes.byref(b)))
        return a.value, c.value, b.value

    def autotune(self, trial_steps=20):
        a, c, b, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self._lib.maxent_autotune_batch(self._h, int(trial_steps), ctypes.byref(a),
                                                    ctypes.byref(c), ctypes.byref(b), ctypes.byref(r)))
        return {'threads': a.value, 'cells_per_thread': c.value, 'wg_per_cu': b.value,
                'cell_updates_per_s': r.value}

    def split(self, field):
        """Per-instance views [14][n_i] of a concatenated field."""
        f = field.reshape(field.shape[0], -1)
        return [f[:, self.offsets[i]:self.offsets[i + 1]] for i in range(self.n_inst)]

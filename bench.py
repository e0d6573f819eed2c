"""Benchmark: 2D crossed supersonic jets, 14-moment maximum-entropy system, 2048 x 2048 cells.

One step = one full SSP-RK2 time step of the whole hot path on every cell (boundary fill,
primitive recovery, common-limiter MUSCL, sigma-limited closure, approximate wave speeds,
HLL, BGK source, update, CFL reduction).  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

The workload: unit square, two Maxwellian jets (width 0.1, centred at y = 0.35 and 0.65,
+-30 degrees, Mach 3, rho = 1, T = 1) entering through the left wall into a background at
rho = 1e-3, T = 1; transmissive elsewhere; Kn = 0.1 through a local BGK collision time;
MUSCL-minmod, HLL, SSP-RK2, CFL 0.4, sigma_lim = 1e-4.  Inputs are synthetic (the problem
definition itself; no dataset).

The timed window: the run starts from rest, advances --advance (1000) steps untimed and
--warmup more, then times --steps steps, so that the window sits in the middle of the 2000-step
workload (where the jets are developed) rather than at its start.

Sub-records beside the headline FP64 value: the same window in mixed precision; the full
2000-step run in FP64 and mixed (average rates, FP64 re-evaluation share, L1 deviation); the
discrete adjoint of the 512^2 jets against its forward run; 512 batched 1D shock tubes (mixed
and FP64, autotuned launch shape); the paper's own crossed-jets geometry at 1200^2 (forward
Euler, van Albada); the two Sod workloads' time per step on the device and in the oracle; and
the CPU oracle on a bounded sample (skip each with its --no-* flag).
"""
import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 2048
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
# algorithmic HBM bytes per cell and stage launch of the 14-moment method: stage 1 reads U^n
# and writes U* (2 x 112 B), stage 2 reads U* and U^n and writes U^{n+1} (3 x 112 B).  These
# are the workload's own counts, whichever kernel runs it, and set roofline.achieved; the
# planar kernel (a planar-symmetric state: ten moments carried, the four z-odd ones
# identically zero) moves 80 B per state, reported beside them as the executed counts
BYTES_PER_CELL_STAGE = {1: 224.0, 2: 336.0}
PLANAR_BYTES_PER_CELL_STAGE = {1: 160.0, 2: 240.0}
# algorithmic FP64 operations per cell and stage launch of the 14-moment method (each face
# once per stage, no halo redundancy; add/sub/mul = 1, fma = 2, div/sqrt/exp/log = 1),
# counted by running the library's own templated device code with a counting scalar:
# paper_2401_15233_amd/csrc/flopcount.cpp (tests/test_flopcount.py keeps these in sync); the
# planar kernel's own count beside it
FLOPS_PER_CELL_STAGE = {1: 4080, 2: 4426}
PLANAR_FLOPS_PER_CELL_STAGE = {1: 2634, 2: 2895}
SOURCES_FOR_TRAFFIC = ('paper_2401_15233_amd/csrc/mx_kernels.hip',
                       'paper_2401_15233_amd/csrc/mx_physics.hpp',
                       'paper_2401_15233_amd/csrc/mx_planar.hpp',
                       'paper_2401_15233_amd/csrc/mx_scheme.hpp',
                       'paper_2401_15233_amd/csrc/mx_bc.hpp',
                       'paper_2401_15233_amd/csrc/mx_internal.hpp')
TRAFFIC_PROFILE = 'profiles/stage_kernel_jets2048_fp64_hbm_traffic.txt'
VALU_PROFILE = 'profiles/stage_kernel_jets2048_fp64_valu.txt'


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES_FOR_TRAFFIC:
        with open(os.path.join(ROOT, f), 'rb') as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per stage launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, or None when the kernel sources changed since those counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ':' in line and not line.startswith(' '):
            k, v = line.split(':', 1)
            kv[k.strip()] = v.strip()
    if kv.get('kernel_source_hash') != kernel_source_hash():
        return None
    return float(kv['hbm_bytes_per_launch'])


def measured_valu_busy():
    """Fraction of cycles the VALU was busy in the FP64 stage kernel, from the committed
    rocprofv3 SQ_ACTIVE_INST_VALU / GRBM_GUI_ACTIVE summary, or None when the kernel sources
    changed since."""
    path = os.path.join(ROOT, VALU_PROFILE)
    if not os.path.exists(path):
        return None
    busy, h = None, None
    for line in open(path):
        if line.startswith('valu_busy_percent'):
            busy = float(line.rsplit(':', 1)[1]) / 100.0
        elif line.startswith('kernel_source_hash:'):
            h = line.split(':', 1)[1].strip()
    return busy if h == kernel_source_hash() else None


def jets_kwargs(n, k_ws=1.2):
    """The crossed-jets workload.  Wave speeds are inflated by k = 1.2: with k = 1 a cell of
    the 2048^2 run becomes unrealizable at step 1730 (the approximate wave speeds under-estimate
    the signal speeds at the jet fronts); with k = 1.1 or 1.2 the 2000 steps complete."""
    return dict(system=14, dim=2, nx=n, ny=n, order=2, integrator='ssprk2', flux='hll',
                limiter='minmod', cfl=0.4, sigma_lim=1e-4, k_ws=k_ws,
                bc=('jet', 'transmissive', 'transmissive', 'transmissive'),
                jets=[(0.35, 0.1, 30.0), (0.65, 0.1, -30.0)], jet_mach=3.0, jet_rho=1.0,
                jet_T=1.0)


def host_cpu():
    """CPU model and the number of host cores this process may run on."""
    model = 'unknown'
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    model = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {'cpu_model': model, 'nproc': avail}


def _cpu_timed(fn):
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    fn()
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return wall, max(1, round(cpu / wall))


def cpu_baseline(n=256, steps=6):
    """The oracle, as it stands, on a bounded sample of the same workload (n x n cells of
    a developed crossed-jets field, `steps` SSP-RK2 steps) on the host cores."""
    from paper_2401_15233_amd import inputs
    from oracle import scheme as sc, moments as mo
    kw = jets_kwargs(n)
    s = sc.Setup(system=14, dim=2, nx=n, ny=n, order=2, integrator='ssprk2', cfl=0.4,
                 bc=kw['bc'], jets=kw['jets'], k_ws=kw['k_ws'])
    U = mo.prim_to_cons14(inputs.crossed_jets_developed(n, n, seed=0))
    tau = inputs.kn_to_tau_ref(0.1, L_ref=0.1)
    wall, cores = _cpu_timed(lambda: sc.run(U, s, tau, nsteps=steps))
    out = {'value': n * n * steps / wall, 'unit': 'cell-updates/s', 'cores': cores, 'kind': 'oracle',
           'sample': f'{n}x{n} developed crossed-jets field, {steps} SSP-RK2 steps, FP64 NumPy, '
                     f'{wall:.1f} s wall'}
    out.update(host_cpu())
    return out


def sod_oracle_record(steps0=2000, steps1=5):
    """The oracle's time per step on the two Sod workloads (bounded samples): the 5-moment
    tube (1000 cells, first order, forward Euler, Kn = 0.01), `steps0` CFL steps; the
    14-moment tube (20000 cells, MUSCL + SSP-RK2, Kn = 0.01), `steps1` CFL steps."""
    from paper_2401_15233_amd import inputs
    from oracle import scheme as sc, moments as mo
    out = {}
    s = sc.Setup(system=5, dim=1, nx=1000, order=1, integrator='fe', cfl=0.5)
    U = mo.prim_to_cons5(inputs.sod_prims(5, 1000))
    wall, cores = _cpu_timed(lambda: sc.run(U, s, inputs.kn_to_tau_ref(0.01), nsteps=steps0))
    out['sod5_1000_kn0.01'] = {'steps': steps0, 'us_per_step': 1e6 * wall / steps0, 'cores': cores,
                               'cell_updates_per_s': 1000 * steps0 / wall}
    s = sc.Setup(system=14, dim=1, nx=20000, order=2, integrator='ssprk2', cfl=0.5)
    U = mo.prim_to_cons14(inputs.sod_prims(14, 20000))
    wall, cores = _cpu_timed(lambda: sc.run(U, s, inputs.kn_to_tau_ref(0.01), nsteps=steps1))
    out['sod14_20000_kn0.01'] = {'steps': steps1, 'us_per_step': 1e6 * wall / steps1, 'cores': cores,
                                 'cell_updates_per_s': 20000 * steps1 / wall}
    return out


def adjoint_record(stream, n=512, steps=400, checkpoint_every=20):
    """Discrete adjoint of the crossed jets (14 moments, FP64): n x n cells from the background
    state, `steps` CFL steps recorded with a checkpoint every `checkpoint_every`, reversed for
    J = dx dy sum of rho u_y over x in [0.05, 0.15], y in [0.5, 1] (a strip the jets reach in
    400 steps).  Times the plain forward run, the recording forward run and the adjoint
    (recomputation of every checkpoint segment included) with HIP events on the solver's
    stream."""
    import numpy as np
    import torch
    from paper_2401_15233_amd import solver, inputs
    tau = inputs.kn_to_tau_ref(0.1, L_ref=0.1)
    W0 = inputs.crossed_jets_initial(n, n)
    s = solver.MaxEntSolver(stream=stream, **jets_kwargs(n))
    w = np.zeros((14, n, n))
    xc = (np.arange(n) + 0.5) / n
    box = ((xc[None, :] >= 0.05) & (xc[None, :] <= 0.15) & (xc[:, None] >= 0.5))
    w[2][box] = 1.0 / (n * n)
    wt = torch.tensor(w, device='cuda')

    def clock(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), r

    s.init_state(W0)
    s.step(3, tau_ref=tau)                       # warm-up
    s.init_state(W0)
    fwd_ms, _ = clock(lambda: s.step(steps, tau_ref=tau))
    s.init_state(W0)
    s.record(checkpoint_every, steps)
    rec_ms, info = clock(lambda: s.step(steps, tau_ref=tau))
    Un = s.get('conserved')
    s.adjoint(wt, want_dU0=False)                # workspace allocation outside the timing
    adj_ms, (gU0, g) = clock(lambda: s.adjoint(wt, want_dU0=True))
    J = float((wt * Un).sum())
    s.set_adjoint_mode('frozen_limiter')
    _, gf = s.adjoint(wt, want_dU0=False)
    s.close()
    return {'workload': f'2D crossed jets, 14-moment FP64, {n}x{n}, {steps} CFL steps '
                        f'(t = {info["t"]:.4f}), checkpoint every {checkpoint_every}',
            'objective': 'dx dy sum of rho u_y over x in [0.05, 0.15], y in [0.5, 1]',
            'J': J,
            'gradient_mode': 'frozen_limiter',
            'gradient': {'dJ_dMach': gf[0], 'dJ_drho_jet': gf[1], 'dJ_dtau_ref': gf[2]},
            'diagnostic': {
                'exact_mode': {'dJ_dMach': g[0], 'dJ_drho_jet': g[1], 'dJ_dtau_ref': g[2]},
                'note': 'the exact derivative of the common-limiter scheme grows without bound '
                        'over long horizons (the limiter\'s cross-variable gains compound); it '
                        'matches the CPU reference gradient on short ones'},
            'forward_ms': fwd_ms, 'forward_recording_ms': rec_ms, 'adjoint_ms': adj_ms,
            'adjoint_over_forward': adj_ms / fwd_ms,
            'forward_cell_updates_per_s': n * n * steps / (fwd_ms / 1e3)}


def batch_record(stream, steps=5000, chunk=500):
    """Batched 1D 14-moment shock tubes: 512 seed-generated instances (cells log-uniform in
    [512, 32768], p_L/p_R ~ U(2, 100), rho_L/rho_R ~ U(2, 20), Kn log-uniform in [1e-3, 10]),
    each with its own CFL dt toward t_end = 0.15, MUSCL-minmod + HLL + SSP-RK2, CFL 0.5, wave
    speeds inflated by k = 1.2 (with k = 1 the strongest tubes, pressure ratio > 80 and density
    ratio > 15, become unrealizable at any CFL).  Mixed precision (FP32 bulk, FP64 closure
    near the Junk subspace and the realizability boundary) is the headline form; FP64 is
    timed beside it.  For each, the launch shape is autotuned, then the first `steps` steps of
    the whole batch are timed (a bounded prefix of the workload: tubes that reach t_end within
    it drop out, and `active_instances_after` says how many are still running at its end)."""
    import torch
    from paper_2401_15233_amd import solver, inputs
    insts = inputs.batch_instances()
    for d in insts:
        d['tau_ref'] = inputs.kn_to_tau_ref(d['kn'])
        d['t_end'] = 0.15
    out = {'workload': f'{len(insts)} batched 1D 14-moment shock tubes, '
                       f'{sum(d["n"] for d in insts)} cells, mixed precision (FP64 beside it)'}
    for prec in ('mixed', 'fp64'):
        b = solver.MaxEntBatch(insts, stream=stream, precision=prec, order=2, integrator='ssprk2',
                               cfl=0.5, k_ws=1.2)
        b.init_state(inputs.batch_sod_prims(insts))
        tuned = b.autotune(trial_steps=10)
        b.init_state(inputs.batch_sod_prims(insts))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        info = b.step(max_steps=steps, chunk=chunk, check=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        reduced = int(b.info()['reduced'])
        b.close()
        rec = {'steps': steps, 'ms': ms, 'cell_updates': info['cell_updates'],
               'value': info['cell_updates'] / (ms / 1e3), 'unit': 'cell-updates/s',
               'launch': {k: tuned[k] for k in ('threads', 'cells_per_thread', 'wg_per_cu')},
               'active_instances_after': info['n_active'],
               # 2: the tubes are axially symmetric and the axial kernel (seven moments) runs
               'reduced_kernel': reduced}
        if prec == 'mixed':
            rec['fp64_reevaluated_face_state_fraction'] = \
                info['n_fp64_states'] / max(info['n_face_states'], 1)
        out[prec] = rec
    out['value'] = out['mixed']['value']
    out['unit'] = 'cell-updates/s'
    out['mixed_speedup_vs_fp64'] = out['mixed']['value'] / out['fp64']['value']
    return out


def batch_full_record(stream, precision='fp64', chunk=400):
    """The batched workload run to completion (every tube to t = 0.15): makespan, total
    cell-updates and the balance efficiency = (full-run rate) / (rate with every tube active,
    from the autotuner's trial), i.e. how much the shrinking active set and the longest tube's
    step latency cost.  About two minutes; progress goes to stderr."""
    import torch
    from paper_2401_15233_amd import solver, inputs
    insts = inputs.batch_instances()
    for d in insts:
        d['tau_ref'] = inputs.kn_to_tau_ref(d['kn'])
        d['t_end'] = 0.15
    b = solver.MaxEntBatch(insts, stream=stream, precision=precision, order=2, integrator='ssprk2',
                           cfl=0.5, k_ws=1.2)
    b.init_state(inputs.batch_sod_prims(insts))
    tuned = b.autotune(trial_steps=20)
    torch.cuda.synchronize()
    t0 = time.time()
    info = None
    for _ in range(1000):
        info = b.step(max_steps=10000, chunk=chunk, check=False)
        print(f'batch {precision}: longest {info["max_steps"]} steps, {info["n_active"]} active, '
              f'{time.time() - t0:.1f} s', file=sys.stderr, flush=True)
        if info['n_active'] == 0 or info['fail_code']:
            break
    torch.cuda.synchronize()
    wall = time.time() - t0
    b.close()
    steps = sorted(p['steps'] for p in info['instances'])
    q = lambda f: steps[int(f * (len(steps) - 1))]  # noqa: E731
    rate = info['cell_updates'] / wall
    return {'precision': precision, 'makespan_s': wall, 'cell_updates': info['cell_updates'],
            'value': rate, 'unit': 'cell-updates/s', 'failed': int(info['fail_code'] != 0),
            'launch': {k: tuned[k] for k in ('threads', 'cells_per_thread', 'wg_per_cu')},
            'all_active_rate': tuned['cell_updates_per_s'],
            'balance_efficiency': rate / tuned['cell_updates_per_s'],
            'steps_min_median_p90_p99_max': [q(0), q(0.5), q(0.9), q(0.99), q(1.0)]}


def _run_to(s, t_end, tau_ref, chunk=5000):
    info = {'t': 0.0}
    while info['t'] < t_end * (1.0 - 1e-12):
        info = s.step(chunk, tau_ref=tau_ref, t_end=t_end, check=False)
        if info['status'] != 'OK':
            break
    return info


def sod_records(stream):
    """The two Sod workloads.  At these sizes a step is bound by launch latency and the
    length of one tile's work, not by throughput, so time per step is the figure:
    (a) 5-moment, 1000 cells, first-order HLL, forward Euler, CFL 0.5, Kn = 0.01, to t = 0.2;
    (b) 14-moment, 20000 cells, MUSCL-minmod + HLL + SSP-RK2, CFL 0.5, Kn in {1e-3, 1e-2, 0.1,
    1, 10}, to t = 0.2: each Knudsen number run alone, and the five as one batch."""
    import torch
    from paper_2401_15233_amd import solver, inputs
    out = {}

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    s = solver.MaxEntSolver(system=5, dim=1, nx=1000, order=1, integrator='fe', flux='hll', cfl=0.5,
                            stream=stream)
    s.init_state(inputs.sod_prims(5, 1000))
    info, ms = timed(lambda: _run_to(s, 0.2, inputs.kn_to_tau_ref(0.01)))
    s.close()
    out['sod5_1000_kn0.01'] = {'steps': info['steps'], 'ms': ms, 'us_per_step': 1e3 * ms / info['steps'],
                               'status': info['status']}
    kns = [1e-3, 1e-2, 0.1, 1.0, 10.0]
    num = dict(order=2, integrator='ssprk2', flux='hll', limiter='minmod', cfl=0.5)
    alone = []
    for kn in kns:
        s = solver.MaxEntSolver(system=14, dim=1, nx=20000, stream=stream, **num)
        s.init_state(inputs.sod_prims(14, 20000))
        info, ms = timed(lambda: _run_to(s, 0.2, inputs.kn_to_tau_ref(kn)))
        s.close()
        alone.append({'kn': kn, 'steps': info['steps'], 'ms': ms, 'us_per_step': 1e3 * ms / info['steps'],
                      'status': info['status']})
    out['sod14_20000_alone'] = alone
    insts = [dict(n=20000, t_end=0.2, tau_ref=inputs.kn_to_tau_ref(kn), rho_ratio=8.0, p_ratio=10.0)
             for kn in kns]
    b = solver.MaxEntBatch(insts, stream=stream, **num)
    b.init_state(inputs.batch_sod_prims(insts))
    tuned = b.autotune(trial_steps=10)
    b.init_state(inputs.batch_sod_prims(insts))
    info, ms = timed(lambda: b.step(max_steps=10 ** 7, chunk=500, check=False))
    b.close()
    out['sod14_20000_batch_of_5'] = {'longest_steps': info['max_steps'], 'ms': ms,
                                     'us_per_step': 1e3 * ms / info['max_steps'],
                                     'sum_alone_ms': sum(r['ms'] for r in alone),
                                     'launch': {k: tuned[k] for k in ('threads', 'cells_per_thread', 'wg_per_cu')},
                                     'status': info['status']}
    return out


def sod_gpu_record(stream, steps1=500):
    """The device's time per step on the two Sod workloads: the 5-moment tube run in full
    (1000 cells, first-order HLL, forward Euler, CFL 0.5, Kn = 0.01, to t = 0.2) and the first
    `steps1` steps of the 14-moment tube (20000 cells, MUSCL-minmod + HLL + SSP-RK2, CFL 0.5,
    Kn = 0.01).  At these sizes a step is bound by launch latency, not throughput."""
    import torch
    from paper_2401_15233_amd import solver, inputs

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        r = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return r, e0.elapsed_time(e1)

    out = {}
    s = solver.MaxEntSolver(system=5, dim=1, nx=1000, order=1, integrator='fe', flux='hll', cfl=0.5,
                            stream=stream)
    s.init_state(inputs.sod_prims(5, 1000))
    s.step(3, tau_ref=inputs.kn_to_tau_ref(0.01))
    s.init_state(inputs.sod_prims(5, 1000))
    info, ms = timed(lambda: _run_to(s, 0.2, inputs.kn_to_tau_ref(0.01)))
    s.close()
    out['sod5_1000_kn0.01'] = {'steps': info['steps'], 'ms': ms, 'us_per_step': 1e3 * ms / info['steps'],
                               'cell_updates_per_s': 1000 * info['steps'] / (ms / 1e3),
                               'status': info['status'], 't': info['t']}
    s = solver.MaxEntSolver(system=14, dim=1, nx=20000, order=2, integrator='ssprk2', flux='hll',
                            limiter='minmod', cfl=0.5, stream=stream)
    s.init_state(inputs.sod_prims(14, 20000))
    s.step(3, tau_ref=inputs.kn_to_tau_ref(0.01))
    s.init_state(inputs.sod_prims(14, 20000))
    info, ms = timed(lambda: s.step(steps1, tau_ref=inputs.kn_to_tau_ref(0.01), check=False))
    s.close()
    out['sod14_20000_kn0.01'] = {'steps': info['steps'], 'ms': ms, 'us_per_step': 1e3 * ms / info['steps'],
                                 'cell_updates_per_s': 20000 * info['steps'] / (ms / 1e3),
                                 'status': info['status'], 'reduced_kernel': int(info['reduced'])}
    return out


def full_run_record(stream, n, steps=2000):
    """The 2048^2 crossed-jets workload in full (all `steps` steps from rest, FP64 and mixed),
    each timed with HIP events: the average rate over the whole run, the mixed form's FP64
    re-evaluation share over it, its L1 deviation from the FP64 run at the end, and beside it
    the FP64 run's own L1 change when its initial state carries one random FP32 rounding
    (+-2^-24 relative), i.e. how far this flow amplifies single-precision-sized rounding."""
    import numpy as np
    import torch
    from paper_2401_15233_amd import solver, inputs
    tau = inputs.kn_to_tau_ref(0.1, L_ref=0.1)
    W0 = inputs.crossed_jets_initial(n, n)

    def run(precision, init):
        s = solver.MaxEntSolver(stream=stream, precision=precision, **jets_kwargs(n))
        s.init_state(init)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        info = s.step(steps, tau_ref=tau, check=False)
        e1.record(stream)
        torch.cuda.synchronize()
        U = s.get('conserved')
        s.close()
        return e0.elapsed_time(e1), info, U

    ms64, info64, U64 = run('fp64', W0)
    msmx, infomx, Umx = run('mixed', W0)
    rng = np.random.default_rng(0)
    _, _, Up = run('fp64', W0 * (1.0 + rng.choice([-1.0, 1.0], W0.shape) * 2.0 ** -24))
    ref = U64.abs().reshape(14, -1).sum(1).clamp_min(1e-300)

    def l1(U):
        return [float(x) for x in ((U - U64).abs().reshape(14, -1).sum(1) / ref).cpu()]

    return {'workload': f'{n}x{n} crossed jets, all {steps} steps from rest',
            'fp64': {'value': n * n * info64['steps'] / (ms64 / 1e3), 'unit': 'cell-updates/s',
                     'ms_per_step': ms64 / max(info64['steps'], 1), 'steps': info64['steps'],
                     'status': info64['status'], 't': info64['t'], 'reduced_kernel': int(info64['reduced'])},
            'mixed': {'value': n * n * infomx['steps'] / (msmx / 1e3), 'unit': 'cell-updates/s',
                      'ms_per_step': msmx / max(infomx['steps'], 1), 'steps': infomx['steps'],
                      'status': infomx['status'], 'speedup_vs_fp64': ms64 / msmx,
                      'fp64_reevaluated_face_state_fraction': infomx['fp64_fraction'],
                      'l1_rel_deviation_from_fp64_per_moment': l1(Umx)},
            'fp64_l1_change_under_fp32_input_rounding_per_moment': l1(Up)}


def paper_jets_record(stream, n=1200, steps=2000):
    """The paper's own crossed jets (Section 6): 1200^2 cells, M = 5 jets of width L/7 on the
    left and bottom walls at a right angle, background 1e-5, van Albada, HLL, forward Euler,
    CFL 0.5, collisionless, FP64.  `steps` CFL steps from rest are timed (the jets cross the
    middle of the domain at about 1700 steps)."""
    import torch
    from paper_2401_15233_amd import solver, inputs
    pj = inputs.PAPER_JETS
    s = solver.MaxEntSolver(system=14, dim=2, nx=n, ny=n, order=2, integrator='fe', flux='hll',
                            limiter='vanalbada', cfl=0.5, sigma_lim=1e-4,
                            bc=('jet', 'transmissive', 'jet', 'transmissive'), jets=list(pj['jets']),
                            jet_mach=pj['mach'], jet_rho=pj['rho'], jet_T=pj['T'], stream=stream)
    s.init_state(inputs.paper_jets_initial(n, n))
    s.step(3, check=False)
    s.init_state(inputs.paper_jets_initial(n, n))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    info = s.step(steps, check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    s.close()
    return {'workload': f'paper crossed jets (M 5, L/7, right angle, background 1e-5), {n}x{n}, '
                        'van Albada + HLL + forward Euler, CFL 0.5, collisionless, FP64',
            'steps': info['steps'], 'status': info['status'], 't': info['t'], 'ms': ms,
            'value': n * n * info['steps'] / (ms / 1e3), 'unit': 'cell-updates/s',
            'ms_per_step': ms / max(info['steps'], 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=5)
    ap.add_argument('--n', type=int, default=N)
    ap.add_argument('--advance', type=int, default=1000,
                    help='untimed steps from rest before the warm-up and the timed steps, so that '
                         'the timed window sits in the middle of the 2000-step workload')
    ap.add_argument('--no-full-kernel', dest='full_kernel', action='store_false',
                    help='skip the timed window with the full 14-moment kernel')
    ap.add_argument('--no-full-run', action='store_true',
                    help='skip the full 2000-step FP64 and mixed runs')
    ap.add_argument('--no-sod', action='store_true',
                    help='skip the Sod time-per-step records (device and oracle)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--precision', default='both', choices=('fp64', 'mixed', 'both'),
                    help='fp64 (the headline value), mixed, or both (fp64 headline plus a mixed '
                         'sub-record with its L1 deviation from the FP64 run)')
    ap.add_argument('--no-adjoint', action='store_true',
                    help='skip the adjoint / forward timing of the 512^2 crossed jets')
    ap.add_argument('--no-batch', action='store_true',
                    help='skip the batched 1D shock-tube record')
    ap.add_argument('--sod', action='store_true',
                    help='only time the two Sod workloads (time per step; about half a minute)')
    ap.add_argument('--batch-full', action='store_true',
                    help='only run the batched tubes to completion (FP64 and mixed; ~4 minutes)')
    ap.add_argument('--no-paper-jets', action='store_true',
                    help="skip the paper's own crossed-jets geometry (1200^2, forward Euler)")
    ap.add_argument('--copy-calibration', action='store_true',
                    help='only run a plain 2 GiB device copy (HBM counter calibration)')
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) != 1:
        print('bench.py runs on exactly one GPU: the solver has no multi-GPU path (a slab '
              'decomposition with ghost-row exchange is the intended design); use --gpus 1',
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2401_15233_amd import solver, inputs

    torch.cuda.set_device(0)
    if a.sod:
        print(json.dumps({'sod': sod_records(torch.cuda.current_stream())}), flush=True)
        return
    if a.batch_full:
        stream = torch.cuda.current_stream()
        print(json.dumps({'batched_full_run': [batch_full_record(stream, p) for p in ('fp64', 'mixed')]}),
              flush=True)
        return
    if a.copy_calibration:
        m = 256 * 1024 * 1024
        src = torch.ones(m, dtype=torch.float64, device='cuda')
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({'copy_kernel_bytes_read': m * 8, 'copy_kernel_bytes_written': m * 8}))
        return
    n = a.n
    # the timed window stays inside the 2000-step workload
    a.advance = max(0, min(a.advance, 2000 - a.warmup - a.steps))
    tau = inputs.kn_to_tau_ref(0.1, L_ref=0.1)
    stream = torch.cuda.current_stream()
    W0 = inputs.crossed_jets_initial(n, n)

    def timed(precision, init=None, planar=True):
        kw = jets_kwargs(n)
        kw['precision'] = precision
        s = solver.MaxEntSolver(stream=stream, **kw)
        s.set_reduced(planar)
        s.init_state(W0 if init is None else init)
        if a.advance:
            s.step(a.advance, tau_ref=tau)
        if a.warmup:
            s.step(a.warmup, tau_ref=tau)
        s.set_profiling(True)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        info = s.step(a.steps, tau_ref=tau)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        stage_ms, launches = s.profile()
        U = s.get('conserved')
        s.close()
        return ms, stage_ms, launches, info, U

    head = 'fp64' if a.precision in ('fp64', 'both') else 'mixed'
    ms, stage_ms, launches, info, U_head = timed(head)
    cells = n * n
    cups = cells * a.steps / (ms / 1e3)
    avg_stage_ms = stage_ms / max(launches, 1)
    planar = info.get('reduced') == 1
    bpc, fpc = BYTES_PER_CELL_STAGE, FLOPS_PER_CELL_STAGE
    bytes_per_launch = cells * 0.5 * (bpc[1] + bpc[2])
    flops_per_launch = cells * 0.5 * (fpc[1] + fpc[2])
    bytes_per_update = bpc[1] + bpc[2]
    sysname = 'Sys14P' if planar else 'Sys14'
    achieved = flops_per_launch / (avg_stage_ms / 1e3) / 1e12
    hbm_achieved = bytes_per_launch / (avg_stage_ms / 1e3) / 1e9
    out = {
        'metric': 'cell-updates/s and HBM GB/s (14-mom 2D jets, FP64 vs mixed); adjoint/forward ratio',
        'value_is': f'cell-updates/s of the {head.upper()} step (HBM GB/s in roofline, mixed and '
                    f'adjoint / forward in their sub-records)',
        'value': cups,
        'unit': 'cell-updates/s',
        'n_gpus': 1,
        'steps': a.steps,
        'warmup': a.warmup,
        'ms_per_step': ms / a.steps,
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f64' if head == 'fp64' else 'f64 state + f32 closure/flux',
        'data': 'synthetic',
        'config': {'workload': f'2D crossed jets, 14-moment, {n}x{n}, MUSCL-minmod + HLL + '
                               f'SSP-RK2, CFL 0.4, Kn 0.1, wave speeds x 1.2', 'cells': cells,
                   'precision': 'fp64',
                   'steps_in_workload': 2000, 'precision_mode': head,
                   'timed_window': f'steps {a.advance + a.warmup + 1}..{a.advance + a.warmup + a.steps} '
                                   f'of the run from rest',
                   'stage_kernel': ('planar: the state is even in v_z, so u_z = P_xz = P_yz = q_z = 0 '
                                    'and the kernel carries the ten other moments' if planar
                                    else 'full 14-moment')},
        'hbm_gbs_algorithmic': cells * bytes_per_update * a.steps / (ms / 1e3) / 1e9,
        'sim_time_reached': info['t'],
        'roofline': {'bound': 'alu', 'achieved': achieved, 'peak': FP64_VECTOR_PEAK_TFLOPS,
                     'unit': 'TFLOP/s', 'frac': achieved / FP64_VECTOR_PEAK_TFLOPS,
                     'traffic': measured_traffic(),
                     'traffic_unit': 'HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a '
                                     'plain copy of known size)',
                     'valu_busy': measured_valu_busy(),
                     'kernel': f'stage_kernel<{sysname},2,2,{0 if head == "fp64" else 1},16,15,256> ({head})',
                     'avg_launch_ms': avg_stage_ms, 'launches': launches,
                     'flops_per_launch': flops_per_launch,
                     'hbm_algorithmic_bytes_per_launch': bytes_per_launch,
                     'hbm_achieved_gbs': hbm_achieved,
                     'hbm_frac': hbm_achieved / HBM_PEAK_GBS},
    }
    if planar:
        # what the symmetry-reduced kernel itself executes and moves (ten of the 14 moments)
        ef = cells * 0.5 * (PLANAR_FLOPS_PER_CELL_STAGE[1] + PLANAR_FLOPS_PER_CELL_STAGE[2])
        eb = cells * 0.5 * (PLANAR_BYTES_PER_CELL_STAGE[1] + PLANAR_BYTES_PER_CELL_STAGE[2])
        et = ef / (avg_stage_ms / 1e3) / 1e12
        eg = eb / (avg_stage_ms / 1e3) / 1e9
        out['roofline']['executed'] = {
            'flops_per_launch': ef, 'tflops': et, 'frac': et / FP64_VECTOR_PEAK_TFLOPS,
            'hbm_bytes_per_launch': eb, 'hbm_gbs': eg, 'hbm_frac': eg / HBM_PEAK_GBS}
    def fp64_sensitivity():
        rng = np.random.default_rng(0)
        Wp = W0 * (1.0 + rng.choice([-1.0, 1.0], W0.shape) * 2.0 ** -24)
        U_p = timed('fp64', init=Wp)[4]
        dd = (U_p - U_head).abs().reshape(14, -1).sum(1)
        rr = U_head.abs().reshape(14, -1).sum(1).clamp_min(1e-300)
        return [float(x) for x in (dd / rr).cpu()]

    if a.precision == 'both':
        ms_m, stage_ms_m, launches_m, info_m, U_m = timed('mixed')
        d = (U_m - U_head).abs().reshape(14, -1).sum(1)
        ref = U_head.abs().reshape(14, -1).sum(1).clamp_min(1e-300)
        avg_m = stage_ms_m / max(launches_m, 1)
        out['mixed'] = {
            'value': cells * a.steps / (ms_m / 1e3), 'unit': 'cell-updates/s',
            'ms_per_step': ms_m / a.steps, 'speedup_vs_fp64': ms / ms_m,
            'avg_stage_launch_ms': avg_m,
            'alu_tflops_algorithmic': flops_per_launch / (avg_m / 1e3) / 1e12,
            'hbm_gbs_algorithmic': cells * bytes_per_update * a.steps / (ms_m / 1e3) / 1e9,
            'l1_rel_deviation_from_fp64_per_moment': [float(x) for x in (d / ref).cpu()],
            # the FP64 run's own L1 change when its initial state carries one random FP32
            # rounding (+-2^-24 relative): how far this flow amplifies single-precision
            # rounding over the same steps
            'fp64_l1_change_under_fp32_input_rounding_per_moment': fp64_sensitivity(),
            'fp64_reevaluated_face_state_fraction':
                info_m['n_fp64_states'] / max(info_m['n_face_states'], 1),
        }
    if planar and a.full_kernel:
        # the same window with the full 14-moment kernel (planar mode off)
        ms_f, stage_ms_f, launches_f, _, U_f = timed(head, planar=False)
        d = (U_f - U_head).abs().reshape(14, -1).sum(1)
        ref = U_head.abs().reshape(14, -1).sum(1).clamp_min(1e-300)
        avg_f = stage_ms_f / max(launches_f, 1)
        out['full_kernel'] = {
            'value': cells * a.steps / (ms_f / 1e3), 'unit': 'cell-updates/s',
            'ms_per_step': ms_f / a.steps, 'avg_stage_launch_ms': avg_f,
            'planar_speedup': ms_f / ms,
            'alu_tflops_algorithmic': cells * 0.5 * (FLOPS_PER_CELL_STAGE[1] + FLOPS_PER_CELL_STAGE[2])
                                      / (avg_f / 1e3) / 1e12,
            # rounding-order differences, amplified over the run like any rounding change
            'l1_rel_deviation_from_planar_per_moment': [float(x) for x in (d / ref).cpu()],
        }
    if not a.no_full_run:
        out['full_run'] = full_run_record(stream, n)
    if not a.no_adjoint:
        out['adjoint'] = adjoint_record(stream)
    if not a.no_batch:
        out['batched'] = batch_record(stream)
    if not a.no_paper_jets:
        out['paper_jets'] = paper_jets_record(stream)
    if not a.no_sod:
        out['sod'] = {'gpu': sod_gpu_record(stream)}
        if not a.no_cpu_baseline:
            out['sod']['oracle'] = sod_oracle_record()
    if not a.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == '__main__':
    main()

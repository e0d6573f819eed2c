"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the CPU oracle.

This module holds none of the method's arithmetic (no closure, wave speed, flux, limiter or
update).  It only builds primitive states W of gas distributions whose moments are known by
definition:
  * Maxwellians: P = p I, q = 0, R = 15 p^2/rho (3V) and q = 0, r = 3 P^2/rho (1V);
  * mixtures of Maxwellian beams: the central moments of a sum of Gaussians, computed in
    closed form (realizable by construction, bimodal where beams cross);
  * weighted discrete particle sets: weighted sums of powers of the peculiar velocity
    (realizable by construction, far from equilibrium for few particles).

Component order (primitives)
  14: [rho, u_x, u_y, u_z, P_xx, P_xy, P_xz, P_yy, P_yz, P_zz, q_x, q_y, q_z, R]
   5: [rho, u, P, q, r]
All arrays are float64 with the component on axis 0; fields are [nv][ny][nx] (x fastest).
"""
import math

import numpy as np

SOD_LEFT = (1.0, 0.0, 1.0)      # rho, u, p
SOD_RIGHT = (0.125, 0.0, 0.1)


def _maxw14(rho, ux, uy, uz, p):
    rho = np.asarray(rho, dtype=np.float64)
    z = np.zeros(np.broadcast(rho, ux, uy, uz, p).shape)
    return np.stack([rho + z, ux + z, uy + z, uz + z, p + z, z, z, p + z, z, p + z,
                     z, z, z, 15.0 * p * p / rho + z], 0)


def _maxw5(rho, u, P):
    z = np.zeros(np.broadcast(rho, u, P).shape)
    return np.stack([rho + z, u + z, P + z, z, 3.0 * P * P / rho + z], 0)


def cell_centres(n, lo=0.0, hi=1.0):
    return lo + (np.arange(n) + 0.5) * ((hi - lo) / n)


def sod_prims(system, nx, left=SOD_LEFT, right=SOD_RIGHT, x_diaphragm=0.5, x0=0.0, x1=1.0):
    """Riemann problem with Maxwellian halves; a centre exactly on the diaphragm goes right."""
    xc = cell_centres(nx, x0, x1)
    isl = xc < x_diaphragm
    rho = np.where(isl, left[0], right[0])
    u = np.where(isl, left[1], right[1])
    p = np.where(isl, left[2], right[2])
    if system == 5:
        return _maxw5(rho, u, p)
    return _maxw14(rho, u, 0.0, 0.0, p)


def uniform_prims14(nx, ny, rho=1e-3, T=1.0, u=(0.0, 0.0, 0.0)):
    W = _maxw14(rho, u[0], u[1], u[2], rho * T)
    return np.broadcast_to(W[:, None, None], (14, ny, nx)).copy()


# --------------------------------------------------------------------------- mixtures
def beam_mixture14(weights, means, temps):
    """Moments of sum_k rho_k * Gaussian(u_k, T_k I).
    weights (K, ...), means (K, 3, ...), temps (K, ...) -> W (14, ...).
    Central moments about the mixture velocity u with d_k = u_k - u:
      P = sum rho_k (T_k I + d d^T),  q = sum rho_k d (|d|^2 + 5 T_k),
      R = sum rho_k (|d|^4 + 10 T_k |d|^2 + 15 T_k^2)."""
    w = np.asarray(weights, dtype=np.float64)
    m = np.asarray(means, dtype=np.float64)
    T = np.asarray(temps, dtype=np.float64)
    rho = w.sum(0)
    u = (w[:, None] * m).sum(0) / rho
    d = m - u[None]
    dd = (d * d).sum(1)
    P = np.zeros((3, 3) + rho.shape)
    for i in range(3):
        for j in range(3):
            P[i, j] = (w * (d[:, i] * d[:, j] + (T if i == j else 0.0))).sum(0)
    q = (w[:, None] * d * (dd + 5.0 * T)[:, None]).sum(0)
    R = (w * (dd * dd + 10.0 * T * dd + 15.0 * T * T)).sum(0)
    return np.stack([rho, u[0], u[1], u[2], P[0, 0], P[0, 1], P[0, 2], P[1, 1], P[1, 2],
                     P[2, 2], q[0], q[1], q[2], R], 0)


def beam_mixture5(weights, means, temps):
    """1V analogue: P = sum rho_k (T_k + d^2), q = sum rho_k d (d^2 + 3 T_k),
    r = sum rho_k (d^4 + 6 T_k d^2 + 3 T_k^2)."""
    w = np.asarray(weights, dtype=np.float64)
    m = np.asarray(means, dtype=np.float64)
    T = np.asarray(temps, dtype=np.float64)
    rho = w.sum(0)
    u = (w * m).sum(0) / rho
    d = m - u
    P = (w * (T + d * d)).sum(0)
    q = (w * d * (d * d + 3.0 * T)).sum(0)
    r = (w * (d**4 + 6.0 * T * d * d + 3.0 * T * T)).sum(0)
    return np.stack([rho, u, P, q, r], 0)


def particle_moments14(weights, vel):
    """Moments of a weighted particle set: weights (M, n), vel (M, 3, n) -> W (14, n)."""
    w = np.asarray(weights, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    rho = w.sum(0)
    u = (w[:, None] * v).sum(0) / rho
    c = v - u[None]
    cc = (c * c).sum(1)
    P = [(w * c[:, i] * c[:, j]).sum(0) for (i, j) in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))]
    q = [(w * c[:, i] * cc).sum(0) for i in range(3)]
    R = (w * cc * cc).sum(0)
    return np.stack([rho, u[0], u[1], u[2]] + P + q + [R], 0)


def particle_moments5(weights, vel):
    w = np.asarray(weights, dtype=np.float64)
    v = np.asarray(vel, dtype=np.float64)
    rho = w.sum(0)
    u = (w * v).sum(0) / rho
    c = v - u
    return np.stack([rho, u, (w * c**2).sum(0), (w * c**3).sum(0), (w * c**4).sum(0)], 0)


def random_states14(n, seed=0):
    """n realizable 14-moment states mixing five families (exact Maxwellians, 2- and
    3-beam mixtures, few-particle sets, many-particle near-equilibrium clouds), with random
    density scale, temperature scale and bulk velocity."""
    rng = np.random.default_rng(seed)
    fam = rng.integers(0, 5, size=n)
    W = np.empty((14, n))
    # family 0: exact Maxwellians
    i0 = np.nonzero(fam == 0)[0]
    W[:, i0] = _maxw14(np.ones(len(i0)), 0.0, 0.0, 0.0, np.ones(len(i0)))
    # families 1, 2: 2 or 3 beams
    for f, K in ((1, 2), (2, 3)):
        ii = np.nonzero(fam == f)[0]
        if len(ii):
            w = rng.uniform(0.05, 1.0, size=(K, len(ii)))
            m = rng.normal(0.0, 1.5, size=(K, 3, len(ii)))
            T = rng.uniform(0.05, 1.5, size=(K, len(ii)))
            W[:, ii] = beam_mixture14(w, m, T)
    # family 3: few particles (5..8, random weights); four points in 3D sit exactly on the
    # sufficient realizability bound, where the wave-speed formula has an infinite slope
    ii = np.nonzero(fam == 3)[0]
    if len(ii):
        M = 8
        w = rng.uniform(0.1, 1.0, size=(M, len(ii)))
        drop = rng.integers(0, 4, size=len(ii))        # keep at least 5 particles
        for k in range(5, M):
            w[k, drop > (k - 5)] = 0.0
        v = rng.normal(0.0, 1.0, size=(M, 3, len(ii)))
        W[:, ii] = particle_moments14(w, v)
    # family 4: many-particle Gaussian clouds (near equilibrium, random anisotropy)
    ii = np.nonzero(fam == 4)[0]
    if len(ii):
        M = 256
        scale = rng.uniform(0.5, 1.5, size=(1, 3, len(ii)))
        v = rng.normal(0.0, 1.0, size=(M, 3, len(ii))) * scale
        w = rng.uniform(0.5, 1.5, size=(M, len(ii)))
        W[:, ii] = particle_moments14(w, v)
    # random Galilean boost, density and temperature scales (exact rescaling of moments)
    a = np.exp(rng.uniform(math.log(1e-3), math.log(10.0), size=n))     # density factor
    b = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=n))       # velocity factor
    boost = rng.normal(0.0, 2.0, size=(3, n))
    W[0] *= a
    W[1:4] = W[1:4] * b + boost
    W[4:10] *= a * b**2
    W[10:13] *= a * b**3
    W[13] *= a * b**4
    return W


def random_planar_states14(n, seed=0):
    """n realizable 14-moment states whose distribution is even in the z velocity (u_z =
    P_xz = P_yz = q_z = 0 exactly): in-plane Maxwellians, 2- and 3-beam mixtures with
    in-plane mean velocities, particle sets mirrored in v_z, with random density scale,
    velocity scale and in-plane boost."""
    rng = np.random.default_rng(seed)
    fam = rng.integers(0, 4, size=n)
    W = np.empty((14, n))
    i0 = np.nonzero(fam == 0)[0]
    W[:, i0] = _maxw14(np.ones(len(i0)), 0.0, 0.0, 0.0, np.ones(len(i0)))
    for f, K in ((1, 2), (2, 3)):
        ii = np.nonzero(fam == f)[0]
        if len(ii):
            w = rng.uniform(0.05, 1.0, size=(K, len(ii)))
            m = rng.normal(0.0, 1.5, size=(K, 3, len(ii)))
            m[:, 2] = 0.0
            T = rng.uniform(0.05, 1.5, size=(K, len(ii)))
            W[:, ii] = beam_mixture14(w, m, T)
    ii = np.nonzero(fam == 3)[0]
    if len(ii):
        M = 4
        w = rng.uniform(0.1, 1.0, size=(M, len(ii)))
        v = rng.normal(0.0, 1.0, size=(M, 3, len(ii)))
        vm = v.copy()
        vm[:, 2] = -vm[:, 2]
        W[:, ii] = particle_moments14(np.concatenate([w, w]), np.concatenate([v, vm]))
    # the z-odd moments vanish by symmetry; drop the sums' rounding residue
    W[[3, 6, 8, 12]] = 0.0
    a = np.exp(rng.uniform(math.log(1e-3), math.log(10.0), size=n))
    b = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=n))
    boost = rng.normal(0.0, 2.0, size=(2, n))
    W[0] *= a
    W[1:3] = W[1:3] * b + boost
    W[4:10] *= a * b**2
    W[10:13] *= a * b**3
    W[13] *= a * b**4
    return W


def random_axial_states14(n, seed=0):
    """n realizable 14-moment states of a 1D flow along x whose distribution is even in v_y
    and in v_z (u_y = u_z = P_xy = P_xz = P_yz = q_y = q_z = 0 exactly): Maxwellians moving
    along x, 2- and 3-beam mixtures with means on the x axis, particle sets mirrored in v_y
    and in v_z (so P_yy and P_zz differ), with random density, velocity scale and x-boost."""
    rng = np.random.default_rng(seed)
    fam = rng.integers(0, 4, size=n)
    W = np.empty((14, n))
    i0 = np.nonzero(fam == 0)[0]
    W[:, i0] = _maxw14(np.ones(len(i0)), 0.0, 0.0, 0.0, np.ones(len(i0)))
    for f, K in ((1, 2), (2, 3)):
        ii = np.nonzero(fam == f)[0]
        if len(ii):
            w = rng.uniform(0.05, 1.0, size=(K, len(ii)))
            m = rng.normal(0.0, 1.5, size=(K, 3, len(ii)))
            m[:, 1:] = 0.0
            T = rng.uniform(0.05, 1.5, size=(K, len(ii)))
            W[:, ii] = beam_mixture14(w, m, T)
    ii = np.nonzero(fam == 3)[0]
    if len(ii):
        M = 3
        w = rng.uniform(0.1, 1.0, size=(M, len(ii)))
        v = rng.normal(0.0, 1.0, size=(M, 3, len(ii)))
        vs, ws = [], []
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                vm = v.copy()
                vm[:, 1] *= sy
                vm[:, 2] *= sz
                vs.append(vm)
                ws.append(w)
        W[:, ii] = particle_moments14(np.concatenate(ws), np.concatenate(vs))
    # the y- and z-odd moments vanish by symmetry; drop the sums' rounding residue
    W[[2, 3, 5, 6, 8, 11, 12]] = 0.0
    a = np.exp(rng.uniform(math.log(1e-3), math.log(10.0), size=n))
    b = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=n))
    W[0] *= a
    W[1] = W[1] * b + rng.normal(0.0, 2.0, size=n)
    W[4:10] *= a * b**2
    W[10:13] *= a * b**3
    W[13] *= a * b**4
    return W


def random_states5(n, seed=0):
    rng = np.random.default_rng(seed)
    fam = rng.integers(0, 4, size=n)
    W = np.empty((5, n))
    i0 = np.nonzero(fam == 0)[0]
    W[:, i0] = _maxw5(np.ones(len(i0)), 0.0, np.ones(len(i0)))
    for f, K in ((1, 2), (2, 3)):
        ii = np.nonzero(fam == f)[0]
        if len(ii):
            W[:, ii] = beam_mixture5(rng.uniform(0.05, 1.0, size=(K, len(ii))),
                                     rng.normal(0.0, 1.5, size=(K, len(ii))),
                                     rng.uniform(0.05, 1.5, size=(K, len(ii))))
    ii = np.nonzero(fam == 3)[0]
    if len(ii):
        M = 6
        W[:, ii] = particle_moments5(rng.uniform(0.1, 1.0, size=(M, len(ii))),
                                     rng.normal(0.0, 1.0, size=(M, len(ii))))
    a = np.exp(rng.uniform(math.log(1e-3), math.log(10.0), size=n))
    b = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=n))
    boost = rng.normal(0.0, 2.0, size=n)
    W[0] *= a
    W[1] = W[1] * b + boost
    W[2] *= a * b**2
    W[3] *= a * b**3
    W[4] *= a * b**4
    return W


# --------------------------------------------------------------------------- workloads
JET_DEFAULTS = dict(mach=3.0, rho=1.0, T=1.0, background_rho=1e-3, background_T=1.0,
                    jets=((0.35, 0.1, 30.0), (0.65, 0.1, -30.0)))


def jet_speed(mach, T):
    """|u| = M sqrt(gamma T) with gamma = 5/3 (monatomic 3V gas, gas constant 1)."""
    return mach * math.sqrt(5.0 / 3.0 * T)


def crossed_jets_initial(nx, ny):
    """Crossed-jets start: uniform Maxwellian background at rho = 1e-3, T = 1, at rest."""
    return uniform_prims14(nx, ny, JET_DEFAULTS['background_rho'], JET_DEFAULTS['background_T'])


# The paper's own crossed jets (Section 6): unit square, two M = 5 jets of width L/7 centred
# on the left and bottom walls, pointing to the centre (at a right angle to each other),
# into a background at 1e-5 of the jet density; forward Euler, CFL 0.5, collisionless.
# Walls: 'xlo' = left, 'ylo' = bottom.
PAPER_JETS = dict(mach=5.0, rho=1.0, T=1.0, background_rho=1e-5, background_T=1.0,
                  jets=((0.5, 1.0 / 7.0, 0.0, 'xlo'), (0.5, 1.0 / 7.0, 90.0, 'ylo')))


def paper_jets_initial(nx, ny):
    """Start of the paper's crossed jets: uniform Maxwellian background at rest."""
    return uniform_prims14(nx, ny, PAPER_JETS['background_rho'], PAPER_JETS['background_T'])


def crossed_jets_developed(nx, ny, seed=0, reach=0.6, smear=0.02):
    """A synthetic mid-run crossed-jets field: two Maxwellian beams (M = 3, T = 1) that have
    penetrated to x = reach from the left wall along +-30 degrees, smoothly tapered, over
    the 1e-3 background, plus a seeded few-percent modulation of beam densities and
    temperatures.  Where the beams overlap the state is bimodal (super-Maxwellian kurtosis,
    non-zero heat flux, anisotropic pressure) -- the structure the crossed jets produce."""
    rng = np.random.default_rng(seed)
    x = cell_centres(nx)[None, :]
    y = cell_centres(ny)[:, None]
    d = JET_DEFAULTS
    spd = jet_speed(d['mach'], d['T'])
    wts, means, temps = [], [], []
    for (yc, w, ang) in d['jets']:
        a = math.radians(ang)
        ex, ey = math.cos(a), math.sin(a)
        # distance along and across the beam axis, from the inlet centre (0, yc)
        along = x * ex + (y - yc) * ey
        across = -x * ey + (y - yc) * ex
        prof = 0.5 * (1.0 - np.tanh((np.abs(across) - 0.5 * w) / smear))
        front = 0.5 * (1.0 - np.tanh((along - reach) / (2 * smear)))
        mod = 1.0 + 0.05 * np.sin(2 * math.pi * (rng.uniform(2, 6) * x + rng.uniform(2, 6) * y
                                                   + rng.uniform()))
        wts.append(d['rho'] * prof * front * mod + 1e-12)
        means.append(np.stack([spd * ex + 0 * x * y, spd * ey + 0 * x * y, 0 * x * y]))
        temps.append(d['T'] * (1.0 + 0.03 * np.cos(2 * math.pi * rng.uniform(1, 4) * (x + y))) + 0 * y)
    wts.append(d['background_rho'] + 0 * x * y)
    means.append(np.zeros((3, ny, nx)))
    temps.append(d['background_T'] + 0 * x * y)
    return beam_mixture14(np.stack(wts), np.stack(means), np.stack(temps))


def random_smooth_field14(nx, ny, seed=0, planar=False):
    """Smooth random realizable 2D field (beam mixtures whose parameters vary smoothly).
    planar=True: the beams move in the x-y plane, so the field is even in v_z (u_z = P_xz =
    P_yz = q_z = 0 exactly); the other parameters are drawn as for planar=False."""
    rng = np.random.default_rng(seed)
    x = cell_centres(nx)[None, :]
    y = cell_centres(ny)[:, None]

    def smooth(amp, base):
        f = np.zeros((ny, nx)) + base
        for _ in range(3):
            kx, ky = rng.integers(1, 4, size=2)
            f = f + amp * np.sin(2 * math.pi * (kx * x + ky * y) + rng.uniform(0, 2 * math.pi))
        return f

    K = 2
    w = np.stack([np.exp(smooth(0.3, 0.0)) for _ in range(K)])
    m = np.stack([np.stack([smooth(0.5, rng.normal()) for _ in range(3)]) for _ in range(K)])
    T = np.stack([np.exp(smooth(0.2, 0.0)) for _ in range(K)])
    if planar:
        m[:, 2] = 0.0
    return beam_mixture14(w, m, T)


def batch_instances(n_inst=512, seed=20240127, n_lo=512, n_hi=32768):
    """Batched shock tubes: per instance the cell count (even, log-uniform), the pressure
    ratio p_L/p_R ~ U(2, 100), the density ratio rho_L/rho_R ~ U(2, 20) and Kn ~
    logU(1e-3, 10), drawn in that order per instance.  Left state (rho, p) = (1, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        N = 2 * int(round(0.5 * math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        pr = rng.uniform(2.0, 100.0)
        rr = rng.uniform(2.0, 20.0)
        kn = math.exp(rng.uniform(math.log(1e-3), math.log(10.0)))
        out.append(dict(n=N, p_ratio=pr, rho_ratio=rr, kn=kn))
    return out


def kn_to_tau_ref(kn, L_ref=1.0, T_ref=1.0):
    """tau_ref = lambda / v_th with lambda = Kn L_ref and v_th = sqrt(8 T_ref / pi)."""
    return kn * L_ref / math.sqrt(8.0 * T_ref / math.pi)


def batch_sod_prims(instances):
    """Concatenated primitive field of batched shock tubes: instance i has left (rho, p) =
    (1, 1) and right (1/rho_ratio, 1/p_ratio), at rest, Maxwellian, diaphragm at 0.5 of [0, 1]."""
    parts = []
    for d in instances:
        right = (1.0 / d['rho_ratio'], 0.0, 1.0 / d['p_ratio'])
        parts.append(sod_prims(14, d['n'], left=(1.0, 0.0, 1.0), right=right))
    return np.concatenate(parts, axis=1)

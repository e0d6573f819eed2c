// Batched independent 1D shock tubes in one launch per stage.
//
// Many 1D problems of uneven length, each with its own collision time, end time and CFL time
// step, are concatenated in one structure-of-arrays field.  The instances form a queue
// ordered by estimated work (cells x steps, from the initial CFL rate).  Each step, a
// one-workgroup finalize kernel gives every instance its time step and compacts the
// instances that still advance, in queue order, into a work list of tiles (tiles never
// straddle instances); the two stage launches of the step split that list into contiguous
// ranges, one per workgroup, so finished instances cost nothing.  A step is finalize + two
// stage launches, so a chunk of steps can be captured once in a hipGraph and replayed.  The
// per-cell arithmetic is the single-instance 1D kernel's (same device functions, same update
// formula), so a batched instance reproduces the same instance run alone bit for bit.
#include "mx_internal.hpp"
#include "mx_physics.hpp"
#include "mx_scheme.hpp"
#include "mx_axial.hpp"
#include "mx_batch.hpp"

namespace mx {

__device__ __forceinline__ double bwave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int bwave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int bwave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int bmap(int g, int n, int lo, int hi, int& refl) {
  if (g < 0) {
    if (lo == 1) g = g + n * ((-g + n - 1) / n);
    else if (lo == 2) { g = -g - 1; refl = 1; }
    else g = 0;
  } else if (g >= n) {
    if (hi == 1) g = g % n;
    else if (hi == 2) { g = 2 * n - 1 - g; refl = 1; }
    else g = n - 1;
  }
  return g < 0 ? 0 : (g >= n ? n - 1 : g);
}

// One workgroup of 1024 threads walks the instance queue (instances ordered by estimated
// work): time step of each instance from its CFL rate, clipped to its t_end; then an ordered
// compaction of the instances that advance, with the exclusive prefix of their tile counts.
// The stage launches of the step split the resulting tile list into contiguous ranges.
__global__ __launch_bounds__(1024) void batch_finalize_kernel(BatchInst* in, const int* order, int n_inst,
                                                             double cfl, int tile_w, int* act_inst,
                                                             int* act_tile0, BatchCtrl* bc, int nb) {
  __shared__ int s_wave[16][2];   // per-wavefront totals of (active, tiles)
  __shared__ int s_carry[2];      // totals of the earlier chunks
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  if (t == 0) { s_carry[0] = 0; s_carry[1] = 0; }
  __syncthreads();
  for (int base = 0; base < n_inst; base += 1024) {
    const int q = base + t;
    int a = 0, nt = 0, inst = 0;
    if (q < n_inst) {
      inst = order[q];
      BatchInst& c = in[inst];
      double dt = 0.0;
      if (c.status == 0) {
        double m = __longlong_as_double((long long)c.maxrate);
        dt = (m > 0.0) ? cfl * c.dx / m : 0.0;
        if (c.t >= c.t_end * (1.0 - 1e-14)) dt = 0.0;
        else dt = fmin(dt, c.t_end - c.t);
      }
      c.dt = dt;
      c.maxrate = 0ull;
      if (dt > 0.0) {
        c.t += dt;
        c.step += 1;
        c.dt_last = dt;
        a = 1;
        nt = (c.n + tile_w - 1) / tile_w;
      }
    }
    // inclusive scans within the wavefront
    int sa = a, sn = nt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int ya = __shfl_up(sa, o, 64), yn = __shfl_up(sn, o, 64);
      if (lane >= o) { sa += ya; sn += yn; }
    }
    if (lane == 63) { s_wave[wid][0] = sa; s_wave[wid][1] = sn; }
    __syncthreads();
    int oa = s_carry[0], on = s_carry[1];
    for (int w = 0; w < wid; ++w) { oa += s_wave[w][0]; on += s_wave[w][1]; }
    if (a) {
      act_inst[oa + sa - 1] = inst;
      act_tile0[oa + sa - 1] = on + sn - nt;
    }
    __syncthreads();  // every thread has read s_carry
    if (t == 1023) { s_carry[0] = oa + sa; s_carry[1] = on + sn; }
    __syncthreads();
  }
  if (t == 0) {
    const int n_tiles = s_carry[1];
    act_tile0[s_carry[0]] = n_tiles;
    bc->n_active = s_carry[0];
    bc->n_tiles = n_tiles;
    // split of the tile list over the nb workgroups of the stage launches: contiguous ranges
    // of `per` tiles.  Hardware deals consecutive workgroups round-robin to the 8 XCDs; each
    // XCD gets a band of neighbouring ranges, so that halos and instance records are shared
    // in its L2.  While the ranges in use fill more than half of the grid the bands are the
    // grid's eighths; once they fill half or less (the end of a batch) the bands divide the
    // ranges in use, which would otherwise all fall on the first XCDs (measured on one
    // 546-tile tube: 85 -> 37.5 us per step)
    const int per = (n_tiles + nb - 1) / nb;
    int band = 0;
    if (nb % 8 == 0 && per > 0) {
      const int used = (n_tiles + per - 1) / per;  // <= nb
      band = (2 * used <= nb) ? (used + 7) / 8 : nb / 8;
    }
    bc->per = per;
    bc->band = band;
  }
}

// Stage kernel: a workgroup of NT threads owns tiles of CPT * NT - 4 cells (CPT cells per
// thread), so the tile plus its two-cell halos fills whole rounds over the threads.  The
// step's tile list (active instances in queue order, each cut into tiles) is split into
// contiguous ranges, one per workgroup, with an XCD-aware order of the ranges; a workgroup
// finds its first tile by a binary search over the tile prefix and then walks forward.
// Two waves per SIMD: the register budget is 256 per lane.
template <class SYS, int ORDER, int PREC, int NT, int CPT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(SYS::NV <= 7 ? 3 : 2)))
void batch_stage_kernel(BatchParams p) {
  constexpr int NV = SYS::NV;
  constexpr int TX = tile_1d(CPT * NT);
  constexpr int G = (ORDER == 2) ? 2 : 1;
  constexpr int LX = TX + 2 * G;
  constexpr int NFX = TX + 1;
  constexpr int NPX = (ORDER == 2) ? TX + 2 : 1;
  __shared__ double sW[NV * LX];
  __shared__ double sFx[NV * NFX];
  __shared__ double sPx[NPX];
  __shared__ double sRed[NT / 64];
  __shared__ int sFlag[3];
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;

  const int n_tiles = p.bctrl->n_tiles;
  const int n_act = p.bctrl->n_active;
  // this workgroup's range of the tile list (split and XCD bands set by the finalize kernel)
  const int per = p.bctrl->per;
  const int band = p.bctrl->band;
  int slot = blockIdx.x;
  if (band > 0) {
    const int kx = blockIdx.x >> 3;
    slot = (kx < band) ? (blockIdx.x & 7) * band + kx : (int)gridDim.x;
  }
  const int k0 = slot * per;   // slot <= grid: at most n_tiles + grid
  const int k1 = min(k0 + per, n_tiles);
  if (k0 >= k1) return;  // uniform over the workgroup
  int j = 0;
  {
    int hi = n_act - 1;  // last active instance whose first tile is <= k0
    while (j < hi) {
      const int mid = (j + hi + 1) >> 1;
      if (p.act_tile0[mid] <= k0) j = mid;
      else hi = mid - 1;
    }
  }
  int first = p.act_tile0[j], next = p.act_tile0[j + 1];

  for (int k = k0; k < k1; ++k) {
    if (k >= next) {  // every active instance has at least one tile
      ++j;
      first = next;
      next = p.act_tile0[j + 1];
    }
    const int inst = p.act_inst[j];
    const int i0 = (k - first) * TX;
    BatchInst* c = p.inst + inst;
    const double dt = c->dt;
    if (!(dt > 0.0)) continue;  // uniform; not reached for a listed instance
    const int n = c->n;
    const long long off = c->off;
    const double inv_dx = c->inv_dx;
    __syncthreads();            // LDS of the previous tile is no longer read
    if (t < 3) sFlag[t] = 0;
    int n64 = 0;

    // 1. tile + halo -> primitives
    for (int cc = t; cc < LX; cc += NT) {
      int rx = 0;
      int si = bmap(i0 + cc - G, n, p.bc_lo, p.bc_hi, rx);
      double Uc[NV], W[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Uc[v] = p.Ub[SYS::plane_of(v) * p.plane + off + si];
      SYS::cons_to_prim(Uc, W);
      if (rx) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (SYS::odd(v, 0)) W[v] = -W[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) sW[v * LX + cc] = W[v];
    }
    __syncthreads();
    auto lds = [&](int ti, double* W) {
#pragma unroll
      for (int v = 0; v < NV; ++v) W[v] = sW[v * LX + ti + G];
    };

    // 2. common limiter factors
    int nfb = 0;
    if constexpr (ORDER == 2) {
      for (int cc = t; cc < NPX; cc += NT) {
        int ti = cc - 1;
        double Wm[NV], Wc[NV], Wp[NV];
        lds(ti - 1, Wm); lds(ti, Wc); lds(ti + 1, Wp);
        double phi = limiter_factor<SYS>(Wm, Wc, Wp, p.limiter);
        if (p.fallback && phi > 0.0) {
          const bool ok = faces_admissible<SYS>(Wm, Wc, Wp, phi);
          if (!ok) {
            phi = 0.0;
            if (ti >= 0 && ti < TX && i0 + ti < n) ++nfb;
          }
        }
        sPx[cc] = phi;
      }
      __syncthreads();
    }

    // 3. faces: face fi lies between tile cells fi - 1 and fi
    for (int fi = t; fi < NFX; fi += NT) {
      double WL[NV], WR[NV];
      if constexpr (ORDER == 2) {
        double A[NV], B[NV], C[NV], D[NV];
        lds(fi - 2, A); lds(fi - 1, B); lds(fi, C); lds(fi + 1, D);
        face_state<SYS>(A, B, C, sPx[fi], 1.0, WL);
        face_state<SYS>(B, C, D, sPx[fi + 1], -1.0, WR);
      } else {
        lds(fi - 1, WL); lds(fi, WR);
      }
      double Fh[NV];
      if constexpr (PREC == 0) face_flux<SYS, 0>(WL, WR, p.sigma_lim, p.kws, p.flux, Fh);
      else face_flux_mixed<SYS, 0>(WL, WR, p.sigma_lim, p.kws, p.flux, Fh, n64);
#pragma unroll
      for (int v = 0; v < NV; ++v) sFx[v * NFX + fi] = Fh[v];
    }
    __syncthreads();

    // 4. update
    int flag = 0;
    double rate = 0.0;
    for (int ci = t; ci < TX; ci += NT) {
      if (i0 + ci >= n) break;
      long long g = off + i0 + ci;
      double Ub[NV], W[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Ub[v] = p.Ub[SYS::plane_of(v) * p.plane + g];
      SYS::cons_to_prim(Ub, W);
      double Cs[NV];
      const double tau_ref = c->tau_ref;
      if (tau_ref > 0.0) {
        double rho = W[0];
        double T = SYS::pressure(W) / rho;
        double tau = (p.tau_mode == 0) ? tau_ref * (p.rho_ref / rho) * sqrt(p.T_ref / T) : tau_ref;
        SYS::source(W, 1.0 / tau, Cs);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Cs[v] = 0.0;
      }
      double Un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double L = -(sFx[v * NFX + ci + 1] - sFx[v * NFX + ci]) * inv_dx;
        L = L + Cs[v];
        double o;
        if (p.mode == MODE_EULER) o = Ub[v] + (p.cdt * dt) * L;
        else if (p.mode == MODE_HEUN2) o = 0.5 * p.Ua[SYS::plane_of(v) * p.plane + g] + 0.5 * (Ub[v] + dt * L);
        else o = p.Ua[SYS::plane_of(v) * p.plane + g] + dt * L;
        Un[v] = o;
        p.Uout[SYS::plane_of(v) * p.plane + g] = o;
      }
      bool fin = true;
#pragma unroll
      for (int v = 0; v < NV; ++v) fin = fin && isfinite(Un[v]);
      if (!fin) {
        flag |= ST_NONFINITE;
      } else if (p.do_cfl) {
        double Wn[NV];
        SYS::cons_to_prim(Un, Wn);
        if (!SYS::admissible(Wn)) flag |= ST_UNREALIZABLE;
        else rate = fmax(rate, SYS::template cell_lambda<0>(Wn, p.sigma_lim, p.kws));
      } else if (!SYS::admissible_cons(Un)) {
        flag |= ST_UNREALIZABLE;
      }
    }
    flag = bwave_or(flag);
    nfb = bwave_sum(nfb);
    if constexpr (PREC != 0) n64 = bwave_sum(n64);
    if (lane == 0) {
      if (flag) atomicOr(&sFlag[0], flag);
      if (nfb) atomicAdd(&sFlag[1], nfb);
      if (PREC != 0 && n64) atomicAdd(&sFlag[2], n64);
    }
    if (p.do_cfl) {
      rate = bwave_max(rate);
      if (lane == 0) sRed[wid] = rate;
    }
    __syncthreads();
    if (t == 0) {
      if (sFlag[0]) {
        atomicOr(&c->status, sFlag[0]);
        atomicMin(&c->fail_step, (int)c->step);
      }
      if (sFlag[1]) atomicAdd((unsigned long long*)&p.ctrl->n_fallback, (unsigned long long)sFlag[1]);
      if (PREC != 0) {
        if (sFlag[2]) atomicAdd((unsigned long long*)&p.ctrl->n_fp64, (unsigned long long)sFlag[2]);
        atomicAdd((unsigned long long*)&p.ctrl->n_states, (unsigned long long)(2 * NFX));
      }
      if (p.do_cfl) {
        double m = sRed[0];
        for (int w = 1; w < NT / 64; ++w) m = fmax(m, sRed[w]);
        atomicMax(&c->maxrate, (unsigned long long)__double_as_longlong(m));
      }
    }
  }
}


// CFL rate of every instance's current state (after init)
template <class SYS>
__global__ __launch_bounds__(256) void batch_cfl_kernel(BatchParams p, long long total) {
  constexpr int NV = SYS::NV;
  for (long long g = (long long)blockIdx.x * 256 + threadIdx.x; g < total;
       g += (long long)gridDim.x * 256) {
    int inst = p.cell_inst[g];
    double U[NV], W[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = p.Ub[v * p.plane + g];
    SYS::cons_to_prim(U, W);
    double r = SYS::template cell_lambda<0>(W, p.sigma_lim, p.kws);
    atomicMax(&p.inst[inst].maxrate, (unsigned long long)__double_as_longlong(r));
  }
}

template <class SYS, int PREC, int NT, int CPT>
static hipError_t launch_bs(const BatchParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_stage_kernel<SYS, 2, PREC, NT, CPT>), dim3(grid), dim3(NT), 0, s, p);
  return hipGetLastError();
}

template <class SYS, int PREC>
static hipError_t launch_bs_p(int nt, int cpt, const BatchParams& p, int grid, hipStream_t s) {
  if (nt == 64 && cpt == 1) return launch_bs<SYS, PREC, 64, 1>(p, grid, s);
  if (nt == 64 && cpt == 2) return launch_bs<SYS, PREC, 64, 2>(p, grid, s);
  if (nt == 64 && cpt == 4) return launch_bs<SYS, PREC, 64, 4>(p, grid, s);
  if (nt == 128 && cpt == 1) return launch_bs<SYS, PREC, 128, 1>(p, grid, s);
  if (nt == 128 && cpt == 2) return launch_bs<SYS, PREC, 128, 2>(p, grid, s);
  if (nt == 256 && cpt == 1) return launch_bs<SYS, PREC, 256, 1>(p, grid, s);
  return hipErrorInvalidValue;
}

bool batch_shape_supported(int nt, int cpt) {
  return (nt == 64 && (cpt == 1 || cpt == 2 || cpt == 4)) || (nt == 128 && (cpt == 1 || cpt == 2)) ||
         (nt == 256 && cpt == 1);
}

hipError_t launch_batch_stage(int precision, bool reduced, int nt, int cpt, const BatchParams& p, int grid,
                              hipStream_t s) {
  if (reduced)
    return precision == 0 ? launch_bs_p<Sys14A, 0>(nt, cpt, p, grid, s) : launch_bs_p<Sys14A, 1>(nt, cpt, p, grid, s);
  return precision == 0 ? launch_bs_p<Sys14, 0>(nt, cpt, p, grid, s) : launch_bs_p<Sys14, 1>(nt, cpt, p, grid, s);
}

hipError_t launch_batch_finalize(BatchInst* in, const int* order, int n_inst, double cfl, int tile_w,
                                 int* act_inst, int* act_tile0, BatchCtrl* bc, int stage_grid,
                                 hipStream_t s) {
  if (stage_grid < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(1), dim3(1024), 0, s, in, order, n_inst, cfl, tile_w,
                     act_inst, act_tile0, bc, stage_grid);
  return hipGetLastError();
}

hipError_t launch_batch_cfl(const BatchParams& p, long long total, hipStream_t s) {
  long long g = (total + 255) / 256;
  int grid = (int)(g > 8192 ? 8192 : g);
  hipLaunchKernelGGL((batch_cfl_kernel<Sys14>), dim3(grid), dim3(256), 0, s, p, total);
  return hipGetLastError();
}

}  // namespace mx

// Batched independent 1D shock tubes in one launch per stage.
//
// Many 1D problems of uneven length, each with its own collision time, end time and CFL time
// step, are concatenated in one structure-of-arrays field.  Each instance is cut into tiles
// of TX cells (tiles never straddle instances); the tile list is static.  A persistent
// launch of a fixed number of workgroups sweeps the tile list with a grid stride, skipping
// the tiles of instances that have reached their end time, so finished instances cost a
// load and a compare; every workgroup leaves the loop when the list is exhausted.  A step is
// finalize (per-instance dt) + two stage launches, so a chunk of steps can be captured once
// in a hipGraph and replayed.  The per-cell arithmetic is the single-instance 1D kernel's
// (same device functions, same update formula), so a batched instance reproduces the same
// instance run alone bit for bit.
#include "mx_internal.hpp"
#include "mx_physics.hpp"
#include "mx_scheme.hpp"
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

// one thread per instance: time step from the instance's CFL rate, clipped to its t_end
__global__ void batch_finalize_kernel(BatchInst* in, int n_inst, double cfl, BatchCtrl* bc) {
  __shared__ int s_active;
  if (threadIdx.x == 0) s_active = 0;
  __syncthreads();
  int active = 0;
  for (int i = threadIdx.x; i < n_inst; i += blockDim.x) {
    BatchInst& c = in[i];
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
      ++active;
    }
  }
  active = bwave_sum(active);
  if ((threadIdx.x & 63) == 0 && active) atomicAdd(&s_active, active);
  __syncthreads();
  if (threadIdx.x == 0) bc->n_active = s_active;
}

template <class SYS, int ORDER, int PREC, int NT>
__global__ __launch_bounds__(NT) void batch_stage_kernel(BatchParams p) {
  constexpr int NV = SYS::NV;
  constexpr int TX = NT - 1;
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

  for (int k = blockIdx.x; k < p.n_tiles; k += gridDim.x) {
    const int2 tl = p.tiles[k];
    const int inst = tl.x;
    const int i0 = tl.y;
    BatchInst* c = p.inst + inst;
    const double dt = c->dt;
    if (!(dt > 0.0)) continue;  // uniform over the workgroup: instance finished or failed
    const int n = c->n;
    const long long off = c->off;
    const double dx = c->dx, inv_dx = c->inv_dx;
    __syncthreads();            // LDS of the previous tile is no longer read
    if (t < 3) sFlag[t] = 0;
    int n64 = 0;

    // 1. tile + halo -> primitives
    for (int cc = t; cc < LX; cc += NT) {
      int rx = 0;
      int si = bmap(i0 + cc - G, n, p.bc_lo, p.bc_hi, rx);
      double Uc[NV], W[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Uc[v] = p.Ub[v * p.plane + off + si];
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
          double Wf[NV];
          face_state<SYS>(Wm, Wc, Wp, phi, 1.0, Wf);
          bool ok = SYS::admissible(Wf);
          face_state<SYS>(Wm, Wc, Wp, phi, -1.0, Wf);
          ok = ok && SYS::admissible(Wf);
          if (!ok) {
            phi = 0.0;
            if (ti >= 0 && ti < TX && i0 + ti < n) ++nfb;
          }
        }
        sPx[cc] = phi;
      }
      __syncthreads();
    }

    // 3. faces
    {
      const int fi = t;
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
    if (t < TX && i0 + t < n) {
      long long g = off + i0 + t;
      double Ub[NV], W[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Ub[v] = p.Ub[v * p.plane + g];
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
        double L = -(sFx[v * NFX + t + 1] - sFx[v * NFX + t]) * inv_dx;
        L = L + Cs[v];
        double o;
        if (p.mode == MODE_EULER) o = Ub[v] + (p.cdt * dt) * L;
        else if (p.mode == MODE_HEUN2) o = 0.5 * p.Ua[v * p.plane + g] + 0.5 * (Ub[v] + dt * L);
        else o = p.Ua[v * p.plane + g] + dt * L;
        Un[v] = o;
        p.Uout[v * p.plane + g] = o;
      }
      bool fin = true;
#pragma unroll
      for (int v = 0; v < NV; ++v) fin = fin && isfinite(Un[v]);
      double Wn[NV];
      SYS::cons_to_prim(Un, Wn);
      if (!fin) flag |= ST_NONFINITE;
      else if (!SYS::admissible(Wn)) flag |= ST_UNREALIZABLE;
      if (p.do_cfl && flag == 0) rate = SYS::template cell_lambda<0>(Wn, p.sigma_lim, p.kws);
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

template <int PREC, int NT>
static hipError_t launch_bs(const BatchParams& p, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batch_stage_kernel<Sys14, 2, PREC, NT>), dim3(grid), dim3(NT), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_batch_stage(int precision, int nt, const BatchParams& p, int grid, hipStream_t s) {
  if (precision == 0) {
    if (nt == 64) return launch_bs<0, 64>(p, grid, s);
    if (nt == 128) return launch_bs<0, 128>(p, grid, s);
    if (nt == 256) return launch_bs<0, 256>(p, grid, s);
  } else {
    if (nt == 64) return launch_bs<1, 64>(p, grid, s);
    if (nt == 128) return launch_bs<1, 128>(p, grid, s);
    if (nt == 256) return launch_bs<1, 256>(p, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_finalize(BatchInst* in, int n_inst, double cfl, BatchCtrl* bc, hipStream_t s) {
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(1), dim3(1024), 0, s, in, n_inst, cfl, bc);
  return hipGetLastError();
}

hipError_t launch_batch_cfl(const BatchParams& p, long long total, hipStream_t s) {
  long long g = (total + 255) / 256;
  int grid = (int)(g > 8192 ? 8192 : g);
  hipLaunchKernelGGL((batch_cfl_kernel<Sys14>), dim3(grid), dim3(256), 0, s, p, total);
  return hipGetLastError();
}

}  // namespace mx

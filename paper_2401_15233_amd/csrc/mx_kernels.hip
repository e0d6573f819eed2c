// gfx950 kernels of the finite-volume step (FP64; FP32 / mixed face evaluation by template).
//
// One fused kernel per Runge-Kutta stage.  A workgroup owns a TX x TY tile of cells and
//   1. loads the tile plus a G-cell halo of the stage input U (structure of arrays, x
//      fastest), applying the boundary conditions while loading (ghost cells are never
//      stored), converts to primitives and keeps them in LDS;
//   2. computes the common (most stringent) limiter factor of every cell that feeds a face
//      of the tile (Section 3.2), with the positivity fallback;
//   3. evaluates every face of the tile once: both reconstructed states, their closure
//      (Sections 2.3-2.4, Appendix A), wave speeds (Section 5.1), physical fluxes and the
//      HLL / Rusanov combination (Section 3.1);
//   4. updates each cell with the flux differences and the BGK source at the cell centre,
//      writes the result, checks it (non-finite, rho <= 0, P not SPD) and, in the last
//      stage of a step, reduces the CFL rate of the new state for the next step.
// The 2D tile is 16 x 15 cells for 256 threads: 255 x-faces and 256 y-faces, one of each
// per thread.  The 1D tile is 60 cells for one 64-wide wavefront: cells plus halo fill the
// wavefront exactly.
#include "mx_internal.hpp"
#include "mx_physics.hpp"
#include "mx_scheme.hpp"
#include "mx_bc.hpp"
#include "mx_planar.hpp"
#include "mx_axial.hpp"

namespace mx {

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ stage kernel
// Waves per SIMD the kernel is compiled for.  The planar 2D kernel (ten moments) fits three
// 256-thread workgroups per CU in LDS (45 KB each, with part of the x-face fluxes kept in
// registers); asking for three waves per SIMD caps it at 168 VGPRs, a few of them spilled,
// which measured faster than two waves without spills.  The full 14-moment kernel needs two.
constexpr int stage_min_waves(int nv, int dim) { return (nv <= 10 && dim == 2) ? 3 : 1; }

template <class SYS, int DIM, int ORDER, int PREC, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(stage_min_waves(SYS::NV, DIM))))
void stage_kernel(StageParams p) {
  constexpr int NV = SYS::NV;
  constexpr int G = (ORDER == 2) ? 2 : 1;
  constexpr int LX = TX + 2 * G;
  constexpr int LY = (DIM == 2) ? TY + 2 * G : 1;
  constexpr int NL = LX * LY;
  constexpr int NFX = (TX + 1) * TY;
  constexpr int NFY = (DIM == 2) ? TX * (TY + 1) : 0;
  constexpr int NPX = (ORDER == 2) ? (TX + 2) * TY : 1;
  constexpr int NPY = (ORDER == 2 && DIM == 2) ? TX * (TY + 2) : 1;
  // planar 2D (XREG): no separate x-flux array.  The x-flux components v >= XK go to LDS at
  // once, past the primitive tile (free during the face phases); the first XK stay in
  // registers through the y-face phase, and all of them overwrite the primitive tile after a
  // barrier.  XK = 1: the largest LDS footprint that still fits three workgroups per CU
  // (52 KB each; all ten components would take 54 KB); each component held in registers
  // instead costs two VGPRs at the kernel's peak, which the three-wavefront build spills
  constexpr bool XREG = (DIM == 2 && NV <= 10);
  constexpr int NFL = XREG ? NV * (NFX + NFY) : NV * NFY;
  constexpr int XK = XREG ? 1 : NV;
  constexpr int NW0 = XREG ? NV * NL + (NV - XK) * NFX : NV * NL;
  constexpr int NW = (NW0 > NFL) ? NW0 : NFL;
  constexpr int XH = NW - (NV - XK) * NFX;      // where the LDS-held x-flux components start
  static_assert(!XREG || XH >= NV * NL, "x-flux slots past the primitive tile");
  static_assert(!XREG || XK * NFX + NV * NFY <= XH, "fluxes after the barrier fit below them");
  static_assert(NFX <= NT || DIM == 1, "one x-face per thread");

  __shared__ double sW[NW];        // primitives of the tile + halo; later the face fluxes
  __shared__ double sFx[XREG ? 1 : NV * NFX];
  __shared__ double sPx[NPX];
  __shared__ double sPy[NPY];
  __shared__ double sRed[NT / 64];
  __shared__ int sFlag[3];

  // XCD-aware tile order: hardware deals consecutive workgroups round-robin to the 8
  // XCDs; give each XCD a contiguous band of tiles so halos are shared in its L2.
  const int nb8 = (p.nblk + 7) / 8;
  const int b = blockIdx.x;
  const int tile = (b % 8) * nb8 + b / 8;
  if (tile >= p.nblk) return;
  const int i0 = (tile % p.ntx) * TX;
  const int j0 = (tile / p.ntx) * TY;
  const int t = threadIdx.x;

  const double dt = p.dt_replay > 0.0 ? p.dt_replay : p.ctrl->dt;
  if (!(dt > 0.0)) {  // uniform: time end reached or a failure stopped the run
    if (p.copy_on_idle && t < TX * TY) {
      int gi = i0 + t % TX, gj = j0 + t / TX;
      if (gi < p.nx && gj < p.ny) {
        long long off = (long long)gj * p.pitch + gi;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const long long o = SYS::plane_of(v) * p.plane + off;
          p.Uout[o] = p.Ub[o];
        }
      }
    }
    return;
  }
  if (t < 3) sFlag[t] = 0;
  int n64 = 0;      // FP64 re-evaluations of face states (mixed precision)
  int nstates = 0;  // face states evaluated

  // 1. tile + halo -> primitives in LDS
  // (a thread issues the loads of all its cells before it converts any)
  {
    constexpr int NR = (NL + NT - 1) / NT;
    double Uh[NR][NV];
    HaloSrc hs[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int c = t + r * NT;
      if (c < NL) {
        const int li = c % LX, lj = c / LX;
        hs[r] = load_cons<SYS>(p, p.Ub, i0 + li - G, (DIM == 2) ? j0 + lj - G : 0, Uh[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int c = t + r * NT;
      if (c < NL) {
        const int li = c % LX, lj = c / LX;
        double W[NV];
        finish_prims<SYS>(p, hs[r], i0 + li - G, (DIM == 2) ? j0 + lj - G : 0, Uh[r], W);
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v * NL + c] = W[v];
      }
    }
  }
  __syncthreads();

  auto lds = [&](int ti, int tj, double* W) {
    int c = (DIM == 2) ? (tj + G) * LX + (ti + G) : (ti + G);
#pragma unroll
    for (int v = 0; v < NV; ++v) W[v] = sW[v * NL + c];
  };

  // 2. common limiter factors, x and y items in one sweep (542 items on 256 threads take
  // three rounds; two separate loops would take four)
  int nfb = 0;
  if constexpr (ORDER == 2) {
    constexpr int NPT = (DIM == 2) ? NPX + NPY : NPX;
    for (int c = t; c < NPT; c += NT) {
      const bool isx = c < NPX;
      int ti, tj, di, dj;
      if (isx) { ti = c % (TX + 2) - 1; tj = c / (TX + 2); di = 1; dj = 0; }
      else { const int cy = c - NPX; ti = cy % TX; tj = cy / TX - 1; di = 0; dj = 1; }
      double Wm[NV], Wc[NV], Wp[NV];
      lds(ti - di, tj - dj, Wm); lds(ti, tj, Wc); lds(ti + di, tj + dj, Wp);
      double phi = limiter_factor<SYS>(Wm, Wc, Wp, p.limiter);
      if (p.fallback && phi > 0.0 && !faces_admissible<SYS>(Wm, Wc, Wp, phi)) {
        phi = 0.0;
        const bool own = isx ? (ti >= 0 && ti < TX) : (tj >= 0 && tj < TY);
        if (own && i0 + ti < p.nx && j0 + tj < p.ny) ++nfb;
      }
      if (isx) sPx[c] = phi;
      else sPy[c - NPX] = phi;
    }
    __syncthreads();
  }

  // 3a. x faces: face f lies between tile cells (fi-1, fj) and (fi, fj)
  double Fx[NV];
  for (int f = t; f < NFX; f += NT) {
    int fi = f % (TX + 1), fj = f / (TX + 1);
    double WL[NV], WR[NV];
    if constexpr (ORDER == 2) {
      double A[NV], B[NV], C[NV], D[NV];
      lds(fi - 2, fj, A); lds(fi - 1, fj, B); lds(fi, fj, C); lds(fi + 1, fj, D);
      face_state<SYS>(A, B, C, sPx[fj * (TX + 2) + fi], 1.0, WL);
      face_state<SYS>(B, C, D, sPx[fj * (TX + 2) + fi + 1], -1.0, WR);
    } else {
      lds(fi - 1, fj, WL); lds(fi, fj, WR);
    }
    double Fh[NV];
    if constexpr (PREC == 0) face_flux<SYS, 0>(WL, WR, p.sigma_lim, p.kws, p.flux, Fh);
    else if constexpr (PREC == 1) face_flux_mixed<SYS, 0>(WL, WR, p.sigma_lim, p.kws, p.flux, Fh, n64);
    else face_flux_fp32<SYS, 0>(WL, WR, p.sigma_lim, p.kws, p.flux, Fh);
    nstates += 2;
    if constexpr (XREG) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v < XK) Fx[v] = Fh[v];
        else sW[XH + (v - XK) * NFX + f] = Fh[v];
      }
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) sFx[v * NFX + f] = Fh[v];
    }
  }

  // 3b. y faces: face f lies between tile cells (fi, fj-1) and (fi, fj)
  double Fy[NV];
  const bool has_y = (DIM == 2) && (t < NFY);
  if constexpr (DIM == 2) {
    static_assert(NFY <= NT, "one y-face per thread");
    if (has_y) {
      int fi = t % TX, fj = t / TX;
      double WL[NV], WR[NV];
      if constexpr (ORDER == 2) {
        double A[NV], B[NV], C[NV], D[NV];
        lds(fi, fj - 2, A); lds(fi, fj - 1, B); lds(fi, fj, C); lds(fi, fj + 1, D);
        face_state<SYS>(A, B, C, sPy[fj * TX + fi], 1.0, WL);
        face_state<SYS>(B, C, D, sPy[(fj + 1) * TX + fi], -1.0, WR);
      } else {
        lds(fi, fj - 1, WL); lds(fi, fj, WR);
      }
      {
        if constexpr (PREC == 0) face_flux<SYS, 1>(WL, WR, p.sigma_lim, p.kws, p.flux, Fy);
        else if constexpr (PREC == 1) face_flux_mixed<SYS, 1>(WL, WR, p.sigma_lim, p.kws, p.flux, Fy, n64);
        else face_flux_fp32<SYS, 1>(WL, WR, p.sigma_lim, p.kws, p.flux, Fy);
      }
      nstates += 2;
    }
  }
  // 3c. the update's inputs, gathered before the barriers so that the global loads overlap
  // the waits: the cell's stage input and (second-stage combinations) U^n from memory, its
  // primitives from the tile in LDS (converted by the load phase, so no second primitive
  // recovery) and the BGK source at the cell centre
  const int ci = t % TX, cj = t / TX;
  const bool own = (t < TX * TY) && (i0 + ci < p.nx) && (j0 + cj < p.ny);
  const long long off = (long long)(j0 + cj) * p.pitch + (i0 + ci);
  const bool implicit_src = p.use_source && p.src_implicit;
  double Ub[NV], Ua[NV], Cs[NV];
  if (own) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Ub[v] = p.Ub[SYS::plane_of(v) * p.plane + off];
    if (p.mode != MODE_EULER) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Ua[v] = p.Ua[SYS::plane_of(v) * p.plane + off];
    }
    if (p.use_source && !implicit_src) {
      double W[NV];
      lds(ci, cj, W);
      const double rho = W[0];
      const double T = SYS::pressure(W) / rho;
      const double tau = (p.tau_mode == 0) ? p.tau_ref * (p.rho_ref / rho) * sqrt(p.T_ref / T) : p.tau_ref;
      SYS::source(W, 1.0 / tau, Cs);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Cs[v] = 0.0;
    }
  }
  __syncthreads();
  // y-face fluxes (and, planar, the x-face fluxes) over the primitive tile
  constexpr int Y0 = XREG ? XK * NFX : 0;
  if constexpr (DIM == 2) {
    if constexpr (XREG) {
      static_assert(NFX <= NT, "one x-face per thread");
      if (t < NFX) {
#pragma unroll
        for (int v = 0; v < XK; ++v) sW[v * NFX + t] = Fx[v];
      }
    }
    if (has_y) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sW[Y0 + v * NFY + t] = Fy[v];
    }
    __syncthreads();
  }

  // 4. update
  int flag = 0;
  double rate = 0.0;
  if (own) {
    {
      double Un[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double* fx = XREG ? sW : sFx;
        const int xb = (XREG && v >= XK) ? XH + (v - XK) * NFX : v * NFX;
        double L = -(fx[xb + cj * (TX + 1) + ci + 1] - fx[xb + cj * (TX + 1) + ci]) * p.inv_dx;
        if constexpr (DIM == 2)
          L = L - (sW[Y0 + v * NFY + (cj + 1) * TX + ci] - sW[Y0 + v * NFY + cj * TX + ci]) * p.inv_dy;
        L = L + Cs[v];
        double o;
        if (p.mode == MODE_EULER) o = Ub[v] + (p.cdt * dt) * L;
        else if (p.mode == MODE_HEUN2) o = 0.5 * Ua[v] + 0.5 * (Ub[v] + dt * L);
        else o = Ua[v] + dt * L;
        Un[v] = o;
        if (!implicit_src) p.Uout[SYS::plane_of(v) * p.plane + off] = o;
      }
      if (implicit_src) {
        // backward-Euler BGK relaxation of the transported state (forward-Euler stages only):
        // the source keeps rho, rho u and the energy, so the Maxwellian and tau of the new
        // state are those of the transported state, and U_new = (U_t + h U_eq) / (1 + h),
        // h = dt / tau
        double Wt[NV], We[NV], Ue[NV];
        SYS::cons_to_prim(Un, Wt);
        const double rho = Wt[0];
        const double T = SYS::pressure(Wt) / rho;
        const double tau = (p.tau_mode == 0) ? p.tau_ref * (p.rho_ref / rho) * sqrt(p.T_ref / T) : p.tau_ref;
        const double h = (p.cdt * dt) / tau;
        const double w = 1.0 / (1.0 + h);
        SYS::equilibrium(Wt, We);
        SYS::prim_to_cons(We, Ue);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          Un[v] = (Un[v] + h * Ue[v]) * w;
          p.Uout[SYS::plane_of(v) * p.plane + off] = Un[v];
        }
      }
      bool fin = true;
#pragma unroll
      for (int v = 0; v < NV; ++v) fin = fin && isfinite(Un[v]);
      if (!fin) {
        flag |= ST_NONFINITE;
      } else if (p.do_cfl) {
        // the last stage of a step: the new state's primitives also give its CFL rate
        double Wn[NV];
        SYS::cons_to_prim(Un, Wn);
        if (!SYS::admissible(Wn)) flag |= ST_UNREALIZABLE;
        else if constexpr (DIM == 1) rate = SYS::template cell_lambda<0>(Wn, p.sigma_lim, p.kws);
        else rate = SYS::cell_rate2d(Wn, p.sigma_lim, p.kws, p.dx, p.dy);
      } else if (!SYS::admissible_cons(Un)) {
        flag |= ST_UNREALIZABLE;
      }
    }
  }
  // block reductions: status, fallback count, CFL rate
  flag = wave_or(flag);
  nfb = wave_sum(nfb);
  if constexpr (PREC == 1) n64 = wave_sum(n64);
  nstates = wave_sum(nstates);
  const int lane = t & 63, wid = t >> 6;
  if (lane == 0) {
    if (flag) atomicOr(&sFlag[0], flag);
    if (nfb) atomicAdd(&sFlag[1], nfb);
    if (PREC == 1 && n64) atomicAdd(&sFlag[2], n64);
  }
  if (p.do_cfl) {
    rate = wave_max(rate);
    if (lane == 0) sRed[wid] = rate;
  }
  __syncthreads();
  if (t == 0) {
    if (sFlag[0]) {
      atomicOr(&p.ctrl->status, sFlag[0]);
      atomicMin(&p.ctrl->fail_step, (int)p.ctrl->step);
    }
    if (sFlag[1]) atomicAdd((unsigned long long*)&p.ctrl->n_fallback, (unsigned long long)sFlag[1]);
    if (PREC != 0) {
      if (sFlag[2]) atomicAdd((unsigned long long*)&p.ctrl->n_fp64, (unsigned long long)sFlag[2]);
      atomicAdd((unsigned long long*)&p.ctrl->n_states,
                (unsigned long long)(2 * (NFX + NFY)));
    }
    if (p.do_cfl) {
      double m = sRed[0];
      for (int k = 1; k < NT / 64; ++k) m = fmax(m, sRed[k]);
      atomicMax(&p.ctrl->maxrate, (unsigned long long)__double_as_longlong(m));
    }
  }
}

// ------------------------------------------------------------------ CFL rate of a state
template <class SYS, int DIM>
__global__ __launch_bounds__(256) void cfl_kernel(CflParams p) {
  constexpr int NV = SYS::NV;
  __shared__ double sRed[4];
  long long n = (long long)p.nx * p.ny;
  double rate = 0.0;
  for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < n; c += (long long)gridDim.x * 256) {
    int i = (int)(c % p.nx), j = (int)(c / p.nx);
    long long off = (long long)j * p.pitch + i;
    double U[NV], W[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = p.U[v * p.plane + off];
    SYS::cons_to_prim(U, W);
    double r;
    if constexpr (DIM == 1) r = SYS::template cell_lambda<0>(W, p.sigma_lim, p.kws);
    else
      r = SYS::cell_rate2d(W, p.sigma_lim, p.kws, p.dx, p.dy);
    rate = fmax(rate, r);
  }
  rate = wave_max(rate);
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = rate;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
    atomicMax(&p.ctrl->maxrate, (unsigned long long)__double_as_longlong(m));
  }
}

// ------------------------------------------------------------------ time control
__global__ void finalize_kernel(DevCtrl* c, int dim, double cfl, double dx) {
  if (threadIdx.x != 0) return;
  double dt = 0.0;
  if (c->status == 0) {
    if (c->dt_fixed > 0.0) {
      dt = c->dt_fixed;
    } else {
      double m = __longlong_as_double((long long)c->maxrate);
      dt = (dim == 1) ? cfl * dx / m : cfl / m;
      if (!(m > 0.0)) dt = 0.0;
    }
    if (c->t_end > 0.0) {
      if (c->t >= c->t_end * (1.0 - 1e-14)) dt = 0.0;
      else dt = fmin(dt, c->t_end - c->t);
    }
  }
  c->dt = dt;
  c->maxrate = 0ull;
  if (dt > 0.0) {
    c->t += dt;
    c->step += 1;
    c->dt_last = dt;
  }
}

__global__ void ctrl_set_kernel(DevCtrl* c, double dt_fixed, double t_end) {
  if (threadIdx.x == 0) {
    c->dt_fixed = dt_fixed;
    c->t_end = t_end;
  }
}

__global__ void ctrl_reset_kernel(DevCtrl* c, double t0) {
  if (threadIdx.x == 0) {
    c->dt = 0.0; c->t = t0; c->t_end = 0.0; c->dt_fixed = 0.0; c->dt_last = 0.0;
    c->maxrate = 0ull; c->step = 0; c->n_fallback = 0; c->status = 0; c->fail_step = 0x7fffffff;
    c->n_fp64 = 0; c->n_states = 0; c->n_sigma_limited = 0; c->asym = 0;
  }
}

// zero the planes no reduced kernel writes (u_y, u_z, P_xy, P_xz, P_yz, q_y, q_z) of a
// 14-moment field
__global__ __launch_bounds__(256) void zero_planes_kernel(double* U, long long plane) {
  const long long n = 7 * plane;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
    const int w = (int)(k / plane);
    const long long o = k - w * plane;
    const int v = w == 0 ? 2 : (w == 1 ? 3 : (w == 2 ? 5 : (w == 3 ? 6 : (w == 4 ? 8 : (w == 5 ? 11 : 12)))));
    U[v * plane + o] = 0.0;
  }
}

// ------------------------------------------------------------------ state in / out
template <class SYS>
__global__ void ingest_kernel(int repr, const double* src, double* U, int nx, int ny, int pitch,
                              DevCtrl* c) {
  constexpr int NV = SYS::NV;
  long long n = (long long)nx * ny;
  long long plane = (long long)ny * pitch;
  int bad = 0, np = 0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    int i = (int)(k % nx), j = (int)(k / nx);
    double A[NV], Uc[NV], W[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) A[v] = src[v * n + k];
    if (repr == 0) {
      SYS::prim_to_cons(A, Uc);
#pragma unroll
      for (int v = 0; v < NV; ++v) W[v] = A[v];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Uc[v] = A[v];
      SYS::cons_to_prim(Uc, W);
    }
    bool fin = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      fin = fin && isfinite(Uc[v]);
      U[v * plane + (long long)j * pitch + i] = Uc[v];
    }
    if (!fin) bad |= ST_NONFINITE;
    else if (!SYS::admissible(W)) bad |= ST_UNREALIZABLE;
    // symmetry (14 moments): z-odd moments u_z, P_xz, P_yz, q_z and y-odd moments u_y, P_xy,
    // P_yz, q_y exactly zero
    if constexpr (NV == 14) {
      if (Uc[3] != 0.0 || Uc[6] != 0.0 || Uc[8] != 0.0 || Uc[12] != 0.0) np |= ASYM_Z;
      if (Uc[2] != 0.0 || Uc[5] != 0.0 || Uc[8] != 0.0 || Uc[11] != 0.0) np |= ASYM_Y;
    }
  }
  bad = wave_or(bad);
  if ((threadIdx.x & 63) == 0 && bad) atomicOr(&c->status, bad);
  if constexpr (NV == 14) {
    np = wave_or(np);
    if ((threadIdx.x & 63) == 0 && np) atomicOr(&c->asym, np);
  }
}

// Closing moments of a cell state (dimensional, at sigma_bar = max(sigma, sigma_lim)):
// 14 moments: Q_ijk (10: xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz), R_ijkk (6: xx xy xz yy yz zz),
// S_ijjkk (3: x y z); 5 moments: s.
constexpr int NCLOSE14 = 19;

MX_HD void closing14(const double* W, double sigma_lim, double* out) {
  Sys14::Core<double> k;
  Sys14::core(W, sigma_lim, k);
  double Q[6], R[3], S;
  Sys14::closure_dir<0>(k, Q, R, S);   // Q_ijx: xxx xyx xzx yyx yzx zzx
  out[0] = Q[0]; out[1] = Q[1]; out[2] = Q[2]; out[3] = Q[3]; out[4] = Q[4]; out[5] = Q[5];
  out[10] = R[0]; out[11] = R[1]; out[12] = R[2];
  out[16] = S;
  Sys14::closure_dir<1>(k, Q, R, S);   // Q_ijy: ... yyy yzy zzy
  out[6] = Q[3]; out[7] = Q[4]; out[8] = Q[5];
  out[13] = R[1]; out[14] = R[2];
  out[17] = S;
  Sys14::closure_dir<2>(k, Q, R, S);   // Q_zzz
  out[9] = Q[5];
  out[15] = R[2];
  out[18] = S;
}

template <class SYS>
__global__ void egress_kernel(int repr, const double* U, double* dst, int nx, int ny, int pitch,
                              double sigma_lim) {
  constexpr int NV = SYS::NV;
  long long n = (long long)nx * ny;
  long long plane = (long long)ny * pitch;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    int i = (int)(k % nx), j = (int)(k / nx);
    double Uc[NV], W[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Uc[v] = U[v * plane + (long long)j * pitch + i];
    if (repr == 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v) dst[v * n + k] = Uc[v];
    } else {
      SYS::cons_to_prim(Uc, W);
      if (repr == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[v * n + k] = W[v];
      } else if (repr == 2) {
        dst[k] = SYS::sigma(W);
      } else if constexpr (NV == 14) {
        double c[NCLOSE14];
        closing14(W, sigma_lim, c);
#pragma unroll
        for (int m = 0; m < NCLOSE14; ++m) dst[m * n + k] = c[m];
      } else {
        typename SYS::template Core<double> kc;
        SYS::core(W, sigma_lim, kc);
        dst[k] = SYS::closing_s(kc);
      }
    }
  }
}

// cells of a state whose unlimited sigma is below sigma_lim (the closure evaluates them at
// sigma_bar = sigma_lim), added to ctrl->n_sigma_limited
template <class SYS>
__global__ __launch_bounds__(256) void count_sigma_limited_kernel(const double* U, int nx, int ny,
                                                                  int pitch, double sigma_lim,
                                                                  DevCtrl* c) {
  constexpr int NV = SYS::NV;
  long long n = (long long)nx * ny;
  long long plane = (long long)ny * pitch;
  int cnt = 0;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
    int i = (int)(k % nx), j = (int)(k / nx);
    double Uc[NV], W[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Uc[v] = U[v * plane + (long long)j * pitch + i];
    SYS::cons_to_prim(Uc, W);
    cnt += (SYS::sigma(W) < sigma_lim) ? 1 : 0;
  }
  cnt = wave_sum(cnt);
  if ((threadIdx.x & 63) == 0 && cnt)
    atomicAdd((unsigned long long*)&c->n_sigma_limited, (unsigned long long)cnt);
}

// ------------------------------------------------------------------ launchers
template <class SYS, int DIM, int ORDER, int PREC>
static hipError_t launch_stage_t(const StageParams& p, hipStream_t s) {
  int grid = ((p.nblk + 7) / 8) * 8;
  if constexpr (DIM == 2) {
    hipLaunchKernelGGL((stage_kernel<SYS, DIM, ORDER, PREC, 16, 15, 256>), dim3(grid), dim3(256), 0, s, p);
  } else {
    hipLaunchKernelGGL((stage_kernel<SYS, DIM, ORDER, PREC, tile_1d(64), 1, 64>), dim3(grid), dim3(64), 0, s, p);
  }
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_stage_p(int system, int dim, int order, bool reduced, const StageParams& p,
                                 hipStream_t s) {
  if (system == 5) {
    if (dim != 1) return hipErrorInvalidValue;
    return order == 2 ? launch_stage_t<Sys5, 1, 2, PREC>(p, s) : launch_stage_t<Sys5, 1, 1, PREC>(p, s);
  }
  if (dim == 1) {
    if (reduced)
      return order == 2 ? launch_stage_t<Sys14A, 1, 2, PREC>(p, s) : launch_stage_t<Sys14A, 1, 1, PREC>(p, s);
    return order == 2 ? launch_stage_t<Sys14, 1, 2, PREC>(p, s) : launch_stage_t<Sys14, 1, 1, PREC>(p, s);
  }
  if (reduced)
    return order == 2 ? launch_stage_t<Sys14P, 2, 2, PREC>(p, s) : launch_stage_t<Sys14P, 2, 1, PREC>(p, s);
  return order == 2 ? launch_stage_t<Sys14, 2, 2, PREC>(p, s) : launch_stage_t<Sys14, 2, 1, PREC>(p, s);
}

hipError_t launch_stage(int system, int dim, int order, int precision, bool reduced,
                        const StageParams& p, hipStream_t s) {
  if (precision == 1) return launch_stage_p<1>(system, dim, order, reduced, p, s);
  if (precision == 2) return launch_stage_p<2>(system, dim, order, reduced, p, s);
  return launch_stage_p<0>(system, dim, order, reduced, p, s);
}

hipError_t launch_cfl(int system, int dim, const CflParams& p, hipStream_t s) {
  long long n = (long long)p.nx * p.ny;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (system == 5) hipLaunchKernelGGL((cfl_kernel<Sys5, 1>), dim3(grid), dim3(256), 0, s, p);
  else if (dim == 1) hipLaunchKernelGGL((cfl_kernel<Sys14, 1>), dim3(grid), dim3(256), 0, s, p);
  else hipLaunchKernelGGL((cfl_kernel<Sys14, 2>), dim3(grid), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_finalize(DevCtrl* c, int dim, double cfl, double dx, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, c, dim, cfl, dx);
  return hipGetLastError();
}

hipError_t launch_ctrl_set(DevCtrl* c, double dt_fixed, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(ctrl_set_kernel, dim3(1), dim3(64), 0, s, c, dt_fixed, t_end);
  return hipGetLastError();
}

hipError_t launch_ctrl_reset(DevCtrl* c, double t0, hipStream_t s) {
  hipLaunchKernelGGL(ctrl_reset_kernel, dim3(1), dim3(64), 0, s, c, t0);
  return hipGetLastError();
}

hipError_t launch_zero_planes(double* U, long long plane, int nv, hipStream_t s) {
  if (nv != 14) return hipSuccess;
  long long n = 7 * plane;
  int grid = (int)((n + 255) / 256);
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(zero_planes_kernel, dim3(grid), dim3(256), 0, s, U, plane);
  return hipGetLastError();
}

hipError_t launch_ingest(int system, int repr, const double* src, double* U, int nx, int ny,
                         int pitch, DevCtrl* c, hipStream_t s) {
  long long n = (long long)nx * ny;
  int grid = (int)((n + 255) / 256);
  if (grid > 8192) grid = 8192;
  if (system == 5) hipLaunchKernelGGL((ingest_kernel<Sys5>), dim3(grid), dim3(256), 0, s, repr, src, U, nx, ny, pitch, c);
  else hipLaunchKernelGGL((ingest_kernel<Sys14>), dim3(grid), dim3(256), 0, s, repr, src, U, nx, ny, pitch, c);
  return hipGetLastError();
}

hipError_t launch_egress(int system, int repr, const double* U, double* dst, int nx, int ny,
                         int pitch, double sigma_lim, hipStream_t s) {
  long long n = (long long)nx * ny;
  int grid = (int)((n + 255) / 256);
  if (grid > 8192) grid = 8192;
  if (system == 5)
    hipLaunchKernelGGL((egress_kernel<Sys5>), dim3(grid), dim3(256), 0, s, repr, U, dst, nx, ny, pitch, sigma_lim);
  else
    hipLaunchKernelGGL((egress_kernel<Sys14>), dim3(grid), dim3(256), 0, s, repr, U, dst, nx, ny, pitch, sigma_lim);
  return hipGetLastError();
}

hipError_t launch_count_sigma_limited(int system, const double* U, int nx, int ny, int pitch,
                                      double sigma_lim, DevCtrl* c, hipStream_t s) {
  long long n = (long long)nx * ny;
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  if (system == 5)
    hipLaunchKernelGGL((count_sigma_limited_kernel<Sys5>), dim3(grid), dim3(256), 0, s, U, nx, ny, pitch, sigma_lim, c);
  else
    hipLaunchKernelGGL((count_sigma_limited_kernel<Sys14>), dim3(grid), dim3(256), 0, s, U, nx, ny, pitch, sigma_lim, c);
  return hipGetLastError();
}

}  // namespace mx

// gfx950 kernels of the discrete adjoint of one stage of the 14-moment finite-volume step.
//
// The forward stage is  Uout = a Ua + beta Ub + mu_coef dt L(Ub)  with
//   L_c = -(F_{c+1/2} - F_{c-1/2}) / dx - (G_{c+1/2} - G_{c-1/2}) / dy + C(W_c)
// (Section 3: HLL / Rusanov interface fluxes of MUSCL face states built with the common
// limiter, BGK source at the cell centre, ghost cells from the boundary conditions).
// Its reverse runs in three deterministic gather passes plus a reduction:
//   1. faces (adj_face_kernel, per direction): rebuild the two face states of every face from
//      the stage input, take the flux adjoint Fb = (mu_right - mu_left) / dx from the two
//      adjacent cells (mu = mu_coef dt lam_out, zero in ghost cells) and reverse the interface
//      flux, closure, wave speeds and conserved map of both face states (branch replayed);
//      store the two face-state adjoints;
//   2. extended cells (adj_cell_kernel): for every cell of the domain and its two ghost
//      layers, gather the reverse of the limited reconstruction of the up to three stencil
//      cells whose face states it feeds (limiter argmin, regime and fallback replayed);
//   3. interior cells (adj_update_kernel): fold the ghost-cell adjoints back onto the cells
//      they copy (transmissive, periodic, reflective with sign flips) or onto the jet
//      parameters, add the reverse of the BGK source (and its tau_ref partial), map the
//      primitive adjoint back to conserved variables and combine with beta lam_out and the
//      later stage's contribution;
//   4. adj_reduce_kernel: sum the per-workgroup parameter partials in a fixed order.
// No atomics: the result is bitwise reproducible.
#include "mx_internal.hpp"
#include "mx_physics.hpp"
#include "mx_scheme.hpp"
#include "mx_bc.hpp"
#include "mx_adjoint.hpp"

namespace mx {

constexpr int ADJ_NT = 256;

__device__ __forceinline__ long long ucell(const StageParams& p, int i, int j) {
  return (long long)j * p.pitch + i;
}

// common limiter factor of the cell with stencil (Wm, Wc, Wp), as the forward stage computes it
__device__ __forceinline__ double forward_phi(const StageParams& p, const double* Wm, const double* Wc,
                                              const double* Wp) {
  double phi = limiter_factor<Sys14>(Wm, Wc, Wp, p.limiter);
  if (p.fallback && phi > 0.0) {
    double Wf[14];
    face_state<Sys14>(Wm, Wc, Wp, phi, 1.0, Wf);
    bool ok = Sys14::admissible(Wf);
    face_state<Sys14>(Wm, Wc, Wp, phi, -1.0, Wf);
    ok = ok && Sys14::admissible(Wf);
    if (!ok) phi = 0.0;
  }
  return phi;
}

// load the primitive state of (possibly ghost) cell c along direction D of line l
template <int D>
__device__ __forceinline__ void line_prims(const StageParams& p, int c, int l, double* W) {
  if (D == 0) load_prims<Sys14>(p, p.Ub, c, l, W);
  else load_prims<Sys14>(p, p.Ub, l, c, W);
}

// ------------------------------------------------------------------ 1. faces
template <int D, int ORDER>
__global__ __launch_bounds__(ADJ_NT) void adj_face_kernel(AdjParams a) {
  const StageParams& p = a.sp;
  const int n = (D == 0) ? p.nx : p.ny;           // cells along D
  const int m = (D == 0) ? p.ny : p.nx;           // lines
  const long long nf = (long long)(n + 1) * m;
  const long long f = (long long)blockIdx.x * ADJ_NT + threadIdx.x;
  if (f >= nf) return;
  int fc, l;                                       // face fc lies between cells fc-1 and fc
  if (D == 0) { fc = (int)(f % (n + 1)); l = (int)(f / (n + 1)); }
  else { fc = (int)(f / m); l = (int)(f % m); }
  double* out = (D == 0) ? a.fbx : a.fby;
  const long long nfs = (D == 0) ? a.nfx : a.nfy;
  const double inv_h = (D == 0) ? p.inv_dx : p.inv_dy;
  const double mc = a.mu_coef * a.dt;

  // flux adjoint from the two adjacent interior cells
  double Fb[14];
  bool any = false;
  {
    long long cl = (D == 0) ? ucell(p, fc - 1, l) : ucell(p, l, fc - 1);
    long long cr = (D == 0) ? ucell(p, fc, l) : ucell(p, l, fc);
    bool hl = fc - 1 >= 0, hr = fc < n;
#pragma unroll
    for (int v = 0; v < 14; ++v) {
      double ml = hl ? mc * a.lam_out[v * p.plane + cl] : 0.0;
      double mr = hr ? mc * a.lam_out[v * p.plane + cr] : 0.0;
      Fb[v] = (mr - ml) * inv_h;
      any = any || (Fb[v] != 0.0);
    }
  }
  double WLb[14], WRb[14];
#pragma unroll
  for (int v = 0; v < 14; ++v) { WLb[v] = 0.0; WRb[v] = 0.0; }
  if (any) {
    double WL[14], WR[14];
    if constexpr (ORDER == 2) {
      double A[14], B[14], C[14], E[14];
      line_prims<D>(p, fc - 2, l, A);
      line_prims<D>(p, fc - 1, l, B);
      line_prims<D>(p, fc, l, C);
      line_prims<D>(p, fc + 1, l, E);
      face_state<Sys14>(A, B, C, forward_phi(p, A, B, C), 1.0, WL);
      face_state<Sys14>(B, C, E, forward_phi(p, B, C, E), -1.0, WR);
    } else {
      line_prims<D>(p, fc - 1, l, WL);
      line_prims<D>(p, fc, l, WR);
    }
    Adj14::face_flux_vjp<D>(WL, WR, p.sigma_lim, p.kws, p.flux, Fb, WLb, WRb);
  }
  // face index in the stored layout: x faces row-major (fc fastest), y faces fc-major
  const long long fo = (D == 0) ? (long long)l * (n + 1) + fc : (long long)fc * m + l;
#pragma unroll
  for (int v = 0; v < 14; ++v) {
    out[v * nfs + fo] = WLb[v];
    out[(14 + v) * nfs + fo] = WRb[v];
  }
}

// ------------------------------------------------------------------ 2. extended cells
// adjoint of the primitive state of cell c (line l, direction D) through the reconstruction
// of the stencil cells c-1, c, c+1
template <int D, int ORDER>
__device__ __forceinline__ void gather_line(const AdjParams& a, int c, int l, double* Wb) {
  const StageParams& p = a.sp;
  const int n = (D == 0) ? p.nx : p.ny;
  const int m = (D == 0) ? p.ny : p.nx;
  const double* fb = (D == 0) ? a.fbx : a.fby;
  const long long nfs = (D == 0) ? a.nfx : a.nfy;
  auto fidx = [&](int fc) -> long long {
    return (D == 0) ? (long long)l * (n + 1) + fc : (long long)fc * m + l;
  };
  if constexpr (ORDER == 1) {
    // face states are the cell states: cell c feeds face c (as its right state) and face c+1
    // (as its left state)
    if (c >= 0 && c <= n) {
#pragma unroll
      for (int v = 0; v < 14; ++v) Wb[v] += fb[(14 + v) * nfs + fidx(c)];
    }
    if (c + 1 >= 0 && c + 1 <= n) {
#pragma unroll
      for (int v = 0; v < 14; ++v) Wb[v] += fb[v * nfs + fidx(c + 1)];
    }
  } else {
    // stencil cells k = c-1, c, c+1 with face states (k in [-1, n]); their stencils span
    // cells c-2 .. c+2
    double S[5][14];
#pragma unroll
    for (int q = 0; q < 5; ++q) line_prims<D>(p, c - 2 + q, l, S[q]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int k = c - 1 + r;
      if (k < -1 || k > n) continue;
      double Op[14], Om[14];
      bool any = false;
#pragma unroll
      for (int v = 0; v < 14; ++v) {
        Op[v] = (k + 1 <= n) ? fb[v * nfs + fidx(k + 1)] : 0.0;        // upper face: its WL
        Om[v] = (k >= 0) ? fb[(14 + v) * nfs + fidx(k)] : 0.0;         // lower face: its WR
        any = any || Op[v] != 0.0 || Om[v] != 0.0;
      }
      if (!any) continue;
      int vstar;
      double phi = Adj14::limiter_select(S[r], S[r + 1], S[r + 2], p.limiter, p.fallback, vstar);
      // cell c is the stencil's Wp (r = 0), Wc (r = 1) or Wm (r = 2)
      Adj14::recon_vjp_role(2 - r, S[r], S[r + 1], S[r + 2], phi, vstar, p.limiter, Op, Om, Wb);
    }
  }
}

template <int DIM, int ORDER>
__global__ __launch_bounds__(ADJ_NT) void adj_cell_kernel(AdjParams a) {
  const StageParams& p = a.sp;
  const long long e = (long long)blockIdx.x * ADJ_NT + threadIdx.x;
  if (e >= a.eplane) return;
  const int ei = (int)(e % a.epitch);
  const int ej = (int)(e / a.epitch);
  const int i = ei - 2;
  const int j = (DIM == 2) ? ej - 2 : 0;
  double Wb[14];
#pragma unroll
  for (int v = 0; v < 14; ++v) Wb[v] = 0.0;
  const bool in_i = i >= 0 && i < p.nx, in_j = j >= 0 && j < p.ny;
  if (in_j) gather_line<0, ORDER>(a, i, j, Wb);
  if (DIM == 2 && in_i) gather_line<1, ORDER>(a, j, i, Wb);
#pragma unroll
  for (int v = 0; v < 14; ++v) a.wb[v * a.eplane + e] = Wb[v];
}

// ------------------------------------------------------------------ 3. interior cells
template <int DIM>
__global__ __launch_bounds__(ADJ_NT) void adj_update_kernel(AdjParams a) {
  const StageParams& p = a.sp;
  __shared__ double sRed[3][ADJ_NT / 64];
  const long long ncell = (long long)p.nx * p.ny;
  const long long k = (long long)blockIdx.x * ADJ_NT + threadIdx.x;
  double gM = 0.0, gR = 0.0, gT = 0.0;
  if (k < ncell) {
    const int i = (int)(k % p.nx), j = (int)(k / p.nx);
    const int ej = (DIM == 2) ? j + 2 : 0;
    auto ext = [&](int ii, int jj) -> long long {
      return (long long)((DIM == 2) ? jj + 2 : 0) * a.epitch + (ii + 2);
    };
    double Wb[14];
    const long long e = (long long)ej * a.epitch + (i + 2);
#pragma unroll
    for (int v = 0; v < 14; ++v) Wb[v] = a.wb[v * a.eplane + e];
    // ghost cells along x in this row that copy cell (i, j)
    const int jet = (p.bc[0] == 3) ? jet_of_row(p, j) : -1;
    const int gx[4] = {-2, -1, p.nx, p.nx + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int g = gx[q];
      int rx = 0;
      const int si = map_axis(g, p.nx, p.bc[0], p.bc[1], rx);
      if (si != i) continue;
      const long long eg = ext(g, j);
      if (g < 0 && jet >= 0) {
        // the ghost holds the jet state: its adjoint goes to the jet parameters
        double sn, cs;
        sincospi(p.jet_ang[jet] / 180.0, &sn, &cs);
        const double T = p.jet_T;
        const double c0 = sqrt(5.0 / 3.0 * T);
        double G[14];
#pragma unroll
        for (int v = 0; v < 14; ++v) G[v] = a.wb[v * a.eplane + eg];
        gM += (G[1] * cs + G[2] * sn) * c0;
        gR += G[0] + T * (G[4] + G[7] + G[9]) + 15.0 * T * T * G[13];
        continue;
      }
#pragma unroll
      for (int v = 0; v < 14; ++v) {
        double gv = a.wb[v * a.eplane + eg];
        Wb[v] += (rx && Sys14::odd(v, 0)) ? -gv : gv;
      }
    }
    if constexpr (DIM == 2) {
      const int gy[4] = {-2, -1, p.ny, p.ny + 1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int g = gy[q];
        int ry = 0;
        const int sj = map_axis(g, p.ny, p.bc[2], p.bc[3], ry);
        if (sj != j) continue;
        const long long eg = ext(i, g);
#pragma unroll
        for (int v = 0; v < 14; ++v) {
          double gv = a.wb[v * a.eplane + eg];
          Wb[v] += (ry && Sys14::odd(v, 1)) ? -gv : gv;
        }
      }
    }
    const long long off = ucell(p, i, j);
    double U[14], lo[14];
#pragma unroll
    for (int v = 0; v < 14; ++v) {
      U[v] = p.Ub[v * p.plane + off];
      lo[v] = a.lam_out[v * p.plane + off];
    }
    if (p.use_source) {
      double W[14];
      Sys14::cons_to_prim(U, W);
      const double rho = W[0];
      const double T = Sys14::pressure(W) / rho;
      const double tau = (p.tau_mode == 0) ? p.tau_ref * (p.rho_ref / rho) * sqrt(p.T_ref / T) : p.tau_ref;
      double mu[14];
      const double mc = a.mu_coef * a.dt;
#pragma unroll
      for (int v = 0; v < 14; ++v) mu[v] = mc * lo[v];
      const double cdot = Adj14::source_vjp(W, 1.0 / tau, p.tau_mode == 0, mu, Wb);
      gT -= cdot / p.tau_ref;
    }
    double Ubar[14];
#pragma unroll
    for (int v = 0; v < 14; ++v) Ubar[v] = 0.0;
    Adj14::cons_to_prim_vjp(U, Wb, Ubar);
#pragma unroll
    for (int v = 0; v < 14; ++v) {
      double r = a.beta * lo[v] + Ubar[v];
      if (a.lam_extra) r += a.extra_coef * a.lam_extra[v * p.plane + off];
      a.lam_in[v * p.plane + off] = r;
    }
  }
  // workgroup partial sums in a fixed order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    gM += __shfl_xor(gM, o, 64);
    gR += __shfl_xor(gR, o, 64);
    gT += __shfl_xor(gT, o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { sRed[0][wid] = gM; sRed[1][wid] = gR; sRed[2][wid] = gT; }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int w = 0; w < ADJ_NT / 64; ++w) s += sRed[threadIdx.x][w];
    a.part[threadIdx.x * a.n_upd_blocks + blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ 4. parameter partials
__global__ __launch_bounds__(ADJ_NT) void adj_reduce_kernel(const double* part, int nb, double* grad) {
  __shared__ double sRed[ADJ_NT / 64];
  for (int m = 0; m < 3; ++m) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += ADJ_NT) s += part[m * nb + b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < ADJ_NT / 64; ++w) t += sRed[w];
      grad[m] += t;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ tape helpers
__global__ void tape_dt_kernel(const DevCtrl* c, double* slot) {
  if (threadIdx.x == 0) *slot = c->dt;
}

__global__ void set_dt_kernel(DevCtrl* c, double dt) {
  if (threadIdx.x == 0) {
    c->dt = dt;
    c->status = 0;
  }
}

__global__ void pad_copy_kernel(const double* src, double* dst, int nv, int nx, int ny, int pitch,
                                int to_padded) {
  const long long n = (long long)nx * ny;
  const long long plane = (long long)ny * pitch;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n * nv;
       k += (long long)gridDim.x * blockDim.x) {
    const long long v = k / n, c = k % n;
    const long long i = c % nx, j = c / nx;
    const long long pk = v * plane + j * pitch + i;
    if (to_padded) dst[pk] = src[k];
    else dst[k] = src[pk];
  }
}

// ------------------------------------------------------------------ launchers
int adjoint_update_blocks(int nx, int ny) {
  return (int)(((long long)nx * ny + ADJ_NT - 1) / ADJ_NT);
}

template <int DIM, int ORDER>
static hipError_t launch_adj_t(AdjParams& a, hipStream_t s) {
  const StageParams& p = a.sp;
  int gx = (int)((a.nfx + ADJ_NT - 1) / ADJ_NT);
  hipLaunchKernelGGL((adj_face_kernel<0, ORDER>), dim3(gx), dim3(ADJ_NT), 0, s, a);
  if constexpr (DIM == 2) {
    int gy = (int)((a.nfy + ADJ_NT - 1) / ADJ_NT);
    hipLaunchKernelGGL((adj_face_kernel<1, ORDER>), dim3(gy), dim3(ADJ_NT), 0, s, a);
  }
  int ge = (int)((a.eplane + ADJ_NT - 1) / ADJ_NT);
  hipLaunchKernelGGL((adj_cell_kernel<DIM, ORDER>), dim3(ge), dim3(ADJ_NT), 0, s, a);
  hipLaunchKernelGGL((adj_update_kernel<DIM>), dim3(a.n_upd_blocks), dim3(ADJ_NT), 0, s, a);
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(1), dim3(ADJ_NT), 0, s, a.part, a.n_upd_blocks, a.grad);
  (void)p;
  return hipGetLastError();
}

hipError_t launch_adjoint_stage(int dim, int order, AdjParams& a, hipStream_t s) {
  if (dim == 2) return order == 2 ? launch_adj_t<2, 2>(a, s) : launch_adj_t<2, 1>(a, s);
  return order == 2 ? launch_adj_t<1, 2>(a, s) : launch_adj_t<1, 1>(a, s);
}

hipError_t launch_tape_dt(const DevCtrl* c, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(tape_dt_kernel, dim3(1), dim3(64), 0, s, c, slot);
  return hipGetLastError();
}

hipError_t launch_set_dt(DevCtrl* c, double dt, hipStream_t s) {
  hipLaunchKernelGGL(set_dt_kernel, dim3(1), dim3(64), 0, s, c, dt);
  return hipGetLastError();
}

hipError_t launch_pad_copy(const double* src, double* dst, int nv, int nx, int ny, int pitch,
                           int to_padded, hipStream_t s) {
  long long n = (long long)nx * ny * nv;
  int grid = (int)((n + 255) / 256);
  if (grid > 8192) grid = 8192;
  hipLaunchKernelGGL(pad_copy_kernel, dim3(grid), dim3(256), 0, s, src, dst, nv, nx, ny, pitch, to_padded);
  return hipGetLastError();
}

}  // namespace mx

// gfx950 kernels of the discrete adjoint of one stage of the 14-moment finite-volume step.
//
// The forward stage is  Uout = a Ua + beta Ub + mu_coef dt L(Ub)  with
//   L_c = -(F_{c+1/2} - F_{c-1/2}) / dx - (G_{c+1/2} - G_{c-1/2}) / dy + C(W_c)
// (Section 3: HLL / Rusanov interface fluxes of MUSCL face states built with the common
// limiter, BGK source at the cell centre, ghost cells from the boundary conditions).
// Its reverse runs as deterministic gather passes plus a reduction:
//   0. prep (adj_prep_kernel, LDS tiles): primitives of every cell of the domain and its two
//      ghost layers, and each cell's common limiter factor and the variable that selected it,
//      per direction (the forward stage's values, bit for bit);
//   1. faces, both directions in one launch (adj_face_kernel, two threads per face, one per
//      face state):
//      each thread takes the flux adjoint Fb = (mu_right - mu_left) / dx from the two
//      adjacent cells (mu = mu_coef dt lam_out, zero in ghost cells), rebuilds its face state
//      and evaluates its closure (kept for the reverse), wave speeds, flux and conserved
//      state; the two threads exchange their wave speeds and the products Fb . F, Fb . U
//      (lane shuffles), which is all the reverse of the HLL / Rusanov combination (branch
//      replayed) needs besides the thread's own side; then each thread reverses closure, wave
//      speeds, physical flux and conserved map of its own face state;
//   2. extended cells (adj_cell_kernel): for every cell of the domain and its two ghost
//      layers, gather the reverse of the limited reconstruction of the up to three stencil
//      cells whose face states it feeds (limiter argmin, regime and fallback replayed);
//   3. interior cells (adj_update_kernel): fold the ghost-cell adjoints back onto the cells
//      they copy (transmissive, periodic, reflective with sign flips) or onto the jet
//      parameters, add the reverse of the BGK source (and its tau_ref partial), map the
//      primitive adjoint back to conserved variables and combine with beta lam_out and the
//      later stage's contribution;
//   4. adj_reduce_kernel: sum the per-workgroup parameter partials in a fixed order.
// No atomics: the result is bitwise reproducible.  Faces whose flux adjoint is exactly zero
// (outside the adjoint's domain of dependence) skip the closure reverse.
//
// Planar runs (template flag PL): when the recorded states are planar-symmetric (u_z = P_xz
// = P_yz = q_z = 0) and so is dJ/dU, the adjoint's z-odd components stay exactly zero too
// (at a planar state the step's Jacobian does not couple z-even and z-odd moments), so the
// kernels read those four components as the constant 0 and never store them.  The file is
// compiled without signed zeros, NaN or infinity (these runs have none), which lets the
// compiler drop every product with such a constant: the same reverse code on ten moments.
#include "mx_internal.hpp"
#include "mx_adjoint_params.hpp"
#include "mx_physics.hpp"
#include "mx_scheme.hpp"
#include "mx_bc.hpp"
#include "mx_planar.hpp"
#include "mx_adjoint.hpp"

namespace mx {

constexpr int ADJ_NT = 256;
// the face reverse runs one wavefront per workgroup: a finished wavefront's slot takes the next
// one at once (a workgroup of four has to wait for four free slots on one CU); at two
// wavefronts per SIMD this made the 512^2 adjoint 4 % faster than 256-thread workgroups
constexpr int FACE_NT = 64;

// XCD-aware block order: the hardware deals consecutive workgroups round-robin to the 8 XCDs;
// give each XCD a contiguous range of blocks so that the neighbour data these gathers re-read
// stays in that XCD's L2
__device__ __forceinline__ long long xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned per = (nb + 7) / 8;
  const unsigned full = nb % 8 == 0 ? 8 : nb % 8;   // XCDs that receive `per` blocks
  const unsigned x = b % 8, k = b / 8;
  // blocks of XCD x in dealing order get the contiguous range starting at its offset
  const unsigned off = (x < full) ? x * per : full * per + (x - full) * (per - 1);
  return (long long)(off + k);
}

__device__ __forceinline__ long long ucell(const StageParams& p, int i, int j) {
  return (long long)j * p.pitch + i;
}

// extended-cell index of cell c of line l along direction D
template <int D, int DIM>
__device__ __forceinline__ long long ext_idx(const AdjParams& a, int c, int l) {
  if (D == 0) return (long long)((DIM == 2) ? l + 2 : 0) * a.epitch + (c + 2);
  return (long long)(c + 2) * a.epitch + (l + 2);
}

// the z-odd moments of the 14-moment state (u_z, P_xz, P_yz, q_z)
__device__ constexpr bool zodd(int v) { return v == 3 || v == 6 || v == 8 || v == 12; }

// value of component v at index k of a 14-plane field, the constant 0 for a z-odd component
// of a planar run
template <bool PL>
__device__ __forceinline__ double ld(const double* f, int v, long long stride, long long k) {
  return (PL && zodd(v)) ? 0.0 : f[v * stride + k];
}

// launders the forward closure core (opaque, mx_adjoint.hpp)
template <class K> __device__ __forceinline__ void opaque_core(K& k) {
  opaque(k.rho); opaque(k.c); opaque(k.t1); opaque(k.t2); opaque(k.A); opaque(k.sig); opaque(k.sb);
#pragma unroll
  for (int m = 0; m < 6; ++m) { opaque(k.Ph[m]); opaque(k.P2[m]); }
#pragma unroll
  for (int i = 0; i < 3; ++i) { opaque(k.qh[i]); opaque(k.z[i]); }
}

template <bool PL>
__device__ __forceinline__ void get_w(const AdjParams& a, long long e, double* W) {
#pragma unroll
  for (int v = 0; v < 14; ++v) W[v] = ld<PL>(a.wext, v, a.eplane, e);
}

// ------------------------------------------------------------------ 0. prep
// Both prep passes in one launch, on tiles of PTX x PTY extended cells: the tile and a ring
// of one cell recover their primitives into LDS (one conversion per cell and thread in a
// loop, the ring's cells by the tile's spare threads), then each cell stores its own to wext
// and forms its limiter factors from its LDS neighbours (the same values as a separate pass
// over wext, bit for bit).
template <int DIM> struct PrepTile;
template <> struct PrepTile<2> { static constexpr int X = 64, Y = 4; };
template <> struct PrepTile<1> { static constexpr int X = 256, Y = 1; };

template <bool PL> struct PrepSys { using S = Sys14; };
template <> struct PrepSys<true> { using S = Sys14P; };

template <int DIM, bool PL>
__device__ __forceinline__ void tile_w(const double* sw, int stride, int k, double* W) {
  using S = typename PrepSys<PL>::S;
#pragma unroll
  for (int v = 0; v < 14; ++v) W[v] = 0.0;
#pragma unroll
  for (int v = 0; v < S::NV; ++v) W[S::plane_of(v)] = sw[v * stride + k];
}

template <int DIM, int ORDER, bool PL>
__global__ __launch_bounds__(ADJ_NT) void adj_prep_kernel(AdjParams a) {
  using S = typename PrepSys<PL>::S;
  constexpr int NV = S::NV;
  constexpr int TX = PrepTile<DIM>::X, TY = PrepTile<DIM>::Y;
  constexpr int R = (ORDER == 2) ? 1 : 0;              // ring of neighbour cells
  constexpr int HX = TX + 2 * R, HY = (DIM == 2) ? TY + 2 * R : 1;
  constexpr int HN = HX * HY;
  __shared__ double sw[NV * HN];
  const StageParams& p = a.sp;
  const int eny = (int)(a.eplane / a.epitch);
  const int ntx = (a.epitch + TX - 1) / TX;
  const int tile = (int)xcd_block();
  const int ex0 = (tile % ntx) * TX, ey0 = (tile / ntx) * TY;
  if (ey0 >= eny) return;                                // uniform per workgroup
#pragma unroll 1
  for (int k = threadIdx.x; k < HN; k += ADJ_NT) {
    const int ex = ex0 - R + k % HX, ey = (DIM == 2) ? ey0 - R + k / HX : 0;
    double W[NV];
    if (ex >= 0 && ex < a.epitch && ey >= 0 && ey < eny) {
      load_prims<S>(p, p.Ub, ex - 2, (DIM == 2) ? ey - 2 : 0, W);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) W[v] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sw[v * HN + k] = W[v];
  }
  __syncthreads();
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int ex = ex0 + tx, ey = ey0 + ty;
  if (ex >= a.epitch || ey >= eny) return;
  const long long e = (long long)ey * a.epitch + ex;
  const int kc = (ty + ((DIM == 2) ? R : 0)) * HX + tx + R;
#pragma unroll
  for (int v = 0; v < NV; ++v) a.wext[S::plane_of(v) * a.eplane + e] = sw[v * HN + kc];
  if constexpr (ORDER == 2) {
    const int i = ex - 2, j = (DIM == 2) ? ey - 2 : 0;
    double Wc[14], Wm[14], Wp[14];
    tile_w<DIM, PL>(sw, HN, kc, Wc);
    double phi = 0.0;
    int vs = -1;
    if (j >= 0 && j < p.ny && i >= -1 && i <= p.nx) {
      tile_w<DIM, PL>(sw, HN, kc - 1, Wm);
      tile_w<DIM, PL>(sw, HN, kc + 1, Wp);
      phi = Adj14::limiter_select(Wm, Wc, Wp, p.limiter, p.fallback, vs);
    }
    a.phix[e] = phi;
    a.vsx[e] = a.frozen_limiter ? -1 : vs;
    if constexpr (DIM == 2) {
      phi = 0.0;
      vs = -1;
      if (i >= 0 && i < p.nx && j >= -1 && j <= p.ny) {
        tile_w<DIM, PL>(sw, HN, kc - HX, Wm);
        tile_w<DIM, PL>(sw, HN, kc + HX, Wp);
        phi = Adj14::limiter_select(Wm, Wc, Wp, p.limiter, p.fallback, vs);
      }
      a.phiy[e] = phi;
      a.vsy[e] = a.frozen_limiter ? -1 : vs;
    }
  }
}

// workgroups of the prep kernel: one per tile
template <int DIM>
static unsigned prep_blocks(const AdjParams& a) {
  const long long eny = a.eplane / a.epitch;
  const long long ntx = (a.epitch + PrepTile<DIM>::X - 1) / PrepTile<DIM>::X;
  const long long nty = (eny + PrepTile<DIM>::Y - 1) / PrepTile<DIM>::Y;
  return (unsigned)(ntx * nty);
}

// ------------------------------------------------------------------ 1. faces
// reverse of face f along D, for its left (right = false) or right state
template <int D, int DIM, int ORDER, bool PL>
__device__ __forceinline__ void face_reverse(const AdjParams& a, long long f, bool right) {
  const StageParams& p = a.sp;
  const int n = (D == 0) ? p.nx : p.ny;           // cells along D
  const int m = (D == 0) ? p.ny : p.nx;           // lines
  const long long nf = (long long)(n + 1) * m;
  if (f >= nf) return;
  int fc, l;                                       // face fc lies between cells fc-1 and fc
  if (D == 0) { fc = (int)(f % (n + 1)); l = (int)(f / (n + 1)); }
  else { fc = (int)(f / m); l = (int)(f % m); }
  const double inv_h = (D == 0) ? p.inv_dx : p.inv_dy;
  const double mc = a.mu_coef * a.dt;
  // face-state adjoints: [0,14) of the face's left state, [14,28) of its right state
  double* out = ((D == 0) ? a.fbx : a.fby) + (right ? 14 * nf : 0) + f;

  // flux adjoint from the two adjacent interior cells
  double Fhb[14];
  bool any = false;
  {
    long long cl = (D == 0) ? ucell(p, fc - 1, l) : ucell(p, l, fc - 1);
    long long cr = (D == 0) ? ucell(p, fc, l) : ucell(p, l, fc);
    bool hl = fc - 1 >= 0, hr = fc < n;
#pragma unroll
    for (int v = 0; v < 14; ++v) {
      double ml = hl ? mc * ld<PL>(a.lam_out, v, p.plane, cl) : 0.0;
      double mr = hr ? mc * ld<PL>(a.lam_out, v, p.plane, cr) : 0.0;
      Fhb[v] = (mr - ml) * inv_h;
      any = any || (Fhb[v] != 0.0);
    }
  }
  if (!any) {
#pragma unroll
    for (int v = 0; v < 14; ++v)
      if (!(PL && zodd(v))) out[v * nf] = 0.0;
    return;
  }
  // this lane's face state: the left state is the upper face state of cell fc-1, the right
  // state the lower face state of cell fc
  const int cc = right ? fc : fc - 1;
  double W[14];
  if constexpr (ORDER == 2) {
    const long long ec = ext_idx<D, DIM>(a, cc, l);
    const long long st = (D == 0) ? 1 : a.epitch;
    double Sm[14], Sc[14], Sp[14];
    get_w<PL>(a, ec - st, Sm);
    get_w<PL>(a, ec, Sc);
    get_w<PL>(a, ec + st, Sp);
    const double ph = (D == 0) ? a.phix[ec] : a.phiy[ec];
    face_state<Sys14>(Sm, Sc, Sp, ph, right ? -1.0 : 1.0, W);
  } else {
    get_w<PL>(a, ext_idx<D, DIM>(a, cc, l), W);
  }
  // forward face terms (Sys14::face_terms, step by step): the closure core and closing values
  // are kept for the reverse below
  Sys14::Core<double> k;
  Sys14::core(W, p.sigma_lim, k);
  double Qd[6], Rd[3], Sd;
  Sys14::closure_dir<D>(k, Qd, Rd, Sd);
  double aF = 0.0, aU = 0.0, lmin, lmax;
  {
    double U[14], F[14];
    Sys14::flux<D>(W, Qd, Rd, Sd, F);
    Sys14::prim_to_cons(W, U);
#pragma unroll
    for (int v = 0; v < 14; ++v) { aF += Fhb[v] * F[v]; aU += Fhb[v] * U[v]; }
  }
  Sys14::wavespeeds<D>(k, W[1 + D], p.kws, lmin, lmax);
  // the partner lane's products and wave speeds
  const double oF = __shfl_xor(aF, 1, 64), oU = __shfl_xor(aU, 1, 64);
  const double omin = __shfl_xor(lmin, 1, 64), omax = __shfl_xor(lmax, 1, 64);
  double Ub[14], Fb[14], lminb, lmaxb;
  Adj14::interface_side_vjp(right, right ? omin : lmin, right ? omax : lmax, right ? lmin : omin,
                            right ? lmax : omax, right ? oF : aF, right ? aF : oF, right ? oU : aU,
                            right ? aU : oU, p.flux, Fhb, Ub, Fb, lminb, lmaxb);
  bool any2 = lminb != 0.0 || lmaxb != 0.0;
#pragma unroll
  for (int v = 0; v < 14; ++v) any2 = any2 || Ub[v] != 0.0 || Fb[v] != 0.0;
  double Wb[14];
#pragma unroll
  for (int v = 0; v < 14; ++v) Wb[v] = 0.0;
  if (any2) {
    // the wave speeds' reverse first, on the forward's own wave-speed values; the rest reads a
    // laundered face state (the flux reverse recomputes what it needs from it rather than
    // holding the forward's flux intermediates); the planar closure reverse may share the
    // forward's closure values, the full one (fourteen moments, more live values) recomputes
    // them from a laundered closure core too
    Adj14::CoreB<double> kb;
    Adj14::zero(kb);
    double udb = 0.0;
    Adj14::wavespeeds_vjp<D>(k, W[1 + D], p.kws, lminb, lmaxb, kb, udb);
#pragma unroll
    for (int v = 0; v < 14; ++v) opaque(W[v]);
    if constexpr (!PL) {
      opaque_core(k);
#pragma unroll
      for (int m = 0; m < 6; ++m) opaque(Qd[m]);
#pragma unroll
      for (int i = 0; i < 3; ++i) opaque(Rd[i]);
      opaque(Sd);
    }
    Adj14::opaque_b(kb);
    opaque(udb);
    Adj14::face_terms_vjp_rest<D>(k, Qd, Rd, Sd, W, p.sigma_lim, Ub, Fb, kb, udb, Wb);
  }
#pragma unroll
  for (int v = 0; v < 14; ++v)
    if (!(PL && zodd(v))) out[v * nf] = Wb[v];
}

// One launch covers both directions: lanes 2k and 2k+1 own the left and the right state of
// a face (two threads per face, so both lanes of a pair pass or fail every face-uniform test
// together); the first bx workgroups take the x faces, the rest the y faces.  One launch
// instead of one per direction leaves one partly filled last round of wavefronts per stage
// instead of two.  Two wavefronts per SIMD: the planar kernel fits 256 registers, the full
// one spills about a hundred (still 13 % faster than one wavefront at 291 registers).
template <int DIM, int ORDER, bool PL>
__global__ __launch_bounds__(FACE_NT) __attribute__((amdgpu_waves_per_eu(2)))
void adj_face_kernel(AdjParams a) {
  const long long b = xcd_block();
  const long long bx = (2 * a.nfx + FACE_NT - 1) / FACE_NT;
  const bool right = (threadIdx.x & 1) != 0;
  if (DIM == 1 || b < bx) face_reverse<0, DIM, ORDER, PL>(a, (b * FACE_NT + threadIdx.x) >> 1, right);
  else if constexpr (DIM == 2)
    face_reverse<1, DIM, ORDER, PL>(a, ((b - bx) * FACE_NT + threadIdx.x) >> 1, right);
}

// ------------------------------------------------------------------ 2. extended cells
// adjoint of the primitive state of cell c (line l, direction D) through the reconstruction
// of the stencil cells c-1, c, c+1
template <int D, int DIM, int ORDER, bool PL>
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
      for (int v = 0; v < 14; ++v) Wb[v] += ld<PL>(fb, 14 + v, nfs, fidx(c));
    }
    if (c + 1 >= 0 && c + 1 <= n) {
#pragma unroll
      for (int v = 0; v < 14; ++v) Wb[v] += ld<PL>(fb, v, nfs, fidx(c + 1));
    }
  } else {
    // stencil cells k = c-1, c, c+1 with face states (k in [-1, n]); each stencil's three
    // cells are read when needed (re-reads hit L2; holding all five cells would cost 140
    // registers)
    const long long st = (D == 0) ? 1 : a.epitch;
    const long long e0 = ext_idx<D, DIM>(a, c, l);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int k = c - 1 + r;
      if (k < -1 || k > n) continue;
      double Op[14], Om[14];
      bool any = false;
#pragma unroll
      for (int v = 0; v < 14; ++v) {
        Op[v] = (k + 1 <= n) ? ld<PL>(fb, v, nfs, fidx(k + 1)) : 0.0;        // upper face: its WL
        Om[v] = (k >= 0) ? ld<PL>(fb, 14 + v, nfs, fidx(k)) : 0.0;          // lower face: its WR
        any = any || Op[v] != 0.0 || Om[v] != 0.0;
      }
      if (!any) continue;
      const long long ek = e0 + (r - 1) * st;
      double Sm[14], Sc[14], Sp[14];
      get_w<PL>(a, ek - st, Sm);
      get_w<PL>(a, ek, Sc);
      get_w<PL>(a, ek + st, Sp);
      const double phi = (D == 0) ? a.phix[ek] : a.phiy[ek];
      const int vstar = (D == 0) ? a.vsx[ek] : a.vsy[ek];
      // cell c is the stencil's Wp (r = 0), Wc (r = 1) or Wm (r = 2)
      Adj14::recon_vjp_role(2 - r, Sm, Sc, Sp, phi, vstar, p.limiter, Op, Om, Wb);
    }
  }
}

template <int DIM, int ORDER, bool PL>
__global__ __launch_bounds__(ADJ_NT) void adj_cell_kernel(AdjParams a) {
  const StageParams& p = a.sp;
  const long long e = xcd_block() * ADJ_NT + threadIdx.x;
  if (e >= a.eplane) return;
  const int ei = (int)(e % a.epitch);
  const int ej = (int)(e / a.epitch);
  const int i = ei - 2;
  const int j = (DIM == 2) ? ej - 2 : 0;
  double Wb[14];
#pragma unroll
  for (int v = 0; v < 14; ++v) Wb[v] = 0.0;
  const bool in_i = i >= 0 && i < p.nx, in_j = j >= 0 && j < p.ny;
  if (in_j) gather_line<0, DIM, ORDER, PL>(a, i, j, Wb);
  if constexpr (DIM == 2) {
    if (in_i) gather_line<1, DIM, ORDER, PL>(a, j, i, Wb);
  }
#pragma unroll
  for (int v = 0; v < 14; ++v)
    if (!(PL && zodd(v))) a.wb[v * a.eplane + e] = Wb[v];
}

// ------------------------------------------------------------------ 3. interior cells
template <int DIM, bool PL>
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
    for (int v = 0; v < 14; ++v) Wb[v] = ld<PL>(a.wb, v, a.eplane, e);
    // a ghost cell holding a jet state: its adjoint goes to the jet parameters
    auto fold_jet = [&](int jet, long long eg) {
      double sn, cs;
      sincospi(p.jet_ang[jet] / 180.0, &sn, &cs);
      const double T = p.jet_T;
      const double c0 = sqrt(5.0 / 3.0 * T);
      double G[14];
#pragma unroll
      for (int v = 0; v < 14; ++v) G[v] = ld<PL>(a.wb, v, a.eplane, eg);
      gM += (G[1] * cs + G[2] * sn) * c0;
      gR += G[0] + T * (G[4] + G[7] + G[9]) + 15.0 * T * T * G[13];
    };
    // ghost cells along x in this row that copy cell (i, j)
    const int jet_lo = (p.n_jets > 0 && p.bc[0] == 3) ? jet_on_wall(p, 0, j) : -1;
    const int jet_hi = (p.n_jets > 0 && p.bc[1] == 3) ? jet_on_wall(p, 1, j) : -1;
    const int gx[4] = {-2, -1, p.nx, p.nx + 1};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int g = gx[q];
      int rx = 0;
      const int si = map_axis(g, p.nx, p.bc[0], p.bc[1], rx);
      if (si != i) continue;
      const long long eg = ext(g, j);
      const int jet = g < 0 ? jet_lo : jet_hi;
      if (jet >= 0) {
        fold_jet(jet, eg);
        continue;
      }
#pragma unroll
      for (int v = 0; v < 14; ++v) {
        double gv = ld<PL>(a.wb, v, a.eplane, eg);
        Wb[v] += (rx && Sys14::odd(v, 0)) ? -gv : gv;
      }
    }
    if constexpr (DIM == 2) {
      const int jet_blo = (p.n_jets > 0 && p.bc[2] == 3) ? jet_on_wall(p, 2, i) : -1;
      const int jet_bhi = (p.n_jets > 0 && p.bc[3] == 3) ? jet_on_wall(p, 3, i) : -1;
      const int gy[4] = {-2, -1, p.ny, p.ny + 1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int g = gy[q];
        int ry = 0;
        const int sj = map_axis(g, p.ny, p.bc[2], p.bc[3], ry);
        if (sj != j) continue;
        const long long eg = ext(i, g);
        const int jet = g < 0 ? jet_blo : jet_bhi;
        if (jet >= 0) {
          fold_jet(jet, eg);
          continue;
        }
#pragma unroll
        for (int v = 0; v < 14; ++v) {
          double gv = ld<PL>(a.wb, v, a.eplane, eg);
          Wb[v] += (ry && Sys14::odd(v, 1)) ? -gv : gv;
        }
      }
    }
    const long long off = ucell(p, i, j);
    double U[14], lo[14];
#pragma unroll
    for (int v = 0; v < 14; ++v) {
      U[v] = ld<PL>(p.Ub, v, p.plane, off);
      lo[v] = ld<PL>(a.lam_out, v, p.plane, off);
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
      if (PL && zodd(v)) continue;
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
    // each workgroup owns its slot and the stages run in order on one stream: the slot sums
    // the workgroup's partials over all reverse stages, summed once at the end (fixed order)
    a.part[threadIdx.x * a.n_upd_blocks + blockIdx.x] += s;
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
      grad[m] = t;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ tape helpers
__global__ void tape_dt_kernel(const DevCtrl* c, double* slot) {
  if (threadIdx.x == 0) *slot = c->dt;
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

template <int DIM, int ORDER, bool PL>
static hipError_t launch_adj_t(AdjParams& a, hipStream_t s) {
  auto blocks = [](long long n) { return dim3((unsigned)((n + ADJ_NT - 1) / ADJ_NT)); };
  hipLaunchKernelGGL((adj_prep_kernel<DIM, ORDER, PL>), dim3(prep_blocks<DIM>(a)), dim3(ADJ_NT), 0, s, a);
  auto fblocks = [](long long n) { return (unsigned)((n + FACE_NT - 1) / FACE_NT); };
  const unsigned nfb = fblocks(2 * a.nfx) + (DIM == 2 ? fblocks(2 * a.nfy) : 0u);
  hipLaunchKernelGGL((adj_face_kernel<DIM, ORDER, PL>), dim3(nfb), dim3(FACE_NT), 0, s, a);
  hipLaunchKernelGGL((adj_cell_kernel<DIM, ORDER, PL>), blocks(a.eplane), dim3(ADJ_NT), 0, s, a);
  hipLaunchKernelGGL((adj_update_kernel<DIM, PL>), dim3(a.n_upd_blocks), dim3(ADJ_NT), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const AdjParams& a, hipStream_t s) {
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(1), dim3(ADJ_NT), 0, s, a.part, a.n_upd_blocks, a.grad);
  return hipGetLastError();
}

hipError_t launch_adjoint_stage(int dim, int order, bool planar, AdjParams& a, hipStream_t s) {
  if (dim == 2) {
    if (planar) return order == 2 ? launch_adj_t<2, 2, true>(a, s) : launch_adj_t<2, 1, true>(a, s);
    return order == 2 ? launch_adj_t<2, 2, false>(a, s) : launch_adj_t<2, 1, false>(a, s);
  }
  return order == 2 ? launch_adj_t<1, 2, false>(a, s) : launch_adj_t<1, 1, false>(a, s);
}

// nonzero z-odd component (3, 6, 8, 12) in a flat 14-moment field of n cells: ctrl->asym
__global__ __launch_bounds__(256) void check_planar_kernel(const double* f, long long n, DevCtrl* c) {
  int np = 0;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256)
    np |= (f[3 * n + k] != 0.0 || f[6 * n + k] != 0.0 || f[8 * n + k] != 0.0 || f[12 * n + k] != 0.0);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) np |= __shfl_xor(np, o, 64);
  if ((threadIdx.x & 63) == 0 && np) atomicOr(&c->asym, ASYM_Z);
}

hipError_t launch_check_planar(const double* f, long long n, DevCtrl* c, hipStream_t s) {
  int grid = (int)((n + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(check_planar_kernel, dim3(grid), dim3(256), 0, s, f, n, c);
  return hipGetLastError();
}

hipError_t launch_tape_dt(const DevCtrl* c, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(tape_dt_kernel, dim3(1), dim3(64), 0, s, c, slot);
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

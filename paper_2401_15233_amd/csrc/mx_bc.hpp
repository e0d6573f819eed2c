// Boundary conditions of the finite-volume stencil: every cell index outside the domain
// (ghost cell) is mapped to a primitive state when the stencil is loaded, so ghost cells are
// never stored.  Transmissive: copy of the edge cell; periodic: wrap; reflective: mirror
// image with the components odd under the reflection negated; jet inflow (any wall,
// 14 moments): the Maxwellian jet state in the ghost cells along each jet's band of the
// wall, transmissive outside.
// Used by the forward stage kernels and by the reverse (adjoint) kernels.
#pragma once
#include "mx_internal.hpp"
#include "mx_physics.hpp"

namespace mx {

__device__ __forceinline__ int map_axis(int g, int n, int lo, int hi, int& refl) {
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

// the jet on `wall` (0 x-low, 1 x-high, 2 y-low, 3 y-high) whose band holds boundary cell s
// (a row for the x walls, a column for the y walls; the last jet listed if bands overlap),
// or -1 (the loop runs over the four parameter slots, so every index into the kernel's
// parameter block is static)
__device__ __forceinline__ int jet_on_wall(const StageParams& p, int wall, int s) {
  const double c = (wall < 2) ? p.y0 + ((double)s + 0.5) * p.dy : p.x0 + ((double)s + 0.5) * p.dx;
  int hit = -1;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < p.n_jets && p.jet_wall[k] == wall && c >= p.jet_yc[k] - 0.5 * p.jet_w[k] &&
        c <= p.jet_yc[k] + 0.5 * p.jet_w[k])
      hit = k;
  return hit;
}

// Maxwellian inflow state of jet k: density rho_j, temperature T_j, speed M sqrt(5/3 T_j)
// along the jet angle, P = rho_j T_j I, q = 0, R = 15 p^2 / rho (the angle is selected over
// the four slots, again so that no index into the parameter block is dynamic)
__device__ __forceinline__ void jet_state(const StageParams& p, int k, double* W) {
  double ang = p.jet_ang[0];
#pragma unroll
  for (int m = 1; m < 4; ++m)
    if (k == m) ang = p.jet_ang[m];
  double sn, cs;
  sincospi(ang / 180.0, &sn, &cs);
  double spd = p.jet_mach * sqrt(5.0 / 3.0 * p.jet_T);
  double pj = p.jet_rho * p.jet_T;
  W[0] = p.jet_rho;
  W[1] = spd * cs; W[2] = spd * sn; W[3] = 0.0;
  W[4] = pj; W[5] = 0.0; W[6] = 0.0; W[7] = pj; W[8] = 0.0; W[9] = pj;
  W[10] = 0.0; W[11] = 0.0; W[12] = 0.0;
  W[13] = 15.0 * pj * pj / p.jet_rho;
}

// where the stencil reads ghost or interior cell (gi, gj): the source cell and whether the
// state is mirrored across an x or a y wall
struct HaloSrc {
  int si, sj, rx, ry;
};

// first half of load_prims: the conserved state of the source cell (the loads only, so that a
// thread can issue the loads of several cells before it converts any)
template <class SYS>
__device__ __forceinline__ HaloSrc load_cons(const StageParams& p, const double* U, int gi, int gj,
                                             double* Uc) {
  HaloSrc h;
  h.rx = 0; h.ry = 0;
  h.si = map_axis(gi, p.nx, p.bc[0], p.bc[1], h.rx);
  h.sj = map_axis(gj, p.ny, p.bc[2], p.bc[3], h.ry);
  const double* src = U + (long long)h.sj * p.pitch + h.si;
#pragma unroll
  for (int v = 0; v < SYS::NV; ++v) Uc[v] = src[SYS::plane_of(v) * p.plane];
  return h;
}

// second half: primitives, mirrored components, jet inflow states in the jets' ghost cells
template <class SYS>
__device__ __forceinline__ void finish_prims(const StageParams& p, const HaloSrc& h, int gi, int gj,
                                             const double* Uc, double* W) {
  constexpr int NV = SYS::NV;
  SYS::cons_to_prim(Uc, W);
  if (h.rx) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (SYS::odd(v, 0)) W[v] = -W[v];
  }
  if (h.ry) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (SYS::odd(v, 1)) W[v] = -W[v];
  }
  if constexpr (SYS::JETS) {
    // ghost cells only (one unsigned compare per axis catches both sides)
    if (p.n_jets > 0 && ((unsigned)gi >= (unsigned)p.nx || (unsigned)gj >= (unsigned)p.ny)) {
      const int wall = gi < 0 ? 0 : (gi >= p.nx ? 1 : (gj < 0 ? 2 : 3));
      const int kind = wall == 0 ? p.bc[0] : (wall == 1 ? p.bc[1] : (wall == 2 ? p.bc[2] : p.bc[3]));
      if (kind == 3) {
        const int k = jet_on_wall(p, wall, wall < 2 ? h.sj : h.si);
        if (k >= 0) {
          double Wj[14];
          jet_state(p, k, Wj);
          SYS::from14(Wj, W);
        }
      }
    }
  }
}

template <class SYS>
__device__ __forceinline__ void load_prims(const StageParams& p, const double* U, int gi, int gj,
                                           double* W) {
  double Uc[SYS::NV];
  const HaloSrc h = load_cons<SYS>(p, U, gi, gj, Uc);
  finish_prims<SYS>(p, h, gi, gj, Uc, W);
}

}  // namespace mx

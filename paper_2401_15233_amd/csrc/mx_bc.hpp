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
// or -1
__device__ __forceinline__ int jet_on_wall(const StageParams& p, int wall, int s) {
  const double c = (wall < 2) ? p.y0 + ((double)s + 0.5) * p.dy : p.x0 + ((double)s + 0.5) * p.dx;
  int hit = -1;
  for (int k = 0; k < p.n_jets; ++k)
    if (p.jet_wall[k] == wall && c >= p.jet_yc[k] - 0.5 * p.jet_w[k] && c <= p.jet_yc[k] + 0.5 * p.jet_w[k])
      hit = k;
  return hit;
}

// Maxwellian inflow state of jet k: density rho_j, temperature T_j, speed M sqrt(5/3 T_j)
// along the jet angle, P = rho_j T_j I, q = 0, R = 15 p^2 / rho
__device__ __forceinline__ void jet_state(const StageParams& p, int k, double* W) {
  double sn, cs;
  sincospi(p.jet_ang[k] / 180.0, &sn, &cs);
  double spd = p.jet_mach * sqrt(5.0 / 3.0 * p.jet_T);
  double pj = p.jet_rho * p.jet_T;
  W[0] = p.jet_rho;
  W[1] = spd * cs; W[2] = spd * sn; W[3] = 0.0;
  W[4] = pj; W[5] = 0.0; W[6] = 0.0; W[7] = pj; W[8] = 0.0; W[9] = pj;
  W[10] = 0.0; W[11] = 0.0; W[12] = 0.0;
  W[13] = 15.0 * pj * pj / p.jet_rho;
}

template <class SYS>
__device__ __forceinline__ void load_prims(const StageParams& p, const double* U, int gi, int gj,
                                           double* W) {
  constexpr int NV = SYS::NV;
  int rx = 0, ry = 0;
  int si = map_axis(gi, p.nx, p.bc[0], p.bc[1], rx);
  int sj = map_axis(gj, p.ny, p.bc[2], p.bc[3], ry);
  double Uc[NV];
  const double* src = U + (long long)sj * p.pitch + si;
#pragma unroll
  for (int v = 0; v < NV; ++v) Uc[v] = src[v * p.plane];
  SYS::cons_to_prim(Uc, W);
  if (rx) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (SYS::odd(v, 0)) W[v] = -W[v];
  }
  if (ry) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (SYS::odd(v, 1)) W[v] = -W[v];
  }
  if constexpr (NV == 14) {
    // ghost cells only (one unsigned compare per axis catches both sides)
    if (p.n_jets > 0 && ((unsigned)gi >= (unsigned)p.nx || (unsigned)gj >= (unsigned)p.ny)) {
      const int wall = gi < 0 ? 0 : (gi >= p.nx ? 1 : (gj < 0 ? 2 : 3));
      const int kind = wall == 0 ? p.bc[0] : (wall == 1 ? p.bc[1] : (wall == 2 ? p.bc[2] : p.bc[3]));
      if (kind == 3) {
        const int k = jet_on_wall(p, wall, wall < 2 ? sj : si);
        if (k >= 0) jet_state(p, k, W);
      }
    }
  }
}

}  // namespace mx

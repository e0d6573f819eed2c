// Algorithmic operation count of one cell-update of the 2D 14-moment step (MUSCL + common
// limiter + closure + wave speeds + HLL + BGK + SSP-RK2 + CFL), obtained by running the
// library's own templated device code on the host with a counting scalar type: the full
// 14-moment kernel and the planar one (ten moments of a planar-symmetric state).
//
// "Algorithmic" means the work the method needs per cell: every face is counted once per
// stage (each cell owns one x-face and one y-face), the cell is converted to primitives once
// per stage, and the halo recomputation a tiled kernel performs is not counted.
// Counting convention: add, sub, mul = 1 flop (a fused multiply-add is two);
// div, sqrt, exp, log = 1 flop each (they are also reported separately, since each costs
// tens of FP64 instructions on the device); comparisons and selects are not counted.
//
// Build and run: hipcc -x hip --offload-arch=gfx950 -O1 -std=c++17 flopcount.cpp -o flopcount
// Prints one JSON object.
#include <cstdio>

struct Ops {
  long long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, log = 0;
  long long flops() const { return add + mul + div + sqrt + exp + log; }
};
static Ops g_ops;

struct CD {
  double v;
  CD() : v(0) {}
  CD(double x) : v(x) {}
};
inline CD operator+(CD a, CD b) { g_ops.add++; return CD(a.v + b.v); }
inline CD operator-(CD a, CD b) { g_ops.add++; return CD(a.v - b.v); }
inline CD operator*(CD a, CD b) { g_ops.mul++; return CD(a.v * b.v); }
inline CD operator/(CD a, CD b) { g_ops.div++; return CD(a.v / b.v); }
inline CD operator-(CD a) { return CD(-a.v); }
inline CD& operator+=(CD& a, CD b) { a = a + b; return a; }
inline CD& operator-=(CD& a, CD b) { a = a - b; return a; }
inline bool operator<(CD a, CD b) { return a.v < b.v; }
inline bool operator>(CD a, CD b) { return a.v > b.v; }
inline bool operator<=(CD a, CD b) { return a.v <= b.v; }
inline bool operator>=(CD a, CD b) { return a.v >= b.v; }
inline bool operator==(CD a, CD b) { return a.v == b.v; }
inline bool operator!(CD a) { return !a.v; }
CD msqrt(CD a);
CD mexp(CD a);
CD mlog(CD a);

#include "mx_scheme.hpp"
#include "mx_planar.hpp"
#include <cmath>

CD msqrt(CD a) { g_ops.sqrt++; return CD(std::sqrt(a.v)); }
CD mexp(CD a) { g_ops.exp++; return CD(std::exp(a.v)); }
CD mlog(CD a) { g_ops.log++; return CD(std::log(a.v)); }

using mx::Sys14;
using mx::Sys14P;

// A bimodal beam-crossing state (anisotropic P, non-zero q, super-Maxwellian R) and two
// slightly different neighbours on each side, so that every branch a typical subsonic face
// of the crossed-jets flow takes is exercised (HLL middle state, limiter with phi in (0,1)).
// (planar-symmetric: u_z = P_xz = P_yz = q_z = 0; SYS::from14 keeps the moments SYS carries)
template <class SYS>
static void state(double f, CD* W) {
  const double base[14] = {0.35, 1.2, 0.1, 0.0, 1.6, 0.4, 0.0, 0.9, 0.0, 0.45,
                           0.6, -0.2, 0.0, 9.0};
  CD W14[14];
  for (int v = 0; v < 14; ++v) W14[v] = CD(base[v] * (1.0 + 0.01 * f * (1 + (v % 3))));
  SYS::from14(W14, W);
}

static Ops delta(const Ops& a, const Ops& b) {
  Ops d;
  d.add = b.add - a.add; d.mul = b.mul - a.mul; d.div = b.div - a.div;
  d.sqrt = b.sqrt - a.sqrt; d.exp = b.exp - a.exp; d.log = b.log - a.log;
  return d;
}

// one stage of one cell; `last` adds the CFL reduction input of the new state
template <class SYS>
static void cell_stage(bool last) {
  constexpr int NV = SYS::NV;
  CD W[5][NV], U[NV], Wc[NV];
  for (int k = 0; k < 5; ++k) state<SYS>(k - 2.0, W[k]);
  SYS::prim_to_cons(W[2], U);
  // primitive recovery of the stage input (once per cell: the update takes the centre's
  // primitives from the loaded tile)
  SYS::cons_to_prim(U, Wc);
  CD sl(1e-4), kws(1.0);
  for (int d = 0; d < 2; ++d) {
    // common limiter factor and the positivity check of the cell's two face states
    CD phi = mx::limiter_factor<SYS>(W[1], W[2], W[3], 0);
    (void)mx::faces_admissible<SYS>(W[1], W[2], W[3], phi);
    // the cell's own face along d: left state from this cell, right state from the next
    CD WL[NV], WR[NV], Fh[NV];
    mx::face_state<SYS>(W[1], W[2], W[3], phi, CD(1.0), WL);
    mx::face_state<SYS>(W[2], W[3], W[4], phi, CD(-1.0), WR);
    if (d == 0) mx::face_flux<SYS, 0>(WL, WR, sl, kws, 0, Fh);
    else mx::face_flux<SYS, 1>(WL, WR, sl, kws, 0, Fh);
  }
  // update: flux differences, BGK source with local tau, Heun combination, admissibility
  CD C[NV], Un[NV], Wn[NV];
  CD rho = Wc[0];
  CD T = SYS::pressure(Wc) / rho;
  CD tau = CD(0.006) * (CD(1.0) / rho) * msqrt(CD(1.0) / T);
  SYS::source(Wc, CD(1.0) / tau, C);
  for (int v = 0; v < NV; ++v) {
    CD L = -(U[v] - Wc[v]) * CD(2048.0);
    L = L - (U[v] - W[1][v]) * CD(2048.0);
    L = L + C[v];
    Un[v] = CD(0.5) * U[v] + CD(0.5) * (U[v] + CD(1e-5) * L);
  }
  if (last) {
    // the last stage: the new state's primitives give the check and the next CFL rate
    SYS::cons_to_prim(Un, Wn);
    (void)SYS::admissible(Wn);
    CD r = SYS::cell_rate2d(Wn, sl, kws, CD(1.0 / 2048), CD(1.0 / 2048));
    (void)r;
  } else {
    (void)SYS::admissible_cons(Un);
  }
}

template <class SYS>
static void count(Ops& s1, Ops& s2, Ops& f) {
  Ops a = g_ops;
  cell_stage<SYS>(false);
  s1 = delta(a, g_ops);
  a = g_ops;
  cell_stage<SYS>(true);
  s2 = delta(a, g_ops);
  // one face evaluation alone, for reference
  CD WL[SYS::NV], WR[SYS::NV], Fh[SYS::NV];
  state<SYS>(0.0, WL);
  state<SYS>(1.0, WR);
  a = g_ops;
  mx::face_flux<SYS, 0>(WL, WR, CD(1e-4), CD(1.0), 0, Fh);
  f = delta(a, g_ops);
}

int main() {
  Ops s1, s2, f, p1, p2, pf;
  count<Sys14>(s1, s2, f);
  count<Sys14P>(p1, p2, pf);
  printf("{\"system\": 14, \"dim\": 2, \"scheme\": \"MUSCL-minmod common limiter + HLL + SSP-RK2 + BGK + CFL\", "
         "\"flops_per_cell_update\": %lld, \"flops_stage1\": %lld, \"flops_stage2\": %lld, "
         "\"div\": %lld, \"sqrt\": %lld, \"exp\": %lld, \"log\": %lld, \"flops_per_face\": %lld, "
         "\"planar_flops_per_cell_update\": %lld, \"planar_flops_stage1\": %lld, "
         "\"planar_flops_stage2\": %lld, \"planar_div\": %lld, \"planar_sqrt\": %lld, "
         "\"planar_flops_per_face\": %lld}\n",
         s1.flops() + s2.flops(), s1.flops(), s2.flops(), s1.div + s2.div, s1.sqrt + s2.sqrt,
         s1.exp + s2.exp, s1.log + s2.log, f.flops(), p1.flops() + p2.flops(), p1.flops(),
         p2.flops(), p1.div + p2.div, p1.sqrt + p2.sqrt, pf.flops());
  return 0;
}

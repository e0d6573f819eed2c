// Per-cell and per-face pieces of the finite-volume scheme (Section 3 of the paper), on
// registers, templated on the system and the real type (host + device).
//   limiter_factor  one common, most stringent limiter factor for all primitives of a cell
//                   along one direction (Section 3.2), relative to the central slope
//   face_state      the cell's reconstructed state at its upper (sgn = +1) or lower face
//   face_flux       HLL or Rusanov combination of the two face states' physical fluxes with
//                   the approximate wave speeds (Section 3.1)
#pragma once
#include "mx_physics.hpp"

namespace mx {

// A variable whose two one-sided jumps are both below NEUTRAL_EPS times its natural scale
// does not take part in the common limiter: round-off is not a discontinuity.
constexpr double NEUTRAL_EPS = 1e-10;

template <class SYS, class T>
MX_HD T limiter_factor(const T* Wm, const T* Wc, const T* Wp, int kind) {
  // running minimum kept as a fraction num/den (den > 0) and compared by cross
  // multiplication, so that only the selected variable's factor is divided out
  constexpr int NV = SYS::NV;
  T sc[NV];
  SYS::scales(Wc, sc);
  T num = T(1), den = T(1);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    T a = Wc[v] - Wm[v];
    T b = Wp[v] - Wc[v];
    T aa = tabs(a), ab = tabs(b);
    T fn, fd;
    if (aa + ab <= T(NEUTRAL_EPS) * sc[v]) { fn = T(1); fd = T(1); }
    else if (a * b <= T(0)) { fn = T(0); fd = T(1); }
    else if (kind == 0) { fn = T(2) * tmin(aa, ab); fd = aa + ab; }
    else { fn = T(2) * a * b; fd = a * a + b * b; }
    if (fn * den < num * fd) { num = fn; den = fd; }
  }
  return (den == T(1)) ? num : num / den;
}

template <class SYS, class T>
MX_HD void face_state(const T* Wm, const T* Wc, const T* Wp, T phi, T sgn, T* Wf) {
#pragma unroll
  for (int v = 0; v < SYS::NV; ++v) {
    T a = Wc[v] - Wm[v];
    T b = Wp[v] - Wc[v];
    T s = phi * (a + b) * T(0.5);
    Wf[v] = Wc[v] + sgn * (s * T(0.5));
  }
}

template <class SYS, int D, class T>
MX_HD void face_flux(const T* WL, const T* WR, T sigma_lim, T kws, int flux_kind, T* Fh) {
  constexpr int NV = SYS::NV;
  T UL[NV], FL[NV], UR[NV], FR[NV];
  T lminL, lmaxL, lminR, lmaxR;
  SYS::template face_terms<D>(WL, sigma_lim, kws, UL, FL, lminL, lmaxL);
  SYS::template face_terms<D>(WR, sigma_lim, kws, UR, FR, lminR, lmaxR);
  if (flux_kind == 0) {
    T SL = tmin(lminL, lminR), SR = tmax(lmaxL, lmaxR);
    if (SL >= T(0)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[v] = FL[v];
    } else if (SR <= T(0)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[v] = FR[v];
    } else {
      T inv = T(1) / (SR - SL);
      T SLR = SL * SR;
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[v] = (SR * FL[v] - SL * FR[v] + SLR * (UR[v] - UL[v])) * inv;
    }
  } else {
    T am = tmax(tmax(tabs(lminL), tabs(lmaxL)), tmax(tabs(lminR), tabs(lmaxR)));
#pragma unroll
    for (int v = 0; v < NV; ++v) Fh[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * am * (UR[v] - UL[v]);
  }
}

}  // namespace mx

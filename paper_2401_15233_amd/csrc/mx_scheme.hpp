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
  return (den == T(1)) ? num : mdiv(num, den);
}

// The cell's state at its upper (sgn = +1) or lower (sgn = -1) face: Wc +- s/2 with the limited
// slope s = phi (a + b)/2 and a + b = Wp - Wm, i.e. Wc + sgn (phi/4)(Wp - Wm), one rounding per
// component.
template <class SYS, class T>
MX_HD void face_state(const T* Wm, const T* Wc, const T* Wp, T phi, T sgn, T* Wf) {
  const T q = sgn * T(0.25) * phi;
#pragma unroll
  for (int v = 0; v < SYS::NV; ++v) Wf[v] = tfma(q, Wp[v] - Wm[v], Wc[v]);
}

// Positivity check of both face states of a cell (rho > 0 and P positive definite): only the
// components the check reads are reconstructed, with face_state's expressions, so the check
// decides on exactly the face states the flux evaluation uses.
template <class SYS, class T>
MX_HD bool faces_admissible(const T* Wm, const T* Wc, const T* Wp, T phi) {
  constexpr int NV = SYS::NV;
  const T q = T(0.25) * phi;
  T Wu[NV], Wd[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (!SYS::admissibility_var(v)) { Wu[v] = Wd[v] = T(0); continue; }
    const T d = Wp[v] - Wm[v];
    Wu[v] = tfma(q, d, Wc[v]);
    Wd[v] = tfma(-q, d, Wc[v]);
  }
  return SYS::admissible(Wu) && SYS::admissible(Wd);
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
      T inv = mrcp(SR - SL);
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

// Mixed precision (Section 3.3: the dimensionless closure is robust in single precision).
// The face states arrive in FP64 (primitive recovery and reconstruction stay FP64).  The
// bracket A of the sigma mapping is formed in FP64 (it cancels near equilibrium); the rest of
// the closure, the wave speeds and the physical flux of each face state are in FP32,
// except near the Junk subspace (A < -MIX_DA and sigma < MIX_SIG_JUNK, where q^3/sigma^2 is
// large) and near the realizability boundary (sigma > 1 - MIX_D1, where 1 - sigma and
// sqrt(3 - 3 sigma) cancel): there the state is re-evaluated in FP64.  The HLL dissipation
// term S_L S_R (U_R - U_L) / (S_R - S_L) uses FP64 conserved states, so that the jump is not
// cancelled in FP32.  Returns the number of FP64 re-evaluations (0, 1 or 2).
constexpr float MIX_DA = 1e-3f;
constexpr float MIX_SIG_JUNK = 1e-2f;
constexpr float MIX_D1 = 1e-3f;

template <class SYS, int D>
MX_HD void face_side_mixed(const double* W64, double sigma_lim, double kws, float* F, float& lmin,
                           float& lmax, int& n64) {
  constexpr int NV = SYS::NV;
  float W[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) W[v] = (float)W64[v];
  typename SYS::template Core<float> k;
  SYS::core_mixed(W64, (float)sigma_lim, k);
  bool near_junk = (k.A < -MIX_DA) && (k.sig < MIX_SIG_JUNK);
  bool near_boundary = k.sig > 1.0f - MIX_D1;
  if (near_junk || near_boundary || !(k.sig == k.sig)) {
    double U[NV], F64[NV], a, b;
    SYS::template face_terms<D>(W64, sigma_lim, kws, U, F64, a, b);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = (float)F64[v];
    lmin = (float)a;
    lmax = (float)b;
    ++n64;
  } else {
    SYS::template flux_speeds<D>(k, W, (float)kws, F, lmin, lmax);
  }
}

template <class SYS, int D>
MX_HD void face_flux_mixed(const double* WL, const double* WR, double sigma_lim, double kws,
                           int flux_kind, double* Fh, int& n64) {
  constexpr int NV = SYS::NV;
  float FL[NV], FR[NV], lminL, lmaxL, lminR, lmaxR;
  face_side_mixed<SYS, D>(WL, sigma_lim, kws, FL, lminL, lmaxL, n64);
  face_side_mixed<SYS, D>(WR, sigma_lim, kws, FR, lminR, lmaxR, n64);
  double UL[NV], UR[NV];
  SYS::prim_to_cons(WL, UL);
  SYS::prim_to_cons(WR, UR);
  if (flux_kind == 0) {
    float SL = tmin(lminL, lminR), SR = tmax(lmaxL, lmaxR);
    if (SL >= 0.0f) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[v] = (double)FL[v];
    } else if (SR <= 0.0f) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fh[v] = (double)FR[v];
    } else {
      float inv = 1.0f / (SR - SL);
      double diss = (double)SL * (double)SR / ((double)SR - (double)SL);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        Fh[v] = (double)((SR * FL[v] - SL * FR[v]) * inv) + diss * (UR[v] - UL[v]);
    }
  } else {
    float am = tmax(tmax(tabs(lminL), tabs(lmaxL)), tmax(tabs(lminR), tabs(lmaxR)));
#pragma unroll
    for (int v = 0; v < NV; ++v)
      Fh[v] = (double)(0.5f * (FL[v] + FR[v])) - 0.5 * (double)am * (UR[v] - UL[v]);
  }
}

// Single precision (the FP32 setting): the closure, wave speeds, physical fluxes and the HLL /
// Rusanov combination of both face states in FP32, with no FP64 re-evaluation; the face
// states arrive in FP64 and the interface flux leaves in FP64.
template <class SYS, int D>
MX_HD void face_flux_fp32(const double* WL, const double* WR, double sigma_lim, double kws,
                          int flux_kind, double* Fh) {
  constexpr int NV = SYS::NV;
  float wl[NV], wr[NV], f[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) { wl[v] = (float)WL[v]; wr[v] = (float)WR[v]; }
  face_flux<SYS, D, float>(wl, wr, (float)sigma_lim, (float)kws, flux_kind, f);
#pragma unroll
  for (int v = 0; v < NV; ++v) Fh[v] = (double)f[v];
}

}  // namespace mx

// The 14-moment system restricted to axially symmetric states of a 1D flow along x (Section
// 2.4 equations, closure and wave speeds of Sections 3.3 and 5.1, with the reduced algebra of
// Sys14).
//
// A 1D flow along x whose distribution function is even in v_y and in v_z (a shock tube
// started from Maxwellians at rest, as in the Sod problems) has u_y = u_z = 0, P_xy = P_xz =
// P_yz = 0 and q_y = q_z = 0.  These seven moments stay exactly zero under the x-direction
// step: each of their fluxes, closing moments and source terms carries a y- or z-odd factor.
// Sys14A carries the seven others,
//   W = (rho, u_x, P_xx, P_yy, P_zz, q_x, R),
// stored in the planes 0 1 4 7 9 10 13 of the 14-moment state, and evaluates the same
// expressions as Sys14 with the vanishing terms left out: the pressure tensor is diagonal,
// the closure along x needs Q_xxx, Q_yyx, Q_zzx, R_xx(kk) and S_x(jjkk), and the flux has
// seven non-zero components.  The results equal Sys14's on such states up to the rounding
// order of the remaining terms.  P_yy and P_zz stay separate (they are equal only if they
// start equal).
#pragma once
#include "mx_physics.hpp"

namespace mx {

struct Sys14A {
  static constexpr int NV = 7;
  static constexpr bool JETS = false;
  MX_HD static constexpr int plane_of(int v) {
    return v < 2 ? v : (v == 2 ? 4 : (v == 3 ? 7 : (v == 4 ? 9 : (v == 5 ? 10 : 13))));
  }

  template <class T> MX_HD static void cons_to_prim(const T* U, T* W) {
    T rho = U[0];
    T ir = mrcp(rho);
    T ux = U[1] * ir;
    T Pxx = U[2] - rho * (ux * ux);
    T Pyy = U[3], Pzz = U[4];
    T uu = ux * ux;
    T trP = Pxx + Pyy + Pzz;
    T Pux = Pxx * ux;
    T qx = U[5] - (rho * uu) * ux - trP * ux - T(2) * Pux;
    T uPu = ux * Pux;
    T uq = ux * qx;
    W[0] = rho; W[1] = ux; W[2] = Pxx; W[3] = Pyy; W[4] = Pzz; W[5] = qx;
    W[6] = U[6] - rho * uu * uu - T(2) * uu * trP - T(4) * uPu - T(4) * uq;
  }

  template <class T> MX_HD static void prim_to_cons(const T* W, T* U) {
    T rho = W[0], ux = W[1], Pxx = W[2], Pyy = W[3], Pzz = W[4];
    T uu = ux * ux;
    T trP = Pxx + Pyy + Pzz;
    T Pux = Pxx * ux;
    T uPu = ux * Pux;
    T uq = ux * W[5];
    U[0] = rho;
    U[1] = rho * ux;
    U[2] = rho * (ux * ux) + Pxx;
    U[3] = Pyy;
    U[4] = Pzz;
    U[5] = (rho * uu) * ux + trP * ux + T(2) * Pux + W[5];
    U[6] = rho * uu * uu + T(2) * uu * trP + T(4) * uPu + T(4) * uq + W[6];
  }

  template <class T> MX_HD static T pressure(const T* W) { return (W[2] + W[3] + W[4]) * T(1.0 / 3.0); }

  // rho > 0 and the diagonal pressure tensor positive definite
  template <class T> MX_HD static bool admissible(const T* W) {
    return (W[0] > T(0)) && (W[2] > T(0)) && (W[3] > T(0)) && (W[4] > T(0));
  }
  MX_HD static constexpr bool admissibility_var(int v) { return v == 0 || (v >= 2 && v <= 4); }
  template <class T> MX_HD static bool admissible_cons(const T* U) {
    T rho = U[0];
    T ux = U[1] * mrcp(rho);
    T Pxx = U[2] - rho * (ux * ux);
    return (rho > T(0)) && (Pxx > T(0)) && (U[3] > T(0)) && (U[4] > T(0));
  }

  template <class T> MX_HD static void scales(const T* W, T* sc) {
    T rho = tabs(W[0]);
    T p = tabs(W[2] + W[3] + W[4]) * T(1.0 / 3.0);
    T c = msqrt(mdiv(p, rho));
    T c3 = rho * c * c * c;
    sc[0] = rho;
    sc[1] = c;
    sc[2] = sc[3] = sc[4] = p;
    sc[5] = c3;
    sc[6] = c3 * c;
  }

  // components odd under reflection of x
  MX_HD static constexpr bool odd(int v, int d) { return d == 0 && (v == 1 || v == 5); }

  template <class T> MX_HD static void from14(const T* W14, T* W) {
    W[0] = W14[0]; W[1] = W14[1]; W[2] = W14[4]; W[3] = W14[7]; W[4] = W14[9];
    W[5] = W14[10]; W[6] = W14[13];
  }

  // dimensionless state: diagonal P* (xx yy zz), q*_x, z_x = q*_x / P*_xx, P*^2 (diagonal)
  template <class T> struct Core {
    T rho, c, Ph[3], qh, z, P2[3], t1, t2, A, sig, sb;
  };

  template <class T> MX_HD static void core(const T* W, T sigma_lim, Core<T>& k) {
    k.rho = W[0];
    T p = (W[2] + W[3] + W[4]) * T(1.0 / 3.0);
    T irho = mrcp(k.rho);
    T ip = mrcp(p);
    k.c = msqrt(p * irho);
    T ic = msqrt(k.rho * ip);          // 1 / c
#pragma unroll
    for (int m = 0; m < 3; ++m) k.Ph[m] = W[2 + m] * ip;
    T is3 = irho * (ic * ic * ic);     // 1 / (rho c^3)
    k.qh = W[5] * is3;
    T Rh = W[6] * (is3 * ic);
    k.t1 = k.Ph[0] + k.Ph[1] + k.Ph[2];
#pragma unroll
    for (int m = 0; m < 3; ++m) k.P2[m] = k.Ph[m] * k.Ph[m];
    k.t2 = k.P2[0] + k.P2[1] + k.P2[2];
    k.z = k.qh * mrcp(k.Ph[0]);
    T D = k.qh * k.z;
    T A = T(2) * k.t2 + k.t1 * k.t1 - Rh;
    T X = A * A + T(8) * k.t2 * D;
    k.A = A;
    k.sig = sigma_root(A, X, T(2) * D, T(4) * k.t2);
    k.sb = tmax(k.sig, sigma_lim);
  }

  // mixed precision: the bracket A and the traces it needs in FP64, the rest in FP32
  MX_HD static void core_mixed(const double* W, float sigma_lim, Core<float>& k) {
    double p = (W[2] + W[3] + W[4]) * (1.0 / 3.0);
    double ip = mrcp(p);
    double Ph[3], P2[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) { Ph[m] = W[2 + m] * ip; P2[m] = Ph[m] * Ph[m]; }
    double t1 = Ph[0] + Ph[1] + Ph[2];
    double t2 = P2[0] + P2[1] + P2[2];
    double A = 2.0 * t2 + t1 * t1 - W[6] * W[0] * ip * ip;
    k.rho = (float)W[0];
    float irho = 1.0f / k.rho;
    float ipf = (float)ip;
    k.c = msqrt((float)p * irho);
    float ic = msqrt(k.rho * ipf);
#pragma unroll
    for (int m = 0; m < 3; ++m) { k.Ph[m] = (float)Ph[m]; k.P2[m] = (float)P2[m]; }
    k.t1 = (float)t1;
    k.t2 = (float)t2;
    k.A = (float)A;
    float is3 = irho * (ic * ic * ic);
    k.qh = (float)W[5] * is3;
    k.z = k.qh / k.Ph[0];
    float D = k.qh * k.z;
    float X = k.A * k.A + 8.0f * k.t2 * D;
    k.sig = sigma_root(k.A, X, 2.0f * D, 4.0f * k.t2);
    k.sb = tmax(k.sig, sigma_lim);
  }

  // Closing values of the flux along x, dimensional: Q_xxx Q_yyx Q_zzx, R_xx(kk), S_x(jjkk)
  // (the other Q_ijx and R_ix(kk) vanish)
  template <int d, class T>
  MX_HD static void closure_dir(const Core<T>& k, T* Qd, T* Rd, T& Sd) {
    static_assert(d == 0, "flows along x only");
    // w = Cm^-1 q with Cm = 2 tr(P^2) I + 4 P^2 (diagonal; w_y = w_z = 0)
    T w = k.qh * mrcp(T(4) * k.P2[0] + T(2) * k.t2);
    T P2z = k.P2[0] * k.z;
    T zP2z = k.z * P2z;
    T wz = w * k.z;
    T s3 = k.rho * (k.c * k.c * k.c);
    T s4 = s3 * k.c;
    T s5 = s4 * k.c;
    Qd[0] = T(2) * (w * k.P2[0] + w * k.P2[0] + w * k.P2[0]) * s3;
    Qd[1] = T(2) * (w * k.P2[1]) * s3;
    Qd[2] = T(2) * (w * k.P2[2]) * s3;
    T isb = mrcp(k.sb);
    T Qz = T(2) * (w * P2z + w * P2z + wz * k.P2[0]);
    Rd[0] = (Qz * isb + T(2) * (T(1) - k.sb) * k.P2[0] + k.t1 * k.Ph[0]) * s4;
    T Pw = k.Ph[0] * w;
    T P2w = k.P2[0] * w;
    T t3 = k.P2[0] * k.Ph[0] + k.P2[1] * k.Ph[1] + k.P2[2] * k.Ph[2];
    T P3w = k.P2[0] * Pw;
    T t1 = k.t1, t2 = k.t2;
    T Wq = (T(2) * t1 * t1 * t1 + T(12) * t3 - T(2) * t2 * t1) * w + (T(14) * t2 - T(6) * t1 * t1) * Pw +
           T(20) * t1 * P2w + T(20) * P3w;
    T Qzz = T(2) * (w * zP2z + T(2) * wz * P2z);
    T rsb = msqrt(k.sb);
    Sd = (Qzz * (isb * isb) + T(2) * rsb * t1 * k.qh + (T(1) - rsb) * Wq) * s5;
  }

  // Physical flux along x (seven components) from primitives and closing values
  template <int d, class T>
  MX_HD static void flux(const T* W, const T* Qd, const T* Rd, T Sd, T* F) {
    static_assert(d == 0, "flows along x only");
    T rho = W[0], ux = W[1], Pxx = W[2], Pyy = W[3], Pzz = W[4], qx = W[5];
    T uu = ux * ux;
    T trP = Pxx + Pyy + Pzz;
    T uPd = ux * Pxx;
    T Pu = Pxx * ux;
    T uPu = ux * Pu;
    T uq = ux * qx;
    T Qu = Qd[0] * ux;
    T uQu = ux * Qu;
    T uR = ux * Rd[0];
    T rud = rho * ux;
    F[0] = rud;
    F[1] = rud * ux + Pxx;
    F[2] = rud * (ux * ux) + ux * Pxx + ux * Pxx + ux * Pxx + Qd[0];
    F[3] = ux * Pyy + Qd[1];
    F[4] = ux * Pzz + Qd[2];
    F[5] = (rud * uu) * ux + (ux * trP) * ux + T(2) * uPd * ux + T(2) * ux * Pu + uu * Pxx + ux * qx +
           ux * qx + T(2) * Qu + Rd[0];
    F[6] = rud * uu * uu + T(2) * ux * uu * trP + T(4) * uu * uPd + T(4) * ux * uPu + T(2) * uu * qx +
           T(4) * ux * uq + T(4) * uQu + T(4) * uR + ux * W[6] + Sd;
  }

  // Approximate minimum / maximum wave speed along x (Section 5.1): no transverse heat flux
  template <int d, class T>
  MX_HD static void wavespeeds(const Core<T>& k, T ud, T kws, T& lmin, T& lmax) {
    static_assert(d == 0, "flows along x only");
    T sw = tmin(k.sb, T(1));
    T Pdd = tmax(k.Ph[0], T(0));
    T qd = k.qh;
    T a = T(0), b = T(0);
    if (Pdd > T(0)) {
      T lP = mlog(Pdd);
      a = T(1.4) * mexp(T(1.1) * lP - Pdd * Pdd);
      b = T(0.9) * Pdd * mexp(T(-0.5) * mexp(T(1.4) * lP));
    }
    BYEC<T> g = byec(sw, Pdd);
    T pref = mdiv(a * sw + b, T(2) * sw);
    T base = T(4) * sw * sw * g.Y;
    T zmax = qd;
    T zmin = -qd;
    T Lmax = pref * hyperbola(zmax, T(-0.8) * zmax * sw * g.C + base) + g.E;
    T Lmin = pref * hyperbola(zmin, T(-0.8) * zmin * sw * g.C + base) + g.E;
    lmax = ud + kws * Lmax * k.c;
    lmin = ud - kws * Lmin * k.c;
  }

  template <int d, class T>
  MX_HD static void face_terms(const T* W, T sigma_lim, T kws, T* U, T* F, T& lmin, T& lmax) {
    Core<T> k;
    core(W, sigma_lim, k);
    T Qd[3], Rd[1], Sd;
    closure_dir<d>(k, Qd, Rd, Sd);
    flux<d>(W, Qd, Rd, Sd, F);
    prim_to_cons(W, U);
    wavespeeds<d>(k, W[1], kws, lmin, lmax);
  }

  template <int d, class T>
  MX_HD static void flux_speeds(const Core<T>& k, const T* W, T kws, T* F, T& lmin, T& lmax) {
    T Qd[3], Rd[1], Sd;
    closure_dir<d>(k, Qd, Rd, Sd);
    flux<d>(W, Qd, Rd, Sd, F);
    wavespeeds<d>(k, W[1], kws, lmin, lmax);
  }

  template <int d, class T> MX_HD static T cell_lambda(const T* W, T sigma_lim, T kws) {
    Core<T> k;
    core(W, sigma_lim, k);
    T lmin, lmax;
    wavespeeds<d>(k, W[1], kws, lmin, lmax);
    return tmax(tabs(lmin), tabs(lmax));
  }

  // local Maxwellian: same rho, u and p, P = p I, q = 0, R = 15 p^2 / rho
  template <class T> MX_HD static void equilibrium(const T* W, T* We) {
    T p = (W[2] + W[3] + W[4]) * T(1.0 / 3.0);
    We[0] = W[0]; We[1] = W[1];
    We[2] = p; We[3] = p; We[4] = p;
    We[5] = T(0);
    We[6] = mdiv(T(15) * p * p, W[0]);
  }

  // BGK source; inv_tau = 1/tau at the cell centre
  template <class T> MX_HD static void source(const T* W, T inv_tau, T* C) {
    T rho = W[0], ux = W[1], qx = W[5];
    T p = (W[2] + W[3] + W[4]) * T(1.0 / 3.0);
    T Pu = W[2] * ux;
    T uPu = ux * Pu;
    T uq = ux * qx;
    T uu = ux * ux;
    C[0] = C[1] = T(0);
    C[2] = -(W[2] - p) * inv_tau;
    C[3] = -(W[3] - p) * inv_tau;
    C[4] = -(W[4] - p) * inv_tau;
    C[5] = -(T(2) * Pu + qx - T(2) * ux * p) * inv_tau;
    C[6] = -((T(4) * uPu + T(4) * uq + W[6]) - (T(4) * uu * p + mdiv(T(15) * p * p, rho))) * inv_tau;
  }
};

}  // namespace mx

// The 14-moment system restricted to planar-symmetric states (Section 2.4 equations, closure
// and wave speeds of Sections 3.3 and 5.1, with the same reduced algebra as Sys14).
//
// A 2D flow in the x-y plane whose distribution function is even in the z velocity has
// u_z = P_xz = P_yz = q_z = 0.  These four moments stay exactly zero under the step: every
// flux, closing moment and source term of a z-odd moment is a product containing a z-odd
// factor, and the jet inflow states lie in the plane.  Sys14P carries the ten other moments,
//   W = (rho, u_x, u_y, P_xx, P_xy, P_yy, P_zz, q_x, q_y, R),
// stored in the planes 0 1 2 4 5 7 9 10 11 13 of the 14-moment state, and evaluates the
// same expressions as Sys14 with the vanishing terms left out: the symmetric 3x3 algebra
// becomes a 2x2 block plus the zz entry, the flux along x or y has ten non-zero components,
// and the closure needs four Q_ijd, two R_id and S_d.  The results equal Sys14's on such
// states up to the rounding order of the remaining terms.
#pragma once
#include "mx_physics.hpp"

namespace mx {

// index of the in-plane symmetric pair (i, j), i, j in {0, 1}: xx 0, xy 1, yy 2
MX_HD constexpr int pidx(int i, int j) { return (i == j) ? (i == 0 ? 0 : 2) : 1; }

struct Sys14P {
  static constexpr int NV = 10;
  static constexpr bool JETS = true;
  // storage plane of each carried moment in the 14-moment state
  MX_HD static constexpr int plane_of(int v) {
    return v < 3 ? v : (v == 3 ? 4 : (v == 4 ? 5 : (v == 5 ? 7 : (v == 6 ? 9 : (v == 7 ? 10 : (v == 8 ? 11 : 13))))));
  }

  template <class T> MX_HD static void cons_to_prim(const T* U, T* W) {
    T rho = U[0];
    T ir = mrcp(rho);
    T ux = U[1] * ir, uy = U[2] * ir;
    T Pxx = U[3] - rho * (ux * ux);
    T Pxy = U[4] - rho * (ux * uy);
    T Pyy = U[5] - rho * (uy * uy);
    T Pzz = U[6];
    T uu = ux * ux + uy * uy;
    T trP = Pxx + Pyy + Pzz;
    T Pux = Pxx * ux + Pxy * uy;
    T Puy = Pxy * ux + Pyy * uy;
    T qx = U[7] - (rho * uu) * ux - trP * ux - T(2) * Pux;
    T qy = U[8] - (rho * uu) * uy - trP * uy - T(2) * Puy;
    T uPu = ux * Pux + uy * Puy;
    T uq = ux * qx + uy * qy;
    W[0] = rho; W[1] = ux; W[2] = uy;
    W[3] = Pxx; W[4] = Pxy; W[5] = Pyy; W[6] = Pzz;
    W[7] = qx; W[8] = qy;
    W[9] = U[9] - rho * uu * uu - T(2) * uu * trP - T(4) * uPu - T(4) * uq;
  }

  template <class T> MX_HD static void prim_to_cons(const T* W, T* U) {
    T rho = W[0], ux = W[1], uy = W[2];
    T Pxx = W[3], Pxy = W[4], Pyy = W[5], Pzz = W[6];
    T uu = ux * ux + uy * uy;
    T trP = Pxx + Pyy + Pzz;
    T Pux = Pxx * ux + Pxy * uy;
    T Puy = Pxy * ux + Pyy * uy;
    T uPu = ux * Pux + uy * Puy;
    T uq = ux * W[7] + uy * W[8];
    U[0] = rho;
    U[1] = rho * ux; U[2] = rho * uy;
    U[3] = rho * (ux * ux) + Pxx;
    U[4] = rho * (ux * uy) + Pxy;
    U[5] = rho * (uy * uy) + Pyy;
    U[6] = Pzz;
    U[7] = (rho * uu) * ux + trP * ux + T(2) * Pux + W[7];
    U[8] = (rho * uu) * uy + trP * uy + T(2) * Puy + W[8];
    U[9] = rho * uu * uu + T(2) * uu * trP + T(4) * uPu + T(4) * uq + W[9];
  }

  template <class T> MX_HD static T pressure(const T* W) { return (W[3] + W[5] + W[6]) * T(1.0 / 3.0); }

  // rho > 0 and P positive definite: the in-plane block's leading minors and P_zz
  template <class T> MX_HD static bool admissible(const T* W) {
    T m2 = W[3] * W[5] - W[4] * W[4];
    return (W[0] > T(0)) && (W[3] > T(0)) && (m2 > T(0)) && (W[6] > T(0));
  }
  MX_HD static constexpr bool admissibility_var(int v) { return v == 0 || (v >= 3 && v <= 6); }
  template <class T> MX_HD static bool admissible_cons(const T* U) {
    T rho = U[0];
    T ir = mrcp(rho);
    T ux = U[1] * ir, uy = U[2] * ir;
    T Pxx = U[3] - rho * (ux * ux);
    T Pxy = U[4] - rho * (ux * uy);
    T Pyy = U[5] - rho * (uy * uy);
    T m2 = Pxx * Pyy - Pxy * Pxy;
    return (rho > T(0)) && (Pxx > T(0)) && (m2 > T(0)) && (U[6] > T(0));
  }

  template <class T> MX_HD static void scales(const T* W, T* sc) {
    T rho = tabs(W[0]);
    T p = tabs(W[3] + W[5] + W[6]) * T(1.0 / 3.0);
    T c = msqrt(mdiv(p, rho));
    T c3 = rho * c * c * c;
    sc[0] = rho;
    sc[1] = sc[2] = c;
    sc[3] = sc[4] = sc[5] = sc[6] = p;
    sc[7] = sc[8] = c3;
    sc[9] = c3 * c;
  }

  // components odd under reflection of axis d (x or y)
  MX_HD static constexpr bool odd(int v, int d) {
    return d == 0 ? (v == 1 || v == 4 || v == 7) : (d == 1 ? (v == 2 || v == 4 || v == 8) : false);
  }

  // the planar state of a 14-moment primitive vector (its z-odd moments are zero)
  template <class T> MX_HD static void from14(const T* W14, T* W) {
    W[0] = W14[0]; W[1] = W14[1]; W[2] = W14[2];
    W[3] = W14[4]; W[4] = W14[5]; W[5] = W14[7]; W[6] = W14[9];
    W[7] = W14[10]; W[8] = W14[11]; W[9] = W14[13];
  }

  // dimensionless state: P* (xx xy yy zz), q* (x y), z = P*^-1 q*, P*^2 (xx xy yy zz)
  template <class T> struct Core {
    T rho, c, Ph[4], qh[2], z[2], P2[4], t1, t2, A, sig, sb;
  };

  template <class T> MX_HD static void core(const T* W, T sigma_lim, Core<T>& k) {
    k.rho = W[0];
    T p = (W[3] + W[5] + W[6]) * T(1.0 / 3.0);
    T irho = mrcp(k.rho);
    T ip = mrcp(p);
    k.c = msqrt(p * irho);
    T ic = msqrt(k.rho * ip);          // 1 / c
#pragma unroll
    for (int m = 0; m < 4; ++m) k.Ph[m] = W[3 + m] * ip;
    T is3 = irho * (ic * ic * ic);     // 1 / (rho c^3)
    k.qh[0] = W[7] * is3;
    k.qh[1] = W[8] * is3;
    T Rh = W[9] * (is3 * ic);
    k.t1 = k.Ph[0] + k.Ph[2] + k.Ph[3];
    k.P2[0] = k.Ph[0] * k.Ph[0] + k.Ph[1] * k.Ph[1];
    k.P2[1] = k.Ph[0] * k.Ph[1] + k.Ph[1] * k.Ph[2];
    k.P2[2] = k.Ph[1] * k.Ph[1] + k.Ph[2] * k.Ph[2];
    k.P2[3] = k.Ph[3] * k.Ph[3];
    k.t2 = k.P2[0] + k.P2[2] + k.P2[3];
    T idet = mrcp(k.Ph[0] * k.Ph[2] - k.Ph[1] * k.Ph[1]);
    k.z[0] = (k.Ph[2] * k.qh[0] - k.Ph[1] * k.qh[1]) * idet;
    k.z[1] = (k.Ph[0] * k.qh[1] - k.Ph[1] * k.qh[0]) * idet;
    T D = k.qh[0] * k.z[0] + k.qh[1] * k.z[1];
    T A = T(2) * k.t2 + k.t1 * k.t1 - Rh;
    T X = A * A + T(8) * k.t2 * D;
    k.A = A;
    k.sig = sigma_root(A, X, T(2) * D, T(4) * k.t2);
    k.sb = tmax(k.sig, sigma_lim);
  }

  // mixed precision: the bracket A and the traces it needs in FP64, the rest in FP32 (as
  // Sys14::core_mixed)
  MX_HD static void core_mixed(const double* W, float sigma_lim, Core<float>& k) {
    double p = (W[3] + W[5] + W[6]) * (1.0 / 3.0);
    double ip = mrcp(p);
    double Ph[4], P2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) Ph[m] = W[3 + m] * ip;
    P2[0] = Ph[0] * Ph[0] + Ph[1] * Ph[1];
    P2[1] = Ph[0] * Ph[1] + Ph[1] * Ph[2];
    P2[2] = Ph[1] * Ph[1] + Ph[2] * Ph[2];
    P2[3] = Ph[3] * Ph[3];
    double t1 = Ph[0] + Ph[2] + Ph[3];
    double t2 = P2[0] + P2[2] + P2[3];
    double A = 2.0 * t2 + t1 * t1 - W[9] * W[0] * ip * ip;
    k.rho = (float)W[0];
    float irho = 1.0f / k.rho;
    float ipf = (float)ip;
    k.c = msqrt((float)p * irho);
    float ic = msqrt(k.rho * ipf);
#pragma unroll
    for (int m = 0; m < 4; ++m) { k.Ph[m] = (float)Ph[m]; k.P2[m] = (float)P2[m]; }
    k.t1 = (float)t1;
    k.t2 = (float)t2;
    k.A = (float)A;
    float is3 = irho * (ic * ic * ic);
    k.qh[0] = (float)W[7] * is3;
    k.qh[1] = (float)W[8] * is3;
    float idet = 1.0f / (k.Ph[0] * k.Ph[2] - k.Ph[1] * k.Ph[1]);
    k.z[0] = (k.Ph[2] * k.qh[0] - k.Ph[1] * k.qh[1]) * idet;
    k.z[1] = (k.Ph[0] * k.qh[1] - k.Ph[1] * k.qh[0]) * idet;
    float D = k.qh[0] * k.z[0] + k.qh[1] * k.z[1];
    float X = k.A * k.A + 8.0f * k.t2 * D;
    k.sig = sigma_root(k.A, X, 2.0f * D, 4.0f * k.t2);
    k.sb = tmax(k.sig, sigma_lim);
  }

  // Closing values of a flux along d (x or y), dimensional: Q_xxd Q_xyd Q_yyd Q_zzd,
  // R_xd(kk) R_yd(kk), S_d(jjkk) (Q_xzd, Q_yzd and R_zd(kk) vanish)
  template <int d, class T>
  MX_HD static void closure_dir(const Core<T>& k, T* Qd, T* Rd, T& Sd) {
    static_assert(d == 0 || d == 1, "in-plane directions only");
    // w = Cm^-1 q with Cm = 2 tr(P^2) I + 4 P^2 (its in-plane block; w_z = 0)
    T C0 = T(4) * k.P2[0] + T(2) * k.t2;
    T C1 = T(4) * k.P2[1];
    T C2 = T(4) * k.P2[2] + T(2) * k.t2;
    T idc = mrcp(C0 * C2 - C1 * C1);
    T w[2] = {(C2 * k.qh[0] - C1 * k.qh[1]) * idc, (C0 * k.qh[1] - C1 * k.qh[0]) * idc};
    T P2z[2] = {k.P2[0] * k.z[0] + k.P2[1] * k.z[1], k.P2[1] * k.z[0] + k.P2[2] * k.z[1]};
    T zP2z = k.z[0] * P2z[0] + k.z[1] * P2z[1];
    T wz = w[0] * k.z[0] + w[1] * k.z[1];
    T s3 = k.rho * (k.c * k.c * k.c);
    T s4 = s3 * k.c;
    T s5 = s4 * k.c;
    constexpr int dx = pidx(0, d), dy = pidx(1, d);   // P2 entries (x,d) and (y,d)
    Qd[0] = T(2) * (w[0] * k.P2[dx] + w[0] * k.P2[dx] + w[d] * k.P2[0]) * s3;
    Qd[1] = T(2) * (w[0] * k.P2[dy] + w[1] * k.P2[dx] + w[d] * k.P2[1]) * s3;
    Qd[2] = T(2) * (w[1] * k.P2[dy] + w[1] * k.P2[dy] + w[d] * k.P2[2]) * s3;
    Qd[3] = T(2) * (w[d] * k.P2[3]) * s3;
    T isb = mrcp(k.sb);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int id = pidx(i, d);
      T Qz = T(2) * (w[i] * P2z[d] + w[d] * P2z[i] + wz * k.P2[id]);
      Rd[i] = (Qz * isb + T(2) * (T(1) - k.sb) * k.P2[id] + k.t1 * k.Ph[id]) * s4;
    }
    T Pw[2] = {k.Ph[0] * w[0] + k.Ph[1] * w[1], k.Ph[1] * w[0] + k.Ph[2] * w[1]};
    T P2w[2] = {k.P2[0] * w[0] + k.P2[1] * w[1], k.P2[1] * w[0] + k.P2[2] * w[1]};
    T t3 = k.P2[0] * k.Ph[0] + k.P2[2] * k.Ph[2] + k.P2[3] * k.Ph[3] + T(2) * (k.P2[1] * k.Ph[1]);
    T P3w_d = k.P2[dx] * Pw[0] + k.P2[dy] * Pw[1];
    T t1 = k.t1, t2 = k.t2;
    T Wq = (T(2) * t1 * t1 * t1 + T(12) * t3 - T(2) * t2 * t1) * w[d] +
           (T(14) * t2 - T(6) * t1 * t1) * Pw[d] + T(20) * t1 * P2w[d] + T(20) * P3w_d;
    T Qzz = T(2) * (w[d] * zP2z + T(2) * wz * P2z[d]);
    T rsb = msqrt(k.sb);
    Sd = (Qzz * (isb * isb) + T(2) * rsb * t1 * k.qh[d] + (T(1) - rsb) * Wq) * s5;
  }

  // Physical flux along d (ten components) from primitives and closing values
  template <int d, class T>
  MX_HD static void flux(const T* W, const T* Qd, const T* Rd, T Sd, T* F) {
    T rho = W[0];
    const T u[2] = {W[1], W[2]};
    const T P[3] = {W[3], W[4], W[5]};   // in-plane block: xx xy yy
    const T Pzz = W[6];
    const T q[2] = {W[7], W[8]};
    T ud = u[d];
    T uu = u[0] * u[0] + u[1] * u[1];
    T trP = P[0] + P[2] + Pzz;
    T Pd[2] = {P[pidx(0, d)], P[pidx(1, d)]};
    T uPd = u[0] * Pd[0] + u[1] * Pd[1];
    T Pu[2] = {P[0] * u[0] + P[1] * u[1], P[1] * u[0] + P[2] * u[1]};
    T uPu = u[0] * Pu[0] + u[1] * Pu[1];
    T uq = u[0] * q[0] + u[1] * q[1];
    T Qu[2] = {Qd[0] * u[0] + Qd[1] * u[1], Qd[1] * u[0] + Qd[2] * u[1]};
    T uQu = u[0] * Qu[0] + u[1] * Qu[1];
    T uR = u[0] * Rd[0] + u[1] * Rd[1];
    T rud = rho * ud;
    F[0] = rud;
    F[1] = rud * u[0] + Pd[0];
    F[2] = rud * u[1] + Pd[1];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = i; j < 2; ++j)
        F[3 + pidx(i, j)] = rud * (u[i] * u[j]) + u[i] * Pd[j] + u[j] * Pd[i] + ud * P[pidx(i, j)] +
                            Qd[pidx(i, j)];
    F[6] = ud * Pzz + Qd[3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      F[7 + i] = (rud * uu) * u[i] + (ud * trP) * u[i] + T(2) * uPd * u[i] + T(2) * ud * Pu[i] +
                 uu * Pd[i] + u[i] * q[d] + ud * q[i] + T(2) * Qu[i] + Rd[i];
    F[9] = rud * uu * uu + T(2) * ud * uu * trP + T(4) * uu * uPd + T(4) * ud * uPu +
           T(2) * uu * q[d] + T(4) * ud * uq + T(4) * uQu + T(4) * uR + ud * W[9] + Sd;
  }

  // Approximate minimum / maximum wave speed along d (Section 5.1); the transverse heat flux
  // magnitude is |q*| of the other in-plane axis (q*_z = 0)
  template <int d, class T>
  MX_HD static void wavespeeds(const Core<T>& k, T ud, T kws, T& lmin, T& lmax) {
    T sw = tmin(k.sb, T(1));
    T Pdd = tmax(k.Ph[pidx(d, d)], T(0));
    T qd = k.qh[d];
    T qt = tabs(k.qh[1 - d]);
    T alpha = T(0.6) * Pdd * Pdd - T(0.38) * Pdd + T(0.35);
    T a = T(0), b = T(0);
    if (Pdd > T(0)) {
      T lP = mlog(Pdd);
      a = T(1.4) * mexp(T(1.1) * lP - Pdd * Pdd);
      b = T(0.9) * Pdd * mexp(T(-0.5) * mexp(T(1.4) * lP));
    }
    BYEC<T> g = byec(sw, Pdd);
    T pref = mdiv(a * sw + b, T(2) * sw);
    T base = T(4) * sw * sw * g.Y + qt * qt * T(0.1);
    T zmax = qd + qt * alpha;
    T zmin = -qd + qt * alpha;
    T Lmax = pref * hyperbola(zmax, T(-0.8) * zmax * sw * g.C + base) + g.E;
    T Lmin = pref * hyperbola(zmin, T(-0.8) * zmin * sw * g.C + base) + g.E;
    lmax = ud + kws * Lmax * k.c;
    lmin = ud - kws * Lmin * k.c;
  }

  template <int d, class T>
  MX_HD static void face_terms(const T* W, T sigma_lim, T kws, T* U, T* F, T& lmin, T& lmax) {
    Core<T> k;
    core(W, sigma_lim, k);
    T Qd[4], Rd[2], Sd;
    closure_dir<d>(k, Qd, Rd, Sd);
    flux<d>(W, Qd, Rd, Sd, F);
    prim_to_cons(W, U);
    wavespeeds<d>(k, W[1 + d], kws, lmin, lmax);
  }

  template <int d, class T>
  MX_HD static void flux_speeds(const Core<T>& k, const T* W, T kws, T* F, T& lmin, T& lmax) {
    T Qd[4], Rd[2], Sd;
    closure_dir<d>(k, Qd, Rd, Sd);
    flux<d>(W, Qd, Rd, Sd, F);
    wavespeeds<d>(k, W[1 + d], kws, lmin, lmax);
  }

  template <int d, class T> MX_HD static T cell_lambda(const T* W, T sigma_lim, T kws) {
    Core<T> k;
    core(W, sigma_lim, k);
    T lmin, lmax;
    wavespeeds<d>(k, W[1 + d], kws, lmin, lmax);
    return tmax(tabs(lmin), tabs(lmax));
  }

  template <class T>
  MX_HD static T cell_rate2d(const T* W, T sigma_lim, T kws, T dx, T dy) {
    Core<T> k;
    core(W, sigma_lim, k);
    T a, b, c, d;
    wavespeeds<0>(k, W[1], kws, a, b);
    wavespeeds<1>(k, W[2], kws, c, d);
    return tmax(tabs(a), tabs(b)) / dx + tmax(tabs(c), tabs(d)) / dy;
  }

  // local Maxwellian: same rho, u and p, P = p I, q = 0, R = 15 p^2 / rho
  template <class T> MX_HD static void equilibrium(const T* W, T* We) {
    T p = (W[3] + W[5] + W[6]) * T(1.0 / 3.0);
    We[0] = W[0]; We[1] = W[1]; We[2] = W[2];
    We[3] = p; We[4] = T(0); We[5] = p; We[6] = p;
    We[7] = T(0); We[8] = T(0);
    We[9] = mdiv(T(15) * p * p, W[0]);
  }

  // BGK source; inv_tau = 1/tau at the cell centre
  template <class T> MX_HD static void source(const T* W, T inv_tau, T* C) {
    T rho = W[0];
    const T u[2] = {W[1], W[2]};
    const T q[2] = {W[7], W[8]};
    T p = (W[3] + W[5] + W[6]) * T(1.0 / 3.0);
    T Pu[2] = {W[3] * u[0] + W[4] * u[1], W[4] * u[0] + W[5] * u[1]};
    T uPu = u[0] * Pu[0] + u[1] * Pu[1];
    T uq = u[0] * q[0] + u[1] * q[1];
    T uu = u[0] * u[0] + u[1] * u[1];
    C[0] = C[1] = C[2] = T(0);
    C[3] = -(W[3] - p) * inv_tau;
    C[4] = -W[4] * inv_tau;
    C[5] = -(W[5] - p) * inv_tau;
    C[6] = -(W[6] - p) * inv_tau;
#pragma unroll
    for (int i = 0; i < 2; ++i) C[7 + i] = -(T(2) * Pu[i] + q[i] - T(2) * u[i] * p) * inv_tau;
    C[9] = -((T(4) * uPu + T(4) * uq + W[9]) - (T(4) * uu * p + mdiv(T(15) * p * p, rho))) * inv_tau;
  }
};

}  // namespace mx

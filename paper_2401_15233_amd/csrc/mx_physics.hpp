// Pointwise physics of the 5- and 14-moment maximum-entropy systems, for gfx950 kernels.
//
// Everything here acts on registers of one thread: primitive <-> conserved maps, the
// sigma-limited interpolative closure evaluated in dimensionless variables, approximate
// wave speeds, physical fluxes along one axis, the BGK source.  All functions are
// __host__ __device__ and templated on the real type so that the same code can run in a
// host-side operation counter.
//
// Paper passages (arXiv 2401.15233):
//   conserved / flux / source terms   Section 2.3 (5-moment system) and Section 2.4 (14-moment
//                                      equations and BGK sources)
//   dimensionless variables           eq. dimensionless-variables; closure evaluated
//                                      dimensionless as Section 3.3 recommends
//   parabolic mapping sigma            eqs. sigma-mapping-5mom, sigma-mapping-14mom
//   closing moments                    eqs. closure-1D1V-s-approx, closure-14mom-*-approx
//   sigma limiting                     Section 2.3 and Appendix A
//   wave speeds                        Section 5.1 (eq. 14mom-approx-ws-equations) and
//                                      Appendix B (Baradaran, eq. ws-max-baradaran-orig)
//
// The 14-moment closure is written in reduced form.  With P, q dimensionless (rho = 1) and
//   Cm = 2 tr(P^2) I + 4 P^2,  w = Cm^-1 q  (= P B^-1 q because B = P Cm and P, Cm commute),
//   z = P^-1 q,
// the closing tensors become
//   Q_ijk   = 2 [w_i (P^2)_jk + w_j (P^2)_ik + w_k (P^2)_ij]
//   Q_idl z_l = 2 [w_i (P^2 z)_d + w_d (P^2 z)_i + (w.z) (P^2)_id]
//   Q_dkl z_k z_l = 2 [w_d (z.P^2 z) + 2 (w.z) (P^2 z)_d]
//   (W q)_d = (2 t1^3 + 12 t3 - 2 t2 t1) w_d + (14 t2 - 6 t1^2)(P w)_d + 20 t1 (P^2 w)_d
//             + 20 (P^3 w)_d,
// t_k = tr(P^k), so only two symmetric 3x3 solves are needed (P^-1 q and Cm^-1 q, Cm is
// always well conditioned) and only the ten closing values a flux along axis d uses.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace mx {

#define MX_HD __host__ __device__ __forceinline__

// storage index of symmetric (i, j): xx xy xz yy yz zz
MX_HD constexpr int sidx(int i, int j) {
  return (i == j) ? (i == 0 ? 0 : (i == 1 ? 3 : 5))
                  : ((i + j) == 1 ? 1 : ((i + j) == 2 ? 2 : 4));
}

template <class T> MX_HD T sq(T a) { return a * a; }
// a * b + c: one rounding for the real types (fused multiply-add), the plain expression for
// the host's counting and dual-number types
template <class T> MX_HD T tfma(T a, T b, T c) { return a * b + c; }
template <> MX_HD double tfma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <> MX_HD float tfma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <class T> MX_HD T tmax(T a, T b) { return a > b ? a : b; }
template <class T> MX_HD T tmin(T a, T b) { return a < b ? a : b; }
template <class T> MX_HD T tabs(T a) { return a < T(0) ? -a : a; }
#if defined(__HIP_DEVICE_COMPILE__)
// on the device: clearing the sign bit is one instruction where the compare and select take
// three; it also maps -0 to +0, so a magnitude (a CFL rate reduced as a positive bit pattern)
// is never negative zero
template <> MX_HD double tabs<double>(double a) { return __builtin_fabs(a); }
template <> MX_HD float tabs<float>(float a) { return __builtin_fabsf(a); }
#endif

// FP64 square root, reciprocal and quotient.  On the device: the hardware reciprocal /
// reciprocal-square-root seed (single-precision accurate) refined by Newton-Raphson -- two
// steps of r <- r + r (1 - b r) for 1/b, then one residual correction of the quotient; for the
// square root two steps of the coupled iteration on g ~ sqrt(a), h ~ 1/(2 sqrt(a)) with
// r = 1/2 - g h, then one residual correction -- about 1 ulp, in fewer instructions than the
// correctly rounded sequences.  The arguments of the step (densities, pressures, determinants,
// positive sums) are positive and far from the exponent range's ends; sqrt(0) = 0 is kept, and
// a negative, zero-divisor or non-finite argument still gives a non-finite result, which the
// step's state check reports.  On the host: the IEEE operations.
#if defined(__HIP_DEVICE_COMPILE__)
MX_HD double msqrt(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  const double d = __builtin_fma(-g, g, a);
  const double s = __builtin_fma(d, h, g);
  return a == 0.0 ? a : s;
}
MX_HD double mrcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
}
MX_HD double mdiv(double a, double b) {
  const double r = mrcp(b);
  const double q = a * r;
  return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
#else
MX_HD double msqrt(double a) { return sqrt(a); }
MX_HD double mrcp(double b) { return 1.0 / b; }
MX_HD double mdiv(double a, double b) { return a / b; }
#endif
template <class T> MX_HD T mrcp(T b) { return T(1) / b; }
template <class T> MX_HD T mdiv(T a, T b) { return a / b; }
MX_HD double mexp(double a) { return exp(a); }
MX_HD double mlog(double a) { return log(a); }
// single precision: the hardware square root / exponential / logarithm (about 1 ulp)
#if defined(__HIP_DEVICE_COMPILE__)
MX_HD float msqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
MX_HD float mexp(float a) { return __expf(a); }
MX_HD float mlog(float a) { return __logf(a); }
#else
MX_HD float msqrt(float a) { return sqrtf(a); }
MX_HD float mexp(float a) { return expf(a); }
MX_HD float mlog(float a) { return logf(a); }
#endif

// symmetric 3x3 (6 stored) times vector
template <class T> MX_HD void symv(const T* S, const T* x, T* y) {
  y[0] = S[0] * x[0] + S[1] * x[1] + S[2] * x[2];
  y[1] = S[1] * x[0] + S[3] * x[1] + S[4] * x[2];
  y[2] = S[2] * x[0] + S[4] * x[1] + S[5] * x[2];
}

// product of two commuting-symmetric matrices stored as 6 (result symmetric): A*A
template <class T> MX_HD void symsq(const T* A, T* B) {
  B[0] = A[0] * A[0] + A[1] * A[1] + A[2] * A[2];
  B[1] = A[0] * A[1] + A[1] * A[3] + A[2] * A[4];
  B[2] = A[0] * A[2] + A[1] * A[4] + A[2] * A[5];
  B[3] = A[1] * A[1] + A[3] * A[3] + A[4] * A[4];
  B[4] = A[1] * A[2] + A[3] * A[4] + A[4] * A[5];
  B[5] = A[2] * A[2] + A[4] * A[4] + A[5] * A[5];
}

// adjugate of a symmetric matrix and its determinant
template <class T> MX_HD T symadj(const T* A, T* C) {
  C[0] = A[3] * A[5] - A[4] * A[4];
  C[1] = A[2] * A[4] - A[1] * A[5];
  C[2] = A[1] * A[4] - A[2] * A[3];
  C[3] = A[0] * A[5] - A[2] * A[2];
  C[4] = A[1] * A[2] - A[0] * A[4];
  C[5] = A[0] * A[3] - A[1] * A[1];
  return A[0] * C[0] + A[1] * C[1] + A[2] * C[2];
}

// rho > 0 and the pressure tensor positive definite (leading principal minors)
template <class T> MX_HD bool spd_ok(T rho, const T* P) {
  T m2 = P[0] * P[3] - P[1] * P[1];
  T m3 = P[0] * (P[3] * P[5] - P[4] * P[4]) - P[1] * (P[1] * P[5] - P[4] * P[2]) +
         P[2] * (P[1] * P[4] - P[3] * P[2]);
  return (rho > T(0)) && (P[0] > T(0)) && (m2 > T(0)) && (m3 > T(0));
}

// positive root of the mapping quadratic, cancellation-free for A < 0
template <class T> MX_HD T sigma_root(T A, T X, T num_small, T denom_big) {
  T sX = msqrt(X);
  return (A >= T(0)) ? mdiv(A + sX, denom_big) : mdiv(num_small, sX - A);
}

// zeta + sqrt(max(0, zeta^2 + rest)), cancellation-free for zeta < 0
template <class T> MX_HD T hyperbola(T zeta, T rest) {
  T X = zeta * zeta + rest;
  if (!(X > T(0))) return zeta;
  T sX = msqrt(X);
  return (zeta >= T(0)) ? zeta + sX : mdiv(rest, sX - zeta);
}

// Baradaran's B, Y, E, C at sigma_w and the normal pressure P*_dd
template <class T> struct BYEC { T B, Y, E, C; };
template <class T> MX_HD BYEC<T> byec(T sw, T Pdd) {
  BYEC<T> r;
  r.C = msqrt(tmax((T(3) - T(3) * sw) * Pdd, T(0)));
  r.E = T(0.8) * r.C;
  T rs = msqrt(sw);
  r.B = T(5) - T(4) * rs + msqrt(tmax(T(10) - T(16) * rs + T(6) * sw, T(0)));
  r.Y = r.B + r.E * r.E - T(2) * r.E * msqrt(r.B);
  return r;
}

// ===================================================================== 14 moments
struct Sys14 {
  static constexpr int NV = 14;
  static constexpr bool JETS = true;       // jet inflow boundaries apply
  MX_HD static constexpr int plane_of(int v) { return v; }   // storage plane of moment v
  template <class T> MX_HD static void from14(const T* W14, T* W) {
#pragma unroll
    for (int v = 0; v < 14; ++v) W[v] = W14[v];
  }

  template <class T> MX_HD static void cons_to_prim(const T* U, T* W) {
    T rho = U[0];
    T ir = mrcp(rho);
    T u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
    T P[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) P[sidx(i, j)] = U[4 + sidx(i, j)] - rho * (u[i] * u[j]);
    T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T trP = P[0] + P[3] + P[5];
    T Pu[3];
    symv(P, u, Pu);
    T q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = U[10 + i] - (rho * uu) * u[i] - trP * u[i] - T(2) * Pu[i];
    T uPu = u[0] * Pu[0] + u[1] * Pu[1] + u[2] * Pu[2];
    T uq = u[0] * q[0] + u[1] * q[1] + u[2] * q[2];
    W[0] = rho;
    W[1] = u[0]; W[2] = u[1]; W[3] = u[2];
#pragma unroll
    for (int k = 0; k < 6; ++k) W[4 + k] = P[k];
    W[10] = q[0]; W[11] = q[1]; W[12] = q[2];
    W[13] = U[13] - rho * uu * uu - T(2) * uu * trP - T(4) * uPu - T(4) * uq;
  }

  template <class T> MX_HD static void prim_to_cons(const T* W, T* U) {
    T rho = W[0];
    const T* u = W + 1;
    const T* P = W + 4;
    const T* q = W + 10;
    T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T trP = P[0] + P[3] + P[5];
    T Pu[3];
    symv(P, u, Pu);
    T uPu = u[0] * Pu[0] + u[1] * Pu[1] + u[2] * Pu[2];
    T uq = u[0] * q[0] + u[1] * q[1] + u[2] * q[2];
    U[0] = rho;
    U[1] = rho * u[0]; U[2] = rho * u[1]; U[3] = rho * u[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) U[4 + sidx(i, j)] = rho * (u[i] * u[j]) + P[sidx(i, j)];
#pragma unroll
    for (int i = 0; i < 3; ++i) U[10 + i] = (rho * uu) * u[i] + trP * u[i] + T(2) * Pu[i] + q[i];
    U[13] = rho * uu * uu + T(2) * uu * trP + T(4) * uPu + T(4) * uq + W[13];
  }

  template <class T> MX_HD static T pressure(const T* W) { return (W[4] + W[7] + W[9]) * T(1.0 / 3.0); }

  template <class T> MX_HD static bool admissible(const T* W) { return spd_ok(W[0], W + 4); }
  // the primitives admissible() reads: rho and the pressure tensor
  MX_HD static constexpr bool admissibility_var(int v) { return v == 0 || (v >= 4 && v < 10); }
  // admissible(cons_to_prim(U)) without recovering q and R (the same expressions for rho, u, P)
  template <class T> MX_HD static bool admissible_cons(const T* U) {
    T rho = U[0];
    T ir = mrcp(rho);
    T u[3] = {U[1] * ir, U[2] * ir, U[3] * ir};
    T P[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) P[sidx(i, j)] = U[4 + sidx(i, j)] - rho * (u[i] * u[j]);
    return spd_ok(rho, P);
  }

  // natural scale of each primitive (rho, c, p, rho c^3, rho c^4) for the neutral-variable
  // test of the common limiter
  template <class T> MX_HD static void scales(const T* W, T* sc) {
    T rho = tabs(W[0]);
    T p = tabs(W[4] + W[7] + W[9]) * T(1.0 / 3.0);
    T c = msqrt(mdiv(p, rho));
    T c3 = rho * c * c * c;
    sc[0] = rho;
    sc[1] = sc[2] = sc[3] = c;
#pragma unroll
    for (int k = 4; k < 10; ++k) sc[k] = p;
    sc[10] = sc[11] = sc[12] = c3;
    sc[13] = c3 * c;
  }

  // components odd under reflection of axis d
  MX_HD static constexpr bool odd(int v, int d) {
    return (v == 1 + d) || (v == 10 + d) ||
           (v >= 4 && v < 10 && ((d == 0 && (v == 5 || v == 6)) || (d == 1 && (v == 5 || v == 8)) ||
                                 (d == 2 && (v == 6 || v == 8))));
  }

  // Dimensionless state, sigma and P^-1 q.
  template <class T> struct Core {
    T rho, c, Ph[6], qh[3], z[3], P2[6], t1, t2, A, sig, sb;
  };

  template <class T> MX_HD static void core(const T* W, T sigma_lim, Core<T>& k) {
    k.rho = W[0];
    T p = (W[4] + W[7] + W[9]) * T(1.0 / 3.0);
    T irho = mrcp(k.rho);
    T ip = mrcp(p);
    k.c = msqrt(p * irho);
    T ic = msqrt(k.rho * ip);          // 1 / c
#pragma unroll
    for (int m = 0; m < 6; ++m) k.Ph[m] = W[4 + m] * ip;
    T is3 = irho * (ic * ic * ic);     // 1 / (rho c^3)
#pragma unroll
    for (int i = 0; i < 3; ++i) k.qh[i] = W[10 + i] * is3;
    T Rh = W[13] * (is3 * ic);
    k.t1 = k.Ph[0] + k.Ph[3] + k.Ph[5];
    symsq(k.Ph, k.P2);
    k.t2 = k.P2[0] + k.P2[3] + k.P2[5];
    T C[6];
    T det = symadj(k.Ph, C);
    T idet = mrcp(det);
    T y[3];
    symv(C, k.qh, y);
#pragma unroll
    for (int i = 0; i < 3; ++i) k.z[i] = y[i] * idet;
    T D = k.qh[0] * k.z[0] + k.qh[1] * k.z[1] + k.qh[2] * k.z[2];
    T A = T(2) * k.t2 + k.t1 * k.t1 - Rh;
    T X = A * A + T(8) * k.t2 * D;
    k.A = A;
    k.sig = sigma_root(A, X, T(2) * D, T(4) * k.t2);
    k.sb = tmax(k.sig, sigma_lim);
  }

  // Mixed precision core: the bracket A = 2 tr(P*^2) + tr(P*)^2 - R* of the sigma mapping
  // cancels near equilibrium (R* ~ 15 against A ~ 0), and the wave speeds scale like
  // 1/sigma, so A and the traces it needs are formed in FP64; the rest in FP32.
  MX_HD static void core_mixed(const double* W, float sigma_lim, Core<float>& k) {
    double p = (W[4] + W[7] + W[9]) * (1.0 / 3.0);
    double ip = mrcp(p);
    double Ph[6], P2[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) Ph[m] = W[4 + m] * ip;
    symsq(Ph, P2);
    double t1 = Ph[0] + Ph[3] + Ph[5];
    double t2 = P2[0] + P2[3] + P2[5];
    double A = 2.0 * t2 + t1 * t1 - W[13] * W[0] * ip * ip;
    k.rho = (float)W[0];
    float irho = 1.0f / k.rho;
    float ipf = (float)ip;
    k.c = msqrt((float)p * irho);
    float ic = msqrt(k.rho * ipf);
#pragma unroll
    for (int m = 0; m < 6; ++m) { k.Ph[m] = (float)Ph[m]; k.P2[m] = (float)P2[m]; }
    k.t1 = (float)t1;
    k.t2 = (float)t2;
    k.A = (float)A;
    float is3 = irho * (ic * ic * ic);
#pragma unroll
    for (int i = 0; i < 3; ++i) k.qh[i] = (float)W[10 + i] * is3;
    float C[6];
    float det = symadj(k.Ph, C);
    float idet = 1.0f / det;
    float y[3];
    symv(C, k.qh, y);
#pragma unroll
    for (int i = 0; i < 3; ++i) k.z[i] = y[i] * idet;
    float D = k.qh[0] * k.z[0] + k.qh[1] * k.z[1] + k.qh[2] * k.z[2];
    float X = k.A * k.A + 8.0f * k.t2 * D;
    k.sig = sigma_root(k.A, X, 2.0f * D, 4.0f * k.t2);
    k.sb = tmax(k.sig, sigma_lim);
  }

  // Closing values used by a flux along axis d: Q_ijd (6), R_id(kk) (3), S_d(jjkk),
  // dimensional.
  template <int d, class T>
  MX_HD static void closure_dir(const Core<T>& k, T* Qd, T* Rd, T& Sd) {
    T Cm[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) Cm[m] = T(4) * k.P2[m];
    Cm[0] += T(2) * k.t2; Cm[3] += T(2) * k.t2; Cm[5] += T(2) * k.t2;
    T Ca[6];
    T detc = symadj(Cm, Ca);
    T y[3];
    symv(Ca, k.qh, y);
    T idc = mrcp(detc);
    T w[3] = {y[0] * idc, y[1] * idc, y[2] * idc};
    T P2z[3];
    symv(k.P2, k.z, P2z);
    T zP2z = k.z[0] * P2z[0] + k.z[1] * P2z[1] + k.z[2] * P2z[2];
    T wz = w[0] * k.z[0] + w[1] * k.z[1] + w[2] * k.z[2];
    T s3 = k.rho * (k.c * k.c * k.c);
    T s4 = s3 * k.c;
    T s5 = s4 * k.c;
    // Q_ijd
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        Qd[sidx(i, j)] = T(2) * (w[i] * k.P2[sidx(j, d)] + w[j] * k.P2[sidx(i, d)] +
                                 w[d] * k.P2[sidx(i, j)]) * s3;
    // R_id(kk)
    T isb = mrcp(k.sb);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T Qz = T(2) * (w[i] * P2z[d] + w[d] * P2z[i] + wz * k.P2[sidx(i, d)]);
      Rd[i] = (Qz * isb + T(2) * (T(1) - k.sb) * k.P2[sidx(i, d)] + k.t1 * k.Ph[sidx(i, d)]) * s4;
    }
    // S_d
    T Pw[3], P2w[3], P3w_d;
    symv(k.Ph, w, Pw);
    symv(k.P2, w, P2w);
    T t3 = k.P2[0] * k.Ph[0] + k.P2[3] * k.Ph[3] + k.P2[5] * k.Ph[5] +
           T(2) * (k.P2[1] * k.Ph[1] + k.P2[2] * k.Ph[2] + k.P2[4] * k.Ph[4]);
    P3w_d = k.P2[sidx(d, 0)] * Pw[0] + k.P2[sidx(d, 1)] * Pw[1] + k.P2[sidx(d, 2)] * Pw[2];
    T t1 = k.t1, t2 = k.t2;
    T Wq = (T(2) * t1 * t1 * t1 + T(12) * t3 - T(2) * t2 * t1) * w[d] +
           (T(14) * t2 - T(6) * t1 * t1) * Pw[d] + T(20) * t1 * P2w[d] + T(20) * P3w_d;
    T Qzz = T(2) * (w[d] * zP2z + T(2) * wz * P2z[d]);
    T rsb = msqrt(k.sb);
    Sd = (Qzz * (isb * isb) + T(2) * rsb * t1 * k.qh[d] + (T(1) - rsb) * Wq) * s5;
  }

  // Physical flux along d (14 components) from primitives and closing values.
  template <int d, class T>
  MX_HD static void flux(const T* W, const T* Qd, const T* Rd, T Sd, T* F) {
    T rho = W[0];
    const T* u = W + 1;
    const T* P = W + 4;
    const T* q = W + 10;
    T ud = u[d];
    T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T trP = P[0] + P[3] + P[5];
    T Pd[3] = {P[sidx(0, d)], P[sidx(1, d)], P[sidx(2, d)]};
    T uPd = u[0] * Pd[0] + u[1] * Pd[1] + u[2] * Pd[2];
    T Pu[3];
    symv(P, u, Pu);
    T uPu = u[0] * Pu[0] + u[1] * Pu[1] + u[2] * Pu[2];
    T uq = u[0] * q[0] + u[1] * q[1] + u[2] * q[2];
    T Qu[3];
    symv(Qd, u, Qu);
    T uQu = u[0] * Qu[0] + u[1] * Qu[1] + u[2] * Qu[2];
    T uR = u[0] * Rd[0] + u[1] * Rd[1] + u[2] * Rd[2];
    T rud = rho * ud;
    F[0] = rud;
#pragma unroll
    for (int i = 0; i < 3; ++i) F[1 + i] = rud * u[i] + Pd[i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        F[4 + sidx(i, j)] = rud * (u[i] * u[j]) + u[i] * Pd[j] + u[j] * Pd[i] + ud * P[sidx(i, j)] +
                            Qd[sidx(i, j)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
      F[10 + i] = (rud * uu) * u[i] + (ud * trP) * u[i] + T(2) * uPd * u[i] + T(2) * ud * Pu[i] +
                  uu * Pd[i] + u[i] * q[d] + ud * q[i] + T(2) * Qu[i] + Rd[i];
    F[13] = rud * uu * uu + T(2) * ud * uu * trP + T(4) * uu * uPd + T(4) * ud * uPu +
            T(2) * uu * q[d] + T(4) * ud * uq + T(4) * uQu + T(4) * uR + ud * W[13] + Sd;
  }

  // Approximate minimum / maximum wave speed along d (Section 5.1).
  template <int d, class T>
  MX_HD static void wavespeeds(const Core<T>& k, T ud, T kws, T& lmin, T& lmax) {
    constexpr int t1i = (d == 0) ? 1 : 0;
    constexpr int t2i = (d == 2) ? 1 : 2;
    T sw = tmin(k.sb, T(1));
    T Pdd = tmax(k.Ph[sidx(d, d)], T(0));
    T qd = k.qh[d];
    T qt = msqrt(k.qh[t1i] * k.qh[t1i] + k.qh[t2i] * k.qh[t2i]);
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

  // U, F_d and the wave speeds of a face state
  template <int d, class T>
  MX_HD static void face_terms(const T* W, T sigma_lim, T kws, T* U, T* F, T& lmin, T& lmax) {
    Core<T> k;
    core(W, sigma_lim, k);
    T Qd[6], Rd[3], Sd;
    closure_dir<d>(k, Qd, Rd, Sd);
    flux<d>(W, Qd, Rd, Sd, F);
    prim_to_cons(W, U);
    wavespeeds<d>(k, W[1 + d], kws, lmin, lmax);
  }

  // F_d and the wave speeds from a prepared core (mixed precision path)
  template <int d, class T>
  MX_HD static void flux_speeds(const Core<T>& k, const T* W, T kws, T* F, T& lmin, T& lmax) {
    T Qd[6], Rd[3], Sd;
    closure_dir<d>(k, Qd, Rd, Sd);
    flux<d>(W, Qd, Rd, Sd, F);
    wavespeeds<d>(k, W[1 + d], kws, lmin, lmax);
  }

  // max(|lambda_min|, |lambda_max|) along d at a cell state
  template <int d, class T> MX_HD static T cell_lambda(const T* W, T sigma_lim, T kws) {
    Core<T> k;
    core(W, sigma_lim, k);
    T lmin, lmax;
    wavespeeds<d>(k, W[1 + d], kws, lmin, lmax);
    return tmax(tabs(lmin), tabs(lmax));
  }

  // 2D CFL rate Lambda_x / dx + Lambda_y / dy of a cell state (one closure core for both
  // directions; the same values as cell_lambda<0> / dx + cell_lambda<1> / dy)
  template <class T>
  MX_HD static T cell_rate2d(const T* W, T sigma_lim, T kws, T dx, T dy) {
    Core<T> k;
    core(W, sigma_lim, k);
    T a, b, c, d;
    wavespeeds<0>(k, W[1], kws, a, b);
    wavespeeds<1>(k, W[2], kws, c, d);
    return tmax(tabs(a), tabs(b)) / dx + tmax(tabs(c), tabs(d)) / dy;
  }

  template <class T> MX_HD static T sigma(const T* W) {
    Core<T> k;
    core(W, T(0), k);
    return k.sig;
  }

  // local Maxwellian of a state: same rho, u and p, P = p I, q = 0, R = 15 p^2 / rho (the
  // state the BGK source relaxes to; it has the same rho, rho u and energy)
  template <class T> MX_HD static void equilibrium(const T* W, T* We) {
    T p = (W[4] + W[7] + W[9]) * T(1.0 / 3.0);
    We[0] = W[0]; We[1] = W[1]; We[2] = W[2]; We[3] = W[3];
    We[4] = p; We[5] = T(0); We[6] = T(0); We[7] = p; We[8] = T(0); We[9] = p;
    We[10] = T(0); We[11] = T(0); We[12] = T(0);
    We[13] = mdiv(T(15) * p * p, W[0]);
  }

  // BGK source; inv_tau = 1/tau at the cell centre
  template <class T> MX_HD static void source(const T* W, T inv_tau, T* C) {
    T rho = W[0];
    const T* u = W + 1;
    const T* P = W + 4;
    const T* q = W + 10;
    T p = (P[0] + P[3] + P[5]) * T(1.0 / 3.0);
    T Pu[3];
    symv(P, u, Pu);
    T uPu = u[0] * Pu[0] + u[1] * Pu[1] + u[2] * Pu[2];
    T uq = u[0] * q[0] + u[1] * q[1] + u[2] * q[2];
    T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    C[0] = C[1] = C[2] = C[3] = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j)
        C[4 + sidx(i, j)] = -(P[sidx(i, j)] - (i == j ? p : T(0))) * inv_tau;
#pragma unroll
    for (int i = 0; i < 3; ++i) C[10 + i] = -(T(2) * Pu[i] + q[i] - T(2) * u[i] * p) * inv_tau;
    C[13] = -((T(4) * uPu + T(4) * uq + W[13]) - (T(4) * uu * p + mdiv(T(15) * p * p, rho))) * inv_tau;
  }
};

// ===================================================================== 5 moments
struct Sys5 {
  static constexpr int NV = 5;
  static constexpr bool JETS = false;
  MX_HD static constexpr int plane_of(int v) { return v; }

  template <class T> MX_HD static void cons_to_prim(const T* U, T* W) {
    T rho = U[0];
    T u = mdiv(U[1], rho);
    T P = U[2] - rho * u * u;
    T q = U[3] - rho * u * u * u - T(3) * u * P;
    T r = U[4] - rho * u * u * u * u - T(6) * u * u * P - T(4) * u * q;
    W[0] = rho; W[1] = u; W[2] = P; W[3] = q; W[4] = r;
  }

  template <class T> MX_HD static void prim_to_cons(const T* W, T* U) {
    T rho = W[0], u = W[1], P = W[2], q = W[3], r = W[4];
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * u * u + P;
    U[3] = rho * u * u * u + T(3) * u * P + q;
    U[4] = rho * u * u * u * u + T(6) * u * u * P + T(4) * u * q + r;
  }

  template <class T> MX_HD static T pressure(const T* W) { return W[2]; }
  template <class T> MX_HD static bool admissible(const T* W) { return W[0] > T(0) && W[2] > T(0); }
  MX_HD static constexpr bool admissibility_var(int v) { return v == 0 || v == 2; }
  template <class T> MX_HD static bool admissible_cons(const T* U) {
    T rho = U[0];
    T u = mdiv(U[1], rho);
    T P = U[2] - rho * u * u;
    return rho > T(0) && P > T(0);
  }

  template <class T> MX_HD static void scales(const T* W, T* sc) {
    T rho = tabs(W[0]);
    T p = tabs(W[2]);
    T c = msqrt(mdiv(p, rho));
    sc[0] = rho; sc[1] = c; sc[2] = p; sc[3] = rho * c * c * c; sc[4] = sc[3] * c;
  }

  MX_HD static constexpr bool odd(int v, int) { return v == 1 || v == 3; }

  template <class T> struct Core { T rho, c, qh, A, sig, sb; };

  template <class T> MX_HD static void core(const T* W, T sigma_lim, Core<T>& k) {
    k.rho = W[0];
    T irho = mrcp(k.rho);
    T ip = mrcp(W[2]);
    k.c = msqrt(W[2] * irho);
    T ic = msqrt(k.rho * ip);
    T is3 = irho * (ic * ic * ic);
    k.qh = W[3] * is3;
    T rh = W[4] * (is3 * ic);
    T A = T(3) - rh;
    T X = A * A + T(8) * k.qh * k.qh;
    k.A = A;
    k.sig = sigma_root(A, X, T(2) * k.qh * k.qh, T(4));
    k.sb = tmax(k.sig, sigma_lim);
  }

  MX_HD static void core_mixed(const double* W, float sigma_lim, Core<float>& k) {
    double ip = mrcp(W[2]);
    double A = 3.0 - W[4] * W[0] * ip * ip;
    k.rho = (float)W[0];
    float irho = 1.0f / k.rho;
    float ipf = (float)ip;
    k.c = msqrt((float)W[2] * irho);
    float ic = msqrt(k.rho * ipf);
    float is3 = irho * (ic * ic * ic);
    k.qh = (float)W[3] * is3;
    k.A = (float)A;
    float X = k.A * k.A + 8.0f * k.qh * k.qh;
    k.sig = sigma_root(k.A, X, 2.0f * k.qh * k.qh, 4.0f);
    k.sb = tmax(k.sig, sigma_lim);
  }

  template <class T> MX_HD static T closing_s(const Core<T>& k) {
    T ss = mdiv(k.qh * k.qh * k.qh, k.sb * k.sb) + (T(10) - T(8) * msqrt(k.sb)) * k.qh;
    T c2 = k.c * k.c;
    return ss * k.rho * (c2 * c2 * k.c);
  }

  template <class T> MX_HD static void flux(const T* W, T s, T* F) {
    T rho = W[0], u = W[1], P = W[2], q = W[3], r = W[4];
    T u2 = u * u;
    F[0] = rho * u;
    F[1] = rho * u2 + P;
    F[2] = rho * u2 * u + T(3) * u * P + q;
    F[3] = rho * u2 * u2 + T(6) * u2 * P + T(4) * u * q + r;
    F[4] = rho * u2 * u2 * u + T(10) * u2 * u * P + T(10) * u2 * q + T(5) * u * r + s;
  }

  template <class T> MX_HD static void wavespeeds(const Core<T>& k, T u, T kws, T& lmin, T& lmax) {
    T sw = tmin(k.sb, T(1));
    BYEC<T> g = byec(sw, T(1));
    T base = T(4) * sw * sw * g.Y;
    T i2s = mrcp(T(2) * sw);
    T Lmax = hyperbola(k.qh, T(-0.8) * k.qh * sw * g.C + base) * i2s + g.E;
    T Lmin = hyperbola(-k.qh, T(0.8) * k.qh * sw * g.C + base) * i2s + g.E;
    lmax = u + kws * Lmax * k.c;
    lmin = u - kws * Lmin * k.c;
  }

  template <int d, class T>
  MX_HD static void face_terms(const T* W, T sigma_lim, T kws, T* U, T* F, T& lmin, T& lmax) {
    Core<T> k;
    core(W, sigma_lim, k);
    flux(W, closing_s(k), F);
    prim_to_cons(W, U);
    wavespeeds(k, W[1], kws, lmin, lmax);
  }

  template <int d, class T>
  MX_HD static void flux_speeds(const Core<T>& k, const T* W, T kws, T* F, T& lmin, T& lmax) {
    flux(W, closing_s(k), F);
    wavespeeds(k, W[1], kws, lmin, lmax);
  }

  template <int d, class T> MX_HD static T cell_lambda(const T* W, T sigma_lim, T kws) {
    Core<T> k;
    core(W, sigma_lim, k);
    T lmin, lmax;
    wavespeeds(k, W[1], kws, lmin, lmax);
    return tmax(tabs(lmin), tabs(lmax));
  }

  template <class T> MX_HD static T sigma(const T* W) {
    Core<T> k;
    core(W, T(0), k);
    return k.sig;
  }

  // 1D1V local Maxwellian: same rho, u, P; q = 0, r = 3 P^2 / rho
  template <class T> MX_HD static void equilibrium(const T* W, T* We) {
    We[0] = W[0]; We[1] = W[1]; We[2] = W[2]; We[3] = T(0);
    We[4] = mdiv(T(3) * W[2] * W[2], W[0]);
  }

  template <class T> MX_HD static void source(const T* W, T inv_tau, T* C) {
    T rho = W[0], u = W[1], P = W[2], q = W[3], r = W[4];
    C[0] = C[1] = C[2] = T(0);
    C[3] = -q * inv_tau;
    C[4] = -(T(4) * u * q + r - mdiv(T(3) * P * P, rho)) * inv_tau;
  }
};

}  // namespace mx

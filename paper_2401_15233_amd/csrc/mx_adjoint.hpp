// Reverse-mode (vector-Jacobian) counterparts of the 14-moment pointwise physics and of the
// per-face scheme pieces: the discrete adjoint of the finite-volume step.
//
// Each *_vjp function reverses the corresponding forward function of mx_physics.hpp /
// mx_scheme.hpp statement by statement: the program variables (including the six stored
// components of every symmetric matrix) are the differentiated variables, and every branch
// (sigma root form, sigma_bar = max(sigma, sigma_lim), sigma_w = min(sigma_bar, 1), the
// square-root clamps, the hyperbola form, the limiter's argmin and regime, HLL's case) is
// the one the forward evaluation takes.  At a kink the derivative of the taken branch is
// used (e.g. sigma_bar = sigma_lim gives no derivative through sigma).  Bars accumulate
// (+=): callers zero them.  Host + device, templated like the forward code, so the host can
// check each one against finite differences.
#pragma once
#include "mx_physics.hpp"
#include "mx_scheme.hpp"

namespace mx {

// Hides a value's origin from the device compiler; no instruction is emitted and host code
// is unchanged.  A reverse that reads the laundered copy recomputes the forward intermediates
// it needs where it needs them, instead of the compiler sharing them with an earlier forward
// evaluation (or hoisting them) and keeping them live across the whole reverse.  Compile-time
// constants (the z-odd zeros of a planar run) are left as they are, so that they still fold.
template <class T> MX_HD void opaque(T& x) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (!__builtin_constant_p(x)) asm volatile("" : "+v"(x));
#else
  (void)x;
#endif
}

// symmetric (stored) y = S x: reverse
template <class T> MX_HD void symv_vjp(const T* S, const T* x, const T* yb, T* Sb, T* xb) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Sb[sidx(i, j)] += yb[i] * x[j];
      xb[j] += yb[i] * S[sidx(i, j)];
    }
}

// B = A*A on stored components: reverse
template <class T> MX_HD void symsq_vjp(const T* A, const T* Bb, T* Ab) {
  // B[sidx(i,j)] = sum_k A[sidx(i,k)] A[sidx(k,j)] for i <= j
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        Ab[sidx(i, k)] += Bb[sidx(i, j)] * A[sidx(k, j)];
        Ab[sidx(k, j)] += Bb[sidx(i, j)] * A[sidx(i, k)];
      }
}

// adjugate C and determinant of a stored symmetric A: reverse (Cb, detb given)
template <class T> MX_HD void symadj_vjp(const T* A, const T* C, const T* Cb, T detb, T* Ab) {
  // det = A0 C0 + A1 C1 + A2 C2
  T Cbt[6] = {Cb[0], Cb[1], Cb[2], Cb[3], Cb[4], Cb[5]};
  Ab[0] += detb * C[0];
  Ab[1] += detb * C[1];
  Ab[2] += detb * C[2];
  Cbt[0] += detb * A[0];
  Cbt[1] += detb * A[1];
  Cbt[2] += detb * A[2];
  // C0 = A3 A5 - A4 A4
  Ab[3] += Cbt[0] * A[5]; Ab[5] += Cbt[0] * A[3]; Ab[4] -= T(2) * Cbt[0] * A[4];
  // C1 = A2 A4 - A1 A5
  Ab[2] += Cbt[1] * A[4]; Ab[4] += Cbt[1] * A[2]; Ab[1] -= Cbt[1] * A[5]; Ab[5] -= Cbt[1] * A[1];
  // C2 = A1 A4 - A2 A3
  Ab[1] += Cbt[2] * A[4]; Ab[4] += Cbt[2] * A[1]; Ab[2] -= Cbt[2] * A[3]; Ab[3] -= Cbt[2] * A[2];
  // C3 = A0 A5 - A2 A2
  Ab[0] += Cbt[3] * A[5]; Ab[5] += Cbt[3] * A[0]; Ab[2] -= T(2) * Cbt[3] * A[2];
  // C4 = A1 A2 - A0 A4
  Ab[1] += Cbt[4] * A[2]; Ab[2] += Cbt[4] * A[1]; Ab[0] -= Cbt[4] * A[4]; Ab[4] -= Cbt[4] * A[0];
  // C5 = A0 A3 - A1 A1
  Ab[0] += Cbt[5] * A[3]; Ab[3] += Cbt[5] * A[0]; Ab[1] -= T(2) * Cbt[5] * A[1];
}

template <class T> MX_HD void sqrt_vjp(T x, T y, T yb, T& xb) {
  // y = sqrt(x); derivative 1/(2y), none at y = 0 (clamped or exact zero)
  if (y > T(0)) xb += mdiv(yb, T(2) * y);
}

// ===================================================================== 14 moments
struct Adj14 {
  using S = Sys14;

  // W = cons_to_prim(U): Ub += (dW/dU)^T Wb
  template <class T> MX_HD static void cons_to_prim_vjp(const T* U, const T* Wb_in, T* Ub) {
    // forward, kept
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
    // reverse
    T rhob = Wb_in[0];
    T ub[3] = {Wb_in[1], Wb_in[2], Wb_in[3]};
    T Pb[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) Pb[m] = Wb_in[4 + m];
    T qb[3] = {Wb_in[10], Wb_in[11], Wb_in[12]};
    T Rb = Wb_in[13];
    T uub = T(0), trPb = T(0), uPub = T(0), uqb = T(0), irb = T(0);
    T Pub[3] = {T(0), T(0), T(0)};
    // R = U13 - rho uu^2 - 2 uu trP - 4 uPu - 4 uq
    Ub[13] += Rb;
    rhob -= Rb * uu * uu;
    uub -= Rb * (T(2) * rho * uu + T(2) * trP);
    trPb -= T(2) * uu * Rb;
    uPub -= T(4) * Rb;
    uqb -= T(4) * Rb;
    // uq = u.q ; uPu = u.Pu
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] += uqb * q[i];
      qb[i] += uqb * u[i];
      ub[i] += uPub * Pu[i];
      Pub[i] += uPub * u[i];
    }
    // q_i = F_i - (rho uu) u_i - trP u_i - 2 Pu_i
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Ub[10 + i] += qb[i];
      rhob -= qb[i] * uu * u[i];
      uub -= qb[i] * rho * u[i];
      ub[i] -= qb[i] * (rho * uu + trP);
      trPb -= qb[i] * u[i];
      Pub[i] -= T(2) * qb[i];
    }
    // Pu = P u
    symv_vjp(P, u, Pub, Pb, ub);
    // trP, uu
    Pb[0] += trPb; Pb[3] += trPb; Pb[5] += trPb;
#pragma unroll
    for (int i = 0; i < 3; ++i) ub[i] += T(2) * uub * u[i];
    // P_ij = E_ij - rho (u_i u_j)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        T b = Pb[sidx(i, j)];
        Ub[4 + sidx(i, j)] += b;
        rhob -= b * (u[i] * u[j]);
        ub[i] -= b * rho * u[j];
        ub[j] -= b * rho * u[i];
      }
    // u_i = U_{1+i} ir ; ir = 1/rho
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Ub[1 + i] += ub[i] * ir;
      irb += ub[i] * U[1 + i];
    }
    rhob -= irb * ir * ir;
    Ub[0] += rhob;
  }

  // U = prim_to_cons(W): Wb += (dU/dW)^T Ub
  template <class T> MX_HD static void prim_to_cons_vjp(const T* W, const T* Ub, T* Wb) {
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
    T rhob = T(0), uub = T(0), trPb = T(0), uPub = T(0), uqb = T(0);
    T ub[3] = {T(0), T(0), T(0)}, Pub[3] = {T(0), T(0), T(0)};
    T* Pb = Wb + 4;
    T* qb = Wb + 10;
    // U13 = rho uu^2 + 2 uu trP + 4 uPu + 4 uq + R
    rhob += Ub[13] * uu * uu;
    uub += Ub[13] * (T(2) * rho * uu + T(2) * trP);
    trPb += T(2) * uu * Ub[13];
    uPub += T(4) * Ub[13];
    uqb += T(4) * Ub[13];
    Wb[13] += Ub[13];
    // U10+i = (rho uu) u_i + trP u_i + 2 Pu_i + q_i
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T b = Ub[10 + i];
      rhob += b * uu * u[i];
      uub += b * rho * u[i];
      ub[i] += b * (rho * uu + trP);
      trPb += b * u[i];
      Pub[i] += T(2) * b;
      qb[i] += b;
    }
    // U4+s = rho (u_i u_j) + P_s
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        T b = Ub[4 + sidx(i, j)];
        rhob += b * (u[i] * u[j]);
        ub[i] += b * rho * u[j];
        ub[j] += b * rho * u[i];
        Pb[sidx(i, j)] += b;
      }
    // U1+i = rho u_i ; U0 = rho
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      rhob += Ub[1 + i] * u[i];
      ub[i] += Ub[1 + i] * rho;
    }
    rhob += Ub[0];
    // uq, uPu, Pu, trP, uu
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] += uqb * q[i];
      qb[i] += uqb * u[i];
      ub[i] += uPub * Pu[i];
      Pub[i] += uPub * u[i];
    }
    symv_vjp(P, u, Pub, Pb, ub);
    Pb[0] += trPb; Pb[3] += trPb; Pb[5] += trPb;
#pragma unroll
    for (int i = 0; i < 3; ++i) ub[i] += T(2) * uub * u[i];
    Wb[0] += rhob;
#pragma unroll
    for (int i = 0; i < 3; ++i) Wb[1 + i] += ub[i];
  }

  // adjoint of the Core fields the downstream code reads
  template <class T> struct CoreB {
    T rho, c, Ph[6], qh[3], z[3], P2[6], t1, t2, sb;
  };

  template <class T> MX_HD static void zero(CoreB<T>& b) {
    b.rho = b.c = b.t1 = b.t2 = b.sb = T(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) { b.Ph[m] = T(0); b.P2[m] = T(0); }
#pragma unroll
    for (int i = 0; i < 3; ++i) { b.qh[i] = T(0); b.z[i] = T(0); }
  }

  // core(W) -> k: Wb += (dk/dW)^T kb
  template <class T>
  MX_HD static void core_vjp(const T* W, T sigma_lim, const CoreB<T>& kb_in, T* Wb) {
    // forward, kept
    T rho = W[0];
    T p = (W[4] + W[7] + W[9]) * T(1.0 / 3.0);
    T irho = mrcp(rho);
    T ip = mrcp(p);
    T c = msqrt(p * irho);
    T ic = msqrt(rho * ip);
    T Ph[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) Ph[m] = W[4 + m] * ip;
    T ic3 = ic * ic * ic;
    T is3 = irho * ic3;
    T qh[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) qh[i] = W[10 + i] * is3;
    T is4 = is3 * ic;
    T Rh = W[13] * is4;
    T t1 = Ph[0] + Ph[3] + Ph[5];
    T P2[6];
    symsq(Ph, P2);
    T t2 = P2[0] + P2[3] + P2[5];
    T C[6];
    T det = symadj(Ph, C);
    T idet = mrcp(det);
    T y[3];
    symv(C, qh, y);
    T z[3] = {y[0] * idet, y[1] * idet, y[2] * idet};
    T D = qh[0] * z[0] + qh[1] * z[1] + qh[2] * z[2];
    T A = T(2) * t2 + t1 * t1 - Rh;
    T X = A * A + T(8) * t2 * D;
    T sX = msqrt(X);
    bool apos = A >= T(0);
    T num = apos ? (A + sX) : T(2) * D;
    T den = apos ? T(4) * t2 : (sX - A);
    T sig = mdiv(num, den);
    // reverse
    T Phb[6], P2b[6], qhb[3], zb[3];
#pragma unroll
    for (int m = 0; m < 6; ++m) { Phb[m] = kb_in.Ph[m]; P2b[m] = kb_in.P2[m]; }
#pragma unroll
    for (int i = 0; i < 3; ++i) { qhb[i] = kb_in.qh[i]; zb[i] = kb_in.z[i]; }
    T rhob = kb_in.rho, cb = kb_in.c, t1b = kb_in.t1, t2b = kb_in.t2;
    T sigb = (sig > sigma_lim) ? kb_in.sb : T(0);  // sigma_bar = max(sigma, sigma_lim)
    T iden = mrcp(den);
    T numb = sigb * iden;
    T denb = -sigb * sig * iden;
    T Ab = T(0), sXb = T(0), Db = T(0);
    if (apos) {
      Ab += numb;
      sXb += numb;
      t2b += T(4) * denb;
    } else {
      Db += T(2) * numb;
      sXb += denb;
      Ab -= denb;
    }
    T Xb = T(0);
    sqrt_vjp(X, sX, sXb, Xb);
    Ab += T(2) * A * Xb;
    t2b += T(8) * D * Xb;
    Db += T(8) * t2 * Xb;
    // A = 2 t2 + t1^2 - Rh
    t2b += T(2) * Ab;
    t1b += T(2) * t1 * Ab;
    T Rhb = -Ab;
    // D = qh . z
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      qhb[i] += Db * z[i];
      zb[i] += Db * qh[i];
    }
    // z = y idet ; y = C qh ; idet = 1/det
    T yb[3], idetb = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      yb[i] = zb[i] * idet;
      idetb += zb[i] * y[i];
    }
    T Cb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    symv_vjp(C, qh, yb, Cb, qhb);
    T detb = -idetb * idet * idet;
    symadj_vjp(Ph, C, Cb, detb, Phb);
    // t2 = tr P2 ; P2 = Ph^2 ; t1 = tr Ph
    P2b[0] += t2b; P2b[3] += t2b; P2b[5] += t2b;
    symsq_vjp(Ph, P2b, Phb);
    Phb[0] += t1b; Phb[3] += t1b; Phb[5] += t1b;
    // Rh = W13 is4 ; is4 = is3 ic ; qh = W10 is3 ; is3 = irho ic3
    T is4b = Rhb * W[13];
    Wb[13] += Rhb * is4;
    T is3b = is4b * ic;
    T icb = is4b * is3;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Wb[10 + i] += qhb[i] * is3;
      is3b += qhb[i] * W[10 + i];
    }
    T irhob = is3b * ic3;
    icb += is3b * irho * T(3) * ic * ic;
    // Ph = W4 ip
    T ipb = T(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      Wb[4 + m] += Phb[m] * ip;
      ipb += Phb[m] * W[4 + m];
    }
    // ic = sqrt(rho ip) ; c = sqrt(p irho)
    T riv = T(0), piv = T(0);
    sqrt_vjp(rho * ip, ic, icb, riv);
    sqrt_vjp(p * irho, c, cb, piv);
    rhob += riv * ip;
    ipb += riv * rho;
    T pb = piv * irho;
    irhob += piv * p;
    // ip = 1/p ; irho = 1/rho
    pb -= ipb * ip * ip;
    rhob -= irhob * irho * irho;
    // p = (W4 + W7 + W9)/3 ; rho = W0
    T pb3 = pb * T(1.0 / 3.0);
    Wb[4] += pb3; Wb[7] += pb3; Wb[9] += pb3;
    Wb[0] += rhob;
  }

  // closure_dir<d>(k) -> (Qd, Rd, Sd): kb += ...
  template <int d, class T>
  MX_HD static void closure_dir_vjp(const S::Core<T>& k, const T* Qdb, const T* Rdb, T Sdb,
                                    CoreB<T>& kb) {
    // forward, kept
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
    T c2 = k.c * k.c;
    T c3 = k.c * c2;
    T s3 = k.rho * c3;
    T s4 = s3 * k.c;
    T s5 = s4 * k.c;
    T isb = mrcp(k.sb);
    T Pw[3], P2w[3];
    symv(k.Ph, w, Pw);
    symv(k.P2, w, P2w);
    T t3 = k.P2[0] * k.Ph[0] + k.P2[3] * k.Ph[3] + k.P2[5] * k.Ph[5] +
           T(2) * (k.P2[1] * k.Ph[1] + k.P2[2] * k.Ph[2] + k.P2[4] * k.Ph[4]);
    T P3w_d = k.P2[sidx(d, 0)] * Pw[0] + k.P2[sidx(d, 1)] * Pw[1] + k.P2[sidx(d, 2)] * Pw[2];
    T t1 = k.t1, t2 = k.t2;
    T cw = T(2) * t1 * t1 * t1 + T(12) * t3 - T(2) * t2 * t1;
    T cpw = T(14) * t2 - T(6) * t1 * t1;
    T Wq = cw * w[d] + cpw * Pw[d] + T(20) * t1 * P2w[d] + T(20) * P3w_d;
    T Qzz = T(2) * (w[d] * zP2z + T(2) * wz * P2z[d]);
    T rsb = msqrt(k.sb);
    T isb2 = isb * isb;
    T inner = Qzz * isb2 + T(2) * rsb * t1 * k.qh[d] + (T(1) - rsb) * Wq;
    // reverse
    T wb[3] = {T(0), T(0), T(0)}, P2zb[3] = {T(0), T(0), T(0)};
    T zP2zb = T(0), wzb = T(0), s3b = T(0), s4b = T(0), s5b = T(0), isbb = T(0);
    // Sd = inner * s5
    T innerb = Sdb * s5;
    s5b += Sdb * inner;
    T Qzzb = innerb * isb2;
    T isb2b = innerb * Qzz;
    T rsbb = innerb * (T(2) * t1 * k.qh[d] - Wq);
    kb.t1 += innerb * T(2) * rsb * k.qh[d];
    kb.qh[d] += innerb * T(2) * rsb * t1;
    T Wqb = innerb * (T(1) - rsb);
    isbb += isb2b * T(2) * isb;
    sqrt_vjp(k.sb, rsb, rsbb, kb.sb);
    // Qzz = 2 (w_d zP2z + 2 wz P2z_d)
    wb[d] += T(2) * Qzzb * zP2z;
    zP2zb += T(2) * Qzzb * w[d];
    wzb += T(4) * Qzzb * P2z[d];
    P2zb[d] += T(4) * Qzzb * wz;
    // Wq = cw w_d + cpw Pw_d + 20 t1 P2w_d + 20 P3w_d
    T cwb = Wqb * w[d];
    wb[d] += Wqb * cw;
    T cpwb = Wqb * Pw[d];
    T Pwb[3] = {T(0), T(0), T(0)}, P2wb[3] = {T(0), T(0), T(0)};
    Pwb[d] += Wqb * cpw;
    kb.t1 += Wqb * T(20) * P2w[d];
    P2wb[d] += Wqb * T(20) * t1;
    T P3wb = Wqb * T(20);
    // cw, cpw
    kb.t1 += cwb * (T(6) * t1 * t1 - T(2) * t2) - cpwb * T(12) * t1;
    T t3b = cwb * T(12);
    kb.t2 += -cwb * T(2) * t1 + cpwb * T(14);
    // P3w_d = sum_m P2[d,m] Pw_m
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      kb.P2[sidx(d, m)] += P3wb * Pw[m];
      Pwb[m] += P3wb * k.P2[sidx(d, m)];
    }
    // t3
    kb.P2[0] += t3b * k.Ph[0]; kb.Ph[0] += t3b * k.P2[0];
    kb.P2[3] += t3b * k.Ph[3]; kb.Ph[3] += t3b * k.P2[3];
    kb.P2[5] += t3b * k.Ph[5]; kb.Ph[5] += t3b * k.P2[5];
    kb.P2[1] += T(2) * t3b * k.Ph[1]; kb.Ph[1] += T(2) * t3b * k.P2[1];
    kb.P2[2] += T(2) * t3b * k.Ph[2]; kb.Ph[2] += T(2) * t3b * k.P2[2];
    kb.P2[4] += T(2) * t3b * k.Ph[4]; kb.Ph[4] += T(2) * t3b * k.P2[4];
    // P2w = P2 w ; Pw = Ph w
    symv_vjp(k.P2, w, P2wb, kb.P2, wb);
    symv_vjp(k.Ph, w, Pwb, kb.Ph, wb);
    // Rd_i = (Qz_i isb + 2 (1 - sb) P2[i,d] + t1 Ph[i,d]) s4,
    // Qz_i = 2 (w_i P2z_d + w_d P2z_i + wz P2[i,d])
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T Qz = T(2) * (w[i] * P2z[d] + w[d] * P2z[i] + wz * k.P2[sidx(i, d)]);
      T inn = Qz * isb + T(2) * (T(1) - k.sb) * k.P2[sidx(i, d)] + t1 * k.Ph[sidx(i, d)];
      T innb = Rdb[i] * s4;
      s4b += Rdb[i] * inn;
      T Qzb = innb * isb;
      isbb += innb * Qz;
      kb.sb -= innb * T(2) * k.P2[sidx(i, d)];
      kb.P2[sidx(i, d)] += innb * T(2) * (T(1) - k.sb);
      kb.t1 += innb * k.Ph[sidx(i, d)];
      kb.Ph[sidx(i, d)] += innb * t1;
      wb[i] += T(2) * Qzb * P2z[d];
      P2zb[d] += T(2) * Qzb * w[i];
      wb[d] += T(2) * Qzb * P2z[i];
      P2zb[i] += T(2) * Qzb * w[d];
      wzb += T(2) * Qzb * k.P2[sidx(i, d)];
      kb.P2[sidx(i, d)] += T(2) * Qzb * wz;
    }
    // isb = 1/sb
    kb.sb -= isbb * isb * isb;
    // Qd_ij = 2 (w_i P2[j,d] + w_j P2[i,d] + w_d P2[i,j]) s3
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        T b = Qdb[sidx(i, j)];
        T inn = T(2) * (w[i] * k.P2[sidx(j, d)] + w[j] * k.P2[sidx(i, d)] + w[d] * k.P2[sidx(i, j)]);
        s3b += b * inn;
        T ib = T(2) * b * s3;
        wb[i] += ib * k.P2[sidx(j, d)];
        kb.P2[sidx(j, d)] += ib * w[i];
        wb[j] += ib * k.P2[sidx(i, d)];
        kb.P2[sidx(i, d)] += ib * w[j];
        wb[d] += ib * k.P2[sidx(i, j)];
        kb.P2[sidx(i, j)] += ib * w[d];
      }
    // s5 = s4 c ; s4 = s3 c ; s3 = rho c3 ; c3 = c c2 ; c2 = c c
    s4b += s5b * k.c;
    T cb = s5b * s4;
    s3b += s4b * k.c;
    cb += s4b * s3;
    kb.rho += s3b * c3;
    T c3b = s3b * k.rho;
    cb += c3b * c2;
    T c2b = c3b * k.c;
    cb += T(2) * c2b * k.c;
    kb.c += cb;
    // wz = w . z ; zP2z = z . P2z ; P2z = P2 z
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      wb[i] += wzb * k.z[i];
      kb.z[i] += wzb * w[i];
      kb.z[i] += zP2zb * P2z[i];
      P2zb[i] += zP2zb * k.z[i];
    }
    symv_vjp(k.P2, k.z, P2zb, kb.P2, kb.z);
    // w = y idc ; y = Ca qh ; idc = 1/detc ; (Ca, detc) = adj(Cm)
    T yb[3], idcb = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      yb[i] = wb[i] * idc;
      idcb += wb[i] * y[i];
    }
    T Cab[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    symv_vjp(Ca, k.qh, yb, Cab, kb.qh);
    T detcb = -idcb * idc * idc;
    T Cmb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    symadj_vjp(Cm, Ca, Cab, detcb, Cmb);
    // Cm = 4 P2 + 2 t2 I
#pragma unroll
    for (int m = 0; m < 6; ++m) kb.P2[m] += T(4) * Cmb[m];
    kb.t2 += T(2) * (Cmb[0] + Cmb[3] + Cmb[5]);
  }

  // hyperbola(zeta, rest) reverse
  template <class T> MX_HD static void hyperbola_vjp(T zeta, T rest, T hb, T& zetab, T& restb) {
    // the partials are formed in locals and added once at the end (no branch writes through
    // the references, which keeps both callers' accumulators in registers)
    T X = zeta * zeta + rest;
    T zb = hb, rb = T(0);
    if (X > T(0)) {
      T sX = msqrt(X);
      T Xb = T(0);
      if (zeta >= T(0)) {
        sqrt_vjp(X, sX, hb, Xb);
      } else {
        T den = sX - zeta;
        T h = mdiv(rest, den);
        T iden = mrcp(den);
        rb = hb * iden;
        T denb = -hb * h * iden;
        sqrt_vjp(X, sX, denb, Xb);
        zb = -denb;
      }
      zb += T(2) * zeta * Xb;
      rb += Xb;
    }
    zetab += zb;
    restb += rb;
  }

  // wavespeeds<d>(k, ud) -> (lmin, lmax): kb, udb
  template <int d, class T>
  MX_HD static void wavespeeds_vjp(const S::Core<T>& k, T ud, T kws, T lminb, T lmaxb, CoreB<T>& kb,
                                   T& udb) {
    constexpr int t1i = (d == 0) ? 1 : 0;
    constexpr int t2i = (d == 2) ? 1 : 2;
    // forward, kept
    bool sw_clamp = !(k.sb < T(1));
    T sw = sw_clamp ? T(1) : k.sb;
    T Pdd_raw = k.Ph[sidx(d, d)];
    bool Pclamp = !(Pdd_raw > T(0));
    T Pdd = Pclamp ? T(0) : Pdd_raw;
    T qd = k.qh[d];
    T qt2 = k.qh[t1i] * k.qh[t1i] + k.qh[t2i] * k.qh[t2i];
    T qt = msqrt(qt2);
    T alpha = T(0.6) * Pdd * Pdd - T(0.38) * Pdd + T(0.35);
    T a = T(0), b = T(0), lP = T(0), ea = T(0), e14 = T(0), eb = T(0);
    if (Pdd > T(0)) {
      lP = mlog(Pdd);
      ea = mexp(T(1.1) * lP - Pdd * Pdd);
      a = T(1.4) * ea;
      e14 = mexp(T(1.4) * lP);
      eb = mexp(T(-0.5) * e14);
      b = T(0.9) * Pdd * eb;
    }
    // byec(sw, Pdd)
    T Carg = (T(3) - T(3) * sw) * Pdd;
    bool Cclamp = !(Carg > T(0));
    T Cc = Cclamp ? T(0) : msqrt(Carg);
    T E = T(0.8) * Cc;
    T rs = msqrt(sw);
    T Barg = T(10) - T(16) * rs + T(6) * sw;
    bool Bclamp = !(Barg > T(0));
    T sBa = Bclamp ? T(0) : msqrt(Barg);
    T B = T(5) - T(4) * rs + sBa;
    T sB = msqrt(B);
    T Y = B + E * E - T(2) * E * sB;
    T twosw = T(2) * sw;
    T pref = mdiv(a * sw + b, twosw);
    T base = T(4) * sw * sw * Y + qt * qt * T(0.1);
    T zmax = qd + qt * alpha;
    T zmin = -qd + qt * alpha;
    T rmax = T(-0.8) * zmax * sw * Cc + base;
    T rmin = T(-0.8) * zmin * sw * Cc + base;
    T hmax = hyperbola(zmax, rmax);
    T hmin = hyperbola(zmin, rmin);
    T Lmax = pref * hmax + E;
    T Lmin = pref * hmin + E;
    // reverse: lmax = ud + kws Lmax c ; lmin = ud - kws Lmin c
    udb += lmaxb + lminb;
    T Lmaxb = lmaxb * kws * k.c;
    T Lminb = -lminb * kws * k.c;
    kb.c += lmaxb * kws * Lmax - lminb * kws * Lmin;
    T prefb = Lmaxb * hmax + Lminb * hmin;
    T hmaxb = Lmaxb * pref, hminb = Lminb * pref;
    T Eb = Lmaxb + Lminb;
    T zmaxb = T(0), rmaxb = T(0), zminb = T(0), rminb = T(0);
    hyperbola_vjp(zmax, rmax, hmaxb, zmaxb, rmaxb);
    hyperbola_vjp(zmin, rmin, hminb, zminb, rminb);
    T baseb = rmaxb + rminb;
    T swb = T(0), Ccb = T(0), qtb = T(0), alphab = T(0), qdb = T(0);
    zmaxb += rmaxb * T(-0.8) * sw * Cc;
    swb += rmaxb * T(-0.8) * zmax * Cc;
    Ccb += rmaxb * T(-0.8) * zmax * sw;
    zminb += rminb * T(-0.8) * sw * Cc;
    swb += rminb * T(-0.8) * zmin * Cc;
    Ccb += rminb * T(-0.8) * zmin * sw;
    // zmax = qd + qt alpha ; zmin = -qd + qt alpha
    qdb += zmaxb - zminb;
    qtb += (zmaxb + zminb) * alpha;
    alphab += (zmaxb + zminb) * qt;
    // base = 4 sw^2 Y + 0.1 qt^2
    swb += baseb * T(8) * sw * Y;
    T Yb = baseb * T(4) * sw * sw;
    qtb += baseb * T(0.2) * qt;
    // pref = (a sw + b) / (2 sw)
    T itw = mrcp(twosw);
    T ab = prefb * sw * itw;
    T bb = prefb * itw;
    swb += prefb * (a - T(2) * pref) * itw;
    // Y = B + E^2 - 2 E sB
    T Bb = Yb;
    Eb += Yb * (T(2) * E - T(2) * sB);
    T sBb = -Yb * T(2) * E;
    sqrt_vjp(B, sB, sBb, Bb);
    // B = 5 - 4 rs + sBa
    T rsb = -T(4) * Bb;
    T sBab = Bb;
    T Bargb = T(0);
    if (!Bclamp) sqrt_vjp(Barg, sBa, sBab, Bargb);
    rsb += -T(16) * Bargb;
    swb += T(6) * Bargb;
    sqrt_vjp(sw, rs, rsb, swb);
    // E = 0.8 Cc ; Cc = sqrt((3 - 3 sw) Pdd)
    Ccb += T(0.8) * Eb;
    T Cargb = T(0);
    if (!Cclamp) sqrt_vjp(Carg, Cc, Ccb, Cargb);
    swb += -T(3) * Pdd * Cargb;
    T Pddb = (T(3) - T(3) * sw) * Cargb;
    // a, b
    if (Pdd > T(0)) {
      // b = 0.9 Pdd eb ; eb = exp(-0.5 e14) ; e14 = exp(1.4 lP)
      Pddb += bb * T(0.9) * eb;
      T ebb = bb * T(0.9) * Pdd;
      T e14b = ebb * eb * T(-0.5);
      T lPb = e14b * e14 * T(1.4);
      // a = 1.4 ea ; ea = exp(1.1 lP - Pdd^2)
      T eab = ab * T(1.4);
      T argb = eab * ea;
      lPb += argb * T(1.1);
      Pddb += -argb * T(2) * Pdd;
      Pddb += mdiv(lPb, Pdd);
    }
    // alpha = 0.6 Pdd^2 - 0.38 Pdd + 0.35
    Pddb += alphab * (T(1.2) * Pdd - T(0.38));
    // qt = sqrt(qt2)
    T qt2b = T(0);
    sqrt_vjp(qt2, qt, qtb, qt2b);
    kb.qh[t1i] += qt2b * T(2) * k.qh[t1i];
    kb.qh[t2i] += qt2b * T(2) * k.qh[t2i];
    kb.qh[d] += qdb;
    if (!Pclamp) kb.Ph[sidx(d, d)] += Pddb;
    if (!sw_clamp) kb.sb += swb;
  }

  // face_terms<d>(W) -> (U, F, lmin, lmax): Wb += ...
  template <int d, class T>
  MX_HD static void face_terms_vjp(const T* W, T sigma_lim, T kws, const T* Ub, const T* Fb, T lminb,
                                   T lmaxb, T* Wb) {
    S::Core<T> k;
    S::core(W, sigma_lim, k);
    T Qd[6], Rd[3], Sd;
    S::closure_dir<d>(k, Qd, Rd, Sd);
    face_terms_vjp_prepared<d>(k, Qd, Rd, Sd, W, sigma_lim, kws, Ub, Fb, lminb, lmaxb, Wb);
  }

  // the same reverse from the forward's own core k = core(W) and closing values
  // (Qd, Rd, Sd) = closure_dir<d>(k), for a caller that has just evaluated them
  template <int d, class T>
  MX_HD static void face_terms_vjp_prepared(const typename S::template Core<T>& k, const T* Qd,
                                            const T* Rd, T Sd, const T* W, T sigma_lim, T kws,
                                            const T* Ub, const T* Fb, T lminb, T lmaxb, T* Wb) {
    CoreB<T> kb;
    zero(kb);
    T udb = T(0);
    wavespeeds_vjp<d>(k, W[1 + d], kws, lminb, lmaxb, kb, udb);
    face_terms_vjp_rest<d>(k, Qd, Rd, Sd, W, sigma_lim, Ub, Fb, kb, udb, Wb);
  }

  // the same reverse after the wave speeds' (kb and udb: their partials of the core and of
  // u_d), so that a caller can reverse the wave speeds while their forward values are live
  template <int d, class T>
  MX_HD static void face_terms_vjp_rest(const typename S::template Core<T>& k, const T* Qd,
                                        const T* Rd, T Sd, const T* W, T sigma_lim, const T* Ub,
                                        const T* Fb, CoreB<T>& kb, T udb, T* Wb) {
    T Qdb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T Rdb[3] = {T(0), T(0), T(0)};
    T Sdb = T(0);
    flux_vjp<d>(W, Qd, Rd, Sd, Fb, Wb, Qdb, Rdb, Sdb);
    prim_to_cons_vjp(W, Ub, Wb);
    Wb[1 + d] += udb;
    closure_dir_vjp<d>(k, Qdb, Rdb, Sdb, kb);
    // core_vjp's forward part depends on W alone: launder W and the accumulated partials so
    // that it is evaluated here, after the closure reverse, not earlier with its values held
    T Wl[14];
#pragma unroll
    for (int v = 0; v < 14; ++v) {
      Wl[v] = W[v];
      opaque(Wl[v]);
      opaque(Wb[v]);
    }
    opaque_b(kb);
    core_vjp(Wl, sigma_lim, kb, Wb);
  }

  template <class T> MX_HD static void opaque_b(CoreB<T>& kb) {
    opaque(kb.rho); opaque(kb.c); opaque(kb.t1); opaque(kb.t2); opaque(kb.sb);
#pragma unroll
    for (int m = 0; m < 6; ++m) { opaque(kb.Ph[m]); opaque(kb.P2[m]); }
#pragma unroll
    for (int i = 0; i < 3; ++i) { opaque(kb.qh[i]); opaque(kb.z[i]); }
  }

  // flux<d>(W, Qd, Rd, Sd) -> F: reverse
  template <int d, class T>
  MX_HD static void flux_vjp(const T* W, const T* Qd, const T* Rd, T Sd, const T* Fb, T* Wb, T* Qdb,
                             T* Rdb, T& Sdb) {
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
    // adjoints of intermediates
    T rhob = T(0), ub[3] = {T(0), T(0), T(0)}, Pb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T qb[3] = {T(0), T(0), T(0)};
    T udb = T(0), uub = T(0), trPb = T(0), uPdb = T(0), uPub = T(0), uqb = T(0), uQub = T(0),
      uRb = T(0), rudb = T(0);
    T Pdb[3] = {T(0), T(0), T(0)}, Pub[3] = {T(0), T(0), T(0)}, Qub[3] = {T(0), T(0), T(0)};
    T Rb = T(0);
    // F13 = rud uu uu + 2 ud uu trP + 4 uu uPd + 4 ud uPu + 2 uu q_d + 4 ud uq + 4 uQu + 4 uR
    //       + ud R + Sd
    {
      T b = Fb[13];
      rudb += b * uu * uu;
      uub += b * (T(2) * rud * uu + T(2) * ud * trP + T(4) * uPd + T(2) * q[d]);
      udb += b * (T(2) * uu * trP + T(4) * uPu + T(4) * uq + W[13]);
      trPb += b * T(2) * ud * uu;
      uPdb += b * T(4) * uu;
      uPub += b * T(4) * ud;
      qb[d] += b * T(2) * uu;
      uqb += b * T(4) * ud;
      uQub += b * T(4);
      uRb += b * T(4);
      Rb += b * ud;
      Sdb += b;
    }
    // F10+i = rud uu u_i + ud trP u_i + 2 uPd u_i + 2 ud Pu_i + uu Pd_i + u_i q_d + ud q_i
    //         + 2 Qu_i + Rd_i
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T b = Fb[10 + i];
      rudb += b * uu * u[i];
      uub += b * (rud * u[i] + Pd[i]);
      ub[i] += b * (rud * uu + ud * trP + T(2) * uPd + q[d]);
      udb += b * (trP * u[i] + T(2) * Pu[i] + q[i]);
      trPb += b * ud * u[i];
      uPdb += b * T(2) * u[i];
      Pub[i] += b * T(2) * ud;
      Pdb[i] += b * uu;
      qb[d] += b * u[i];
      qb[i] += b * ud;
      Qub[i] += b * T(2);
      Rdb[i] += b;
    }
    // F4+s = rud (u_i u_j) + u_i Pd_j + u_j Pd_i + ud P_s + Qd_s
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        T b = Fb[4 + sidx(i, j)];
        rudb += b * (u[i] * u[j]);
        ub[i] += b * (rud * u[j] + Pd[j]);
        ub[j] += b * (rud * u[i] + Pd[i]);
        Pdb[j] += b * u[i];
        Pdb[i] += b * u[j];
        udb += b * P[sidx(i, j)];
        Pb[sidx(i, j)] += b * ud;
        Qdb[sidx(i, j)] += b;
      }
    // F1+i = rud u_i + Pd_i ; F0 = rud
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      rudb += Fb[1 + i] * u[i];
      ub[i] += Fb[1 + i] * rud;
      Pdb[i] += Fb[1 + i];
    }
    rudb += Fb[0];
    // rud = rho ud
    rhob += rudb * ud;
    udb += rudb * rho;
    // uR = u . Rd ; uQu = u . Qu ; Qu = Qd u
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] += uRb * Rd[i];
      Rdb[i] += uRb * u[i];
      ub[i] += uQub * Qu[i];
      Qub[i] += uQub * u[i];
    }
    symv_vjp(Qd, u, Qub, Qdb, ub);
    // uq, uPu, Pu
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] += uqb * q[i];
      qb[i] += uqb * u[i];
      ub[i] += uPub * Pu[i];
      Pub[i] += uPub * u[i];
    }
    symv_vjp(P, u, Pub, Pb, ub);
    // uPd = u . Pd ; Pd_i = P[i,d]
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] += uPdb * Pd[i];
      Pdb[i] += uPdb * u[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) Pb[sidx(i, d)] += Pdb[i];
    // trP, uu, ud
    Pb[0] += trPb; Pb[3] += trPb; Pb[5] += trPb;
#pragma unroll
    for (int i = 0; i < 3; ++i) ub[i] += T(2) * uub * u[i];
    ub[d] += udb;
    Wb[0] += rhob;
#pragma unroll
    for (int i = 0; i < 3; ++i) { Wb[1 + i] += ub[i]; Wb[10 + i] += qb[i]; }
#pragma unroll
    for (int m = 0; m < 6; ++m) Wb[4 + m] += Pb[m];
    Wb[13] += Rb;
  }

  // BGK source with inv_tau = 1/tau.  Local tau: inv_tau = kappa sqrt(rho p) with kappa fixed
  // by tau_ref, rho_ref, T_ref, so d inv_tau/d rho = inv_tau/(2 rho), d inv_tau/d p =
  // inv_tau/(2 p).  Reverse: Wb += (dC/dW)^T Cb, and returns Cb . C (for d/d tau_ref:
  // dC/d tau_ref = -C / tau_ref).
  template <class T>
  MX_HD static T source_vjp(const T* W, T inv_tau, bool local_tau, const T* Cb, T* Wb) {
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
    // C = -B inv_tau
    T Bv[14];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) Bv[4 + sidx(i, j)] = P[sidx(i, j)] - (i == j ? p : T(0));
#pragma unroll
    for (int i = 0; i < 3; ++i) Bv[10 + i] = T(2) * Pu[i] + q[i] - T(2) * u[i] * p;
    Bv[13] = (T(4) * uPu + T(4) * uq + W[13]) - (T(4) * uu * p + mdiv(T(15) * p * p, rho));
    T cdotb = T(0);  // Cb . C
    T itb = T(0);    // adjoint of inv_tau
    T Bb[14];
#pragma unroll
    for (int v = 4; v < 14; ++v) {
      T C = -Bv[v] * inv_tau;
      cdotb += Cb[v] * C;
      Bb[v] = -Cb[v] * inv_tau;
      itb -= Cb[v] * Bv[v];
    }
    T rhob = T(0), ub[3] = {T(0), T(0), T(0)}, Pb[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T qb[3] = {T(0), T(0), T(0)}, pb = T(0), Pub[3] = {T(0), T(0), T(0)};
    T uPub = T(0), uqb = T(0), uub = T(0);
    // B13
    uPub += T(4) * Bb[13];
    uqb += T(4) * Bb[13];
    Wb[13] += Bb[13];
    uub -= T(4) * p * Bb[13];
    const T irho = mrcp(rho);
    pb -= Bb[13] * (T(4) * uu + T(30) * p * irho);
    rhob += Bb[13] * T(15) * p * p * irho * irho;
    // B10+i = 2 Pu_i + q_i - 2 u_i p
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Pub[i] += T(2) * Bb[10 + i];
      qb[i] += Bb[10 + i];
      ub[i] -= T(2) * p * Bb[10 + i];
      pb -= T(2) * u[i] * Bb[10 + i];
    }
    // B4+s = P_s - p delta
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = i; j < 3; ++j) {
        Pb[sidx(i, j)] += Bb[4 + sidx(i, j)];
        if (i == j) pb -= Bb[4 + sidx(i, j)];
      }
    // inv_tau = kappa sqrt(rho p) (local)
    if (local_tau) {
      rhob += itb * inv_tau * T(0.5) * irho;
      pb += itb * inv_tau * T(0.5) * mrcp(p);
    }
    // uu, uq, uPu, Pu
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      ub[i] += T(2) * uub * u[i];
      ub[i] += uqb * q[i];
      qb[i] += uqb * u[i];
      ub[i] += uPub * Pu[i];
      Pub[i] += uPub * u[i];
    }
    symv_vjp(P, u, Pub, Pb, ub);
    T pb3 = pb * T(1.0 / 3.0);
    Pb[0] += pb3; Pb[3] += pb3; Pb[5] += pb3;
    Wb[0] += rhob;
#pragma unroll
    for (int i = 0; i < 3; ++i) { Wb[1 + i] += ub[i]; Wb[10 + i] += qb[i]; }
#pragma unroll
    for (int m = 0; m < 6; ++m) Wb[4 + m] += Pb[m];
    return cdotb;
  }

  // Reverse of the HLL / Rusanov combination of two face states' (U, F, lambda_min,
  // lambda_max): given Fhb, sets the adjoints of both sides' U, F and speeds (overwritten).
  template <class T>
  MX_HD static void interface_vjp(const T* UL, const T* FL, T lminL, T lmaxL, const T* UR,
                                  const T* FR, T lminR, T lmaxR, int flux_kind, const T* Fhb,
                                  T* ULb, T* FLb, T& lminLb, T& lmaxLb, T* URb, T* FRb, T& lminRb,
                                  T& lmaxRb) {
    constexpr int NV = 14;
#pragma unroll
    for (int v = 0; v < NV; ++v) { ULb[v] = FLb[v] = URb[v] = FRb[v] = T(0); }
    lminLb = lmaxLb = lminRb = lmaxRb = T(0);
    if (flux_kind == 0) {
      T SL = tmin(lminL, lminR), SR = tmax(lmaxL, lmaxR);
      if (SL >= T(0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) FLb[v] = Fhb[v];
      } else if (SR <= T(0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) FRb[v] = Fhb[v];
      } else {
        T inv = mrcp(SR - SL);
        T SLR = SL * SR;
        T SLb = T(0), SRb = T(0), invb = T(0), SLRb = T(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          T num = SR * FL[v] - SL * FR[v] + SLR * (UR[v] - UL[v]);
          T nb = Fhb[v] * inv;
          invb += Fhb[v] * num;
          SRb += nb * FL[v];
          FLb[v] += nb * SR;
          SLb -= nb * FR[v];
          FRb[v] -= nb * SL;
          SLRb += nb * (UR[v] - UL[v]);
          URb[v] += nb * SLR;
          ULb[v] -= nb * SLR;
        }
        SLb += SLRb * SR;
        SRb += SLRb * SL;
        T db = -invb * inv * inv;  // d/d(SR - SL)
        SRb += db;
        SLb -= db;
        // SL = min(lminL, lminR), SR = max(lmaxL, lmaxR): the branch the forward took
        if (lminL < lminR) lminLb += SLb; else lminRb += SLb;
        if (lmaxL > lmaxR) lmaxLb += SRb; else lmaxRb += SRb;
      }
    } else {
      T aL1 = tabs(lminL), aL2 = tabs(lmaxL), aR1 = tabs(lminR), aR2 = tabs(lmaxR);
      T mL = tmax(aL1, aL2), mR = tmax(aR1, aR2);
      T am = tmax(mL, mR);
      T amb = T(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        FLb[v] += T(0.5) * Fhb[v];
        FRb[v] += T(0.5) * Fhb[v];
        amb -= T(0.5) * Fhb[v] * (UR[v] - UL[v]);
        URb[v] -= T(0.5) * am * Fhb[v];
        ULb[v] += T(0.5) * am * Fhb[v];
      }
      // am = max(max(|lminL|, |lmaxL|), max(|lminR|, |lmaxR|)): the branch taken
      if (mL > mR) {
        if (aL1 > aL2) lminLb += amb * (lminL < T(0) ? T(-1) : T(1));
        else lmaxLb += amb * (lmaxL < T(0) ? T(-1) : T(1));
      } else {
        if (aR1 > aR2) lminRb += amb * (lminR < T(0) ? T(-1) : T(1));
        else lmaxRb += amb * (lmaxR < T(0) ? T(-1) : T(1));
      }
    }
  }

  // One side's share of interface_vjp, for two threads that each own one face state of the
  // face.  Besides its own side it needs only both sides' wave speeds and the products
  // aFL = Fhb . FL, aFR = Fhb . FR, aUL = Fhb . UL, aUR = Fhb . UR, which each side forms from
  // its own U and F.  Same branches and tie rules as interface_vjp; the sums over the 14
  // components are taken before the scalar factors are applied (rounding order differs).
  template <class T>
  MX_HD static void interface_side_vjp(bool right, T lminL, T lmaxL, T lminR, T lmaxR, T aFL, T aFR,
                                       T aUL, T aUR, int flux_kind, const T* Fhb, T* Ub, T* Fb,
                                       T& lminb, T& lmaxb) {
    constexpr int NV = 14;
#pragma unroll
    for (int v = 0; v < NV; ++v) { Ub[v] = Fb[v] = T(0); }
    lminb = lmaxb = T(0);
    if (flux_kind == 0) {
      T SL = tmin(lminL, lminR), SR = tmax(lmaxL, lmaxR);
      if (SL >= T(0)) {
        if (!right) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fb[v] = Fhb[v];
        }
      } else if (SR <= T(0)) {
        if (right) {
#pragma unroll
          for (int v = 0; v < NV; ++v) Fb[v] = Fhb[v];
        }
      } else {
        T inv = mrcp(SR - SL);
        T SLR = SL * SR;
        // F = (SR FL - SL FR + SL SR (UR - UL)) inv
        T invb = SR * aFL - SL * aFR + SLR * (aUR - aUL);
        T SRb = inv * aFL;
        T SLb = -(inv * aFR);
        T SLRb = inv * (aUR - aUL);
        const T cF = right ? -SL : SR;
        const T cU = right ? SLR : -SLR;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          T nb = Fhb[v] * inv;
          Fb[v] = nb * cF;
          Ub[v] = nb * cU;
        }
        SLb += SLRb * SR;
        SRb += SLRb * SL;
        T db = -invb * inv * inv;  // d/d(SR - SL)
        SRb += db;
        SLb -= db;
        // SL = min(lminL, lminR), SR = max(lmaxL, lmaxR): the branch the forward took
        if ((lminL < lminR) != right) lminb = SLb;
        if ((lmaxL > lmaxR) != right) lmaxb = SRb;
      }
    } else {
      T aL1 = tabs(lminL), aL2 = tabs(lmaxL), aR1 = tabs(lminR), aR2 = tabs(lmaxR);
      T mL = tmax(aL1, aL2), mR = tmax(aR1, aR2);
      T am = tmax(mL, mR);
      T amb = -(T(0.5) * (aUR - aUL));
      const T cU = right ? -(T(0.5) * am) : T(0.5) * am;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Fb[v] = T(0.5) * Fhb[v];
        Ub[v] = cU * Fhb[v];
      }
      // am = max(max(|lminL|, |lmaxL|), max(|lminR|, |lmaxR|)): the branch taken
      if ((mL > mR) != right) {
        const T a1 = right ? aR1 : aL1, a2 = right ? aR2 : aL2;
        const T l1 = right ? lminR : lminL, l2 = right ? lmaxR : lmaxL;
        if (a1 > a2) lminb = amb * (l1 < T(0) ? T(-1) : T(1));
        else lmaxb = amb * (l2 < T(0) ? T(-1) : T(1));
      }
    }
  }

  // face_flux<d> (HLL or Rusanov of two face states): WLb, WRb += ...
  template <int d, class T>
  MX_HD static void face_flux_vjp(const T* WL, const T* WR, T sigma_lim, T kws, int flux_kind,
                                  const T* Fhb, T* WLb, T* WRb) {
    constexpr int NV = 14;
    T UL[NV], FL[NV], UR[NV], FR[NV];
    T lminL, lmaxL, lminR, lmaxR;
    S::face_terms<d>(WL, sigma_lim, kws, UL, FL, lminL, lmaxL);
    S::face_terms<d>(WR, sigma_lim, kws, UR, FR, lminR, lmaxR);
    T ULb[NV], FLb[NV], URb[NV], FRb[NV];
    T lminLb, lmaxLb, lminRb, lmaxRb;
    interface_vjp(UL, FL, lminL, lmaxL, UR, FR, lminR, lmaxR, flux_kind, Fhb, ULb, FLb, lminLb,
                  lmaxLb, URb, FRb, lminRb, lmaxRb);
    face_terms_vjp<d>(WL, sigma_lim, kws, ULb, FLb, lminLb, lmaxLb, WLb);
    face_terms_vjp<d>(WR, sigma_lim, kws, URb, FRb, lminRb, lmaxRb, WRb);
  }

  // The cell's common limiter factor phi (minmod / van Albada, neutral variables, positivity
  // fallback) and, for the adjoint, which variable and regime selected it: returns phi and
  // sets vstar (-1 when phi is a constant 0 or 1, i.e. carries no derivative).
  template <class T>
  MX_HD static T limiter_select(const T* Wm, const T* Wc, const T* Wp, int kind, int fallback, int& vstar) {
    constexpr int NV = 14;
    T sc[NV];
    S::scales(Wc, sc);
    T num = T(1), den = T(1);
    vstar = -1;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T a = Wc[v] - Wm[v];
      T b = Wp[v] - Wc[v];
      T aa = tabs(a), ab = tabs(b);
      T fn, fd;
      int var = -1;
      if (aa + ab <= T(NEUTRAL_EPS) * sc[v]) { fn = T(1); fd = T(1); }
      else if (a * b <= T(0)) { fn = T(0); fd = T(1); }
      else if (kind == 0) { fn = T(2) * tmin(aa, ab); fd = aa + ab; var = v; }
      else { fn = T(2) * a * b; fd = a * a + b * b; var = v; }
      if (fn * den < num * fd) { num = fn; den = fd; vstar = var; }
    }
    T phi = (den == T(1)) ? num : mdiv(num, den);
    if (fallback && phi > T(0)) {
      if (!faces_admissible<S>(Wm, Wc, Wp, phi)) { phi = T(0); vstar = -1; }
    }
    return phi;
  }

  // Reverse of the two face states of a cell along one direction (face_state with the
  // common factor phi), given their adjoints Op (upper face state) and Om (lower): the part
  // that lands on one cell of the stencil, role 0 = Wm, 1 = Wc, 2 = Wp, accumulated into Wb.
  // vstar and phi come from limiter_select on the same stencil.
  template <class T>
  MX_HD static void recon_vjp_role(int role, const T* Wm, const T* Wc, const T* Wp, T phi, int vstar,
                                   int kind, const T* Op, const T* Om, T* Wb) {
    constexpr int NV = 14;
    T phib = T(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T a = Wc[v] - Wm[v];
      T b = Wp[v] - Wc[v];
      // Wf = Wc +- (s * 0.5), s = phi (a + b) * 0.5, and a + b = Wp - Wm
      T sb = (Op[v] - Om[v]) * T(0.5);
      phib += sb * (a + b) * T(0.5);
      T abb = sb * phi * T(0.5);
      if (role == 1) Wb[v] += Op[v] + Om[v];
      else if (role == 2) Wb[v] += abb;
      else Wb[v] -= abb;
    }
    if (vstar >= 0) {
      // the selected variable's jumps, picked without a runtime array index (keeps the
      // arrays in registers)
      T a = T(0), b = T(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v == vstar) {
          a = Wc[v] - Wm[v];
          b = Wp[v] - Wc[v];
        }
      }
      T dpa, dpb;
      if (kind == 0) {
        T aa = tabs(a), ab = tabs(b), s = aa + ab;
        // phi = 2 min(|a|, |b|) / (|a| + |b|), the smaller one as the forward's tmin picks it
        const T is2 = mrcp(s * s);
        if (aa < ab) { dpa = T(2) * ab * is2; dpb = -T(2) * aa * is2; }
        else { dpa = -T(2) * ab * is2; dpb = T(2) * aa * is2; }
        dpa = (a < T(0)) ? -dpa : dpa;
        dpb = (b < T(0)) ? -dpb : dpb;
      } else {
        T s = a * a + b * b;
        // phi = 2 a b / (a^2 + b^2)
        const T is2 = mrcp(s * s);
        dpa = T(2) * b * (b * b - a * a) * is2;
        dpb = T(2) * a * (a * a - b * b) * is2;
      }
      T ab_ = phib * dpa, bb_ = phib * dpb;
      // a = Wc - Wm, b = Wp - Wc
      const T add = (role == 1) ? ab_ - bb_ : ((role == 0) ? -ab_ : bb_);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (v == vstar) Wb[v] += add;
    }
  }

  // all three parts of recon_vjp_role
  template <class T>
  MX_HD static void recon_vjp(const T* Wm, const T* Wc, const T* Wp, T phi, int vstar, int kind,
                              const T* Op, const T* Om, T* Wmb, T* Wcb, T* Wpb) {
    recon_vjp_role(0, Wm, Wc, Wp, phi, vstar, kind, Op, Om, Wmb);
    recon_vjp_role(1, Wm, Wc, Wp, phi, vstar, kind, Op, Om, Wcb);
    recon_vjp_role(2, Wm, Wc, Wp, phi, vstar, kind, Op, Om, Wpb);
  }
};

}  // namespace mx

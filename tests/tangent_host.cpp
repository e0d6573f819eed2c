// Host tangent-linear reference for the discrete adjoint: the crossed-jets scheme (14 moments,
// 2D, jet inflow on up to four walls, transmissive elsewhere, MUSCL with the common minmod or
// van Albada limiter and positivity fallback, HLL, local-tau BGK source, SSP-RK2 or forward
// Euler), written as plain loops over the
// library's own templated pointwise functions and run with a dual-number scalar.  One run gives
// the exact forward-mode derivative dJ/dp of J = sum(w * U_n) along one input direction: the jet
// Mach number, the jet density, tau_ref, or a given direction of U_0.  With "frozen" the limiter
// factor is held at its value (no derivative through the limiter), the linearization the
// adjoint's frozen-limiter mode transposes.  Time steps are read from the input (frozen).
//
// Input (binary, native endianness): int32 nx, ny, nsteps, seed (0 Mach, 1 jet rho, 2 tau_ref,
// 3 U0 direction), frozen; float64 mach, rho_j, T_j, tau_ref; int32 integrator (0 forward
// Euler, 1 SSP-RK2), limiter (0 minmod, 1 van Albada), n_jets; n_jets x float64 (centre along
// the wall, width, angle in degrees, wall 0 x-low / 1 x-high / 2 y-low / 3 y-high);
// nsteps float64 dt; U0 [14][ny][nx]; v [14][ny][nx]; w [14][ny][nx].
// Output: "J dJ" as two numbers.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mx_physics.hpp"
#include "mx_scheme.hpp"

namespace dual {
struct D {
  double v, d;
  D() : v(0), d(0) {}
  D(double x) : v(x), d(0) {}
  D(double x, double dx) : v(x), d(dx) {}
};
inline D operator+(D a, D b) { return D(a.v + b.v, a.d + b.d); }
inline D operator-(D a, D b) { return D(a.v - b.v, a.d - b.d); }
inline D operator-(D a) { return D(-a.v, -a.d); }
inline D operator*(D a, D b) { return D(a.v * b.v, a.d * b.v + a.v * b.d); }
inline D operator/(D a, D b) { return D(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline D& operator+=(D& a, D b) { a = a + b; return a; }
inline D& operator-=(D& a, D b) { a = a - b; return a; }
inline D& operator*=(D& a, D b) { a = a * b; return a; }
inline bool operator<(D a, D b) { return a.v < b.v; }
inline bool operator>(D a, D b) { return a.v > b.v; }
inline bool operator<=(D a, D b) { return a.v <= b.v; }
inline bool operator>=(D a, D b) { return a.v >= b.v; }
inline bool operator==(D a, D b) { return a.v == b.v; }
inline bool operator!=(D a, D b) { return a.v != b.v; }
inline D msqrt(D a) {
  double s = std::sqrt(a.v);
  return D(s, s > 0 ? a.d / (2 * s) : 0.0);
}
inline D mexp(D a) { double e = std::exp(a.v); return D(e, e * a.d); }
inline D mlog(D a) { return D(std::log(a.v), a.d / a.v); }
}  // namespace dual

using dual::D;
using mx::Sys14;

static int NX, NY, INTEG = 1, LIMITER = 0, NJ = 0;
static double DX, DY;
static double JC[4], JW[4], JANG[4];
static int JWALL[4];

struct Scheme {
  D mach, rhoj, tau_ref;
  double Tj = 1.0;
  bool frozen = false;
  std::vector<D> U;  // [14][NY][NX]

  D& at(std::vector<D>& A, int v, int i, int j) { return A[((size_t)v * NY + j) * NX + i]; }

  // primitive state of cell (gi, gj), ghost cells by the boundary conditions
  void prims(const std::vector<D>& A, int gi, int gj, D* W) {
    int si = gi < 0 ? 0 : (gi >= NX ? NX - 1 : gi);
    int sj = gj < 0 ? 0 : (gj >= NY ? NY - 1 : gj);
    D Uc[14];
    for (int v = 0; v < 14; ++v) Uc[v] = A[((size_t)v * NY + sj) * NX + si];
    Sys14::cons_to_prim(Uc, W);
    int wall = -1, s = 0;
    if (gi < 0) { wall = 0; s = sj; }
    else if (gi >= NX) { wall = 1; s = sj; }
    else if (gj < 0) { wall = 2; s = si; }
    else if (gj >= NY) { wall = 3; s = si; }
    if (wall >= 0) {
      double c = (wall < 2) ? (s + 0.5) * DY : (s + 0.5) * DX;
      int hit = -1;
      for (int k = 0; k < NJ; ++k)
        if (JWALL[k] == wall && c >= JC[k] - 0.5 * JW[k] && c <= JC[k] + 0.5 * JW[k]) hit = k;
      if (hit >= 0) {
        double a = JANG[hit] * M_PI / 180.0;
        D spd = mach * D(std::sqrt(5.0 / 3.0 * Tj));
        D pj = rhoj * D(Tj);
        W[0] = rhoj;
        W[1] = spd * D(std::cos(a)); W[2] = spd * D(std::sin(a)); W[3] = D(0);
        W[4] = pj; W[5] = D(0); W[6] = D(0); W[7] = pj; W[8] = D(0); W[9] = pj;
        W[10] = D(0); W[11] = D(0); W[12] = D(0);
        W[13] = D(15.0) * pj * pj / rhoj;
      }
    }
  }

  D phi_of(const D* Wm, const D* Wc, const D* Wp) {
    D phi = mx::limiter_factor<Sys14>(Wm, Wc, Wp, LIMITER);
    if (phi > D(0)) {
      D Wf[14];
      mx::face_state<Sys14>(Wm, Wc, Wp, phi, D(1), Wf);
      bool ok = Sys14::admissible(Wf);
      mx::face_state<Sys14>(Wm, Wc, Wp, phi, D(-1), Wf);
      ok = ok && Sys14::admissible(Wf);
      if (!ok) phi = D(0);
    }
    if (frozen) phi = D(phi.v);
    return phi;
  }

  void residual(const std::vector<D>& A, std::vector<D>& Lo) {
    const int ex = NX + 4, ey = NY + 4;
    std::vector<D> W((size_t)14 * ex * ey);
    auto w = [&](int v, int i, int j) -> D& { return W[((size_t)v * ey + (j + 2)) * ex + (i + 2)]; };
    for (int j = -2; j < NY + 2; ++j)
      for (int i = -2; i < NX + 2; ++i) {
        if ((i < 0 || i >= NX) && (j < 0 || j >= NY)) continue;
        D Wc[14];
        prims(A, i, j, Wc);
        for (int v = 0; v < 14; ++v) w(v, i, j) = Wc[v];
      }
    auto cell = [&](int i, int j, D* o) { for (int v = 0; v < 14; ++v) o[v] = w(v, i, j); };
    Lo.assign(A.size(), D(0));
    for (int j = 0; j < NY; ++j)
      for (int f = 0; f <= NX; ++f) {
        D a[14], b[14], c[14], e[14], WL[14], WR[14], F[14];
        cell(f - 2, j, a); cell(f - 1, j, b); cell(f, j, c); cell(f + 1, j, e);
        mx::face_state<Sys14>(a, b, c, phi_of(a, b, c), D(1), WL);
        mx::face_state<Sys14>(b, c, e, phi_of(b, c, e), D(-1), WR);
        mx::face_flux<Sys14, 0>(WL, WR, D(1e-4), D(1.0), 0, F);
        for (int v = 0; v < 14; ++v) {
          if (f - 1 >= 0) at(Lo, v, f - 1, j) -= F[v] * D(1.0 / DX);
          if (f < NX) at(Lo, v, f, j) += F[v] * D(1.0 / DX);
        }
      }
    for (int i = 0; i < NX; ++i)
      for (int f = 0; f <= NY; ++f) {
        D a[14], b[14], c[14], e[14], WL[14], WR[14], F[14];
        cell(i, f - 2, a); cell(i, f - 1, b); cell(i, f, c); cell(i, f + 1, e);
        mx::face_state<Sys14>(a, b, c, phi_of(a, b, c), D(1), WL);
        mx::face_state<Sys14>(b, c, e, phi_of(b, c, e), D(-1), WR);
        mx::face_flux<Sys14, 1>(WL, WR, D(1e-4), D(1.0), 0, F);
        for (int v = 0; v < 14; ++v) {
          if (f - 1 >= 0) at(Lo, v, i, f - 1) -= F[v] * D(1.0 / DY);
          if (f < NY) at(Lo, v, i, f) += F[v] * D(1.0 / DY);
        }
      }
    for (int j = 0; j < NY; ++j)
      for (int i = 0; i < NX; ++i) {
        D Wc[14], Cs[14];
        cell(i, j, Wc);
        D rho = Wc[0];
        D T = Sys14::pressure(Wc) / rho;
        D tau = tau_ref * (D(1.0) / rho) * dual::msqrt(D(1.0) / T);   // rho_ref = T_ref = 1
        Sys14::source(Wc, D(1.0) / tau, Cs);
        for (int v = 0; v < 14; ++v) at(Lo, v, i, j) += Cs[v];
      }
  }

  void step(double dt) {
    std::vector<D> L1, L2, Us(U.size());
    residual(U, L1);
    for (size_t k = 0; k < U.size(); ++k) Us[k] = U[k] + D(dt) * L1[k];
    if (INTEG == 0) {
      U = Us;
      return;
    }
    residual(Us, L2);
    for (size_t k = 0; k < U.size(); ++k) U[k] = D(0.5) * U[k] + D(0.5) * (Us[k] + D(dt) * L2[k]);
  }
};

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int hdr[5];
  double par[4];
  if (std::fread(hdr, 4, 5, f) != 5 || std::fread(par, 8, 4, f) != 4) return 2;
  int opt[3];
  if (std::fread(opt, 4, 3, f) != 3) return 2;
  INTEG = opt[0]; LIMITER = opt[1]; NJ = opt[2];
  if (NJ < 0 || NJ > 4) return 2;
  for (int k = 0; k < NJ; ++k) {
    double jd[4];
    if (std::fread(jd, 8, 4, f) != 4) return 2;
    JC[k] = jd[0]; JW[k] = jd[1]; JANG[k] = jd[2]; JWALL[k] = (int)jd[3];
  }
  NX = hdr[0]; NY = hdr[1];
  const int nsteps = hdr[2], seed = hdr[3];
  DX = 1.0 / NX; DY = 1.0 / NY;
  std::vector<double> dts(nsteps), U0((size_t)14 * NX * NY), v(U0.size()), w(U0.size());
  if (std::fread(dts.data(), 8, nsteps, f) != (size_t)nsteps) return 2;
  if (std::fread(U0.data(), 8, U0.size(), f) != U0.size()) return 2;
  if (std::fread(v.data(), 8, v.size(), f) != v.size()) return 2;
  if (std::fread(w.data(), 8, w.size(), f) != w.size()) return 2;
  std::fclose(f);
  Scheme s;
  s.frozen = hdr[4] != 0;
  s.mach = D(par[0], seed == 0 ? 1.0 : 0.0);
  s.rhoj = D(par[1], seed == 1 ? 1.0 : 0.0);
  s.Tj = par[2];
  s.tau_ref = D(par[3], seed == 2 ? 1.0 : 0.0);
  s.U.resize(U0.size());
  for (size_t k = 0; k < U0.size(); ++k) s.U[k] = D(U0[k], seed == 3 ? v[k] : 0.0);
  for (int n = 0; n < nsteps; ++n) s.step(dts[n]);
  double J = 0, dJ = 0;
  for (size_t k = 0; k < U0.size(); ++k) {
    J += w[k] * s.U[k].v;
    dJ += w[k] * s.U[k].d;
  }
  std::printf("%.17e %.17e\n", J, dJ);
  return 0;
}

// Host check of the hand-written reverse-mode pieces of the finite-volume step.
//
// Forward-mode derivatives of the same templated forward code, taken with a dual-number
// type, give J xdot exactly (to rounding); each reverse function gives J^T ybar.  The
// transposition identity  ybar . (J xdot) = (J^T ybar) . xdot  must then hold to rounding
// for every function and every state.  The dual type is itself checked against central
// differences of the plain double code.
//
// Input file: int32 n, then n x 14 primitive states (float64, row-major).
// Output: one line per check, "name max_rel_err count".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "mx_adjoint.hpp"

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
using mx::Adj14;
using mx::Sys14;

static std::mt19937_64 rng(12345);
static double gauss() { static std::normal_distribution<double> n(0.0, 1.0); return n(rng); }

struct Stat {
  std::string name;
  double worst = 0.0;
  int n = 0;
  void add(double lhs, double rhs, double scale) {
    double e = std::fabs(lhs - rhs) / (scale > 0 ? scale : 1.0);
    if (!(e <= worst)) worst = e;  // NaN propagates as worst
    ++n;
  }
  void print() const { std::printf("%s %.3e %d\n", name.c_str(), worst, n); }
};

// dot products with an absolute-value scale for the rounding bound
struct Dot {
  double s = 0, a = 0;
  void add(double x, double y) { s += x * y; a += std::fabs(x * y); }
};

// ---------------------------------------------------------------- generic driver
// f: (const D* x, D* y) ; fb: (const double* x, const double* yb, double* xb)
template <class F, class FB>
static void check(Stat& st, const std::vector<double>& x, int ny, F f, FB fb) {
  int nx = (int)x.size();
  std::vector<double> xd(nx), yb(ny), xb(nx, 0.0);
  for (int i = 0; i < nx; ++i) xd[i] = gauss() * (1e-3 + std::fabs(x[i]));
  for (int i = 0; i < ny; ++i) yb[i] = gauss();
  std::vector<D> X(nx), Y(ny);
  for (int i = 0; i < nx; ++i) X[i] = D(x[i], xd[i]);
  f(X.data(), Y.data());
  fb(x.data(), yb.data(), xb.data());
  Dot l, r;
  for (int i = 0; i < ny; ++i) l.add(yb[i], Y[i].d);
  for (int i = 0; i < nx; ++i) r.add(xb[i], xd[i]);
  st.add(l.s, r.s, l.a + r.a);
}

static void perturb(const double* W, double rel, double* Wo) {
  // a nearby realizable state: perturb, keep rho > 0 and P SPD by shrinking the step
  for (double s = rel; s > 1e-6; s *= 0.5) {
    for (int v = 0; v < 14; ++v) {
      double sc = std::fabs(W[v]) + (v >= 1 && v <= 3 ? std::sqrt(std::fabs(W[4] + W[7] + W[9]) / 3 / W[0]) : 0.0);
      if (v >= 4 && v < 10) sc = std::fabs(W[v]) + std::fabs(W[4] + W[7] + W[9]) / 3;
      Wo[v] = W[v] + s * gauss() * sc;
    }
    if (Sys14::admissible(Wo) && Sys14::sigma(Wo) > 0.0) return;
  }
  for (int v = 0; v < 14; ++v) Wo[v] = W[v];
}

int main(int argc, char** argv) {
  if (argc < 2) { std::fprintf(stderr, "usage: %s states.bin\n", argv[0]); return 2; }
  FILE* fp = std::fopen(argv[1], "rb");
  if (!fp) return 2;
  int n = 0;
  if (std::fread(&n, 4, 1, fp) != 1) return 2;
  std::vector<double> all(14 * (size_t)n);
  if (std::fread(all.data(), 8, all.size(), fp) != all.size()) return 2;
  std::fclose(fp);

  const double sl = 1e-4, kws = 1.0;
  Stat s_c2p{"cons_to_prim"}, s_p2c{"prim_to_cons"}, s_ft0{"face_terms_x"}, s_ft1{"face_terms_y"},
      s_src_l{"source_local"}, s_src_c{"source_const"}, s_tau{"source_tau_ref"},
      s_hll{"face_flux_hll"}, s_rus{"face_flux_rusanov"}, s_rec_mm{"recon_minmod"},
      s_rec_va{"recon_vanalbada"}, s_phi{"limiter_phi_equal"}, s_fd{"dual_vs_fd"},
      s_side{"interface_side_split"}, s_side_l{"interface_side_speeds"};
  int hll_branch[3] = {0, 0, 0};

  for (int c = 0; c < n; ++c) {
    std::vector<double> W(all.begin() + 14 * c, all.begin() + 14 * (c + 1));
    double U[14];
    Sys14::prim_to_cons(W.data(), U);
    std::vector<double> Uv(U, U + 14);

    check(s_c2p, Uv, 14, [](const D* x, D* y) { Sys14::cons_to_prim(x, y); },
          [](const double* x, const double* yb, double* xb) { Adj14::cons_to_prim_vjp(x, yb, xb); });
    check(s_p2c, W, 14, [](const D* x, D* y) { Sys14::prim_to_cons(x, y); },
          [](const double* x, const double* yb, double* xb) { Adj14::prim_to_cons_vjp(x, yb, xb); });

    auto ft = [&](auto dtag, Stat& st) {
      constexpr int d = decltype(dtag)::value;
      check(st, W, 30,
            [&](const D* x, D* y) { Sys14::face_terms<d>(x, D(sl), D(kws), y, y + 14, y[28], y[29]); },
            [&](const double* x, const double* yb, double* xb) {
              Adj14::face_terms_vjp<d>(x, sl, kws, yb, yb + 14, yb[28], yb[29], xb);
            });
    };
    ft(std::integral_constant<int, 0>(), s_ft0);
    ft(std::integral_constant<int, 1>(), s_ft1);

    // BGK source with the local relaxation time tau = tau_ref (rho_ref/rho) sqrt(T_ref/T)
    const double tau_ref = 0.037, rho_ref = 1.3, T_ref = 0.9;
    check(s_src_l, W, 14,
          [&](const D* x, D* y) {
            D rho = x[0];
            D T = Sys14::pressure(x) / rho;
            D tau = D(tau_ref) * (D(rho_ref) / rho) * dual::msqrt(D(T_ref) / T);
            Sys14::source(x, D(1.0) / tau, y);
          },
          [&](const double* x, const double* yb, double* xb) {
            double rho = x[0];
            double T = Sys14::pressure(x) / rho;
            double tau = tau_ref * (rho_ref / rho) * std::sqrt(T_ref / T);
            Adj14::source_vjp(x, 1.0 / tau, true, yb, xb);
          });
    check(s_src_c, W, 14, [&](const D* x, D* y) { Sys14::source(x, D(1.0) / D(tau_ref), y); },
          [&](const double* x, const double* yb, double* xb) { Adj14::source_vjp(x, 1.0 / tau_ref, false, yb, xb); });
    {
      // d/d tau_ref: the reverse returns Cb . C, and dC/dtau_ref = -C / tau_ref
      std::vector<double> yb(14);
      for (auto& v : yb) v = gauss();
      double rho = W[0], T = Sys14::pressure(W.data()) / rho;
      D tr(tau_ref, 1.0);
      D tau = tr * (D(rho_ref) / D(rho)) * dual::msqrt(D(T_ref) / D(T));
      std::vector<D> Wd(W.begin(), W.end()), C(14);
      Sys14::source(Wd.data(), D(1.0) / tau, C.data());
      Dot l;
      for (int v = 0; v < 14; ++v) l.add(yb[v], C[v].d);
      double xb[14] = {0};
      double cdot = Adj14::source_vjp(W.data(), 1.0 / tau.v, true, yb.data(), xb);
      double r = -cdot / tau_ref;
      s_tau.add(l.s, r, l.a + std::fabs(r));
    }

    // interface flux between this state and a nearby one (and a shifted copy to reach
    // every HLL case)
    for (int rep = 0; rep < 3; ++rep) {
      double WL[14], WR[14];
      for (int v = 0; v < 14; ++v) WL[v] = W[v];
      perturb(W.data(), 0.2, WR);
      if (rep > 0) {
        // add a bulk velocity of +-3 sound speeds along x: supersonic faces
        double cs = std::sqrt((W[4] + W[7] + W[9]) / 3 / W[0]);
        double sh = (rep == 1 ? 4.0 : -4.0) * cs;
        WL[1] += sh; WR[1] += sh;
      }
      std::vector<double> x(28);
      for (int v = 0; v < 14; ++v) { x[v] = WL[v]; x[14 + v] = WR[v]; }
      for (int kind = 0; kind < 2; ++kind) {
        check(kind == 0 ? s_hll : s_rus, x, 14,
              [&](const D* xx, D* y) { mx::face_flux<Sys14, 0>(xx, xx + 14, D(sl), D(kws), kind, y); },
              [&](const double* xx, const double* yb, double* xb) {
                Adj14::face_flux_vjp<0>(xx, xx + 14, sl, kws, kind, yb, xb, xb + 14);
              });
      }
      {
        double UL[14], FL[14], UR[14], FR[14], a, b, c2, d2;
        Sys14::face_terms<0>(WL, sl, kws, UL, FL, a, b);
        Sys14::face_terms<0>(WR, sl, kws, UR, FR, c2, d2);
        double SL = a < c2 ? a : c2, SR = b > d2 ? b : d2;
        hll_branch[SL >= 0 ? 0 : (SR <= 0 ? 1 : 2)]++;
        // the interface reverse split over two threads, one per face state, against the
        // whole; on the second pass both sides are the same state (every min / max a tie)
        for (int tie = 0; tie < 2; ++tie) {
          const double* uR = tie ? UL : UR;
          const double* fR = tie ? FL : FR;
          const double lR = tie ? a : c2, mR = tie ? b : d2;
          for (int kind = 0; kind < 2; ++kind) {
            double Fhb[14], ULb[14], FLb[14], URb[14], FRb[14], lLb, mLb, lRb, mRb;
            for (int v = 0; v < 14; ++v) Fhb[v] = gauss();
            Adj14::interface_vjp(UL, FL, a, b, uR, fR, lR, mR, kind, Fhb, ULb, FLb, lLb, mLb, URb, FRb,
                                 lRb, mRb);
            double aFL = 0, aFR = 0, aUL = 0, aUR = 0;
            for (int v = 0; v < 14; ++v) {
              aFL += Fhb[v] * FL[v]; aFR += Fhb[v] * fR[v];
              aUL += Fhb[v] * UL[v]; aUR += Fhb[v] * uR[v];
            }
            // the U and F adjoints are the same products as in interface_vjp (compared exactly);
            // the speed adjoints sum the 14 components before scaling, so they agree to the
            // rounding of those sums: scale = the absolute sums they are formed from
            double bFL = 0, bFR = 0, bU = 0;
            for (int v = 0; v < 14; ++v) {
              bFL += std::fabs(Fhb[v] * FL[v]); bFR += std::fabs(Fhb[v] * fR[v]);
              bU += std::fabs(Fhb[v] * uR[v]) + std::fabs(Fhb[v] * UL[v]);
            }
            double sscale = 0.5 * bU;   // Rusanov: the speed adjoint is -(aUR - aUL) / 2
            if (kind == 0) {
              const double sL = a < lR ? a : lR, sR = b > mR ? b : mR;
              const double inv = (sL < 0 && sR > 0) ? 1.0 / (sR - sL) : 0.0;
              sscale = inv * (bFL + bFR) + inv * (std::fabs(sL) + std::fabs(sR)) * bU +
                       inv * inv * (std::fabs(sR) * bFL + std::fabs(sL) * bFR + std::fabs(sL * sR) * bU);
            }
            for (int side = 0; side < 2; ++side) {
              double Ub[14], Fb[14], lb, mb;
              Adj14::interface_side_vjp(side == 1, a, b, lR, mR, aFL, aFR, aUL, aUR, kind, Fhb, Ub, Fb,
                                        lb, mb);
              const double* rU = side ? URb : ULb;
              const double* rF = side ? FRb : FLb;
              for (int v = 0; v < 14; ++v) {
                s_side.add(rU[v], Ub[v], 1.0);
                s_side.add(rF[v], Fb[v], 1.0);
              }
              s_side_l.add(side ? lRb : lLb, lb, sscale);
              s_side_l.add(side ? mRb : mLb, mb, sscale);
            }
          }
        }
      }
    }

    // reconstruction of the two face states of a cell from (Wm, Wc, Wp)
    for (int rep = 0; rep < 4; ++rep) {
      double Wm[14], Wp[14];
      double rel = rep == 0 ? 0.02 : (rep == 1 ? 0.3 : (rep == 2 ? 1e-13 : 0.05));
      perturb(W.data(), rel, Wm);
      perturb(W.data(), rel, Wp);
      if (rep == 3) {
        // a monotone profile: Wp - Wc and Wc - Wm of one sign in every variable
        for (int v = 0; v < 14; ++v) Wp[v] = 2 * W[v] - Wm[v] + 0.3 * (W[v] - Wm[v]);
        if (!Sys14::admissible(Wp)) perturb(W.data(), 0.05, Wp);
      }
      std::vector<double> x(42);
      for (int v = 0; v < 14; ++v) { x[v] = Wm[v]; x[14 + v] = W[v]; x[28 + v] = Wp[v]; }
      for (int kind = 0; kind < 2; ++kind) {
        // phi from the reverse's own selection equals the forward factor bit for bit
        double phi_f = mx::limiter_factor<Sys14>(Wm, W.data(), Wp, kind);
        {
          double Wf[14];
          mx::face_state<Sys14>(Wm, W.data(), Wp, phi_f, 1.0, Wf);
          bool ok = Sys14::admissible(Wf);
          mx::face_state<Sys14>(Wm, W.data(), Wp, phi_f, -1.0, Wf);
          ok = ok && Sys14::admissible(Wf);
          if (phi_f > 0 && !ok) phi_f = 0.0;
        }
        int vs;
        double phi_s = Adj14::limiter_select(Wm, W.data(), Wp, kind, 1, vs);
        s_phi.add(phi_f, phi_s, 1.0);
        check(kind == 0 ? s_rec_mm : s_rec_va, x, 28,
              [&](const D* xx, D* y) {
                D phi = mx::limiter_factor<Sys14>(xx, xx + 14, xx + 28, kind);
                if (phi > D(0)) {
                  D Wf[14];
                  mx::face_state<Sys14>(xx, xx + 14, xx + 28, phi, D(1.0), Wf);
                  bool ok = Sys14::admissible(Wf);
                  mx::face_state<Sys14>(xx, xx + 14, xx + 28, phi, D(-1.0), Wf);
                  ok = ok && Sys14::admissible(Wf);
                  if (!ok) phi = D(0);
                }
                mx::face_state<Sys14>(xx, xx + 14, xx + 28, phi, D(1.0), y);
                mx::face_state<Sys14>(xx, xx + 14, xx + 28, phi, D(-1.0), y + 14);
              },
              [&](const double* xx, const double* yb, double* xb) {
                int v2;
                double phi = Adj14::limiter_select(xx, xx + 14, xx + 28, kind, 1, v2);
                Adj14::recon_vjp(xx, xx + 14, xx + 28, phi, v2, kind, yb, yb + 14, xb, xb + 14, xb + 28);
              });
      }
    }

    // the dual type against central differences of the double code (face terms along x);
    // states with sigma near sigma_lim or near 1 are skipped: there the wave-speed hyperbola
    // in q has a curvature scale of order sigma_lim, and sqrt(3 - 3 sigma_w) an unbounded
    // curvature, so central differences are not accurate
    double sgm = Sys14::sigma(W.data());
    if (c % 2 == 0 && sgm > 1e-2 && sgm < 0.99) {
      std::vector<double> xd(14);
      double sc[14];
      Sys14::scales(W.data(), sc);
      for (int v = 0; v < 14; ++v) xd[v] = gauss() * (std::fabs(W[v]) + 1e-2 * sc[v]);
      std::vector<D> X(14), Y(30);
      for (int v = 0; v < 14; ++v) X[v] = D(W[v], xd[v]);
      Sys14::face_terms<0>(X.data(), D(sl), D(kws), Y.data(), Y.data() + 14, Y[28], Y[29]);
      double h = 1e-6;
      double Wp[14], Wm2[14], yp[30], ym[30];
      for (int v = 0; v < 14; ++v) { Wp[v] = W[v] + h * xd[v]; Wm2[v] = W[v] - h * xd[v]; }
      Sys14::face_terms<0>(Wp, sl, kws, yp, yp + 14, yp[28], yp[29]);
      Sys14::face_terms<0>(Wm2, sl, kws, ym, ym + 14, ym[28], ym[29]);
      for (int k = 0; k < 30; ++k) {
        double fd = (yp[k] - ym[k]) / (2 * h);
        s_fd.add(fd, Y[k].d, std::fabs(fd) + std::fabs(Y[k].d) + 1e-8 * (std::fabs(yp[k]) + 1.0));
      }
    }
  }
  for (const Stat* st : {&s_c2p, &s_p2c, &s_ft0, &s_ft1, &s_src_l, &s_src_c, &s_tau, &s_hll, &s_rus,
                         &s_rec_mm, &s_rec_va, &s_phi, &s_fd, &s_side, &s_side_l})
    st->print();
  std::printf("hll_branches %d %d %d\n", hll_branch[0], hll_branch[1], hll_branch[2]);
  return 0;
}

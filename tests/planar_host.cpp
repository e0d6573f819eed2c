// Host check of the planar 14-moment system (csrc/mx_planar.hpp) against the full one
// (csrc/mx_physics.hpp, csrc/mx_scheme.hpp) on planar-symmetric states: every function the
// stage kernel calls gives, on the ten moments it carries, the full system's values to
// rounding, and the full system's z-odd outputs vanish exactly.
//
// Input file: int32 n, then n x 14 primitive states (float64, row-major), each with
// u_z = P_xz = P_yz = q_z = 0.
// Output: one line per check, "name max_rel_err max_abs_zodd count".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "mx_scheme.hpp"
#include "mx_planar.hpp"

using mx::Sys14;
using mx::Sys14P;

static const int kPlane[10] = {0, 1, 2, 4, 5, 7, 9, 10, 11, 13};
static const int kZodd[4] = {3, 6, 8, 12};

struct Check {
  std::string name;
  double rel = 0.0, zodd = 0.0;
  long long n = 0;
  // planar values p[10] against full values g[14]: error relative to the largest |g|
  void add14(const double* p, const double* g) {
    double s = 0.0;
    for (int v = 0; v < 14; ++v) s = std::fmax(s, std::fabs(g[v]));
    for (int k = 0; k < 10; ++k) rel = std::fmax(rel, std::fabs(p[k] - g[kPlane[k]]) / std::fmax(s, 1e-300));
    for (int k = 0; k < 4; ++k) zodd = std::fmax(zodd, std::fabs(g[kZodd[k]]));
    ++n;
  }
  void add(const double* p, const double* g, int m) {
    double s = 0.0;
    for (int v = 0; v < m; ++v) s = std::fmax(s, std::fabs(g[v]));
    for (int v = 0; v < m; ++v) rel = std::fmax(rel, std::fabs(p[v] - g[v]) / std::fmax(s, 1e-300));
    ++n;
  }
  void print() const { std::printf("%s %.3e %.3e %lld\n", name.c_str(), rel, zodd, n); }
};

template <int d>
static void closure_check(const double* W14, Check& c) {
  double Wp[10];
  Sys14P::from14(W14, Wp);
  Sys14::Core<double> k;
  Sys14::core(W14, 1e-4, k);
  Sys14P::Core<double> kp;
  Sys14P::core(Wp, 1e-4, kp);
  double Q[6], R[3], S, Qp[4], Rp[2], Sp;
  Sys14::closure_dir<d>(k, Q, R, S);
  Sys14P::closure_dir<d>(kp, Qp, Rp, Sp);
  // Q_ijd: xx xy yy zz carried; xz yz vanish.  R_id: x y carried; z vanishes.
  const double g[9] = {Q[0], Q[1], Q[3], Q[5], R[0], R[1], S, k.sig, k.sb};
  const double p[9] = {Qp[0], Qp[1], Qp[2], Qp[3], Rp[0], Rp[1], Sp, kp.sig, kp.sb};
  c.add(p, g, 9);
  c.zodd = std::fmax(c.zodd, std::fmax(std::fabs(Q[2]), std::fmax(std::fabs(Q[4]), std::fabs(R[2]))));
}

template <int d>
static void face_check(const double* W14, Check& flux, Check& speeds) {
  double Wp[10];
  Sys14P::from14(W14, Wp);
  double U[14], F[14], lmin, lmax, Up[10], Fp[10], lminp, lmaxp;
  Sys14::face_terms<d>(W14, 1e-4, 1.2, U, F, lmin, lmax);
  Sys14P::face_terms<d>(Wp, 1e-4, 1.2, Up, Fp, lminp, lmaxp);
  flux.add14(Fp, F);
  const double g[2] = {lmin, lmax}, p[2] = {lminp, lmaxp};
  speeds.add(p, g, 2);
}

template <int d>
static void interface_check(const double* WL14, const double* WR14, int kind, Check& c) {
  double WL[10], WR[10], F[14], Fp[10];
  Sys14P::from14(WL14, WL);
  Sys14P::from14(WR14, WR);
  mx::face_flux<Sys14, d>(WL14, WR14, 1e-4, 1.2, kind, F);
  mx::face_flux<Sys14P, d>(WL, WR, 1e-4, 1.2, kind, Fp);
  c.add14(Fp, F);
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int n = 0;
  if (std::fread(&n, sizeof(int), 1, f) != 1) return 2;
  std::vector<double> W((size_t)n * 14);
  if (std::fread(W.data(), sizeof(double), W.size(), f) != W.size()) return 2;
  std::fclose(f);

  Check c2p{"cons_to_prim"}, p2c{"prim_to_cons"}, clo0{"closure_x"}, clo1{"closure_y"};
  Check fl0{"flux_x"}, fl1{"flux_y"}, ws0{"wavespeeds_x"}, ws1{"wavespeeds_y"};
  Check src{"source"}, eq{"equilibrium"}, rate{"cell_rate2d"}, hll0{"hll_x"}, hll1{"hll_y"};
  Check rus0{"rusanov_x"}, rus1{"rusanov_y"}, lim{"limiter_factor"}, fst{"face_state"};
  long long adm_mismatch = 0, adm_n = 0;
  for (int i = 0; i < n; ++i) {
    const double* W14 = &W[(size_t)i * 14];
    double Wp[10];
    Sys14P::from14(W14, Wp);
    double U[14], Up[10], Wb[14], Wbp[10];
    Sys14::prim_to_cons(W14, U);
    Sys14P::prim_to_cons(Wp, Up);
    p2c.add14(Up, U);
    // primitive recovery of the same conserved state
    double Uq[10];
    for (int k = 0; k < 10; ++k) Uq[k] = U[kPlane[k]];
    Sys14::cons_to_prim(U, Wb);
    Sys14P::cons_to_prim(Uq, Wbp);
    c2p.add14(Wbp, Wb);
    closure_check<0>(W14, clo0);
    closure_check<1>(W14, clo1);
    face_check<0>(W14, fl0, ws0);
    face_check<1>(W14, fl1, ws1);
    double C[14], Cp[10], E[14], Ep[10];
    Sys14::source(W14, 3.7, C);
    Sys14P::source(Wp, 3.7, Cp);
    src.add14(Cp, C);
    Sys14::equilibrium(W14, E);
    Sys14P::equilibrium(Wp, Ep);
    eq.add14(Ep, E);
    const double r = Sys14::cell_rate2d(W14, 1e-4, 1.2, 1.0 / 512, 1.0 / 384);
    const double rp = Sys14P::cell_rate2d(Wp, 1e-4, 1.2, 1.0 / 512, 1.0 / 384);
    rate.add(&rp, &r, 1);
    adm_n++;
    if (Sys14::admissible(W14) != Sys14P::admissible(Wp)) adm_mismatch++;
    if (Sys14::admissible_cons(U) != Sys14P::admissible_cons(Uq)) adm_mismatch++;
    // pairs and triples of neighbouring states (cyclic)
    const double* Wn = &W[(size_t)((i + 1) % n) * 14];
    const double* Wm = &W[(size_t)((i + n - 1) % n) * 14];
    interface_check<0>(W14, Wn, 0, hll0);
    interface_check<1>(W14, Wn, 0, hll1);
    interface_check<0>(W14, Wn, 1, rus0);
    interface_check<1>(W14, Wn, 1, rus1);
    // a triple that is a small perturbation of one state (a smooth stencil) and the raw one
    for (int kind = 0; kind < 2; ++kind) {
      for (int smooth = 0; smooth < 2; ++smooth) {
        double A[14], B[14], Cc[14];
        for (int v = 0; v < 14; ++v) {
          A[v] = smooth ? W14[v] * (1.0 - 0.01 * ((v % 3) + 1)) : Wm[v];
          B[v] = W14[v];
          Cc[v] = smooth ? W14[v] * (1.0 + 0.013 * ((v % 2) + 1)) : Wn[v];
        }
        double Ap[10], Bp[10], Cp2[10];
        Sys14P::from14(A, Ap);
        Sys14P::from14(B, Bp);
        Sys14P::from14(Cc, Cp2);
        const double phi = mx::limiter_factor<Sys14>(A, B, Cc, kind);
        const double phip = mx::limiter_factor<Sys14P>(Ap, Bp, Cp2, kind);
        lim.add(&phip, &phi, 1);
        double Wf[14], Wfp[10];
        mx::face_state<Sys14>(A, B, Cc, phi, 1.0, Wf);
        mx::face_state<Sys14P>(Ap, Bp, Cp2, phi, 1.0, Wfp);
        fst.add14(Wfp, Wf);
        adm_n++;
        if (mx::faces_admissible<Sys14>(A, B, Cc, phi) != mx::faces_admissible<Sys14P>(Ap, Bp, Cp2, phi))
          adm_mismatch++;
      }
    }
  }
  for (const Check* c : {&c2p, &p2c, &clo0, &clo1, &fl0, &fl1, &ws0, &ws1, &src, &eq, &rate, &hll0,
                         &hll1, &rus0, &rus1, &lim, &fst})
    c->print();
  std::printf("admissible_mismatch %lld 0 %lld\n", adm_mismatch, adm_n);
  return 0;
}

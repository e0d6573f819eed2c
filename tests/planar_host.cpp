// Host check of the symmetry-reduced 14-moment systems against the full one (csrc/mx_physics.hpp,
// csrc/mx_scheme.hpp): the planar system (csrc/mx_planar.hpp) on planar-symmetric states and
// the axial system (csrc/mx_axial.hpp) on axially symmetric 1D states.  Every function the
// stage kernels call gives, on the moments it carries, the full system's values to rounding,
// and the full system's outputs for the moments left out vanish exactly.
//
// Usage: planarcheck planar|axial file.  Input file: int32 n, then n x 14 primitive states
// (float64, row-major) with the symmetry's vanishing moments exactly zero.
// Output: one line per check, "name max_rel_err max_abs_dropped count".
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "mx_scheme.hpp"
#include "mx_planar.hpp"
#include "mx_axial.hpp"

using mx::Sys14;
using mx::Sys14P;
using mx::Sys14A;

struct Check {
  std::string name;
  double rel = 0.0, zodd = 0.0;
  long long n = 0;
  // reduced values p[R::NV] against full values g[14]: error relative to the largest |g|;
  // the largest |g| of a moment the reduced system leaves out
  template <class R> void add14(const double* p, const double* g) {
    double s = 0.0;
    for (int v = 0; v < 14; ++v) s = std::fmax(s, std::fabs(g[v]));
    bool kept[14] = {};
    for (int k = 0; k < R::NV; ++k) {
      kept[R::plane_of(k)] = true;
      rel = std::fmax(rel, std::fabs(p[k] - g[R::plane_of(k)]) / std::fmax(s, 1e-300));
    }
    for (int v = 0; v < 14; ++v)
      if (!kept[v]) zodd = std::fmax(zodd, std::fabs(g[v]));
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

// closing values along d: the reduced system's against the full system's (the carried ones),
// and the full system's values the reduced one drops (zero)
template <class R, int d>
static void closure_check(const double* W14, Check& c) {
  double Wr[R::NV];
  R::from14(W14, Wr);
  Sys14::Core<double> k;
  Sys14::core(W14, 1e-4, k);
  typename R::template Core<double> kr;
  R::core(Wr, 1e-4, kr);
  double Q[6], Rf[3], S, Qr[4], Rr[2], Sr;
  Sys14::closure_dir<d>(k, Q, Rf, S);
  R::template closure_dir<d>(kr, Qr, Rr, Sr);
  if constexpr (R::NV == 10) {
    // Q_ijd: xx xy yy zz carried, xz yz dropped; R_id: x y carried, z dropped
    const double g[9] = {Q[0], Q[1], Q[3], Q[5], Rf[0], Rf[1], S, k.sig, k.sb};
    const double p[9] = {Qr[0], Qr[1], Qr[2], Qr[3], Rr[0], Rr[1], Sr, kr.sig, kr.sb};
    c.add(p, g, 9);
    c.zodd = std::fmax(c.zodd, std::fmax(std::fabs(Q[2]), std::fmax(std::fabs(Q[4]), std::fabs(Rf[2]))));
  } else {
    // along x: Q_xxx Q_yyx Q_zzx and R_xx carried; the off-diagonal Q_ijx and R_yx, R_zx dropped
    const double g[7] = {Q[0], Q[3], Q[5], Rf[0], S, k.sig, k.sb};
    const double p[7] = {Qr[0], Qr[1], Qr[2], Rr[0], Sr, kr.sig, kr.sb};
    c.add(p, g, 7);
    for (double x : {Q[1], Q[2], Q[4], Rf[1], Rf[2]}) c.zodd = std::fmax(c.zodd, std::fabs(x));
  }
}

template <class R, int d>
static void face_check(const double* W14, Check& flux, Check& speeds) {
  double Wr[R::NV];
  R::from14(W14, Wr);
  double U[14], F[14], lmin, lmax, Ur[R::NV], Fr[R::NV], lminr, lmaxr;
  Sys14::face_terms<d>(W14, 1e-4, 1.2, U, F, lmin, lmax);
  R::template face_terms<d>(Wr, 1e-4, 1.2, Ur, Fr, lminr, lmaxr);
  flux.add14<R>(Fr, F);
  const double g[2] = {lmin, lmax}, p[2] = {lminr, lmaxr};
  speeds.add(p, g, 2);
}

template <class R, int d>
static void interface_check(const double* WL14, const double* WR14, int kind, Check& c) {
  double WL[R::NV], WR[R::NV], F[14], Fr[R::NV];
  R::from14(WL14, WL);
  R::from14(WR14, WR);
  mx::face_flux<Sys14, d>(WL14, WR14, 1e-4, 1.2, kind, F);
  mx::face_flux<R, d>(WL, WR, 1e-4, 1.2, kind, Fr);
  c.add14<R>(Fr, F);
}

template <class R>
static void run(const std::vector<double>& W, int n) {
  constexpr int NV = R::NV;
  constexpr bool two_d = NV == 10;
  Check c2p{"cons_to_prim"}, p2c{"prim_to_cons"}, clo0{"closure_x"}, clo1{"closure_y"};
  Check fl0{"flux_x"}, fl1{"flux_y"}, ws0{"wavespeeds_x"}, ws1{"wavespeeds_y"};
  Check src{"source"}, eq{"equilibrium"}, rate{"cfl_rate"}, hll0{"hll_x"}, hll1{"hll_y"};
  Check rus0{"rusanov_x"}, rus1{"rusanov_y"}, lim{"limiter_factor"}, fst{"face_state"};
  long long adm_mismatch = 0, adm_n = 0;
  for (int i = 0; i < n; ++i) {
    const double* W14 = &W[(size_t)i * 14];
    double Wr[NV];
    R::from14(W14, Wr);
    double U[14], Ur[NV], Wb[14], Wbr[NV];
    Sys14::prim_to_cons(W14, U);
    R::prim_to_cons(Wr, Ur);
    p2c.add14<R>(Ur, U);
    // primitive recovery of the same conserved state
    double Uq[NV];
    for (int k = 0; k < NV; ++k) Uq[k] = U[R::plane_of(k)];
    Sys14::cons_to_prim(U, Wb);
    R::cons_to_prim(Uq, Wbr);
    c2p.add14<R>(Wbr, Wb);
    closure_check<R, 0>(W14, clo0);
    face_check<R, 0>(W14, fl0, ws0);
    if constexpr (two_d) {
      closure_check<R, 1>(W14, clo1);
      face_check<R, 1>(W14, fl1, ws1);
    }
    double C[14], Cr[NV], E[14], Er[NV];
    Sys14::source(W14, 3.7, C);
    R::source(Wr, 3.7, Cr);
    src.add14<R>(Cr, C);
    Sys14::equilibrium(W14, E);
    R::equilibrium(Wr, Er);
    eq.add14<R>(Er, E);
    double r, rr;
    if constexpr (two_d) {
      r = Sys14::cell_rate2d(W14, 1e-4, 1.2, 1.0 / 512, 1.0 / 384);
      rr = R::cell_rate2d(Wr, 1e-4, 1.2, 1.0 / 512, 1.0 / 384);
    } else {
      r = Sys14::cell_lambda<0>(W14, 1e-4, 1.2);
      rr = R::template cell_lambda<0>(Wr, 1e-4, 1.2);
    }
    rate.add(&rr, &r, 1);
    adm_n++;
    if (Sys14::admissible(W14) != R::admissible(Wr)) adm_mismatch++;
    if (Sys14::admissible_cons(U) != R::admissible_cons(Uq)) adm_mismatch++;
    // pairs and triples of neighbouring states (cyclic)
    const double* Wn = &W[(size_t)((i + 1) % n) * 14];
    const double* Wm = &W[(size_t)((i + n - 1) % n) * 14];
    interface_check<R, 0>(W14, Wn, 0, hll0);
    interface_check<R, 0>(W14, Wn, 1, rus0);
    if constexpr (two_d) {
      interface_check<R, 1>(W14, Wn, 0, hll1);
      interface_check<R, 1>(W14, Wn, 1, rus1);
    }
    // a triple that is a small perturbation of one state (a smooth stencil) and the raw one
    for (int kind = 0; kind < 2; ++kind) {
      for (int smooth = 0; smooth < 2; ++smooth) {
        double A[14], B[14], Cc[14];
        for (int v = 0; v < 14; ++v) {
          A[v] = smooth ? W14[v] * (1.0 - 0.01 * ((v % 3) + 1)) : Wm[v];
          B[v] = W14[v];
          Cc[v] = smooth ? W14[v] * (1.0 + 0.013 * ((v % 2) + 1)) : Wn[v];
        }
        double Ar[NV], Br[NV], Cr2[NV];
        R::from14(A, Ar);
        R::from14(B, Br);
        R::from14(Cc, Cr2);
        const double phi = mx::limiter_factor<Sys14>(A, B, Cc, kind);
        const double phir = mx::limiter_factor<R>(Ar, Br, Cr2, kind);
        lim.add(&phir, &phi, 1);
        double Wf[14], Wfr[NV];
        mx::face_state<Sys14>(A, B, Cc, phi, 1.0, Wf);
        mx::face_state<R>(Ar, Br, Cr2, phi, 1.0, Wfr);
        fst.add14<R>(Wfr, Wf);
        adm_n++;
        if (mx::faces_admissible<Sys14>(A, B, Cc, phi) != mx::faces_admissible<R>(Ar, Br, Cr2, phi))
          adm_mismatch++;
      }
    }
  }
  for (const Check* c : {&c2p, &p2c, &clo0, &fl0, &ws0, &src, &eq, &rate, &hll0, &rus0, &lim, &fst})
    c->print();
  if (two_d)
    for (const Check* c : {&clo1, &fl1, &ws1, &hll1, &rus1}) c->print();
  std::printf("admissible_mismatch %lld 0 %lld\n", adm_mismatch, adm_n);
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const std::string which = argv[1];
  FILE* f = std::fopen(argv[2], "rb");
  if (!f) return 2;
  int n = 0;
  if (std::fread(&n, sizeof(int), 1, f) != 1) return 2;
  std::vector<double> W((size_t)n * 14);
  if (std::fread(W.data(), sizeof(double), W.size(), f) != W.size()) return 2;
  std::fclose(f);
  if (which == "planar") run<Sys14P>(W, n);
  else if (which == "axial") run<Sys14A>(W, n);
  else return 2;
  return 0;
}

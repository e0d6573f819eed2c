// Interface between the C-ABI runtime and the reverse (adjoint) kernels.
#pragma once
#include "mx_internal.hpp"

namespace mx {

// Reverse (adjoint) of one stage  Uout = a Ua + beta Ub + mu_coef dt L(Ub)  (14 moments, FP64).
// Given lam_out (adjoint of Uout) the reverse writes
//   lam_in = extra_coef lam_extra + beta lam_out + (dL/dUb)^T (mu_coef dt lam_out)
// and adds the stage's parameter partials (jet Mach, jet density, tau_ref), per workgroup of
// the update kernel, to part (zeroed by the caller before the first reverse stage);
// launch_adjoint_reduce then sums part into grad[3].
// The coefficient a of Ua is applied by the caller through the next reverse stage's
// lam_extra.  All fields are padded SoA like the state.
struct AdjParams {
  StageParams sp;            // sp.Ub = stage input; geometry, BCs, physics of the stage
  const double* lam_out;
  const double* lam_extra;   // may be null
  double extra_coef;
  double beta;
  double mu_coef;
  double dt;
  double* lam_in;
  double* fbx;               // x-face state adjoints [28][(nx+1) ny]: WL then WR
  double* fby;               // y-face state adjoints [28][nx (ny+1)]
  long long nfx, nfy;
  double* wb;                // primitive adjoints of the ghost-extended cells [14][eny][nx+4]
  int epitch;                // nx + 4
  long long eplane;          // epitch * eny (eny = ny + 4 in 2D, 1 in 1D)
  double* wext;              // primitives of the ghost-extended cells [14][eplane]
  double* phix;              // common limiter factor of each extended cell along x [eplane]
  double* phiy;              //   ... along y
  int* vsx;                  // variable that selected it (-1: a constant factor) [eplane]
  int* vsy;
  int frozen_limiter;        // 1: no derivative through the limiter factors
  double* part;              // per-workgroup partial sums over the reverse pass [3][n_upd_blocks]
  int n_upd_blocks;
  double* grad;              // [3] sums of part: d/d jet Mach, d/d jet rho, d/d tau_ref
};

// launchers (mx_adjoint.hip)
// planar: the recorded states and dJ/dU are planar-symmetric (2D only): the z-odd adjoint
// components are zero and are neither read nor written
hipError_t launch_adjoint_stage(int dim, int order, bool planar, AdjParams& a, hipStream_t s);
// sets ASYM_Z in ctrl->asym when a z-odd component of the flat 14-moment field f (n cells) is
// nonzero
hipError_t launch_check_planar(const double* f, long long n, DevCtrl* c, hipStream_t s);
// grad[m] = sum over the workgroups of part[m] (fixed order)
hipError_t launch_adjoint_reduce(const AdjParams& a, hipStream_t s);
int adjoint_update_blocks(int nx, int ny);
hipError_t launch_tape_dt(const DevCtrl* c, double* slot, hipStream_t s);
hipError_t launch_pad_copy(const double* src, double* dst, int nv, int nx, int ny, int pitch,
                           int to_padded, hipStream_t s);
}  // namespace mx

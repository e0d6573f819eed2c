// Device records and launchers of the batched 1D shock tubes.
#pragma once
#include <hip/hip_runtime.h>
#include "mx_internal.hpp"

namespace mx {

struct BatchInst {
  double dt, t, t_end, dt_last;
  double dx, inv_dx, tau_ref;
  unsigned long long maxrate;    // bit pattern of the max CFL rate (positive double)
  long long step;
  long long off;                 // first cell in the concatenated field
  int n;                         // cells
  int status;                    // bit 1 non-finite, bit 2 unrealizable
  int fail_step;
  int pad;
};

struct BatchCtrl {
  int n_active;                  // instances that advance in the current step
  int n_tiles;                   // their tiles: the work list of the step's stage launches
  int per;                       // tiles per workgroup range of the stage launches (0: none)
  int band;                      // ranges per XCD band (0: no bands, range = workgroup index)
};

struct BatchParams {
  const double* Ub;
  const double* Ua;
  double* Uout;
  long long plane;               // padded total cells
  BatchInst* inst;
  const int* act_inst;           // instances that advance, in queue order
  const int* act_tile0;          // first work-list tile of each; [n_active] = n_tiles
  const BatchCtrl* bctrl;        // n_active and n_tiles of the current step
  const int* cell_inst;          // instance of every cell (CFL initialisation)
  int bc_lo, bc_hi;
  int tau_mode;
  double rho_ref, T_ref;
  double sigma_lim, kws;
  int limiter, flux, fallback;
  int mode;
  double cdt;
  int do_cfl;
  DevCtrl* ctrl;                 // shared counters (fallbacks, FP64 re-evaluations)
};

// launch shapes: nt threads per workgroup, cpt cells per thread (tiles of tile_1d(nt * cpt))
bool batch_shape_supported(int nt, int cpt);
// reduced: every tube's state is axially symmetric (u_y = u_z = P_xy = P_xz = P_yz = q_y = q_z = 0)
// and the stages carry the seven other moments (Sys14A)
hipError_t launch_batch_stage(int precision, bool reduced, int nt, int cpt, const BatchParams& p, int grid,
                              hipStream_t s);
hipError_t launch_batch_finalize(BatchInst* in, const int* order, int n_inst, double cfl, int tile_w,
                                 int* act_inst, int* act_tile0, BatchCtrl* bc, int stage_grid,
                                 hipStream_t s);
hipError_t launch_batch_cfl(const BatchParams& p, long long total, hipStream_t s);

}  // namespace mx

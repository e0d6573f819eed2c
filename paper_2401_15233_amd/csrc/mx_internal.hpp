// Internal interface between the C-ABI runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mx {

// Device-resident control block: time step, time and status live on the device so that a
// sequence of steps needs no host round trip.
struct DevCtrl {
  double dt;                     // time step of the current step (0: step is a no-op)
  double t;                      // time after the current step's update
  double t_end;                  // > 0: clip to t_end
  double dt_fixed;               // > 0: fixed time step
  double dt_last;
  unsigned long long maxrate;    // bit pattern of the max CFL rate (positive double)
  long long step;                // steps taken (1-based index of the current step)
  long long n_fallback;          // positivity fallbacks
  int status;                    // bit 1 non-finite, bit 2 unrealizable
  int fail_step;                 // first failing step (0: none)
  long long n_fp64;              // mixed precision: face states re-evaluated in FP64
  long long n_states;            // mixed precision: face states evaluated
  long long n_sigma_limited;     // cells with sigma < sigma_lim (set by the counting kernel)
  int asym;                      // set by the ingest kernel: bit 1 a z-odd moment (u_z, P_xz,
                                 // P_yz, q_z) is non-zero somewhere, bit 2 a y-odd one (u_y,
                                 // P_xy, P_yz, q_y)
};
enum { ASYM_Z = 1, ASYM_Y = 2 };

// 1D tiles: a workgroup of NT threads owns NT - 4 cells, so that the cells plus the two-cell
// halo on each side (NT), the limiter items (NT - 2) and the faces (NT - 3) each take a single
// round over the threads.
constexpr int tile_1d(int nt) { return nt - 4; }

enum { MODE_EULER = 0, MODE_HEUN2 = 1, MODE_MID2 = 2 };
enum { ST_NONFINITE = 1, ST_UNREALIZABLE = 2 };

struct StageParams {
  const double* Ub;        // stage input, read with its neighbourhood
  const double* Ua;        // U^n for the second-stage combinations (may equal Uout)
  double* Uout;
  int nx, ny, pitch;
  long long plane;         // ny * pitch
  double x0, y0, dx, dy, inv_dx, inv_dy;
  int bc[4];
  int n_jets;
  double jet_yc[4], jet_w[4], jet_ang[4];   // centre along the jet's wall, width, angle
  int jet_wall[4];         // 0 x-low, 1 x-high, 2 y-low, 3 y-high
  double jet_mach, jet_rho, jet_T;
  int use_source, tau_mode;
  int src_implicit;        // BGK source by backward Euler on the transported state (EULER mode)
  double tau_ref, rho_ref, T_ref;
  double sigma_lim, kws;
  int limiter, flux, fallback;
  int mode;
  double cdt;              // stage step = cdt * dt (EULER mode)
  int do_cfl;
  int copy_on_idle;        // dt == 0: copy Ub to Uout (forward-Euler ping-pong) instead of skipping
  int ntx, nty;            // tile grid
  int nblk;                // real number of tiles
  double dt_replay;        // > 0: the step's dt (a replayed recorded step); else ctrl->dt
  DevCtrl* ctrl;
};

struct CflParams {
  const double* U;
  int nx, ny, pitch;
  long long plane;
  double dx, dy;
  double sigma_lim, kws;
  DevCtrl* ctrl;
};

// launchers (mx_kernels.hip)
// reduced (14 moments): the state is symmetric and the stage carries only the moments that can
// be non-zero -- 2D planar (u_z = P_xz = P_yz = q_z = 0; ten moments, Sys14P), 1D axial (also
// u_y = P_xy = q_y = 0; seven moments, Sys14A)
hipError_t launch_stage(int system, int dim, int order, int precision, bool reduced,
                        const StageParams& p, hipStream_t s);
hipError_t launch_cfl(int system, int dim, const CflParams& p, hipStream_t s);
hipError_t launch_finalize(DevCtrl* c, int dim, double cfl, double dx, hipStream_t s);
hipError_t launch_ctrl_set(DevCtrl* c, double dt_fixed, double t_end, hipStream_t s);
hipError_t launch_ctrl_reset(DevCtrl* c, double t0, hipStream_t s);
// zero the planes a reduced kernel never writes (2, 3, 5, 6, 8, 11, 12: u_y, u_z, P_xy, P_xz,
// P_yz, q_y, q_z) of a 14-moment field of `plane` doubles per plane (a kernel, no memset);
// nothing for nv != 14
hipError_t launch_zero_planes(double* U, long long plane, int nv, hipStream_t s);
// src/dst: unpadded [nv][ny][nx]; U: padded [nv][ny][pitch]
hipError_t launch_ingest(int system, int repr, const double* src, double* U, int nx, int ny,
                         int pitch, DevCtrl* c, hipStream_t s);
// repr 0 primitive, 1 conserved, 2 sigma, 3 closing moments (19 values per 14-moment cell)
hipError_t launch_egress(int system, int repr, const double* U, double* dst, int nx, int ny,
                         int pitch, double sigma_lim, hipStream_t s);
// zero ctrl->n_sigma_limited first; adds the cells of U with sigma < sigma_lim
hipError_t launch_count_sigma_limited(int system, const double* U, int nx, int ny, int pitch,
                                      double sigma_lim, DevCtrl* c, hipStream_t s);

}  // namespace mx

// C-ABI runtime: handle, device buffers, argument validation, step sequencing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/maxent.h"
#include "mx_internal.hpp"
#include "mx_adjoint_params.hpp"
#include "mx_batch.hpp"

using mx::DevCtrl;

// batched 1D tubes: per-instance records, the work-ordered instance queue, the per-step work
// list, graph of a chunk
struct BatchState {
  int n_inst = 0;
  long long total = 0;
  std::vector<mx::BatchInst> init;       // records as created (t = 0)
  mx::BatchInst* d_inst = nullptr;
  mx::BatchInst* h_inst = nullptr;       // pinned read-back
  mx::BatchCtrl* d_ctrl = nullptr;
  mx::BatchCtrl* h_ctrl = nullptr;       // pinned read-back
  std::vector<int> order;                // instance queue, largest estimated work first
  int* d_order = nullptr;
  int* d_act_inst = nullptr;             // per step: instances that advance, in queue order
  int* d_act_tile0 = nullptr;            // per step: their first tile in the work list (n_inst + 1)
  int* d_cell_inst = nullptr;
  int nt = 64;                           // threads per workgroup
  int cpt = 1;                           // cells per thread: tiles of tile_1d(nt * cpt) cells
  int wg_per_cu = 4;
  int n_cu = 256;
  hipStream_t gstream = nullptr;         // capture stream (a captured graph cannot use the null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_chunk = 0;
  bool graph_valid = false;
};

// recorded run for the discrete adjoint, and the adjoint's workspace
struct TapeState {
  int K = 0;                             // checkpoint every K steps
  int max_steps = 0;
  long long n = 0;                       // steps recorded
  bool failed = false;
  std::vector<double*> ckpt;             // states at steps 0, K, 2K, ... (padded SoA)
  double* d_dt = nullptr;                // time step of every recorded step (device)
  std::vector<double> tau;               // tau_ref of every recorded step
  // adjoint workspace (allocated by the first maxent_step_adjoint)
  std::vector<double*> seg;              // 2K states: states after each step, stage-1 outputs
  double* lam[3] = {nullptr, nullptr, nullptr};
  double* fbx = nullptr;
  double* fby = nullptr;
  double* wb = nullptr;
  double* wext = nullptr;
  double* phix = nullptr;
  double* phiy = nullptr;
  int* vsx = nullptr;
  int* vsy = nullptr;
  double* part = nullptr;
  double* grad = nullptr;
  DevCtrl* actrl = nullptr;              // control block of the replayed stages
};

struct maxent_solver {
  maxent_problem prob;
  maxent_numerics num;
  hipStream_t stream = nullptr;
  int device = 0;
  int nv = 14;
  int pitch = 0;
  long long plane = 0;
  double* U = nullptr;       // current state (padded SoA)
  double* Us = nullptr;      // stage / ping-pong buffer
  double* stage = nullptr;   // unpadded staging for init / get_moments
  DevCtrl* ctrl = nullptr;
  DevCtrl* ctrl_host = nullptr;  // pinned read-back
  bool ready = false;
  bool rate_valid = false;
  // optional per-launch timing of the stage kernels with HIP events
  bool prof = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  long long prof_n = 0;
  BatchState* batch = nullptr;
  TapeState* tape = nullptr;
  int adj_mode = MAXENT_ADJ_EXACT;
  int asym = mx::ASYM_Z | mx::ASYM_Y;  // symmetry of the loaded state (set by the ingest)
  bool reduced_on = true;               // maxent_set_reduced
  std::string err;
  // the 14-moment stage kernels carry only the moments the state's symmetry leaves non-zero:
  // 2D planar (no z-odd moment; ten moments), 1D axial (no y- or z-odd moment; seven)
  bool reduced() const {
    if (!reduced_on || prob.system != 14) return false;
    return prob.dim == 2 ? (asym & mx::ASYM_Z) == 0 : asym == 0;
  }
  bool planar() const { return reduced() && prob.dim == 2; }
};

// message of the last failed call without a handle (maxent_create, maxent_create_batch,
// maxent_step_noalloc); a fixed buffer, so that reporting needs no host allocation
static char g_create_err[512] = "";

static void set_create_err(const char* msg) {
  std::snprintf(g_create_err, sizeof(g_create_err), "%s", msg);
}

static int fail(maxent_solver* s, int code, const std::string& msg) {
  if (s) s->err = msg; else set_create_err(msg.c_str());
  // a failed runtime call (e.g. an allocation beyond the card's memory) leaves its error as the
  // runtime's last error, which the next launch check would report: the error is reported
  // here, so clear it
  if (code == MAXENT_E_NOMEM || code == MAXENT_E_DEVICE) (void)hipGetLastError();
  return code;
}

#define HIP_TRY(s, call)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((s), MAXENT_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// "" when the problem and numerics are consistent, else what is wrong (a literal)
static const char* validate(const maxent_problem& p, const maxent_numerics& n) {
  if (p.system != 5 && p.system != 14) return "system must be 5 or 14";
  if (p.dim != 1 && p.dim != 2) return "dim must be 1 or 2";
  if (p.system == 5 && p.dim != 1) return "the 5-moment system is one-dimensional";
  if (p.nx < 4) return "nx must be >= 4";
  if (p.dim == 1 && p.ny != 1) return "ny must be 1 when dim = 1";
  if (p.dim == 2 && p.ny < 4) return "ny must be >= 4";
  if ((long long)p.nx * p.ny > (1ll << 31)) return "too many cells";
  if (!(p.x1 > p.x0)) return "x1 must exceed x0";
  if (p.dim == 2 && !(p.y1 > p.y0)) return "y1 must exceed y0";
  int nb = p.dim == 2 ? 4 : 2;
  for (int k = 0; k < nb; ++k)
    if (p.bc[k] < 0 || p.bc[k] > 3) return "unknown boundary kind";
  if ((p.bc[0] == MAXENT_BC_PERIODIC) != (p.bc[1] == MAXENT_BC_PERIODIC))
    return "periodic x needs both x sides periodic";
  if (p.dim == 2 && ((p.bc[2] == MAXENT_BC_PERIODIC) != (p.bc[3] == MAXENT_BC_PERIODIC)))
    return "periodic y needs both y sides periodic";
  bool any_jet = false;
  for (int k = 0; k < nb; ++k) any_jet = any_jet || p.bc[k] == MAXENT_BC_JET;
  if (any_jet) {
    if (p.system != 14 || p.dim != 2) return "jet inflow needs the 2D 14-moment system";
    if (p.n_jets < 1 || p.n_jets > 4) return "n_jets must be 1..4";
    if (!(p.jet_rho > 0) || !(p.jet_T > 0) || !(p.jet_mach >= 0)) return "bad jet state";
    for (int k = 0; k < p.n_jets; ++k) {
      if (!(p.jet_width[k] > 0)) return "jet width must be positive";
      if (p.jet_wall[k] < 0 || p.jet_wall[k] > 3) return "jet_wall must be 0..3";
      if (p.bc[p.jet_wall[k]] != MAXENT_BC_JET) return "a jet's wall must have the JET boundary kind";
    }
    for (int w = 0; w < 4; ++w) {
      if (p.bc[w] != MAXENT_BC_JET) continue;
      bool has = false;
      for (int k = 0; k < p.n_jets; ++k) has = has || p.jet_wall[k] == w;
      if (!has) return "a JET side needs at least one jet on it";
    }
  }
  if (p.tau_mode != MAXENT_TAU_LOCAL && p.tau_mode != MAXENT_TAU_CONST) return "bad tau_mode";
  if (p.tau_mode == MAXENT_TAU_LOCAL && !(p.rho_ref > 0 && p.T_ref > 0)) return "bad rho_ref/T_ref";
  if (n.precision != MAXENT_FP64 && n.precision != MAXENT_FP32 && n.precision != MAXENT_MIXED)
    return "unsupported precision";
  if (n.order != 1 && n.order != 2) return "order must be 1 or 2";
  if (n.limiter != MAXENT_MINMOD && n.limiter != MAXENT_VANALBADA) return "bad limiter";
  if (n.flux != MAXENT_HLL && n.flux != MAXENT_RUSANOV) return "bad flux";
  if (n.integrator < MAXENT_FE || n.integrator > MAXENT_MIDPOINT) return "bad integrator";
  if (!(n.cfl > 0 && n.cfl <= 1)) return "cfl must be in (0, 1]";
  if (!(n.sigma_lim > 0 && n.sigma_lim < 1)) return "sigma_lim must be in (0, 1)";
  if (!(n.k_ws >= 1)) return "k_ws must be >= 1";
  if (n.source_implicit != 0 && n.source_implicit != 1) return "source_implicit must be 0 or 1";
  if (n.source_implicit && n.integrator != MAXENT_FE) return "the implicit source needs the FE integrator";
  return "";
}

extern "C" int maxent_abi_version(void) { return MAXENT_ABI_VERSION; }

extern "C" const char* maxent_last_error(const maxent_solver* s) {
  return s ? s->err.c_str() : g_create_err;
}

extern "C" int maxent_num_vars(const maxent_solver* s) { return s ? s->nv : 0; }

static void free_tape(maxent_solver* s) {
  TapeState* t = s->tape;
  if (!t) return;
  (void)hipStreamSynchronize(s->stream);
  for (double* p : t->ckpt) if (p) (void)hipFree(p);
  for (double* p : t->seg) if (p) (void)hipFree(p);
  for (double* p : t->lam) if (p) (void)hipFree(p);
  double* bufs[] = {t->d_dt, t->fbx, t->fby, t->wb, t->wext, t->phix, t->phiy, t->part, t->grad};
  for (double* p : bufs) if (p) (void)hipFree(p);
  if (t->vsx) (void)hipFree(t->vsx);
  if (t->vsy) (void)hipFree(t->vsy);
  if (t->actrl) (void)hipFree(t->actrl);
  delete t;
  s->tape = nullptr;
}

extern "C" void maxent_destroy(maxent_solver* s) {
  if (!s) return;
  free_tape(s);
  (void)hipStreamSynchronize(s->stream);
  if (s->U) (void)hipFree(s->U);
  if (s->Us) (void)hipFree(s->Us);
  if (s->stage) (void)hipFree(s->stage);
  if (s->ctrl) (void)hipFree(s->ctrl);
  if (s->ctrl_host) (void)hipHostFree(s->ctrl_host);
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  if (BatchState* b = s->batch) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->h_inst) (void)hipHostFree(b->h_inst);
    if (b->d_ctrl) (void)hipFree(b->d_ctrl);
    if (b->h_ctrl) (void)hipHostFree(b->h_ctrl);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_act_inst) (void)hipFree(b->d_act_inst);
    if (b->d_act_tile0) (void)hipFree(b->d_act_tile0);
    if (b->d_cell_inst) (void)hipFree(b->d_cell_inst);
    delete b;
  }
  delete s;
}

extern "C" int maxent_create(const maxent_problem* problem, const maxent_numerics* numerics,
                             void* stream, maxent_solver** out) {
  if (!problem || !numerics || !out) return fail(nullptr, MAXENT_E_INVAL, "null argument");
  *out = nullptr;
  std::string why = validate(*problem, *numerics);
  if (!why.empty()) return fail(nullptr, MAXENT_E_INVAL, why);
  maxent_solver* s = new (std::nothrow) maxent_solver();
  if (!s) return fail(nullptr, MAXENT_E_NOMEM, "host allocation failed");
  s->prob = *problem;
  s->num = *numerics;
  if (s->prob.dim == 1) { s->prob.bc[2] = s->prob.bc[3] = MAXENT_BC_TRANSMISSIVE; }
  s->stream = (hipStream_t)stream;
  s->nv = problem->system;
  s->pitch = ((problem->nx + 15) / 16) * 16;   // rows start on 128-byte boundaries
  s->plane = (long long)problem->ny * s->pitch;
  size_t field = (size_t)s->nv * s->plane * sizeof(double);
  // unpadded staging: a field of nv components, or the closing moments (19 per 14-moment cell)
  const int n_stage = s->nv == 14 ? MAXENT_CLOSING_COMPONENTS_14 : s->nv;
  size_t flat = (size_t)n_stage * problem->nx * problem->ny * sizeof(double);
  hipError_t e = hipGetDevice(&s->device);
  if (e == hipSuccess) e = hipMalloc(&s->U, field);
  if (e == hipSuccess) e = hipMalloc(&s->Us, field);
  if (e == hipSuccess) e = hipMalloc(&s->stage, flat);
  if (e == hipSuccess) e = hipMalloc(&s->ctrl, sizeof(DevCtrl));
  if (e == hipSuccess) e = hipHostMalloc(&s->ctrl_host, sizeof(DevCtrl));
  if (e == hipSuccess) e = hipMemsetAsync(s->U, 0, field, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->Us, 0, field, s->stream);
  if (e == hipSuccess) e = mx::launch_ctrl_reset(s->ctrl, 0.0, s->stream);
  if (e != hipSuccess) {
    int code = (e == hipErrorOutOfMemory) ? MAXENT_E_NOMEM : MAXENT_E_DEVICE;
    std::string m = std::string("allocation failed: ") + hipGetErrorString(e);
    maxent_destroy(s);
    return fail(nullptr, code, m);
  }
  *out = s;
  return MAXENT_OK;
}

static mx::StageParams stage_params(maxent_solver* s, double tau_ref) {
  mx::StageParams p;
  std::memset(&p, 0, sizeof(p));
  const maxent_problem& q = s->prob;
  p.nx = q.nx; p.ny = q.ny; p.pitch = s->pitch; p.plane = s->plane;
  p.x0 = q.x0; p.y0 = q.y0;
  p.dx = (q.x1 - q.x0) / q.nx;
  p.dy = q.dim == 2 ? (q.y1 - q.y0) / q.ny : 1.0;
  p.inv_dx = 1.0 / p.dx;
  p.inv_dy = 1.0 / p.dy;
  for (int k = 0; k < 4; ++k) p.bc[k] = q.bc[k];
  bool any_jet = false;
  for (int k = 0; k < 4; ++k) any_jet = any_jet || q.bc[k] == MAXENT_BC_JET;
  p.n_jets = any_jet ? q.n_jets : 0;
  for (int k = 0; k < 4; ++k) {
    p.jet_yc[k] = q.jet_yc[k]; p.jet_w[k] = q.jet_width[k]; p.jet_ang[k] = q.jet_angle_deg[k];
    p.jet_wall[k] = q.jet_wall[k];
  }
  p.jet_mach = q.jet_mach; p.jet_rho = q.jet_rho; p.jet_T = q.jet_T;
  p.use_source = (tau_ref > 0 && std::isfinite(tau_ref)) ? 1 : 0;
  p.src_implicit = s->num.source_implicit;
  p.tau_mode = q.tau_mode; p.tau_ref = tau_ref; p.rho_ref = q.rho_ref; p.T_ref = q.T_ref;
  p.sigma_lim = s->num.sigma_lim; p.kws = s->num.k_ws;
  p.limiter = s->num.limiter; p.flux = s->num.flux; p.fallback = s->num.positivity_fallback;
  if (q.dim == 2) { p.ntx = (q.nx + 15) / 16; p.nty = (q.ny + 14) / 15; }
  else { p.ntx = (q.nx + mx::tile_1d(64) - 1) / mx::tile_1d(64); p.nty = 1; }
  p.nblk = p.ntx * p.nty;
  p.ctrl = s->ctrl;
  return p;
}

static int stage_precision(const maxent_numerics& n) {
  return n.precision == MAXENT_MIXED ? 1 : (n.precision == MAXENT_FP32 ? 2 : 0);
}

static hipError_t stage(maxent_solver* s, int sys, int dim, int ord, const mx::StageParams& p) {
  const int prec = stage_precision(s->num);
  if (!s->prof) return mx::launch_stage(sys, dim, ord, prec, s->reduced(), p, s->stream);
  while (s->ev.size() < s->ev_used + 2) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    try {
      s->ev.push_back(e);
    } catch (const std::bad_alloc&) {
      (void)hipEventDestroy(e);
      return hipErrorOutOfMemory;
    }
  }
  hipError_t r = hipEventRecord(s->ev[s->ev_used], s->stream);
  if (r == hipSuccess) r = mx::launch_stage(sys, dim, ord, prec, s->reduced(), p, s->stream);
  if (r == hipSuccess) r = hipEventRecord(s->ev[s->ev_used + 1], s->stream);
  s->ev_used += 2;
  return r;
}

static hipError_t collect_profile(maxent_solver* s) {
  for (size_t k = 0; k + 1 < s->ev_used; k += 2) {
    float ms = 0.f;
    hipError_t r = hipEventElapsedTime(&ms, s->ev[k], s->ev[k + 1]);
    if (r != hipSuccess) return r;
    s->prof_ms += ms;
    s->prof_n += 1;
  }
  s->ev_used = 0;
  return hipSuccess;
}

static hipError_t run_cfl(maxent_solver* s) {
  mx::CflParams c;
  c.U = s->U; c.nx = s->prob.nx; c.ny = s->prob.ny; c.pitch = s->pitch; c.plane = s->plane;
  c.dx = (s->prob.x1 - s->prob.x0) / s->prob.nx;
  c.dy = s->prob.dim == 2 ? (s->prob.y1 - s->prob.y0) / s->prob.ny : 1.0;
  c.sigma_lim = s->num.sigma_lim; c.kws = s->num.k_ws; c.ctrl = s->ctrl;
  return mx::launch_cfl(s->prob.system, s->prob.dim, c, s->stream);
}

static int read_ctrl(maxent_solver* s) {
  HIP_TRY(s, hipMemcpyAsync(s->ctrl_host, s->ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return MAXENT_OK;
}

static void fill_info(maxent_solver* s, maxent_info* info) {
  if (!info) return;
  const DevCtrl& c = *s->ctrl_host;
  info->t = c.t;
  info->dt_last = c.dt_last;
  info->steps = c.step;
  info->n_fallback = c.n_fallback;
  info->fail_step = (c.fail_step == 0x7fffffff) ? 0 : c.fail_step;
  info->fail_code = c.status;
  info->n_fp64_states = c.n_fp64;
  info->n_face_states = c.n_states;
  info->n_sigma_limited = -1;     // counted by maxent_get_info only
  info->fp64_fraction = c.n_states > 0 ? (double)c.n_fp64 / (double)c.n_states
                                       : (s->num.precision == MAXENT_FP64 ? 1.0 : 0.0);
  info->reduced = s->reduced() ? (s->prob.dim == 2 ? 1 : 2) : 0;
  info->reserved = 0;
}

static mx::BatchParams batch_params(maxent_solver* s) {
  BatchState* b = s->batch;
  mx::BatchParams p;
  std::memset(&p, 0, sizeof(p));
  p.plane = s->plane;
  p.inst = b->d_inst;
  p.act_inst = b->d_act_inst;
  p.act_tile0 = b->d_act_tile0;
  p.bctrl = b->d_ctrl;
  p.cell_inst = b->d_cell_inst;
  p.bc_lo = s->prob.bc[0];
  p.bc_hi = s->prob.bc[1];
  p.tau_mode = s->prob.tau_mode;
  p.rho_ref = s->prob.rho_ref;
  p.T_ref = s->prob.T_ref;
  p.sigma_lim = s->num.sigma_lim;
  p.kws = s->num.k_ws;
  p.limiter = s->num.limiter;
  p.flux = s->num.flux;
  p.fallback = s->num.positivity_fallback;
  p.ctrl = s->ctrl;
  return p;
}

// restore the per-instance records to t = 0 and reduce each instance's first CFL rate
static int batch_reset(maxent_solver* s) {
  BatchState* b = s->batch;
  HIP_TRY(s, hipMemcpyAsync(b->d_inst, b->init.data(), b->init.size() * sizeof(mx::BatchInst),
                            hipMemcpyHostToDevice, s->stream));
  mx::BatchParams p = batch_params(s);
  p.Ub = s->U;
  HIP_TRY(s, mx::launch_batch_cfl(p, b->total, s->stream));
  // instance queue: estimated work = cells x steps to t_end at the initial CFL rate
  HIP_TRY(s, hipMemcpyAsync(b->h_inst, b->d_inst, b->n_inst * sizeof(mx::BatchInst), hipMemcpyDeviceToHost,
                            s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  std::vector<double> work;
  try {
    work.resize(b->n_inst);
  } catch (const std::bad_alloc&) {
    return fail(s, MAXENT_E_NOMEM, "host allocation failed");
  }
  for (int i = 0; i < b->n_inst; ++i) {
    const mx::BatchInst& r = b->h_inst[i];
    double rate = __builtin_bit_cast(double, r.maxrate);
    double w = (double)r.n * r.t_end * rate / (s->num.cfl * r.dx);
    work[i] = std::isfinite(w) ? w : 0.0;
  }
  for (int i = 0; i < b->n_inst; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return work[x] > work[y]; });
  HIP_TRY(s, hipMemcpyAsync(b->d_order, b->order.data(), b->n_inst * sizeof(int), hipMemcpyHostToDevice,
                            s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return MAXENT_OK;
}

extern "C" int maxent_init_state(maxent_solver* s, int repr, const double* src, int src_on_device,
                                 double t0) {
  if (!s) return MAXENT_E_INVAL;
  if (!src) return fail(s, MAXENT_E_INVAL, "null src");
  if (repr != MAXENT_PRIMITIVE && repr != MAXENT_CONSERVED)
    return fail(s, MAXENT_E_INVAL, "repr must be PRIMITIVE or CONSERVED");
  if (!std::isfinite(t0)) return fail(s, MAXENT_E_INVAL, "t0 must be finite");
  free_tape(s);
  size_t flat = (size_t)s->nv * s->prob.nx * s->prob.ny * sizeof(double);
  HIP_TRY(s, hipMemcpyAsync(s->stage, src, flat,
                            src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
  HIP_TRY(s, mx::launch_ctrl_reset(s->ctrl, t0, s->stream));
  HIP_TRY(s, mx::launch_ingest(s->prob.system, repr, s->stage, s->U, s->prob.nx, s->prob.ny,
                               s->pitch, s->ctrl, s->stream));
  if (s->batch) {
    int rc = batch_reset(s);
    if (rc) return rc;
  } else {
    HIP_TRY(s, run_cfl(s));
  }
  // the reduced kernels never write the moments they leave out: the stage / ping-pong buffer
  // starts from zeros there, so that a forward-Euler swap hands back a symmetric state
  HIP_TRY(s, mx::launch_zero_planes(s->Us, s->plane, s->nv, s->stream));
  int rc = read_ctrl(s);
  if (rc) return rc;
  s->asym = s->ctrl_host->asym;
  s->ready = true;
  s->rate_valid = true;
  int st = s->ctrl_host->status;
  if (st) {
    // keep the loaded state but clear the status so that the caller may inspect it
    HIP_TRY(s, mx::launch_ctrl_reset(s->ctrl, t0, s->stream));
    if (!s->batch) HIP_TRY(s, run_cfl(s));
    s->ready = false;
    if (st & mx::ST_NONFINITE) return fail(s, MAXENT_E_NONFINITE, "initial state has non-finite values");
    return fail(s, MAXENT_E_UNREALIZABLE, "initial state has rho <= 0 or a non-SPD pressure tensor");
  }
  return MAXENT_OK;
}

// Enqueue n steps on the solver's stream (no host synchronisation, no allocation): the
// control block sets dt (fixed or CFL) and t_end; each step is the finalize kernel, then one
// stage kernel (FE) or two (SSP-RK2, midpoint); with a tape, each step's dt and tau_ref are
// kept and a checkpoint every K steps.  FE ping-pongs between U and Us (the pointers swap).
static hipError_t enqueue_steps(maxent_solver* s, int n, double dt, double tau_ref, double t_end) {
  TapeState* tape = s->tape;
  const size_t field_bytes = (size_t)s->nv * s->plane * sizeof(double);
  const bool cfl_mode = !(dt > 0);
  mx::StageParams p = stage_params(s, tau_ref);
  const int sys = s->prob.system, dim = s->prob.dim, ord = s->num.order;
  const double dx = (s->prob.x1 - s->prob.x0) / s->prob.nx;
  hipError_t e = mx::launch_ctrl_set(s->ctrl, cfl_mode ? 0.0 : dt, t_end > 0 ? t_end : 0.0, s->stream);
  if (e != hipSuccess) return e;
  if (cfl_mode && !s->rate_valid && (e = run_cfl(s)) != hipSuccess) return e;
  for (int k = 0; k < n; ++k) {
    if ((e = mx::launch_finalize(s->ctrl, dim, s->num.cfl, dx, s->stream)) != hipSuccess) return e;
    if (tape) {
      if ((e = mx::launch_tape_dt(s->ctrl, tape->d_dt + tape->n, s->stream)) != hipSuccess) return e;
      tape->tau.push_back(tau_ref);   // capacity reserved by maxent_record
    }
    if (s->num.integrator == MAXENT_FE) {
      p.Ub = s->U; p.Ua = s->U; p.Uout = s->Us;
      p.mode = mx::MODE_EULER; p.cdt = 1.0; p.do_cfl = cfl_mode; p.copy_on_idle = 1;
      if ((e = stage(s, sys, dim, ord, p)) != hipSuccess) return e;
      // the result lives in Us; swap so that U is always the current state
      double* tmp = s->U; s->U = s->Us; s->Us = tmp;
    } else {
      p.Ub = s->U; p.Ua = s->U; p.Uout = s->Us;
      p.mode = mx::MODE_EULER;
      p.copy_on_idle = 0;
      p.cdt = (s->num.integrator == MAXENT_MIDPOINT) ? 0.5 : 1.0;
      p.do_cfl = 0;
      if ((e = stage(s, sys, dim, ord, p)) != hipSuccess) return e;
      p.Ub = s->Us; p.Ua = s->U; p.Uout = s->U;
      p.mode = (s->num.integrator == MAXENT_MIDPOINT) ? mx::MODE_MID2 : mx::MODE_HEUN2;
      p.cdt = 1.0;
      p.do_cfl = cfl_mode;
      if ((e = stage(s, sys, dim, ord, p)) != hipSuccess) return e;
    }
    if (tape && ++tape->n % tape->K == 0) {
      e = hipMemcpyAsync(tape->ckpt[tape->n / tape->K], s->U, field_bytes, hipMemcpyDeviceToDevice,
                         s->stream);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

extern "C" int maxent_step(maxent_solver* s, int n, double dt, double tau_ref, double t_end,
                           maxent_info* info) {
  if (!s) return MAXENT_E_INVAL;
  if (n < 0) return fail(s, MAXENT_E_INVAL, "n must be >= 0");
  if (std::isnan(dt) || std::isinf(dt)) return fail(s, MAXENT_E_INVAL, "dt must be finite");
  if (std::isnan(tau_ref)) return fail(s, MAXENT_E_INVAL, "tau_ref is NaN");
  if (std::isnan(t_end)) return fail(s, MAXENT_E_INVAL, "t_end is NaN");
  if (!s->ready) return fail(s, MAXENT_E_STATE, "step before a valid init_state");
  if (s->batch) return fail(s, MAXENT_E_STATE, "a batch solver advances with maxent_step_batch");
  TapeState* tape = s->tape;
  if (tape && tape->n + n > tape->max_steps)
    return fail(s, MAXENT_E_INVAL, "the tape would exceed its max_steps");
  const bool cfl_mode = !(dt > 0);
  HIP_TRY(s, enqueue_steps(s, n, dt, tau_ref, t_end));
  int rc = read_ctrl(s);
  if (rc) return rc;
  if (s->prof) HIP_TRY(s, collect_profile(s));
  if (n > 0) s->rate_valid = cfl_mode;  // the last stage reduced the rate of the new state
  fill_info(s, info);
  int st = s->ctrl_host->status;
  if (st && tape) tape->failed = true;
  if (st & mx::ST_NONFINITE) return fail(s, MAXENT_E_NONFINITE, "non-finite cell state");
  if (st & mx::ST_UNREALIZABLE) return fail(s, MAXENT_E_UNREALIZABLE, "rho <= 0 or P not SPD at a cell");
  return MAXENT_OK;
}

// ------------------------------------------------------------------ no-allocation stepping
// Device scratch of maxent_step_noalloc: the control block, then one intermediate state.  Each
// device holds its own copy of this array once the library's code runs on it; host code uses
// the per-device address from hipGetSymbolAddress, never the array's name.
static __device__ __align__(256) unsigned char scratch[MAXENT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

static int noalloc_fail(int code, const char* what, hipError_t e = hipSuccess) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    std::snprintf(g_create_err, sizeof(g_create_err), "%s: %s", what, hipGetErrorString(e));
  } else {
    set_create_err(what);
  }
  return code;
}

extern "C" int maxent_step_noalloc(const maxent_problem* problem, const maxent_numerics* numerics,
                                   double* U, int n, double dt, double tau_ref, double t_end,
                                   double t0, void* stream, maxent_info* info) {
  if (!problem || !numerics || !U) return noalloc_fail(MAXENT_E_INVAL, "null argument");
  if (n < 0) return noalloc_fail(MAXENT_E_INVAL, "n must be >= 0");
  if (!std::isfinite(dt) || std::isnan(tau_ref) || std::isnan(t_end) || !std::isfinite(t0))
    return noalloc_fail(MAXENT_E_INVAL, "dt and t0 must be finite, tau_ref and t_end not NaN");
  const char* why = validate(*problem, *numerics);
  if (*why) return noalloc_fail(MAXENT_E_INVAL, why);
  const int nv = problem->system;
  const long long cells = (long long)problem->nx * problem->ny;
  const long long need = 256 + (long long)nv * cells * (long long)sizeof(double);
  if (need > (long long)MAXENT_NOALLOC_SCRATCH_BYTES)
    return noalloc_fail(MAXENT_E_INVAL, "problem too large for the no-allocation scratch "
                                        "(nv * nx * ny * 8 + 256 bytes must not exceed "
                                        "MAXENT_NOALLOC_SCRATCH_BYTES)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return noalloc_fail(MAXENT_E_DEVICE, "hipGetDevice", e);
  if (dev < 0 || dev >= MAX_DEVICES) return noalloc_fail(MAXENT_E_DEVICE, "device index out of range");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) return noalloc_fail(MAXENT_E_DEVICE, "hipGetSymbolAddress(scratch)", e);
      g_scratch_ptr[dev] = ptr;
    }
    base = g_scratch_ptr[dev];
  }
  // a handle on the stack over the caller's state (pitch = nx: the caller's unpadded layout)
  // and the scratch; it owns nothing, and nothing below allocates
  maxent_solver t;
  t.prob = *problem;
  t.num = *numerics;
  if (t.prob.dim == 1) { t.prob.bc[2] = t.prob.bc[3] = MAXENT_BC_TRANSMISSIVE; }
  t.stream = (hipStream_t)stream;
  t.device = dev;
  t.nv = nv;
  t.pitch = problem->nx;
  t.plane = (long long)problem->ny * problem->nx;
  t.ctrl = (DevCtrl*)base;
  t.U = U;
  t.Us = (double*)((unsigned char*)base + 256);
  t.rate_valid = false;
  static_assert(sizeof(DevCtrl) <= 256, "the control block fits its scratch slot");
  // the control block starts from zero (a kernel, not a memset); the input state is checked
  // in place (conserved in, the same values out) and its first CFL rate reduced
  e = mx::launch_ctrl_reset(t.ctrl, t0, t.stream);
  if (e == hipSuccess)
    e = mx::launch_ingest(nv, MAXENT_CONSERVED, U, U, problem->nx, problem->ny, problem->nx, t.ctrl, t.stream);
  // symmetry of a 14-moment state: read the ingest's flags, and give the scratch state zero
  // planes where a reduced kernel writes none
  if (e == hipSuccess && nv == 14) {
    int asym = mx::ASYM_Z | mx::ASYM_Y;
    e = hipMemcpyAsync(&asym, &t.ctrl->asym, sizeof(int), hipMemcpyDeviceToHost, t.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t.stream);
    if (e == hipSuccess) t.asym = asym;
    if (e == hipSuccess && t.reduced()) e = mx::launch_zero_planes(t.Us, t.plane, nv, t.stream);
  }
  if (e == hipSuccess) e = enqueue_steps(&t, n, dt, tau_ref, t_end);
  // FE ping-pongs: after an odd number of steps the state sits in the scratch
  if (e == hipSuccess && t.U != U)
    e = hipMemcpyAsync(U, t.U, (size_t)nv * cells * sizeof(double), hipMemcpyDeviceToDevice, t.stream);
  DevCtrl host;
  if (e == hipSuccess) e = hipMemcpyAsync(&host, t.ctrl, sizeof(DevCtrl), hipMemcpyDeviceToHost, t.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(t.stream);
  if (e != hipSuccess) return noalloc_fail(MAXENT_E_DEVICE, "maxent_step_noalloc", e);
  if (info) {
    info->t = host.t;
    info->dt_last = host.dt_last;
    info->steps = host.step;
    info->n_fallback = host.n_fallback;
    info->fail_step = (host.fail_step == 0x7fffffff) ? 0 : host.fail_step;
    info->fail_code = host.status;
    info->n_fp64_states = host.n_fp64;
    info->n_face_states = host.n_states;
    info->n_sigma_limited = -1;
    info->fp64_fraction = host.n_states > 0 ? (double)host.n_fp64 / (double)host.n_states
                                            : (numerics->precision == MAXENT_FP64 ? 1.0 : 0.0);
    info->reduced = t.reduced() ? (problem->dim == 2 ? 1 : 2) : 0;
    info->reserved = 0;
  }
  if (host.status & mx::ST_NONFINITE) return noalloc_fail(MAXENT_E_NONFINITE, "non-finite cell state");
  if (host.status & mx::ST_UNREALIZABLE)
    return noalloc_fail(MAXENT_E_UNREALIZABLE, "rho <= 0 or P not SPD at a cell");
  return MAXENT_OK;
}

extern "C" int maxent_get_info(maxent_solver* s, maxent_info* info) {
  if (!s || !info) return MAXENT_E_INVAL;
  if (s->ready || s->batch) {
    HIP_TRY(s, hipMemsetAsync(&s->ctrl->n_sigma_limited, 0, sizeof(long long), s->stream));
    HIP_TRY(s, mx::launch_count_sigma_limited(s->prob.system, s->U, s->prob.nx, s->prob.ny, s->pitch,
                                              s->num.sigma_lim, s->ctrl, s->stream));
  }
  int rc = read_ctrl(s);
  if (rc) return rc;
  fill_info(s, info);
  info->n_sigma_limited = (s->ready || s->batch) ? s->ctrl_host->n_sigma_limited : 0;
  return MAXENT_OK;
}

extern "C" int maxent_get_moments(maxent_solver* s, int repr, double* dst, int dst_on_device) {
  if (!s) return MAXENT_E_INVAL;
  if (!dst) return fail(s, MAXENT_E_INVAL, "null dst");
  if (repr != MAXENT_PRIMITIVE && repr != MAXENT_CONSERVED && repr != MAXENT_SIGMA &&
      repr != MAXENT_CLOSING)
    return fail(s, MAXENT_E_INVAL, "repr must be PRIMITIVE, CONSERVED, SIGMA or CLOSING");
  size_t cells = (size_t)s->prob.nx * s->prob.ny;
  size_t comps = (size_t)s->nv;
  if (repr == MAXENT_SIGMA) comps = 1;
  if (repr == MAXENT_CLOSING) comps = s->nv == 14 ? MAXENT_CLOSING_COMPONENTS_14 : 1;
  size_t bytes = comps * cells * sizeof(double);
  HIP_TRY(s, mx::launch_egress(s->prob.system, repr, s->U, s->stage, s->prob.nx, s->prob.ny,
                               s->pitch, s->num.sigma_lim, s->stream));
  HIP_TRY(s, hipMemcpyAsync(dst, s->stage, bytes,
                            dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  return MAXENT_OK;
}

// ------------------------------------------------------------------ discrete adjoint
extern "C" int maxent_record(maxent_solver* s, int checkpoint_every, int max_steps) {
  if (!s) return MAXENT_E_INVAL;
  if (checkpoint_every < 0) return fail(s, MAXENT_E_INVAL, "checkpoint_every must be >= 0");
  if (checkpoint_every == 0) {
    free_tape(s);
    return MAXENT_OK;
  }
  if (max_steps < 1) return fail(s, MAXENT_E_INVAL, "max_steps must be >= 1");
  if (s->batch) return fail(s, MAXENT_E_STATE, "the adjoint is not available for batch solvers");
  if (s->prob.system != 14) return fail(s, MAXENT_E_INVAL, "the adjoint needs the 14-moment system");
  if (s->num.precision != MAXENT_FP64) return fail(s, MAXENT_E_INVAL, "the adjoint needs FP64 precision");
  if (s->num.source_implicit)
    return fail(s, MAXENT_E_INVAL, "the adjoint needs the explicit BGK source (source_implicit = 0)");
  if (!s->ready) return fail(s, MAXENT_E_STATE, "record before a valid init_state");
  free_tape(s);
  TapeState* t = new (std::nothrow) TapeState();
  if (!t) return fail(s, MAXENT_E_NOMEM, "host allocation failed");
  s->tape = t;
  t->K = checkpoint_every;
  t->max_steps = max_steps;
  const size_t field = (size_t)s->nv * s->plane * sizeof(double);
  const int n_ck = max_steps / checkpoint_every + 1;
  try {
    t->ckpt.assign(n_ck, nullptr);
    t->tau.reserve(max_steps);   // maxent_step appends one entry per step, up to max_steps
  } catch (const std::bad_alloc&) {
    free_tape(s);
    return fail(s, MAXENT_E_NOMEM, "host allocation failed");
  }
  hipError_t e = hipMalloc(&t->d_dt, (size_t)max_steps * sizeof(double));
  for (int k = 0; k < n_ck && e == hipSuccess; ++k) e = hipMalloc(&t->ckpt[k], field);
  if (e == hipSuccess) e = hipMemcpyAsync(t->ckpt[0], s->U, field, hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) {
    free_tape(s);
    return fail(s, e == hipErrorOutOfMemory ? MAXENT_E_NOMEM : MAXENT_E_DEVICE,
                std::string("tape allocation failed: ") + hipGetErrorString(e));
  }
  return MAXENT_OK;
}

extern "C" int maxent_set_adjoint_mode(maxent_solver* s, int mode) {
  if (!s) return MAXENT_E_INVAL;
  if (mode != MAXENT_ADJ_EXACT && mode != MAXENT_ADJ_FROZEN_LIMITER)
    return fail(s, MAXENT_E_INVAL, "unknown adjoint mode");
  s->adj_mode = mode;
  return MAXENT_OK;
}

extern "C" int maxent_set_inflow(maxent_solver* s, double mach, double rho) {
  if (!s) return MAXENT_E_INVAL;
  if (!(mach > 0) || !(rho > 0) || !std::isfinite(mach) || !std::isfinite(rho))
    return fail(s, MAXENT_E_INVAL, "jet Mach number and density must be finite and > 0");
  if (s->tape && s->tape->n > 0)
    return fail(s, MAXENT_E_STATE, "the inflow cannot change while a tape holds recorded steps");
  s->prob.jet_mach = mach;
  s->prob.jet_rho = rho;
  return MAXENT_OK;
}

extern "C" int maxent_tape_info(maxent_solver* s, long long* n_steps, double* dt) {
  if (!s) return MAXENT_E_INVAL;
  TapeState* t = s->tape;
  if (!t) return fail(s, MAXENT_E_STATE, "no tape");
  if (n_steps) *n_steps = t->n;
  if (dt && t->n > 0) {
    HIP_TRY(s, hipMemcpyAsync(dt, t->d_dt, (size_t)t->n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
  }
  return MAXENT_OK;
}

static hipError_t adjoint_workspace(maxent_solver* s) {
  TapeState* t = s->tape;
  if (t->actrl) return hipSuccess;
  const int nx = s->prob.nx, ny = s->prob.ny, dim = s->prob.dim;
  const size_t field = (size_t)s->nv * s->plane * sizeof(double);
  const long long nfx = (long long)(nx + 1) * ny;
  const long long nfy = dim == 2 ? (long long)nx * (ny + 1) : 0;
  const long long eplane = (long long)(nx + 4) * (dim == 2 ? ny + 4 : 1);
  const int nb = mx::adjoint_update_blocks(nx, ny);
  hipError_t e = hipSuccess;
  try {
    t->seg.assign(2 * t->K, nullptr);
  } catch (const std::bad_alloc&) {
    return hipErrorOutOfMemory;
  }
  for (auto& p : t->seg)
    if (e == hipSuccess) e = hipMalloc(&p, field);
  for (auto& p : t->lam)
    if (e == hipSuccess) e = hipMalloc(&p, field);
  if (e == hipSuccess) e = hipMalloc(&t->fbx, (size_t)28 * nfx * sizeof(double));
  if (e == hipSuccess && nfy) e = hipMalloc(&t->fby, (size_t)28 * nfy * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t->wb, (size_t)14 * eplane * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t->wext, (size_t)14 * eplane * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t->phix, (size_t)eplane * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t->phiy, (size_t)eplane * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t->vsx, (size_t)eplane * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&t->vsy, (size_t)eplane * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&t->part, (size_t)3 * nb * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&t->grad, 3 * sizeof(double));
  for (auto& p : t->lam)
    if (e == hipSuccess) e = hipMemsetAsync(p, 0, field, s->stream);
  // the recomputed stage states: the reduced kernels leave the moments they drop as they are
  for (auto& p : t->seg)
    if (e == hipSuccess) e = hipMemsetAsync(p, 0, field, s->stream);
  if (e == hipSuccess) e = hipMalloc(&t->actrl, sizeof(DevCtrl));
  if (e == hipSuccess) e = mx::launch_ctrl_reset(t->actrl, 0.0, s->stream);
  return e;
}

extern "C" int maxent_step_adjoint(maxent_solver* s, const double* dJ_dU, int dJ_on_device,
                                   double* dJ_dU0, int dU0_on_device, double* dJ_dparams) {
  if (!s) return MAXENT_E_INVAL;
  if (!dJ_dU) return fail(s, MAXENT_E_INVAL, "null dJ_dU");
  TapeState* t = s->tape;
  if (!t) return fail(s, MAXENT_E_STATE, "no tape: call maxent_record before stepping");
  if (t->failed) return fail(s, MAXENT_E_STATE, "the recorded run failed; its adjoint is undefined");
  hipError_t e = adjoint_workspace(s);
  if (e != hipSuccess) {
    // leave the tape usable for the forward run; drop the partial workspace
    for (auto& p : t->seg) { if (p) (void)hipFree(p); p = nullptr; }
    for (auto& p : t->lam) { if (p) (void)hipFree(p); p = nullptr; }
    double** bufs[] = {&t->fbx, &t->fby, &t->wb, &t->wext, &t->phix, &t->phiy, &t->part, &t->grad};
    for (double** p : bufs) { if (*p) (void)hipFree(*p); *p = nullptr; }
    int** ibufs[] = {&t->vsx, &t->vsy};
    for (int** p : ibufs) { if (*p) (void)hipFree(*p); *p = nullptr; }
    if (t->actrl) (void)hipFree(t->actrl);
    t->actrl = nullptr;
    t->seg.clear();
    return fail(s, e == hipErrorOutOfMemory ? MAXENT_E_NOMEM : MAXENT_E_DEVICE,
                std::string("adjoint workspace: ") + hipGetErrorString(e));
  }
  const int nx = s->prob.nx, ny = s->prob.ny, dim = s->prob.dim, ord = s->num.order;
  const int integ = s->num.integrator;
  const long long n = t->n;
  const long long K = t->K;
  std::vector<double> dts;
  std::vector<const double*> segU, segS;
  try {
    dts.resize((size_t)n);
    segU.resize((size_t)K + 1);
    segS.resize((size_t)K);
  } catch (const std::bad_alloc&) {
    return fail(s, MAXENT_E_NOMEM, "host allocation failed");
  }
  if (n > 0)
    HIP_TRY(s, hipMemcpyAsync(dts.data(), t->d_dt, (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                              s->stream));
  // lambda <- dJ/dU_final
  const size_t flat = (size_t)s->nv * nx * ny * sizeof(double);
  HIP_TRY(s, hipMemcpyAsync(s->stage, dJ_dU, flat,
                            dJ_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
  // planar run: planar-symmetric recorded states (the planar kernels ran them) and a
  // planar-symmetric dJ/dU keep the z-odd adjoint components at zero
  int nonplanar = 1;
  if (s->planar()) {
    HIP_TRY(s, mx::launch_ctrl_reset(t->actrl, 0.0, s->stream));
    HIP_TRY(s, mx::launch_check_planar(s->stage, (long long)nx * ny, t->actrl, s->stream));
    HIP_TRY(s, hipMemcpyAsync(&nonplanar, &t->actrl->asym, sizeof(int), hipMemcpyDeviceToHost,
                              s->stream));
  }
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  const bool pl = s->planar() && nonplanar == 0;
  double* lamA = t->lam[0];
  double* lamB = t->lam[1];
  double* lamC = t->lam[2];
  if (pl)  // never written in a planar run: they start (and stay) zero
    for (double* l : {lamA, lamB, lamC}) HIP_TRY(s, mx::launch_zero_planes(l, s->plane, 14, s->stream));
  HIP_TRY(s, mx::launch_pad_copy(s->stage, lamA, s->nv, nx, ny, s->pitch, 1, s->stream));
  HIP_TRY(s, hipMemsetAsync(t->part, 0, (size_t)3 * mx::adjoint_update_blocks(nx, ny) * sizeof(double),
                            s->stream));

  mx::AdjParams a;
  std::memset(&a, 0, sizeof(a));
  a.fbx = t->fbx;
  a.fby = t->fby;
  a.nfx = (long long)(nx + 1) * ny;
  a.nfy = dim == 2 ? (long long)nx * (ny + 1) : 0;
  a.wb = t->wb;
  a.wext = t->wext;
  a.phix = t->phix;
  a.phiy = t->phiy;
  a.vsx = t->vsx;
  a.vsy = t->vsy;
  a.frozen_limiter = s->adj_mode == MAXENT_ADJ_FROZEN_LIMITER ? 1 : 0;
  a.epitch = nx + 4;
  a.eplane = (long long)(nx + 4) * (dim == 2 ? ny + 4 : 1);
  a.part = t->part;
  a.n_upd_blocks = mx::adjoint_update_blocks(nx, ny);
  a.grad = t->grad;
  const double cdt1 = (integ == MAXENT_MIDPOINT) ? 0.5 : 1.0;

  const long long nseg = (n + K - 1) / K;
  for (long long sg = nseg - 1; sg >= 0; --sg) {
    const long long k0 = sg * K, k1 = std::min(n, k0 + K);
    const int m = (int)(k1 - k0);
    // 1. recompute the segment's stage inputs from its checkpoint with the recorded dt
    segU[0] = t->ckpt[sg];
    for (int j = 0; j < m; ++j) {
      const double dtk = dts[(size_t)(k0 + j)];
      segS[j] = nullptr;
      if (!(dtk > 0.0)) {  // a no-op step (t_end reached): the state does not change
        segU[j + 1] = segU[j];
        continue;
      }
      const bool need_next = j + 1 < m;  // the last step's output is not an input of any stage
      mx::StageParams p = stage_params(s, t->tau[(size_t)(k0 + j)]);
      p.ctrl = t->actrl;
      p.dt_replay = dtk;   // the recorded dt, passed by value (no control-block update)
      p.do_cfl = 0;
      p.copy_on_idle = 0;
      double* outU = t->seg[(size_t)j];
      if (integ == MAXENT_FE) {
        if (need_next) {
          p.Ub = segU[j]; p.Ua = segU[j]; p.Uout = outU;
          p.mode = mx::MODE_EULER; p.cdt = 1.0;
          HIP_TRY(s, mx::launch_stage(14, dim, ord, 0, s->reduced(), p, s->stream));
        }
        segU[j + 1] = outU;
        continue;
      }
      double* outS = t->seg[(size_t)(K + j)];
      p.Ub = segU[j]; p.Ua = segU[j]; p.Uout = outS;
      p.mode = mx::MODE_EULER; p.cdt = cdt1;
      HIP_TRY(s, mx::launch_stage(14, dim, ord, 0, s->reduced(), p, s->stream));
      segS[j] = outS;
      if (need_next) {
        p.Ub = outS; p.Ua = segU[j]; p.Uout = outU;
        p.mode = (integ == MAXENT_MIDPOINT) ? mx::MODE_MID2 : mx::MODE_HEUN2;
        p.cdt = 1.0;
        HIP_TRY(s, mx::launch_stage(14, dim, ord, 0, s->reduced(), p, s->stream));
      }
      segU[j + 1] = outU;
    }
    // 2. reverse the segment's steps, newest first
    for (int j = m - 1; j >= 0; --j) {
      const double dtk = dts[(size_t)(k0 + j)];
      if (!(dtk > 0.0)) continue;
      a.sp = stage_params(s, t->tau[(size_t)(k0 + j)]);
      a.dt = dtk;
      if (integ == MAXENT_FE) {
        a.sp.Ub = segU[j];
        a.lam_out = lamA; a.lam_extra = nullptr; a.extra_coef = 0.0;
        a.beta = 1.0; a.mu_coef = 1.0; a.lam_in = lamC;
        HIP_TRY(s, mx::launch_adjoint_stage(dim, ord, pl, a, s->stream));
      } else {
        const bool mid = integ == MAXENT_MIDPOINT;
        // second stage: Uout = alpha U^n + beta U* + mu dt L(U*)
        a.sp.Ub = segS[j];
        a.lam_out = lamA; a.lam_extra = nullptr; a.extra_coef = 0.0;
        a.beta = mid ? 0.0 : 0.5; a.mu_coef = mid ? 1.0 : 0.5; a.lam_in = lamB;
        HIP_TRY(s, mx::launch_adjoint_stage(dim, ord, pl, a, s->stream));
        // first stage: U* = U^n + cdt dt L(U^n); U^n also enters the second stage with alpha
        a.sp.Ub = segU[j];
        a.lam_out = lamB; a.lam_extra = lamA; a.extra_coef = mid ? 1.0 : 0.5;
        a.beta = 1.0; a.mu_coef = cdt1; a.lam_in = lamC;
        HIP_TRY(s, mx::launch_adjoint_stage(dim, ord, pl, a, s->stream));
      }
      std::swap(lamA, lamC);
    }
  }
  HIP_TRY(s, mx::launch_adjoint_reduce(a, s->stream));
  if (dJ_dU0) {
    HIP_TRY(s, mx::launch_pad_copy(lamA, s->stage, s->nv, nx, ny, s->pitch, 0, s->stream));
    HIP_TRY(s, hipMemcpyAsync(dJ_dU0, s->stage, flat,
                              dU0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  }
  double g[3] = {0.0, 0.0, 0.0};
  HIP_TRY(s, hipMemcpyAsync(g, t->grad, sizeof(g), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(s, hipStreamSynchronize(s->stream));
  if (dJ_dparams) {
    bool jet = false;
    for (int k = 0; k < 4; ++k) jet = jet || s->prob.bc[k] == MAXENT_BC_JET;
    jet = jet && s->prob.n_jets > 0;
    dJ_dparams[0] = jet ? g[0] : 0.0;
    dJ_dparams[1] = jet ? g[1] : 0.0;
    dJ_dparams[2] = g[2];
  }
  return MAXENT_OK;
}

extern "C" int maxent_set_reduced(maxent_solver* s, int enable) {
  if (!s) return MAXENT_E_INVAL;
  if (s->tape && (enable != 0) != s->reduced_on)
    return fail(s, MAXENT_E_STATE, "the reduced-kernel mode cannot change while a tape is recorded");
  s->reduced_on = enable != 0;
  return MAXENT_OK;
}

extern "C" int maxent_set_profiling(maxent_solver* s, int enable) {
  if (!s) return MAXENT_E_INVAL;
  s->prof = enable != 0;
  s->prof_ms = 0.0;
  s->prof_n = 0;
  s->ev_used = 0;
  return MAXENT_OK;
}

extern "C" int maxent_get_profile(maxent_solver* s, double* stage_ms_total, long long* stage_launches) {
  if (!s || !stage_ms_total || !stage_launches) return MAXENT_E_INVAL;
  *stage_ms_total = s->prof_ms;
  *stage_launches = s->prof_n;
  return MAXENT_OK;
}

// ------------------------------------------------------------------------- batched tubes
extern "C" int maxent_create_batch(const maxent_problem* common, const maxent_numerics* num,
                                   int n_inst, const maxent_instance* inst, void* stream,
                                   maxent_solver** out) {
  if (!common || !num || !inst || !out) return fail(nullptr, MAXENT_E_INVAL, "null argument");
  *out = nullptr;
  if (common->system != 14) return fail(nullptr, MAXENT_E_INVAL, "batched tubes use the 14-moment system");
  if (n_inst < 1 || n_inst > 65536) return fail(nullptr, MAXENT_E_INVAL, "n_inst must be 1..65536");
  if (num->order != 2) return fail(nullptr, MAXENT_E_INVAL, "batched tubes use the second-order scheme");
  if (num->integrator != MAXENT_SSPRK2 && num->integrator != MAXENT_MIDPOINT)
    return fail(nullptr, MAXENT_E_INVAL, "batched tubes use SSPRK2 or MIDPOINT");
  if (num->precision != MAXENT_FP64 && num->precision != MAXENT_MIXED)
    return fail(nullptr, MAXENT_E_INVAL, "batched tubes use FP64 or MIXED precision");
  long long total = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (inst[i].n_cells < 4) return fail(nullptr, MAXENT_E_INVAL, "every instance needs >= 4 cells");
    if (!(inst[i].x1 > inst[i].x0)) return fail(nullptr, MAXENT_E_INVAL, "instance x1 must exceed x0");
    if (!(inst[i].t_end > 0)) return fail(nullptr, MAXENT_E_INVAL, "instance t_end must be > 0");
    if (std::isnan(inst[i].tau_ref)) return fail(nullptr, MAXENT_E_INVAL, "instance tau_ref is NaN");
    total += inst[i].n_cells;
  }
  if (total > (1ll << 31)) return fail(nullptr, MAXENT_E_INVAL, "too many cells");
  maxent_problem p = *common;
  p.dim = 1;
  p.nx = (int)total;
  p.ny = 1;
  p.x0 = 0.0;
  p.x1 = 1.0;
  p.bc[2] = p.bc[3] = MAXENT_BC_TRANSMISSIVE;
  if (p.bc[0] == MAXENT_BC_JET || p.bc[1] == MAXENT_BC_JET) return fail(nullptr, MAXENT_E_INVAL, "no jet inflow in 1D");
  maxent_solver* s = nullptr;
  int rc = maxent_create(&p, num, stream, &s);
  if (rc) return rc;
  BatchState* b = new (std::nothrow) BatchState();
  if (!b) { maxent_destroy(s); return fail(nullptr, MAXENT_E_NOMEM, "host allocation failed"); }
  s->batch = b;
  b->n_inst = n_inst;
  b->total = total;
  std::vector<int> cell_inst;
  try {
    b->init.resize(n_inst);
    b->order.resize(n_inst);
    cell_inst.resize(total);
  } catch (const std::bad_alloc&) {
    maxent_destroy(s);
    return fail(nullptr, MAXENT_E_NOMEM, "host allocation failed");
  }
  long long off = 0;
  for (int i = 0; i < n_inst; ++i) {
    mx::BatchInst r;
    std::memset(&r, 0, sizeof(r));
    r.t_end = inst[i].t_end;
    r.dx = (inst[i].x1 - inst[i].x0) / inst[i].n_cells;
    r.inv_dx = 1.0 / r.dx;
    r.tau_ref = inst[i].tau_ref;
    r.off = off;
    r.n = inst[i].n_cells;
    r.fail_step = 0x7fffffff;
    b->init[i] = r;
    for (int c = 0; c < r.n; ++c) cell_inst[off + c] = i;
    off += r.n;
  }
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, s->device);
  if (e == hipSuccess) b->n_cu = prop.multiProcessorCount;
  if (e == hipSuccess) e = hipMalloc(&b->d_inst, n_inst * sizeof(mx::BatchInst));
  if (e == hipSuccess) e = hipHostMalloc(&b->h_inst, n_inst * sizeof(mx::BatchInst));
  if (e == hipSuccess) e = hipMalloc(&b->d_ctrl, sizeof(mx::BatchCtrl));
  if (e == hipSuccess) e = hipHostMalloc(&b->h_ctrl, sizeof(mx::BatchCtrl));
  if (e == hipSuccess) e = hipMalloc(&b->d_cell_inst, total * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(b->d_cell_inst, cell_inst.data(), total * sizeof(int), hipMemcpyHostToDevice);
  for (int i = 0; i < n_inst; ++i) b->order[i] = i;
  if (e == hipSuccess) e = hipMalloc(&b->d_order, n_inst * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(b->d_order, b->order.data(), n_inst * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&b->d_act_inst, n_inst * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&b->d_act_tile0, (n_inst + 1) * sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(b->d_inst, b->init.data(), n_inst * sizeof(mx::BatchInst), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e != hipSuccess) {
    std::string m = std::string("batch allocation failed: ") + hipGetErrorString(e);
    maxent_destroy(s);
    return fail(nullptr, e == hipErrorOutOfMemory ? MAXENT_E_NOMEM : MAXENT_E_DEVICE, m);
  }
  *out = s;
  return MAXENT_OK;
}

// enqueue `steps` batched steps on stream st
static hipError_t batch_enqueue(maxent_solver* s, int steps, hipStream_t st) {
  BatchState* b = s->batch;
  mx::BatchParams p = batch_params(s);
  const int grid = b->wg_per_cu * b->n_cu;
  const bool mid = s->num.integrator == MAXENT_MIDPOINT;
  const int prec = s->num.precision == MAXENT_MIXED ? 1 : 0;
  for (int k = 0; k < steps; ++k) {
    hipError_t e = mx::launch_batch_finalize(b->d_inst, b->d_order, b->n_inst, s->num.cfl,
                                             mx::tile_1d(b->nt * b->cpt), b->d_act_inst, b->d_act_tile0,
                                             b->d_ctrl, grid, st);
    if (e != hipSuccess) return e;
    p.Ub = s->U; p.Ua = s->U; p.Uout = s->Us;
    p.mode = mx::MODE_EULER; p.cdt = mid ? 0.5 : 1.0; p.do_cfl = 0;
    e = mx::launch_batch_stage(prec, s->reduced(), b->nt, b->cpt, p, grid, st);
    if (e != hipSuccess) return e;
    p.Ub = s->Us; p.Ua = s->U; p.Uout = s->U;
    p.mode = mid ? mx::MODE_MID2 : mx::MODE_HEUN2; p.cdt = 1.0; p.do_cfl = 1;
    e = mx::launch_batch_stage(prec, s->reduced(), b->nt, b->cpt, p, grid, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static int batch_capture(maxent_solver* s, int chunk) {
  BatchState* b = s->batch;
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  b->graph_valid = false;
  hipGraph_t g = nullptr;
  HIP_TRY(s, hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
  hipError_t e = batch_enqueue(s, chunk, b->gstream);
  hipError_t e2 = hipStreamEndCapture(b->gstream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(s, MAXENT_E_DEVICE, std::string("graph capture failed: ") +
                                        hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(s, MAXENT_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  b->graph_chunk = chunk;
  b->graph_valid = true;
  return MAXENT_OK;
}

extern "C" int maxent_step_batch(maxent_solver* s, int max_steps, int chunk, maxent_batch_info* info,
                                 maxent_instance_info* per_inst) {
  if (!s) return MAXENT_E_INVAL;
  if (!s->batch) return fail(s, MAXENT_E_STATE, "not a batch solver (maxent_create_batch)");
  if (!s->ready) return fail(s, MAXENT_E_STATE, "step before a valid init_state");
  if (max_steps < 0 || chunk < 1 || chunk > 100000) return fail(s, MAXENT_E_INVAL, "bad max_steps or chunk");
  BatchState* b = s->batch;
  if (!b->graph_valid || b->graph_chunk != chunk) {
    int rc = batch_capture(s, chunk);
    if (rc) return rc;
  }
  // order the graph replays after earlier work on the caller's stream, and back
  HIP_TRY(s, hipEventRecord(b->ev_in, s->stream));
  HIP_TRY(s, hipStreamWaitEvent(b->gstream, b->ev_in, 0));
  int done = 0;
  while (done < max_steps) {
    HIP_TRY(s, hipGraphLaunch(b->exec, b->gstream));
    done += chunk;
    HIP_TRY(s, hipMemcpyAsync(b->h_ctrl, b->d_ctrl, sizeof(mx::BatchCtrl), hipMemcpyDeviceToHost, b->gstream));
    HIP_TRY(s, hipStreamSynchronize(b->gstream));
    if (b->h_ctrl->n_active == 0) break;
  }
  HIP_TRY(s, hipEventRecord(b->ev_out, b->gstream));
  HIP_TRY(s, hipStreamWaitEvent(s->stream, b->ev_out, 0));
  HIP_TRY(s, hipMemcpyAsync(b->h_inst, b->d_inst, b->n_inst * sizeof(mx::BatchInst), hipMemcpyDeviceToHost,
                            s->stream));
  int rc = read_ctrl(s);
  if (rc) return rc;
  long long max_steps_taken = 0, cell_updates = 0, active = 0;
  int status = 0, first_fail = 0x7fffffff;
  for (int i = 0; i < b->n_inst; ++i) {
    const mx::BatchInst& r = b->h_inst[i];
    if (r.step > max_steps_taken) max_steps_taken = r.step;
    cell_updates += r.step * (long long)r.n;
    if (r.t < r.t_end * (1.0 - 1e-14) && r.status == 0) ++active;
    status |= r.status;
    if (r.status && r.fail_step < first_fail) first_fail = r.fail_step;
    if (per_inst) {
      per_inst[i].t = r.t;
      per_inst[i].dt_last = r.dt_last;
      per_inst[i].steps = r.step;
      per_inst[i].fail_step = r.fail_step == 0x7fffffff ? 0 : r.fail_step;
      per_inst[i].fail_code = r.status;
    }
  }
  if (info) {
    info->max_steps = max_steps_taken;
    info->cell_updates = cell_updates;
    info->n_active = active;
    info->n_fallback = s->ctrl_host->n_fallback;
    info->n_fp64_states = s->ctrl_host->n_fp64;
    info->n_face_states = s->ctrl_host->n_states;
    info->fail_code = status;
    info->fail_step = status ? first_fail : 0;
  }
  if (status & mx::ST_NONFINITE) return fail(s, MAXENT_E_NONFINITE, "non-finite cell state in an instance");
  if (status & mx::ST_UNREALIZABLE) return fail(s, MAXENT_E_UNREALIZABLE, "rho <= 0 or P not SPD in an instance");
  return MAXENT_OK;
}

extern "C" int maxent_set_batch_launch(maxent_solver* s, int threads, int cells_per_thread, int wg_per_cu) {
  if (!s || !s->batch) return MAXENT_E_INVAL;
  if (!mx::batch_shape_supported(threads, cells_per_thread))
    return fail(s, MAXENT_E_INVAL, "threads x cells per thread must be 64x1, 64x2, 64x4, 128x1, 128x2 or 256x1");
  if (wg_per_cu < 1 || wg_per_cu > 32) return fail(s, MAXENT_E_INVAL, "wg_per_cu must be 1..32");
  s->batch->nt = threads;
  s->batch->cpt = cells_per_thread;
  s->batch->wg_per_cu = wg_per_cu;
  s->batch->graph_valid = false;
  return MAXENT_OK;
}

extern "C" int maxent_get_batch_launch(maxent_solver* s, int* threads, int* cells_per_thread, int* wg_per_cu) {
  if (!s || !s->batch || !threads || !cells_per_thread || !wg_per_cu) return MAXENT_E_INVAL;
  *threads = s->batch->nt;
  *cells_per_thread = s->batch->cpt;
  *wg_per_cu = s->batch->wg_per_cu;
  return MAXENT_OK;
}

// Time `trial_steps` steps of every launch shape from the current state and keep the fastest
// (cell-updates per second).  The state and the per-instance records are restored after each
// trial, so the call leaves the solution untouched.
extern "C" int maxent_autotune_batch(maxent_solver* s, int trial_steps, int* threads, int* cells_per_thread,
                                     int* wg_per_cu, double* best_rate) {
  if (!s || !s->batch) return MAXENT_E_INVAL;
  if (!s->ready) return fail(s, MAXENT_E_STATE, "autotune before a valid init_state");
  if (trial_steps < 1 || trial_steps > 10000) return fail(s, MAXENT_E_INVAL, "trial_steps must be 1..10000");
  BatchState* b = s->batch;
  size_t field = (size_t)s->nv * s->plane * sizeof(double);
  size_t recs = b->n_inst * sizeof(mx::BatchInst);
  double* saveU = nullptr;
  mx::BatchInst* saveI = nullptr;
  hipError_t e = hipMalloc(&saveU, field);
  if (e == hipSuccess) e = hipMalloc(&saveI, recs);
  if (e != hipSuccess) {
    if (saveU) (void)hipFree(saveU);
    return fail(s, e == hipErrorOutOfMemory ? MAXENT_E_NOMEM : MAXENT_E_DEVICE,
                std::string("autotune snapshot: ") + hipGetErrorString(e));
  }
  e = hipMemcpyAsync(saveU, s->U, field, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(saveI, b->d_inst, recs, hipMemcpyDeviceToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  const int shapes[6][2] = {{64, 1}, {64, 2}, {64, 4}, {128, 1}, {128, 2}, {256, 1}};
  const int wgs[4] = {2, 4, 8, 16};
  double best = -1.0;
  const int nt0 = b->nt, cpt0 = b->cpt, wg0 = b->wg_per_cu;
  int bt = nt0, bc = cpt0, bw = wg0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int a = 0; a < 6 && e == hipSuccess; ++a) {
    for (int w = 0; w < 4 && e == hipSuccess; ++w) {
      b->nt = shapes[a][0];
      b->cpt = shapes[a][1];
      b->wg_per_cu = wgs[w];
      e = batch_enqueue(s, 1, s->stream);  // warm-up step (first use of the shape)
      if (e == hipSuccess) e = hipMemcpyAsync(s->U, saveU, field, hipMemcpyDeviceToDevice, s->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(b->d_inst, saveI, recs, hipMemcpyDeviceToDevice, s->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
      if (e == hipSuccess) e = batch_enqueue(s, trial_steps, s->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(b->h_inst, b->d_inst, recs, hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) break;
      long long cu = 0;
      for (int i = 0; i < b->n_inst; ++i) cu += b->h_inst[i].step * (long long)b->h_inst[i].n;
      double rate = ms > 0 ? cu / (ms * 1e-3) : 0.0;
      if (rate > best) { best = rate; bt = shapes[a][0]; bc = shapes[a][1]; bw = wgs[w]; }
      e = hipMemcpyAsync(s->U, saveU, field, hipMemcpyDeviceToDevice, s->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(b->d_inst, saveI, recs, hipMemcpyDeviceToDevice, s->stream);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(saveU);
  (void)hipFree(saveI);
  if (e != hipSuccess) {
    // keep the launch shape the solver had before the call
    b->nt = nt0;
    b->cpt = cpt0;
    b->wg_per_cu = wg0;
    b->graph_valid = false;
    return fail(s, MAXENT_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  }
  b->nt = bt;
  b->cpt = bc;
  b->wg_per_cu = bw;
  b->graph_valid = false;
  // counters polluted by the trials
  HIP_TRY(s, mx::launch_ctrl_reset(s->ctrl, 0.0, s->stream));
  if (threads) *threads = bt;
  if (cells_per_thread) *cells_per_thread = bc;
  if (wg_per_cu) *wg_per_cu = bw;
  if (best_rate) *best_rate = best;
  return MAXENT_OK;
}

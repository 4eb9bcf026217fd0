// npw_runtime.cpp -- host runtime behind the C ABI of include/npweno.h: parameter validation,
// device buffers, the tile table, captured HIP graphs of whole SSP-RK3 steps, and readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/npweno.h"
#include "npw_internal.h"

using npw::Ctl;
using npw::InstDev;
using npw::StageArgs;
using npw::Tile;

struct npw_solver {
  int precision = NPW_FP64, flux = 0, ncomp = 1, dim = 1;
  size_t esize = 8;
  int ninst = 0;
  int block = 256;
  hipStream_t user = nullptr;   // caller's stream (ordering only)
  hipStream_t stream = nullptr; // stream of all library work (graphs are captured and replayed here)
  bool own_stream = false;      // the caller passed the default stream: use a private one
  hipEvent_t ev = nullptr;
  std::vector<InstDev> h_inst;  // host copy of the static part of every instance
  InstDev* d_inst = nullptr;
  InstDev* h_pin = nullptr;     // pinned readback of the instance table
  Tile* d_tiles = nullptr;
  int ntiles = 0;
  size_t total = 0;             // elements per state buffer
  void* P0 = nullptr;
  void* P1 = nullptr;
  void* C = nullptr;
  void* scratch = nullptr;      // rhs destination when the caller passes host memory
  std::map<int, hipGraphExec_t> graphs;  // steps per graph -> executable graph
  int sticky_err = 0;
};

namespace {

constexpr int kMaxGraphSteps = 256;  // steps per captured graph (3 stage kernels each)

#define HIP_TRY(expr)                          \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return NPW_EHIP;     \
  } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const npw_params* p) {
  if (!p) return NPW_EINVAL;
  if (p->abi_version != NPW_ABI_VERSION) return NPW_EINVAL;
  if (p->dim != 1 && p->dim != 2) return NPW_EINVAL;
  if (p->nx < 1 || (p->dim == 2 && p->ny < 1)) return NPW_EINVAL;
  if (p->flux == NPW_ADVECTION || p->flux == NPW_BURGERS) {
    if (p->ncomp != 1) return NPW_EINVAL;
  } else if (p->flux == NPW_EULER) {
    if ((p->dim == 1 && p->ncomp != 3) || (p->dim == 2 && p->ncomp != 4)) return NPW_EINVAL;
    if (!(std::isfinite(p->gamma) && p->gamma > 1.0)) return NPW_EINVAL;
  } else {
    return NPW_EINVAL;
  }
  if (p->bc != NPW_PERIODIC && p->bc != NPW_TRANSMISSIVE) return NPW_EINVAL;
  if (p->precision != NPW_FP64 && p->precision != NPW_FP32) return NPW_EINVAL;
  if (p->recon != NPW_RBF_WENO5 && p->recon != NPW_WENO5_JS) return NPW_EINVAL;
  if (p->switch_mode != NPW_SWITCH_MONOTONE && p->switch_mode != NPW_SWITCH_OFF) return NPW_EINVAL;
  if (!(std::isfinite(p->x0) && std::isfinite(p->x1) && p->x1 > p->x0)) return NPW_EINVAL;
  if (p->dim == 2 && !(std::isfinite(p->y0) && std::isfinite(p->y1) && p->y1 > p->y0)) return NPW_EINVAL;
  if (!finite_pos(p->cfl) || !finite_pos(p->eps_weno) || !finite_pos(p->eps_m)) return NPW_EINVAL;
  if (!(std::isfinite(p->dt_fixed) && p->dt_fixed >= 0.0)) return NPW_EINVAL;
  if (!std::isfinite(p->speed_x) || !std::isfinite(p->speed_y)) return NPW_EINVAL;
  if (p->dim == 2) return NPW_EINVAL;  // the 2D stage kernel is not part of this build
  return NPW_OK;
}

int env_block() {
  const char* s = std::getenv("NPW_BLOCK");
  if (!s) return 256;
  int b = std::atoi(s);
  return (b == 128 || b == 256 || b == 512) ? b : 256;
}

hipError_t launch_stage(const npw_solver* s, const StageArgs& a, hipStream_t st) {
  return s->precision == NPW_FP64 ? npw::launch_stage_f64(s->flux, s->ncomp, s->block, a, st)
                                  : npw::launch_stage_f32(s->flux, s->ncomp, s->block, a, st);
}

hipError_t launch_init(const npw_solver* s, hipStream_t st) {
  return s->precision == NPW_FP64 ? npw::launch_init_f64(s->flux, s->ncomp, s->d_inst, s->ninst, s->P0, s->P1, st)
                                  : npw::launch_init_f32(s->flux, s->ncomp, s->d_inst, s->ninst, s->P0, s->P1, st);
}

StageArgs stage_args(const npw_solver* s, int stage, void* out) {
  StageArgs a;
  a.inst = s->d_inst;
  a.tiles = s->d_tiles;
  a.ntiles = s->ntiles;
  a.ntiles_dev = nullptr;
  a.P0 = s->P0;
  a.P1 = s->P1;
  a.C = s->C;
  a.out = out;
  a.stage = stage;
  return a;
}

// Order library work after everything already queued on the caller's stream.
int enter(const npw_solver* s) {
  if (!s->own_stream) return NPW_OK;
  HIP_TRY(hipEventRecord(s->ev, s->user));
  HIP_TRY(hipStreamWaitEvent(s->stream, s->ev, 0));
  return NPW_OK;
}
// Make the caller's stream wait for the library's work.
int leave(const npw_solver* s) {
  if (!s->own_stream) return NPW_OK;
  HIP_TRY(hipEventRecord(s->ev, s->stream));
  HIP_TRY(hipStreamWaitEvent(s->user, s->ev, 0));
  return NPW_OK;
}

// Pull the dynamic part of every instance into pinned memory.
int pull(npw_solver* s) {
  HIP_TRY(hipMemcpyAsync(s->h_pin, s->d_inst, sizeof(InstDev) * s->ninst, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NPW_OK;
}

// Push the static part of every instance (everything before ctl) to the device.
int push_static(npw_solver* s) {
  const size_t width = offsetof(InstDev, ctl);
  HIP_TRY(hipMemcpy2DAsync(s->d_inst, sizeof(InstDev), s->h_inst.data(), sizeof(InstDev), width, s->ninst,
                           hipMemcpyHostToDevice, s->stream));
  return NPW_OK;
}

hipGraphExec_t graph_for(npw_solver* s, int k) {
  auto it = s->graphs.find(k);
  if (it != s->graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  bool ok = true;
  for (int i = 0; i < k && ok; ++i)
    for (int st = 1; st <= 3 && ok; ++st) ok = launch_stage(s, stage_args(s, st, nullptr), s->stream) == hipSuccess;
  hipError_t e = hipStreamEndCapture(s->stream, &g);
  if (!ok || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return nullptr;
  }
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return nullptr;
  s->graphs[k] = ex;
  return ex;
}

// After a failed step: put the control word back at the last good step (its state is still in
// P[n & 1]) and refresh alpha and the sums of that state.
int settle_error(npw_solver* s) {
  for (int b = 0; b < s->ninst; ++b) {
    const InstDev& h = s->h_pin[b];
    if (!h.err) continue;
    Ctl c;
    c.t = h.err_t;
    c.dt = 0.0;
    c.n = h.err_n;
    c.active = 0;
    c.pad = 0;
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(s->d_inst + b) + offsetof(InstDev, ctl), &c, sizeof(Ctl),
                           hipMemcpyHostToDevice, s->stream));
    if (s->sticky_err == 0) s->sticky_err = h.err;
  }
  HIP_TRY(launch_init(s, s->stream));
  return pull(s);
}

void fill_stats(const npw_solver* s, int b, npw_stats* st) {
  const InstDev& h = s->h_pin[b];
  st->t = h.ctl[0].t;
  st->nsteps = h.ctl[0].n;
  for (int d = 0; d < 2; ++d) {
    double v;
    std::memcpy(&v, &h.alpha[0][d], sizeof v);
    st->alpha[d] = v;
  }
  for (int c = 0; c < 4; ++c) st->mass[c] = h.mass[c];
  st->err = h.err;
  st->err_stage = h.err_stage;
}

void release(npw_solver* s) {
  if (!s) return;
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  if (s->P0) (void)hipFree(s->P0);
  if (s->P1) (void)hipFree(s->P1);
  if (s->C) (void)hipFree(s->C);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->d_inst) (void)hipFree(s->d_inst);
  if (s->d_tiles) (void)hipFree(s->d_tiles);
  if (s->h_pin) (void)hipHostFree(s->h_pin);
  if (s->ev) (void)hipEventDestroy(s->ev);
  if (s->stream && s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

InstDev make_inst(const npw_params* p, long long off) {
  InstDev d;
  std::memset(&d, 0, sizeof d);
  d.off = off;
  d.nx = p->nx;
  d.ny = p->dim == 2 ? p->ny : 1;
  d.dx = (p->x1 - p->x0) / (double)p->nx;
  d.dy = p->dim == 2 ? (p->y1 - p->y0) / (double)p->ny : 1.0;
  d.cfl = p->cfl;
  d.dt_fixed = p->dt_fixed;
  d.T = 0.0;
  d.tol = 1e-12;
  d.speed_x = p->speed_x;
  d.speed_y = p->speed_y;
  d.gamma = p->gamma;
  d.eps_weno = p->eps_weno;
  d.eps_m = p->eps_m;
  d.bc = p->bc;
  d.recon = p->recon;
  d.sw = p->switch_mode;
  d.dim = p->dim;
  return d;
}

int upload_state(npw_solver* s, const void* u, int on_device, double t) {
  const size_t bytes = s->total * s->esize;
  HIP_TRY(hipMemcpyAsync(s->P0, u, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream));
  for (int b = 0; b < s->ninst; ++b) {
    InstDev& h = s->h_inst[b];
    std::memset(h.ctl, 0, sizeof h.ctl);
    std::memset(h.alpha, 0, sizeof h.alpha);
    h.ctl[0].t = t;
    h.err = 0;
    h.err_stage = 0;
    h.err_n = 0;
    h.err_t = 0.0;
  }
  HIP_TRY(hipMemcpyAsync(s->d_inst, s->h_inst.data(), sizeof(InstDev) * s->ninst, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(launch_init(s, s->stream));
  int rc = pull(s);
  if (rc) return rc;
  s->sticky_err = 0;
  return s->h_pin[0].err;
}

}  // namespace

extern "C" {

int npweno_abi_version(void) { return NPW_ABI_VERSION; }

const char* npweno_strerror(int code) {
  switch (code) {
    case NPW_OK: return "ok";
    case NPW_EINVAL: return "invalid argument";
    case NPW_ENOMEM: return "out of memory";
    case NPW_EHIP: return "HIP runtime error";
    case NPW_ENONFINITE: return "non-finite cell average";
    case NPW_ENONPHYSICAL: return "non-physical Euler state (density or pressure <= 0)";
    case NPW_EBUSY: return "request not finished";
    case NPW_ENOTFOUND: return "unknown request";
    default: return "unknown error";
  }
}

void npweno_default_params(npw_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->abi_version = NPW_ABI_VERSION;
  p->dim = 1;
  p->flux = NPW_ADVECTION;
  p->ncomp = 1;
  p->bc = NPW_PERIODIC;
  p->precision = NPW_FP64;
  p->recon = NPW_RBF_WENO5;
  p->switch_mode = NPW_SWITCH_MONOTONE;
  p->nx = 80;
  p->ny = 1;
  p->x0 = -1.0;
  p->x1 = 1.0;
  p->y0 = 0.0;
  p->y1 = 1.0;
  p->speed_x = 1.0;
  p->speed_y = 0.0;
  p->gamma = 1.4;
  p->cfl = 0.5;
  p->eps_weno = 1e-6;
  p->eps_m = 1e-12;
  p->dt_fixed = 0.0;
}

int npweno_create(const npw_params* p, const void* u0, int u0_on_device, void* hip_stream, npw_solver** out) {
  if (!out) return NPW_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!u0) return NPW_EINVAL;
  npw_solver* s = new (std::nothrow) npw_solver();
  if (!s) return NPW_ENOMEM;
  s->precision = p->precision;
  s->flux = p->flux;
  s->ncomp = p->ncomp;
  s->dim = p->dim;
  s->esize = p->precision == NPW_FP64 ? sizeof(double) : sizeof(float);
  s->ninst = 1;
  s->block = env_block();
  s->user = reinterpret_cast<hipStream_t>(hip_stream);
  const long long ncell = p->nx * (p->dim == 2 ? p->ny : 1);
  s->total = (size_t)ncell * (size_t)p->ncomp;
  s->h_inst.push_back(make_inst(p, 0));
  const int tile = s->block - 2;
  std::vector<Tile> tiles;
  for (long long st = 0; st < p->nx; st += tile) {
    Tile t;
    t.inst = 0;
    t.pad = 0;
    t.start = st;
    tiles.push_back(t);
  }
  s->ntiles = (int)tiles.size();
  const size_t bytes = s->total * s->esize;
  // Graph capture needs a real stream: the legacy default stream gets a private stream that is
  // ordered against it with an event at every entry point.
  s->own_stream = (s->user == nullptr);
  if (s->own_stream) {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      release(s);
      return NPW_EHIP;
    }
  } else {
    s->stream = s->user;
  }
  if (hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess) {
    release(s);
    return NPW_EHIP;
  }
  if (hipMalloc(&s->P0, bytes) != hipSuccess || hipMalloc(&s->P1, bytes) != hipSuccess ||
      hipMalloc(&s->C, bytes) != hipSuccess || hipMalloc(&s->d_inst, sizeof(InstDev)) != hipSuccess ||
      hipMalloc(&s->d_tiles, sizeof(Tile) * tiles.size()) != hipSuccess ||
      hipHostMalloc(&s->h_pin, sizeof(InstDev), hipHostMallocDefault) != hipSuccess) {
    release(s);
    return NPW_ENOMEM;
  }
  if (enter(s) || hipMemcpyAsync(s->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice,
                                 s->stream) != hipSuccess) {
    release(s);
    return NPW_EHIP;
  }
  rc = upload_state(s, u0, u0_on_device, 0.0);
  if (rc == NPW_OK) rc = leave(s);
  if (rc) {
    release(s);
    return rc;
  }
  *out = s;
  return NPW_OK;
}

int npweno_write(npw_solver* s, const void* u, int on_device, double t) {
  if (!s || !u || !std::isfinite(t)) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  rc = upload_state(s, u, on_device, t);
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

static int run_steps(npw_solver* s, double t_final, int64_t max_steps, int64_t* taken) {
  if (taken) *taken = 0;
  if (!std::isfinite(t_final)) return NPW_EINVAL;
  if (s->sticky_err) return s->sticky_err;
  for (auto& h : s->h_inst) {
    h.T = t_final;
    h.tol = 1e-12 * std::max(1.0, std::fabs(t_final));
  }
  int rc = push_static(s);
  if (rc) return rc;
  int64_t done_steps = 0;
  int k = 1;  // steps per graph replay; grows while the solve is far from its end
  rc = pull(s);
  if (rc) return rc;
  const long long n_start = s->h_pin[0].ctl[0].n;
  while (true) {
    bool all_done = true;
    for (int b = 0; b < s->ninst; ++b) {
      const InstDev& h = s->h_pin[b];
      if (h.err) return settle_error(s) ? NPW_EHIP : h.err;
      if (t_final - h.ctl[0].t > s->h_inst[b].tol) all_done = false;
    }
    done_steps = s->h_pin[0].ctl[0].n - n_start;
    if (taken) *taken = done_steps;
    if (all_done || (max_steps >= 0 && done_steps >= max_steps)) break;
    // choose the graph size: estimate the remaining steps from the last dt
    int want = kMaxGraphSteps;
    const InstDev& h0 = s->h_pin[0];
    if (s->ninst == 1 && h0.ctl[1].dt > 0.0) {
      const double est = (t_final - h0.ctl[0].t) / h0.ctl[1].dt;
      want = est < 1.0 ? 1 : (int)std::min((double)kMaxGraphSteps, std::ceil(est));
    }
    if (max_steps >= 0) want = (int)std::min<int64_t>(want, max_steps - done_steps);
    k = 1;
    while (k * 4 <= want) k *= 4;
    hipGraphExec_t g = graph_for(s, k);
    if (!g) return NPW_EHIP;
    HIP_TRY(hipGraphLaunch(g, s->stream));
    rc = pull(s);
    if (rc) return rc;
  }
  return NPW_OK;
}

int npweno_step(npw_solver* s, double t_final, double* dt_taken) {
  if (!s) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  int64_t taken = 0;
  rc = run_steps(s, t_final, 1, &taken);
  if (dt_taken) *dt_taken = (rc == NPW_OK && taken == 1) ? s->h_pin[0].ctl[1].dt : 0.0;
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

int npweno_solve(npw_solver* s, double t_final, int64_t max_steps, npw_stats* stats) {
  if (!s) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  rc = run_steps(s, t_final, max_steps, nullptr);
  if (stats) {
    HIP_TRY(launch_init(s, s->stream));
    if (pull(s) == NPW_OK) fill_stats(s, 0, stats);
  }
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

int npweno_rhs(npw_solver* s, void* L_out, int out_on_device) {
  if (!s || !L_out) return NPW_EINVAL;
  if (s->sticky_err) return s->sticky_err;
  int rc = enter(s);
  if (rc) return rc;
  const size_t bytes = s->total * s->esize;
  void* dst = L_out;
  if (!out_on_device) {
    if (!s->scratch && hipMalloc(&s->scratch, bytes) != hipSuccess) return NPW_ENOMEM;
    dst = s->scratch;
  }
  HIP_TRY(launch_stage(s, stage_args(s, 0, dst), s->stream));
  if (!out_on_device) HIP_TRY(hipMemcpyAsync(L_out, dst, bytes, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return leave(s);
}

int npweno_read(const npw_solver* cs, void* u_out, int out_on_device) {
  if (!cs || !u_out) return NPW_EINVAL;
  npw_solver* s = const_cast<npw_solver*>(cs);
  int rc = enter(s);
  if (rc) return rc;
  rc = pull(s);
  if (rc) return rc;
  const long long n = s->h_pin[0].ctl[0].n;
  const void* src = (n & 1) ? s->P1 : s->P0;
  HIP_TRY(hipMemcpyAsync(u_out, src, s->total * s->esize, out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return leave(s);
}

int npweno_get_stats(const npw_solver* cs, npw_stats* stats) {
  if (!cs || !stats) return NPW_EINVAL;
  npw_solver* s = const_cast<npw_solver*>(cs);
  int rc = enter(s);
  if (rc) return rc;
  HIP_TRY(launch_init(s, s->stream));
  rc = pull(s);
  if (rc) return rc;
  fill_stats(s, 0, stats);
  if (s->sticky_err) stats->err = s->sticky_err;
  return leave(s);
}

void npweno_destroy(npw_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  release(s);
}

}  // extern "C"

// npw_runtime.cpp -- host runtime behind the C ABI of include/npweno.h: parameter validation,
// device buffers, the tile table, captured HIP graphs of whole SSP-RK3 steps, and readback.
#include <hip/hip_runtime.h>
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
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
  int charw = 0;                // characteristic-wise Euler reconstruction (all instances)
  int any_k2 = 0;               // some instance reconstructs with k = 2
  size_t esize = 8;
  int ninst = 0;
  int block = 256;              // 1D stage workgroup size (tile = block - 2 cells)
  int shape2d = 0;              // 2D tile shape (see npw_internal.h)
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
  unsigned long long* spread = nullptr;  // spread alpha slots (single-grid solvers)
  void* pack = nullptr;                   // packed alpha slots (1D single grids), after the spread
  unsigned long long* bsp = nullptr;      // per-instance spread alpha entries (batches)
  int bsp_k = 0;
  long long most_cells = 0;               // cells of the largest instance
  void* check_part = nullptr;   // partial records of the state check
  int check_G = 1;              // workgroups per instance in the state check
  std::map<int, hipGraphExec_t> graphs;  // (steps per graph, start parity) -> executable graph
  int sticky_err = 0;
  bool batch = false;              // created by npweno_create_batch
  std::vector<Tile> tiles_all;     // every tile of every instance
  std::vector<Tile> tiles_live;    // host source of the last tile-table upload (kept until the next)
  std::vector<char> settled;       // per instance: error already handled
  long long seq_limit = 1LL << 30; // steps after seq_base at which the spread tags are rebased
};

constexpr long long kMaxNy2D = 4LL * 65535;  // tallest 2D grid (126 x 4 tiles, 65535 rows of them)
constexpr long long kMaxElems1D = (1LL << 31) - (1LL << 16);  // largest 1D instance, ncomp * nx

namespace {

// Steps per captured graph (3 stage kernels each).  The host reads the instance table back after
// every graph, which leaves the device idle for ~40 us; a single grid amortises that over 1024
// steps once at least 8 such graphs remain (instantiating a 3072-node graph costs milliseconds,
// which a short solve would not earn back), while a batch keeps 64 so that its tile table drops
// finished instances sooner (4096 Euler Riemann problems to T: 0.567 s with 256, 0.553 s with 64,
// 0.565 s with 16, whose extra graph captures and host round trips cost more than they save).
constexpr int kMaxGraphStepsSingle = 1024;
constexpr int kMaxGraphStepsSingleTail = 256;  // a single grid's graphs once fewer than 8 x 1024 steps remain
constexpr int kMaxGraphStepsBatch = 64;

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
  // 1D kernels index an instance's state with 32-bit integers, including the ghost and halo cells
  // of its last tile (up to BS + 3 past nx), so ncomp * nx keeps a 2^16 margin below 2^31; the 2D
  // grid spans ceil(ny / 4) workgroups along y, at most 65535.
  if (p->dim == 1 && (long long)(p->ncomp > 0 ? p->ncomp : 1) * p->nx > kMaxElems1D) return NPW_EINVAL;
  if (p->dim == 2 && (p->nx > (1 << 30) || p->ny > kMaxNy2D)) return NPW_EINVAL;
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
  if (p->recon < NPW_RBF_WENO5 || p->recon > NPW_RBF_ENO2_2D) return NPW_EINVAL;
  if (p->recon == NPW_RBF_ENO2_2D && (p->dim != 2 || p->variables != NPW_COMPONENTWISE)) return NPW_EINVAL;
  if (p->switch_mode != NPW_SWITCH_MONOTONE && p->switch_mode != NPW_SWITCH_OFF) return NPW_EINVAL;
  if (!(std::isfinite(p->x0) && std::isfinite(p->x1) && p->x1 > p->x0)) return NPW_EINVAL;
  if (p->dim == 2 && !(std::isfinite(p->y0) && std::isfinite(p->y1) && p->y1 > p->y0)) return NPW_EINVAL;
  if (!finite_pos(p->cfl) || !finite_pos(p->eps_weno) || !finite_pos(p->eps_m)) return NPW_EINVAL;
  if (!(std::isfinite(p->dt_fixed) && p->dt_fixed >= 0.0)) return NPW_EINVAL;
  if (!std::isfinite(p->speed_x) || !std::isfinite(p->speed_y)) return NPW_EINVAL;
  if (p->variables != NPW_COMPONENTWISE && (p->variables != NPW_CHARACTERISTIC || p->flux != NPW_EULER))
    return NPW_EINVAL;
  if (p->reserved != 0) return NPW_EINVAL;
  return NPW_OK;
}

int env_block() {
  const char* s = std::getenv("NPW_BLOCK");
  if (!s) return 256;
  int b = std::atoi(s);
  return (b == 64 || b == 128 || b == 256 || b == 512) ? b : 256;
}

hipError_t launch_stage(const npw_solver* s, const StageArgs& a, hipStream_t st) {
  if (s->dim == 2)
    return s->precision == NPW_FP64 ? npw::launch_stage2d_f64(s->flux, s->ncomp, s->shape2d, a, st)
                                    : npw::launch_stage2d_f32(s->flux, s->ncomp, s->shape2d, a, st);
  return s->precision == NPW_FP64 ? npw::launch_stage_f64(s->flux, s->ncomp, s->block, a, st)
                                  : npw::launch_stage_f32(s->flux, s->ncomp, s->block, a, st);
}

hipError_t launch_init(const npw_solver* s, hipStream_t st) {
  return s->precision == NPW_FP64 ? npw::launch_init_f64(s->flux, s->ncomp, s->d_inst, s->ninst, s->P0, s->P1,
                                                         s->spread, s->pack, s->bsp, s->bsp_k, s->check_part, s->check_G,
                                                         st)
                                  : npw::launch_init_f32(s->flux, s->ncomp, s->d_inst, s->ninst, s->P0, s->P1,
                                                         s->spread, s->pack, s->bsp, s->bsp_k, s->check_part, s->check_G,
                                                         st);
}

// A 1D single grid launched with at most 128 threads per workgroup over at most kPackMax tiles
// exchanges alpha through its packed slots (see StageArgs::pack); the block size and so the tile
// count are fixed between state checks, which clear those slots.
// The scheme every instance of the solver uses, when a kernel is built for it alone.
int one_scheme(const npw_solver* s) {
  for (const InstDev& h : s->h_inst)
    if (h.recon != NPW_RBF_WENO5 || h.sw != NPW_SWITCH_MONOTONE) return npw::kSchemeAny;
  return npw::kSchemeRbfWeno5Switch;
}

bool use_pack(const npw_solver* s) { return s->pack != nullptr && s->block <= 128 && s->ntiles <= npw::kPackMax; }

StageArgs stage_args(const npw_solver* s, int stage, int par, void* out) {
  StageArgs a;
  a.inst = s->d_inst;
  a.tiles = s->ninst == 1 ? nullptr : s->d_tiles;
  a.ntiles = s->ntiles;
  a.ntiles_dev = nullptr;
  a.nx = s->h_inst[0].nx;
  a.ny = s->h_inst[0].ny;
  a.bc = s->h_inst[0].bc;
  a.par = par;
  a.P0 = s->P0;
  a.P1 = s->P1;
  a.C = s->C;
  a.out = out;
  a.stage = stage;
  a.charw = s->charw;
  a.any_k2 = s->any_k2;
  a.spread = s->spread;
  a.pack = use_pack(s) ? s->pack : nullptr;
  a.bsp = s->bsp && s->most_cells > (long long)npw::kBspLaunchTiles * (s->block - 2) ? s->bsp : nullptr;
  a.bsp_k = s->bsp_k;
  a.scheme = one_scheme(s);
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

// Graph of k whole steps whose first step reads u^n from P[par]; the buffers alternate per step.
hipGraphExec_t graph_for(npw_solver* s, int k, int par) {
  const int key = 2 * k + par;
  auto it = s->graphs.find(key);
  if (it != s->graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  bool ok = true;
  for (int i = 0; i < k && ok; ++i)
    for (int st = 1; st <= 3 && ok; ++st)
      ok = launch_stage(s, stage_args(s, st, par ^ (i & 1), nullptr), s->stream) == hipSuccess;
  hipError_t e = hipStreamEndCapture(s->stream, &g);
  if (!ok || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return nullptr;
  }
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return nullptr;
  s->graphs[key] = ex;
  return ex;
}

// After a failed step of instance b: put its control word back at the last good step (that
// state is still in its home buffer) and refresh alpha and the sums of every state.
int settle_error(npw_solver* s, int b) {
  const InstDev& h = s->h_pin[b];
  Ctl c;
  c.t = h.err_t;
  c.dt = 0.0;
  c.n = h.err_n;
  c.active = 0;
  c.home = h.err_home;
  HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(s->d_inst + b) + offsetof(InstDev, ctl), &c, sizeof(Ctl),
                         hipMemcpyHostToDevice, s->stream));
  if (s->sticky_err == 0 && !s->batch) s->sticky_err = h.err;
  HIP_TRY(launch_init(s, s->stream));
  return pull(s);
}

void clear_graphs(npw_solver* s) {
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
}

// Float-bulk single grids tag their spread alpha entries with 32 bits of 3 (n - seq_base) + stage.
// Before a graph could take that past 3 * seq_limit (2^30 steps by default, far below 2^32 / 3),
// move seq_base to the current step and run the state check, which clears every entry and seeds
// slot 0 with alpha of u^n under sequence 0.  NPW_SEQ_REBASE lowers the limit (for tests).
bool tagged_spread(const npw_solver* s) { return s->spread != nullptr && s->precision == NPW_FP32; }

int maybe_rebase(npw_solver* s, int k) {
  if (!tagged_spread(s)) return NPW_OK;
  const long long n = s->h_pin[0].ctl[0].n;
  if (n + k - s->h_inst[0].seq_base <= s->seq_limit) return NPW_OK;
  s->h_inst[0].seq_base = n;
  int rc = push_static(s);
  if (rc) return rc;
  HIP_TRY(launch_init(s, s->stream));
  return pull(s);
}

// Tile table of the instances flagged in `want`.  Tiles of finished instances cost one
// early-exit workgroup each, so the table is only rebuilt when it is forced (start of a solve)
// or when at most 3/4 of its tiles still belong to running instances.  Graphs hold the tile
// count, so they are re-captured when it changes.
int set_tiles(npw_solver* s, const std::vector<char>& want, bool force) {
  if (!s->batch) return NPW_OK;  // a single grid derives its tiles from the block index
  size_t n = 0;
  for (const Tile& x : s->tiles_all) n += want[x.inst] ? 1 : 0;
  if (!force && 4 * n > 3 * (size_t)s->ntiles) return NPW_OK;
  // the asynchronous copy reads tiles_live after this returns; the caller synchronizes the stream
  // (pull) before the next call can refill it
  std::vector<Tile>& t = s->tiles_live;
  t.clear();
  t.reserve(n);
  for (const Tile& x : s->tiles_all)
    if (want[x.inst]) t.push_back(x);
  if (!t.empty())
    HIP_TRY(hipMemcpyAsync(s->d_tiles, t.data(), sizeof(Tile) * t.size(), hipMemcpyHostToDevice, s->stream));
  if ((int)t.size() != s->ntiles) clear_graphs(s);
  s->ntiles = (int)t.size();
  return NPW_OK;
}

// Stepped instances advance in lockstep, so their u^n must sit in the same ping-pong buffer:
// move the minority to the majority's buffer (device copies) and report that buffer.
int align_homes(npw_solver* s, int* gp_out) {
  int votes[2] = {0, 0};
  for (int b = 0; b < s->ninst; ++b)
    if (!s->h_pin[b].err) votes[s->h_pin[b].ctl[0].home & 1]++;
  const int gp = votes[1] > votes[0] ? 1 : 0;
  bool moved = false;
  for (int b = 0; b < s->ninst; ++b) {
    const InstDev& h = s->h_pin[b];
    if (h.err || h.ctl[0].home == gp) continue;
    const size_t len = (size_t)s->ncomp * (size_t)(h.nx * h.ny) * s->esize;
    char* from = static_cast<char*>(h.ctl[0].home ? s->P1 : s->P0) + (size_t)h.off * s->esize;
    char* to = static_cast<char*>(gp ? s->P1 : s->P0) + (size_t)h.off * s->esize;
    HIP_TRY(hipMemcpyAsync(to, from, len, hipMemcpyDeviceToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(s->d_inst + b) + offsetof(InstDev, ctl) + offsetof(Ctl, home),
                           &gp, sizeof(int), hipMemcpyHostToDevice, s->stream));
    moved = true;
  }
  *gp_out = gp;
  return moved ? pull(s) : NPW_OK;
}

int reset_instances(npw_solver* s, double t);

// ---- tiles and block size --------------------------------------------------------------------
constexpr int kBlocks[4] = {64, 128, 256, 512};  // smallest first (max_tiles)

size_t max_tiles(const npw_solver* s) {
  if (!s->batch) return 1;  // no table: tiles follow from the block index
  size_t n = 0;
  for (const InstDev& h : s->h_inst) n += (size_t)((h.nx + kBlocks[0] - 3) / (kBlocks[0] - 2));
  return std::max<size_t>(n, 1);
}

// Tile list of every instance for the current block size (BS - 2 owned cells per tile).
void build_tiles(npw_solver* s) {
  const int tile = s->block - 2;
  s->tiles_all.clear();
  if (!s->batch) {  // one placeholder entry; the grid covers ceil(nx / tile) tiles
    const InstDev& h = s->h_inst[0];
    Tile t;
    t.inst = 0;
    t.bc = h.bc;
    t.start = 0;
    t.nx = h.nx;
    t.off = 0;
    s->tiles_all.push_back(t);
    s->ntiles = (int)((h.nx + tile - 1) / tile);
    return;
  }
  for (int b = 0; b < s->ninst; ++b) {
    const InstDev& h = s->h_inst[b];
    for (long long st = 0; st < h.nx; st += tile) {
      Tile t;
      t.inst = b;
      t.bc = h.bc;
      t.start = st;
      t.nx = h.nx;
      t.off = h.off;
      s->tiles_all.push_back(t);
    }
  }
  s->ntiles = (int)s->tiles_all.size();
}

int set_block(npw_solver* s, int block) {
  s->block = block;
  build_tiles(s);
  clear_graphs(s);
  HIP_TRY(hipMemcpyAsync(s->d_tiles, s->tiles_all.data(), sizeof(Tile) * s->tiles_all.size(), hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NPW_OK;
}

std::string tune_path() {
  if (const char* p = std::getenv("NPW_TUNE_CACHE")) return p;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/npweno_tune.txt";
  return "";
}

std::string tune_key(const npw_solver* s) {
  long long cells = 0;
  for (const InstDev& h : s->h_inst) cells += h.nx * h.ny;
  int lg = 0;
  while ((1ll << (lg + 1)) <= cells) ++lg;
  std::ostringstream k;
  k << "v3_d" << s->dim << "_f" << s->flux << "_m" << s->ncomp << "_p" << s->precision << "_n" << lg << "_i"
    << (s->ninst > 1 ? 1 : 0) << (s->charw ? "_c" : "");
  return k.str();
}

int tune_lookup(const std::string& key) {
  std::ifstream f(tune_path());
  std::string k;
  int b;
  int found = -1;
  const bool two_d = key.find("_d2_") != std::string::npos;
  while (f >> k >> b)
    if (k == key && (two_d ? (b >= 0 && b < npw::k2dShapes) : (b == 64 || b == 128 || b == 256 || b == 512))) found = b;
  return found;
}

void tune_store(const std::string& key, int block) {
  const std::string path = tune_path();
  if (path.empty()) return;
  // create missing parent directories (no shell: plain mkdir calls)
  for (size_t at = path.find('/', 1); at != std::string::npos; at = path.find('/', at + 1))
    (void)::mkdir(path.substr(0, at).c_str(), 0755);
  std::ofstream f(path, std::ios::app);
  if (f) f << key << " " << block << "\n";
}

// Autotuner: pick the 1D stage block size (or the 2D tile shape) by timing a short graph with
// every candidate on a copy of the initial state, then restore that state.  The choice is cached
// per (dimension, flux, components, precision, log2 cells, batch) in a small text file.  Every
// candidate computes each cell with the same arithmetic, so the choice never changes results.
// NPW_BLOCK / NPW_TILE2D fix the knob; NPW_AUTOTUNE=0 keeps the default.
// Candidate c of the tuned knob: the 1D block size, or the 2D tile shape.
int candidate_count(const npw_solver* s) { return s->dim == 1 ? 4 : npw::k2dShapes; }
int candidate_value(const npw_solver* s, int c) { return s->dim == 1 ? kBlocks[c] : c; }
int apply_candidate(npw_solver* s, int v) {
  if (s->dim == 1) return set_block(s, v);
  s->shape2d = v;
  clear_graphs(s);
  return NPW_OK;
}

int autotune(npw_solver* s) {
  if (s->dim == 1 && std::getenv("NPW_BLOCK")) return NPW_OK;
  if (s->dim == 2 && std::getenv("NPW_TILE2D")) {
    const int v = std::atoi(std::getenv("NPW_TILE2D"));
    return apply_candidate(s, (v >= 0 && v < npw::k2dShapes) ? v : 0);
  }
  const char* at = std::getenv("NPW_AUTOTUNE");
  if (at && std::strcmp(at, "0") == 0) return NPW_OK;
  const std::string key = tune_key(s);
  const int cached = tune_lookup(key);
  if (cached >= 0) return apply_candidate(s, cached);
  const size_t bytes = s->total * s->esize;
  void* backup = nullptr;
  if (hipMalloc(&backup, bytes) != hipSuccess) return NPW_OK;  // tuning is optional
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int best = s->dim == 1 ? s->block : s->shape2d;
  int rc = NPW_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMemcpyAsync(backup, s->P0, bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess) {
    rc = NPW_EHIP;
  }
  // Every candidate is timed once per round, rounds interleaved, and keeps its fastest round, so
  // a transient slowdown cannot decide the choice.  1D grids time 64 steps (16 beyond 4 Mi
  // cells), 2D grids 2.
  long long cells = 0;
  for (const InstDev& h : s->h_inst) cells += h.nx * h.ny;
  const int steps = s->dim == 1 ? (cells <= (1ll << 22) ? 64 : 16) : 2;
  const int nc = candidate_count(s);
  std::vector<float> fastest(nc, 1e30f);
  for (int round = 0; round < 3 && rc == NPW_OK; ++round) {
    for (int ci = 0; ci < nc && rc == NPW_OK; ++ci) {
      rc = apply_candidate(s, candidate_value(s, ci));
      for (auto& h : s->h_inst) {
        h.T = 1e300;
        h.tol = 0.0;
      }
      float ms = 0.0f;
      for (int rep = 0; rep < 2 && rc == NPW_OK; ++rep) {  // the first replay of a new graph warms up
        if (hipMemcpyAsync(s->P0, backup, bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess) rc = NPW_EHIP;
        if (rc == NPW_OK) rc = reset_instances(s, 0.0);
        if (rc != NPW_OK) break;
        hipGraphExec_t g = graph_for(s, steps, 0);
        if (!g) {
          rc = NPW_EHIP;
          break;
        }
        if (hipEventRecord(e0, s->stream) != hipSuccess || hipGraphLaunch(g, s->stream) != hipSuccess ||
            hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          rc = NPW_EHIP;
      }
      if (rc == NPW_OK && ms < fastest[ci]) fastest[ci] = ms;
    }
  }
  float best_ms = 1e30f;
  for (int ci = 0; ci < nc; ++ci)
    if (fastest[ci] < best_ms) {
      best_ms = fastest[ci];
      best = candidate_value(s, ci);
    }
  for (auto& h : s->h_inst) {
    h.T = 0.0;
    h.tol = 1e-12;
  }
  if (rc == NPW_OK) rc = apply_candidate(s, best);
  if (rc == NPW_OK && hipMemcpyAsync(s->P0, backup, bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess)
    rc = NPW_EHIP;
  if (rc == NPW_OK) rc = reset_instances(s, 0.0);
  if (rc == NPW_OK) rc = push_static(s);
  (void)hipStreamSynchronize(s->stream);
  (void)hipFree(backup);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc == NPW_OK) tune_store(key, best);
  return rc;
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
  if (s->spread) (void)hipFree(s->spread);
  if (s->bsp) (void)hipFree(s->bsp);
  if (s->check_part) (void)hipFree(s->check_part);
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
  d.inv_dx = 1.0 / d.dx;
  d.inv_dy = 1.0 / d.dy;
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

// Every instance restarts at time t from the state in P0 (step count, error and home reset),
// followed by the state check.  Returns the first error the check finds.
int reset_instances(npw_solver* s, double t) {
  for (int b = 0; b < s->ninst; ++b) {
    InstDev& h = s->h_inst[b];
    std::memset(h.ctl, 0, sizeof h.ctl);
    std::memset(h.alpha, 0, sizeof h.alpha);
    h.ctl[0].t = t;
    h.seq_base = 0;
    h.err = 0;
    h.err_stage = 0;
    h.err_n = 0;
    h.err_t = 0.0;
    h.err_home = 0;
  }
  HIP_TRY(hipMemcpyAsync(s->d_inst, s->h_inst.data(), sizeof(InstDev) * s->ninst, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(launch_init(s, s->stream));
  int rc = pull(s);
  if (rc) return rc;
  s->sticky_err = 0;
  for (int b = 0; b < s->ninst; ++b)
    if (s->h_pin[b].err) return s->h_pin[b].err;
  return NPW_OK;
}

}  // namespace

static int run_steps(npw_solver* s, const double* T, int64_t max_steps, int64_t* taken);

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
    case NPW_ESCRATCH: return "the grid needs more scratch than the fixed device array holds";
    default: return "unknown error";
  }
}

static void npweno_default_params_impl(npw_params* p) {
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
  p->variables = NPW_COMPONENTWISE;
  p->reserved = 0;
}

// Build a solver for `count` instances sharing precision, flux and dimension.  u0[b] holds the
// initial state of instance b.
static int create_common(const npw_params* p, int32_t count, const void* const* u0, int on_device, void* hip_stream,
                         bool batch, npw_solver** out) {
  if (!out) return NPW_EINVAL;
  *out = nullptr;
  if (!p || !u0 || count < 1) return NPW_EINVAL;
  for (int b = 0; b < count; ++b) {
    int rc = validate(&p[b]);
    if (rc) return rc;
    if (batch && p[b].dim != 1) return NPW_EINVAL;  // batches are 1D
    if (!u0[b]) return NPW_EINVAL;
    if (p[b].precision != p[0].precision || p[b].flux != p[0].flux || p[b].ncomp != p[0].ncomp ||
        p[b].dim != p[0].dim || p[b].variables != p[0].variables)
      return NPW_EINVAL;
  }
  npw_solver* s = new (std::nothrow) npw_solver();
  if (!s) return NPW_ENOMEM;
  s->precision = p[0].precision;
  s->flux = p[0].flux;
  s->ncomp = p[0].ncomp;
  s->dim = p[0].dim;
  s->charw = p[0].variables == NPW_CHARACTERISTIC ? 1 : 0;
  for (int b = 0; b < count; ++b) s->any_k2 |= p[b].recon >= NPW_RBF_WENO3 ? 1 : 0;
  s->esize = p[0].precision == NPW_FP64 ? sizeof(double) : sizeof(float);
  s->ninst = count;
  s->batch = batch;
  s->block = env_block();
  if (const char* e = std::getenv("NPW_SEQ_REBASE")) {
    const long long v = std::atoll(e);
    if (v >= 1 && v <= (1LL << 30)) s->seq_limit = v;
  }
  s->user = reinterpret_cast<hipStream_t>(hip_stream);
  long long off = 0;
  for (int b = 0; b < count; ++b) {
    s->h_inst.push_back(make_inst(&p[b], off));
    off += (long long)p[b].ncomp * p[b].nx * (p[b].dim == 2 ? p[b].ny : 1);
  }
  build_tiles(s);  // also sets ntiles
  s->total = (size_t)off;
  // state-check workgroups per instance: one per 16 Ki cells of a single grid, at most 512
  if (!batch) {
    const long long cells = s->h_inst[0].nx * s->h_inst[0].ny;
    s->check_G = (int)std::min<long long>(512, std::max<long long>(1, cells / 16384));
  }
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
      hipMalloc(&s->C, bytes) != hipSuccess || hipMalloc(&s->d_inst, sizeof(InstDev) * count) != hipSuccess ||
      hipMalloc(&s->d_tiles, sizeof(Tile) * max_tiles(s)) != hipSuccess ||
      hipHostMalloc(&s->h_pin, sizeof(InstDev) * count, hipHostMallocDefault) != hipSuccess ||
      (!batch && hipMalloc(&s->spread, sizeof(unsigned long long) * (npw::kSpreadWords + npw::kPackWords)) !=
                     hipSuccess) ||
      hipMalloc(&s->check_part, (size_t)npw::kCheckPartialBytes * s->check_G * count) != hipSuccess) {
    release(s);
    return NPW_ENOMEM;
  }
  if (s->spread && s->dim == 1) s->pack = s->spread + npw::kSpreadWords;
  if (batch) {  // spread entries per instance, as many as its largest instance's tiles call for
    for (const InstDev& h : s->h_inst) s->most_cells = std::max(s->most_cells, h.nx);
    s->bsp_k = npw::bsp_entries((s->most_cells + kBlocks[0] - 3) / (kBlocks[0] - 2));
    if (hipMalloc(&s->bsp, sizeof(unsigned long long) * (size_t)count * 3 * s->bsp_k * npw::kSpreadStride) !=
        hipSuccess) {
      release(s);
      return NPW_ENOMEM;
    }
  }
  if (enter(s) || hipMemcpyAsync(s->d_tiles, s->tiles_all.data(), sizeof(Tile) * s->tiles_all.size(),
                                 hipMemcpyHostToDevice, s->stream) != hipSuccess) {
    release(s);
    return NPW_EHIP;
  }
  int rc = NPW_OK;
  for (int b = 0; b < count && rc == NPW_OK; ++b) {
    const size_t len = (size_t)p[b].ncomp * (size_t)(p[b].nx * (p[b].dim == 2 ? p[b].ny : 1)) * s->esize;
    char* dst = static_cast<char*>(s->P0) + (size_t)s->h_inst[b].off * s->esize;
    if (hipMemcpyAsync(dst, u0[b], len, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s->stream) !=
        hipSuccess)
      rc = NPW_EHIP;
  }
  if (rc == NPW_OK) rc = reset_instances(s, 0.0);
  if (rc == NPW_OK) rc = autotune(s);
  if (rc == NPW_OK) rc = leave(s);
  if (rc) {
    release(s);
    return rc;
  }
  *out = s;
  return NPW_OK;
}

static int npweno_create_impl(const npw_params* p, const void* u0, int u0_on_device, void* hip_stream, npw_solver** out) {
  const void* one[1] = {u0};
  return create_common(p, 1, one, u0_on_device, hip_stream, false, out);
}

static int npweno_create_batch_impl(const npw_params* params, int32_t count, const void* const* u0, int on_device,
                        void* hip_stream, npw_solver** out) {
  return create_common(params, count, u0, on_device, hip_stream, true, out);
}

static int npweno_solve_batch_impl(npw_solver* s, const double* t_final, int64_t max_steps, npw_stats* per_instance) {
  if (!s || !t_final) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  rc = run_steps(s, t_final, max_steps, nullptr);
  if (per_instance) {
    HIP_TRY(launch_init(s, s->stream));
    if (pull(s) == NPW_OK)
      for (int b = 0; b < s->ninst; ++b) fill_stats(s, b, &per_instance[b]);
  }
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

static int npweno_read_instance_impl(const npw_solver* cs, int32_t index, void* u_out, int out_on_device) {
  if (!cs || !u_out || index < 0 || index >= cs->ninst) return NPW_EINVAL;
  npw_solver* s = const_cast<npw_solver*>(cs);
  int rc = enter(s);
  if (rc) return rc;
  rc = pull(s);
  if (rc) return rc;
  const InstDev& h = s->h_pin[index];
  const size_t len = (size_t)s->ncomp * (size_t)(h.nx * h.ny) * s->esize;
  const char* src = static_cast<const char*>(h.ctl[0].home ? s->P1 : s->P0) + (size_t)h.off * s->esize;
  HIP_TRY(hipMemcpyAsync(u_out, src, len, out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return leave(s);
}

static int npweno_get_stats_instance_impl(const npw_solver* cs, int32_t index, npw_stats* stats) {
  if (!cs || !stats || index < 0 || index >= cs->ninst) return NPW_EINVAL;
  npw_solver* s = const_cast<npw_solver*>(cs);
  int rc = enter(s);
  if (rc) return rc;
  HIP_TRY(launch_init(s, s->stream));
  rc = pull(s);
  if (rc) return rc;
  fill_stats(s, index, stats);
  return leave(s);
}

int npweno_instance_count(const npw_solver* s) { return s ? s->ninst : 0; }

static int npweno_launch_shape_impl(const npw_solver* s, int32_t* block_1d, int32_t* tile_x, int32_t* tile_y,
                        int32_t* lds_shared) {
  if (!s) return NPW_EINVAL;
  static const int kTx[npw::k2dShapes] = {64, 62, 126, 64, 62, 126, 62, 62, 62};
  static const int kTy[npw::k2dShapes] = {8, 8, 4, 8, 8, 4, 16, 32, 64};
  // the strips run only 2D Euler with component-wise k = 3; other schemes take the 62 x 8 tile
  const bool strip_ok = s->flux == npw::kEuler && s->ncomp == 4 && !s->charw && !s->any_k2;
  const int shape = s->shape2d >= npw::k2dStripFirst && !strip_ok ? 4 : s->shape2d;
  if (block_1d) *block_1d = s->block;
  if (tile_x) *tile_x = s->dim == 2 ? kTx[shape] : 0;
  if (tile_y) *tile_y = s->dim == 2 ? kTy[shape] : 0;
  // characteristic-wise 2D reconstruction works per interface and shares nothing per cell
  if (lds_shared) *lds_shared = s->dim == 2 ? (s->shape2d < 3 && !s->charw ? 1 : 0) : 1;
  return NPW_OK;
}

static int npweno_write_impl(npw_solver* s, const void* u, int on_device, double t) {
  if (!s || !u || !std::isfinite(t)) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(s->P0, u, s->total * s->esize, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         s->stream));
  rc = reset_instances(s, t);
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

// Advance every instance towards its target T[b] (same stopping rule as a single solve) or until
// max_steps graph steps were launched.  Instances that fail are restored to their last good
// step and left behind; the others continue.  Returns the first error seen (NPW_OK if none).
static int run_steps(npw_solver* s, const double* T, int64_t max_steps, int64_t* taken) {
  if (taken) *taken = 0;
  for (int b = 0; b < s->ninst; ++b)
    if (!std::isfinite(T[b])) return NPW_EINVAL;
  if (s->sticky_err) return s->sticky_err;
  for (int b = 0; b < s->ninst; ++b) {
    s->h_inst[b].T = T[b];
    s->h_inst[b].tol = 1e-12 * std::max(1.0, std::fabs(T[b]));
  }
  int rc = push_static(s);
  if (rc) return rc;
  rc = pull(s);
  if (rc) return rc;
  s->settled.assign(s->ninst, 0);
  int gp = 0;
  rc = align_homes(s, &gp);
  if (rc) return rc;
  const long long n0 = s->h_pin[0].ctl[0].n;
  int64_t launched = 0;
  int first_err = 0;
  std::vector<char> active(s->ninst, 0);
  const int max_k = s->batch ? kMaxGraphStepsBatch : kMaxGraphStepsSingle;
  while (true) {
    int nactive = 0;
    double est = 0.0;
    int home = gp;
    for (int b = 0; b < s->ninst; ++b) {
      const InstDev& h = s->h_pin[b];
      active[b] = 0;
      if (h.err) {
        if (!s->settled[b]) {
          s->settled[b] = 1;
          if (!first_err) first_err = h.err;
          if (settle_error(s, b)) return NPW_EHIP;
        }
        continue;
      }
      const double rem = s->h_inst[b].T - h.ctl[0].t;
      if (rem > s->h_inst[b].tol) {
        active[b] = 1;
        ++nactive;
        home = h.ctl[0].home;
        const double dt = h.ctl[1].dt;
        est = std::max(est, dt > 0.0 ? rem / dt : (double)max_k);
      }
    }
    if (taken) *taken = s->ninst == 1 ? (int64_t)(s->h_pin[0].ctl[0].n - n0) : launched;
    const int64_t progress = s->ninst == 1 ? (int64_t)(s->h_pin[0].ctl[0].n - n0) : launched;
    if (nactive == 0 || (max_steps >= 0 && progress >= max_steps)) break;
    if (s->batch) {
      rc = set_tiles(s, active, launched == 0);
      if (rc) return rc;
    }
    const int cap = (!s->batch && est < 8.0 * max_k) ? kMaxGraphStepsSingleTail : max_k;
    int want = est < 1.0 ? 1 : (int)std::min((double)cap, std::ceil(est));
    if (max_steps >= 0) want = (int)std::min<int64_t>(want, max_steps - progress);
    int k = 1;
    while (k * 4 <= want) k *= 4;
    rc = maybe_rebase(s, k);
    if (rc) return rc;
    hipGraphExec_t g = graph_for(s, k, home);
    if (!g) return NPW_EHIP;
    HIP_TRY(hipGraphLaunch(g, s->stream));
    launched += k;
    rc = pull(s);
    if (rc) return rc;
  }
  return first_err;
}

static int npweno_step_impl(npw_solver* s, double t_final, double* dt_taken) {
  if (!s) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  int64_t taken = 0;
  std::vector<double> T(s->ninst, t_final);
  rc = run_steps(s, T.data(), 1, &taken);
  if (dt_taken) *dt_taken = (rc == NPW_OK && taken == 1) ? s->h_pin[0].ctl[1].dt : 0.0;
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

static int npweno_solve_impl(npw_solver* s, double t_final, int64_t max_steps, npw_stats* stats) {
  if (!s) return NPW_EINVAL;
  int rc = enter(s);
  if (rc) return rc;
  std::vector<double> T(s->ninst, t_final);
  rc = run_steps(s, T.data(), max_steps, nullptr);
  if (stats) {
    HIP_TRY(launch_init(s, s->stream));
    if (pull(s) == NPW_OK) fill_stats(s, 0, stats);
  }
  int rc2 = leave(s);
  return rc ? rc : rc2;
}

static int npweno_rhs_impl(npw_solver* s, void* L_out, int out_on_device) {
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
  rc = pull(s);
  if (rc) return rc;
  int gp = 0;
  rc = align_homes(s, &gp);
  if (rc) return rc;
  if (s->batch) {  // every tile, including those of finished instances
    std::vector<char> all(s->ninst, 1);
    rc = set_tiles(s, all, true);
    if (rc) return rc;
  }
  HIP_TRY(launch_stage(s, stage_args(s, 0, gp, dst), s->stream));
  if (!out_on_device) HIP_TRY(hipMemcpyAsync(L_out, dst, bytes, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return leave(s);
}

static int npweno_read_impl(const npw_solver* cs, void* u_out, int out_on_device) {
  if (!cs || !u_out) return NPW_EINVAL;
  npw_solver* s = const_cast<npw_solver*>(cs);
  int rc = enter(s);
  if (rc) return rc;
  rc = pull(s);
  if (rc) return rc;
  const hipMemcpyKind kind = out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  for (int b = 0; b < s->ninst; ++b) {  // each instance from the buffer that holds its u^n
    const InstDev& h = s->h_pin[b];
    const size_t at = (size_t)h.off * s->esize;
    const size_t len = (size_t)s->ncomp * (size_t)(h.nx * h.ny) * s->esize;
    const char* src = static_cast<const char*>(h.ctl[0].home ? s->P1 : s->P0) + at;
    HIP_TRY(hipMemcpyAsync(static_cast<char*>(u_out) + at, src, len, kind, s->stream));
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return leave(s);
}

static int npweno_get_stats_impl(const npw_solver* cs, npw_stats* stats) {
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

static void npweno_destroy_impl(npw_solver* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  release(s);
}

}  // extern "C"

// ---- The allocation-free right-hand side ---------------------------------------------------
// Its scratch lives in one fixed device array of this translation unit, one copy per GPU:
//   [0, 512)                 the instance record (InstDev)
//   [512, 512 + 49152)       the spread alpha entries of a single grid (kSpreadWords words)
//   [49664, 49664 + 28672)   the state check's partial records (kCheckMaxG records)
// Every grid within the limits of npweno_create fits, since the check uses at most kCheckMaxG
// workgroups.  Host code reaches the array only through the address hipGetSymbolAddress gives
// for the current device (the array's name in host code is a stand-in, not a device address).
namespace {
constexpr size_t kNaRecordBytes = 512;
constexpr size_t kNaSpreadBytes = sizeof(unsigned long long) * npw::kSpreadWords;
constexpr int kCheckMaxG = 512;
constexpr size_t kNaPartialBytes = (size_t)npw::kCheckPartialBytes * kCheckMaxG;
constexpr size_t kNoAllocScratchBytes = kNaRecordBytes + kNaSpreadBytes + kNaPartialBytes;
static_assert(sizeof(InstDev) <= kNaRecordBytes, "the instance record fits its slot");
static_assert(kNoAllocScratchBytes <= 80 * 1024, "the scratch array stays modest");
static_assert(kNaSpreadBytes % 256 == 0, "the partial records start 256-byte aligned");
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return NPW_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return NPW_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NPW_OK;
}

// Write the instance record (static part from the parameters, dynamic part zero: t = 0, step 0,
// no error, alpha slots clear) without a host copy, so nothing reads host memory after return.
__global__ void noalloc_record_kernel(InstDev* rec, InstDev v) {
  const unsigned* src = reinterpret_cast<const unsigned*>(&v);
  unsigned* dst = reinterpret_cast<unsigned*>(rec);
  for (int k = threadIdx.x; k < (int)(sizeof(InstDev) / sizeof(unsigned)); k += blockDim.x) dst[k] = src[k];
}

// Copy the state check's verdict (NPW_OK, NPW_ENONFINITE or NPW_ENONPHYSICAL) to the caller.
__global__ void noalloc_status_kernel(const InstDev* rec, int32_t* status) { *status = rec->err; }

int rhs_noalloc_impl(const npw_params* p, const void* u, void* L_out, void* hip_stream, int32_t* status_dev) {
  if (!p || !u || !L_out) return NPW_EINVAL;
  int rc = validate(p);
  if (rc) return rc;
  const long long ny = p->dim == 2 ? p->ny : 1;
  const size_t esize = p->precision == NPW_FP64 ? sizeof(double) : sizeof(float);
  const size_t bytes = (size_t)p->ncomp * (size_t)(p->nx * ny) * esize;
  const char* ub = static_cast<const char*>(u);
  const char* lb = static_cast<const char*>(L_out);
  if (ub < lb + bytes && lb < ub + bytes) return NPW_EINVAL;  // L_out must not overlap u
  const long long cells = p->nx * ny;
  const int G = (int)std::min<long long>(kCheckMaxG, std::max<long long>(1, cells / 16384));
  if (kNaRecordBytes + kNaSpreadBytes + (size_t)npw::kCheckPartialBytes * G > kNoAllocScratchBytes)
    return NPW_ESCRATCH;
  void* base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  char* sc = static_cast<char*>(base);
  InstDev* rec = reinterpret_cast<InstDev*>(sc);
  unsigned long long* spread = reinterpret_cast<unsigned long long*>(sc + kNaRecordBytes);
  void* part = sc + kNaRecordBytes + kNaSpreadBytes;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);

  noalloc_record_kernel<<<1, 64, 0, st>>>(rec, make_inst(p, 0));
  HIP_TRY(hipGetLastError());
  void* uu = const_cast<void*>(u);  // read only: rhs mode loads the state and writes L_out
  const int flux = p->flux, m = p->ncomp;
  HIP_TRY(p->precision == NPW_FP64 ? npw::launch_init_f64(flux, m, rec, 1, uu, uu, spread, nullptr, nullptr, 0, part, G, st)
                                   : npw::launch_init_f32(flux, m, rec, 1, uu, uu, spread, nullptr, nullptr, 0, part, G, st));
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.inst = rec;
  a.tiles = nullptr;
  a.nx = p->nx;
  a.ny = ny;
  a.bc = p->bc;
  a.par = 0;
  a.P0 = uu;
  a.P1 = uu;
  a.C = uu;
  a.out = L_out;
  a.stage = 0;
  a.charw = p->variables == NPW_CHARACTERISTIC ? 1 : 0;
  a.any_k2 = p->recon >= NPW_RBF_WENO3 ? 1 : 0;
  a.spread = spread;
  a.pack = nullptr;  // the spread entries: the scratch array holds no packed slots
  // the same kernel as a solver of these parameters (the 2D strip has a build for one scheme)
  a.scheme = p->recon == NPW_RBF_WENO5 && p->switch_mode == NPW_SWITCH_MONOTONE ? npw::kSchemeRbfWeno5Switch
                                                                               : npw::kSchemeAny;
  if (p->dim == 1) {
    const int block = env_block();
    a.ntiles = (int)((p->nx + block - 3) / (block - 2));
    HIP_TRY(p->precision == NPW_FP64 ? npw::launch_stage_f64(flux, m, block, a, st)
                                     : npw::launch_stage_f32(flux, m, block, a, st));
  } else {
    int shape = 4;  // 62 x 8 cells, per-interface recompute
    if (const char* e = std::getenv("NPW_TILE2D")) {
      const int v = std::atoi(e);
      if (v >= 0 && v < npw::k2dShapes) shape = v;
    }
    HIP_TRY(p->precision == NPW_FP64 ? npw::launch_stage2d_f64(flux, m, shape, a, st)
                                     : npw::launch_stage2d_f32(flux, m, shape, a, st));
  }
  if (status_dev) {
    noalloc_status_kernel<<<1, 1, 0, st>>>(rec, status_dev);
    HIP_TRY(hipGetLastError());
  }
  return NPW_OK;
}
}  // namespace

// ---- C ABI entry points: no C++ exception crosses the boundary ------------------------
// (std containers may throw std::bad_alloc; every entry point maps that to NPW_ENOMEM.)
template <typename F>
static int guarded(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return NPW_ENOMEM;
  } catch (...) {
    return NPW_EINVAL;
  }
}

void npweno_default_params(npw_params* p) {
  try {
    npweno_default_params_impl(p);
  } catch (...) {
  }
}

int npweno_create(const npw_params* p, const void* u0, int u0_on_device, void* hip_stream, npw_solver** out) {
  return guarded([&] { return npweno_create_impl(p, u0, u0_on_device, hip_stream, out); });
}

int npweno_create_batch(const npw_params* params, int32_t count, const void* const* u0, int on_device,
                        void* hip_stream, npw_solver** out) {
  return guarded([&] { return npweno_create_batch_impl(params, count, u0, on_device, hip_stream, out); });
}

int npweno_solve_batch(npw_solver* s, const double* t_final, int64_t max_steps, npw_stats* per_instance) {
  return guarded([&] { return npweno_solve_batch_impl(s, t_final, max_steps, per_instance); });
}

int npweno_read_instance(const npw_solver* cs, int32_t index, void* u_out, int out_on_device) {
  return guarded([&] { return npweno_read_instance_impl(cs, index, u_out, out_on_device); });
}

int npweno_get_stats_instance(const npw_solver* cs, int32_t index, npw_stats* stats) {
  return guarded([&] { return npweno_get_stats_instance_impl(cs, index, stats); });
}

int npweno_launch_shape(const npw_solver* s, int32_t* block_1d, int32_t* tile_x, int32_t* tile_y,
                        int32_t* lds_shared) {
  return guarded([&] { return npweno_launch_shape_impl(s, block_1d, tile_x, tile_y, lds_shared); });
}

int npweno_write(npw_solver* s, const void* u, int on_device, double t) {
  return guarded([&] { return npweno_write_impl(s, u, on_device, t); });
}

int npweno_step(npw_solver* s, double t_final, double* dt_taken) {
  return guarded([&] { return npweno_step_impl(s, t_final, dt_taken); });
}

int npweno_solve(npw_solver* s, double t_final, int64_t max_steps, npw_stats* stats) {
  return guarded([&] { return npweno_solve_impl(s, t_final, max_steps, stats); });
}

int npweno_rhs(npw_solver* s, void* L_out, int out_on_device) {
  return guarded([&] { return npweno_rhs_impl(s, L_out, out_on_device); });
}

int npweno_read(const npw_solver* cs, void* u_out, int out_on_device) {
  return guarded([&] { return npweno_read_impl(cs, u_out, out_on_device); });
}

int npweno_rhs_noalloc(const npw_params* p, const void* u, void* L_out, void* hip_stream, int32_t* status_dev) {
  return guarded([&] { return rhs_noalloc_impl(p, u, L_out, hip_stream, status_dev); });
}

int npweno_get_stats(const npw_solver* cs, npw_stats* stats) {
  return guarded([&] { return npweno_get_stats_impl(cs, stats); });
}

void npweno_destroy(npw_solver* s) {
  try {
    npweno_destroy_impl(s);
  } catch (...) {
  }
}

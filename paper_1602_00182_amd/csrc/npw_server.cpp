// npw_server.cpp -- continuous-batching serving loop behind npw_server_* (include/npweno.h).
//
// Requests are 1D solves of any flux type.  They share one device arena (three state buffers
// sized by the HBM budget) and are grouped into one pool per flux type; every pool steps all of
// its running requests with one launch of the batched stage kernel per RK stage.  Admission is
// FIFO: the head request enters as soon as its pool has a free slot and the arena a free range
// large enough; finished requests leave at the end of a pump and free their slot and range.
// The stage kernels read the pool's tile count from device memory, so the captured graphs stay
// valid while requests come and go.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/npweno.h"
#include "npw_internal.h"

using npw::Ctl;
using npw::InstDev;
using npw::StageArgs;
using npw::Tile;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  npw_params p{};
  std::vector<char> u0;      // host copy of the initial state
  std::vector<char> result;  // final (or last good) state once finished
  double T = 0.0;
  int state = 0;             // 0 queued, 1 running, 2 done, 3 failed
  int pool = -1, slot = -1;
  size_t off = 0, len = 0;   // arena range in elements
  npw_stats stats{};
  int err = 0;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

struct Pool {
  int flux = 0, ncomp = 1;
  int charw = 0;              // Euler characteristic-wise reconstruction
  hipStream_t stream = nullptr;
  InstDev* d_inst = nullptr;
  InstDev* h_pin = nullptr;
  Tile* d_tiles = nullptr;
  int* d_ntiles = nullptr;
  void* d_check = nullptr;    // state-check partial records (kCheckMaxG)
  unsigned long long* d_bsp = nullptr;  // per-slot spread alpha entries (StageArgs::bsp)
  int bsp_k = 1;
  int tile_cap = 0;
  std::vector<int> slot_req;  // request index (into server order) per slot, -1 if free
  std::vector<uint64_t> slot_id;
  int par = 0;                // ping-pong buffer of u^n for every running request
  std::map<int, hipGraphExec_t> graphs;
  bool dirty = true;          // tile table must be rebuilt
};

// Stage workgroup size of the pools (tile = block - 2 cells); NPW_BLOCK overrides.  Measured on the
// 2000-request trace (64 MiB arena): 4.58e10-4.60e10 cell-updates/s at 512 against 3.41e10-3.47e10 at
// 256 and 2.18e10-2.20e10 at 128 (earlier kernels: 2.89e10 at 256, 1.92e10 at 128, 1.06e10 at 64),
// so the pools take the largest tiles even though single batches tune to smaller blocks.
constexpr int kDefaultBlock = 512;

int server_block() {
  const char* e = std::getenv("NPW_BLOCK");
  const int b = e ? std::atoi(e) : kDefaultBlock;
  return (b == 64 || b == 128 || b == 256 || b == 512) ? b : kDefaultBlock;
}
constexpr int kGridThreads = 2048 * 256;  // threads of a pool launch (grid-stride over its tiles)
constexpr int kCheckMaxG = 512;  // state-check workgroups of one request: one per 16 Ki cells, at most this

int check_groups(long long cells) { return (int)std::min<long long>(kCheckMaxG, std::max<long long>(1, cells / 16384)); }


// Free-list allocator over [0, cap) elements (first fit, coalescing).
struct Arena {
  size_t cap = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t c) {
    cap = c;
    free_.clear();
    if (c) free_[0] = c;
  }
  bool alloc(size_t len, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        *off = it->first;
        const size_t rest = it->second - len;
        const size_t at = it->first + len;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t len) {
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct npw_server {
  size_t budget = 0;
  int max_slots = 0;
  int block = 256;  // stage workgroup size of every pool
  int precision = NPW_FP32;
  size_t esize = 4;
  void* P0 = nullptr;
  void* P1 = nullptr;
  void* C = nullptr;
  Arena arena;
  Pool pools[4];  // advection, Burgers, Euler, Euler (characteristic-wise)
  std::deque<size_t> queue;       // indices into reqs (FIFO)
  std::vector<Request> reqs;      // every request ever submitted (by index)
  std::map<uint64_t, size_t> index;
  uint64_t next_id = 1;
};

namespace {

#define HIP_TRY(expr)                      \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return NPW_EHIP; \
  } while (0)

int pool_of(const npw_params* p) {  // advection 0, Burgers 1, Euler 2, Euler characteristic-wise 3
  return p->flux == NPW_EULER && p->variables == NPW_CHARACTERISTIC ? 3 : p->flux;
}

unsigned long long* slot_bsp(const Pool& pl, int slot) {
  return pl.d_bsp + (size_t)slot * 3 * pl.bsp_k * npw::kSpreadStride;
}

// State check of one request (alpha, validity, FP64 sums of its current state) on its pool's
// stream.  Checks on one stream run in order, so they share the pool's partial records.
hipError_t launch_check(const npw_server* s, const Pool& pl, int slot, long long cells) {
  return s->precision == NPW_FP64
             ? npw::launch_init_f64(pl.flux, pl.ncomp, pl.d_inst + slot, 1, s->P0, s->P1, nullptr, nullptr,
                                    slot_bsp(pl, slot), pl.bsp_k, pl.d_check, check_groups(cells), pl.stream)
             : npw::launch_init_f32(pl.flux, pl.ncomp, pl.d_inst + slot, 1, s->P0, s->P1, nullptr, nullptr,
                                    slot_bsp(pl, slot), pl.bsp_k, pl.d_check, check_groups(cells), pl.stream);
}

hipError_t launch_stage(const npw_server* s, int flux, int ncomp, const StageArgs& a, hipStream_t st) {
  return s->precision == NPW_FP64 ? npw::launch_stage_f64(flux, ncomp, s->block, a, st)
                                  : npw::launch_stage_f32(flux, ncomp, s->block, a, st);
}

StageArgs pool_args(const npw_server* s, const Pool& pl, int stage, int par) {
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.inst = pl.d_inst;
  a.tiles = pl.d_tiles;
  a.ntiles = kGridThreads / s->block;  // grid size; the tile count comes from d_ntiles
  a.ntiles_dev = pl.d_ntiles;
  a.par = par;
  a.P0 = s->P0;
  a.P1 = s->P1;
  a.C = s->C;
  a.stage = stage;
  a.spread = nullptr;
  a.bsp = pl.d_bsp;
  a.bsp_k = pl.bsp_k;
  a.charw = pl.charw;
  a.any_k2 = 1;  // requests of either order share the pool's graphs
  return a;
}

hipGraphExec_t pool_graph(npw_server* s, Pool& pl, int k, int par) {
  const int key = 2 * k + par;
  auto it = pl.graphs.find(key);
  if (it != pl.graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  if (hipStreamBeginCapture(pl.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  bool ok = true;
  for (int i = 0; i < k && ok; ++i)
    for (int st = 1; st <= 3 && ok; ++st)
      ok = launch_stage(s, pl.flux, pl.ncomp, pool_args(s, pl, st, par ^ (i & 1)), pl.stream) == hipSuccess;
  hipError_t e = hipStreamEndCapture(pl.stream, &g);
  if (!ok || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return nullptr;
  }
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return nullptr;
  pl.graphs[key] = ex;
  return ex;
}

int rebuild_tiles(npw_server* s, Pool& pl) {
  std::vector<Tile> t;
  for (int b = 0; b < s->max_slots; ++b) {
    if (pl.slot_req[b] < 0) continue;
    const Request& r = s->reqs[pl.slot_req[b]];
    if (r.state != 1) continue;
    for (long long st = 0; st < r.p.nx; st += s->block - 2) {
      Tile x;
      x.inst = b;
      x.bc = r.p.bc;
      x.start = st;
      x.nx = r.p.nx;
      x.off = (long long)r.off;
      t.push_back(x);
    }
  }
  if ((int)t.size() > pl.tile_cap) return NPW_ENOMEM;
  if (!t.empty())
    HIP_TRY(hipMemcpyAsync(pl.d_tiles, t.data(), sizeof(Tile) * t.size(), hipMemcpyHostToDevice, pl.stream));
  const int n = (int)t.size();
  HIP_TRY(hipMemcpyAsync(pl.d_ntiles, &n, sizeof(int), hipMemcpyHostToDevice, pl.stream));
  HIP_TRY(hipStreamSynchronize(pl.stream));  // the host vector goes out of scope
  pl.dirty = false;
  return NPW_OK;
}

int validate_request(const npw_server* s, const npw_params* p) {
  if (!p || p->abi_version != NPW_ABI_VERSION || p->dim != 1) return NPW_EINVAL;
  if (p->precision != s->precision) return NPW_EINVAL;
  if (p->nx < 1 || (long long)(p->ncomp > 0 ? p->ncomp : 1) * p->nx > (1LL << 31) - (1LL << 16)) return NPW_EINVAL;
  if ((p->flux == NPW_ADVECTION || p->flux == NPW_BURGERS) && p->ncomp != 1) return NPW_EINVAL;
  if (p->flux == NPW_EULER && (p->ncomp != 3 || !(p->gamma > 1.0))) return NPW_EINVAL;
  if (p->flux < 0 || p->flux > 2) return NPW_EINVAL;
  if (p->bc != NPW_PERIODIC && p->bc != NPW_TRANSMISSIVE) return NPW_EINVAL;
  if (p->recon < NPW_RBF_WENO5 || p->recon > NPW_ENO2) return NPW_EINVAL;
  if (p->switch_mode != NPW_SWITCH_MONOTONE && p->switch_mode != NPW_SWITCH_OFF) return NPW_EINVAL;
  if (!(std::isfinite(p->x0) && std::isfinite(p->x1) && p->x1 > p->x0)) return NPW_EINVAL;
  if (!(p->cfl > 0.0) || !(p->eps_weno > 0.0) || !(p->eps_m > 0.0) || !(p->dt_fixed >= 0.0)) return NPW_EINVAL;
  if (!std::isfinite(p->cfl) || !std::isfinite(p->eps_weno) || !std::isfinite(p->eps_m)) return NPW_EINVAL;
  if (!std::isfinite(p->speed_x)) return NPW_EINVAL;
  if (p->variables != NPW_COMPONENTWISE && (p->variables != NPW_CHARACTERISTIC || p->flux != NPW_EULER))
    return NPW_EINVAL;
  if (p->reserved != 0) return NPW_EINVAL;
  return NPW_OK;
}

InstDev make_slot(const Request& r, int par) {
  InstDev d;
  std::memset(&d, 0, sizeof d);
  const npw_params* p = &r.p;
  d.off = (long long)r.off;
  d.nx = p->nx;
  d.ny = 1;
  d.dx = (p->x1 - p->x0) / (double)p->nx;
  d.dy = 1.0;
  d.inv_dx = 1.0 / d.dx;
  d.inv_dy = 1.0;
  d.cfl = p->cfl;
  d.dt_fixed = p->dt_fixed;
  d.T = r.T;
  d.tol = 1e-12 * std::max(1.0, std::fabs(r.T));
  d.speed_x = p->speed_x;
  d.speed_y = 0.0;
  d.gamma = p->gamma;
  d.eps_weno = p->eps_weno;
  d.eps_m = p->eps_m;
  d.bc = p->bc;
  d.recon = p->recon;
  d.sw = p->switch_mode;
  d.dim = 1;
  d.ctl[0].home = par;
  return d;
}

// Admit queued requests in FIFO order while slots and arena space allow.  Every admitted
// request's state and record are copied and checked (alpha, validity, FP64 sums) on its pool's
// stream; one synchronization at the end covers all of them.
int admit(npw_server* s) {
  std::vector<size_t> admitted;
  std::vector<InstDev> staged;
  staged.reserve(s->queue.size());  // the copies below read these records until the final sync
  bool used[4] = {false, false, false, false};
  int rc = NPW_OK;
  while (!s->queue.empty()) {
    Request& r = s->reqs[s->queue.front()];
    Pool& pl = s->pools[r.pool];
    int slot = -1;
    for (int b = 0; b < s->max_slots; ++b)
      if (pl.slot_req[b] < 0) {
        slot = b;
        break;
      }
    if (slot < 0) break;
    size_t off = 0;
    if (!s->arena.alloc(r.len, &off)) break;
    r.off = off;
    r.slot = slot;
    r.state = 1;
    r.t_admit = now_s();
    pl.slot_req[slot] = (int)s->queue.front();
    pl.slot_id[slot] = r.id;
    s->queue.pop_front();
    admitted.push_back(pl.slot_req[slot]);
    used[r.pool] = true;
    pl.dirty = true;
    char* dst = static_cast<char*>(pl.par ? s->P1 : s->P0) + off * s->esize;
    staged.push_back(make_slot(r, pl.par));
    if (hipMemcpyAsync(dst, r.u0.data(), r.len * s->esize, hipMemcpyHostToDevice, pl.stream) != hipSuccess ||
        hipMemcpyAsync(pl.d_inst + slot, &staged.back(), sizeof(InstDev), hipMemcpyHostToDevice, pl.stream) !=
            hipSuccess ||
        launch_check(s, pl, slot, r.p.nx) != hipSuccess) {
      rc = NPW_EHIP;
      break;
    }
  }
  // the host copies of the states and records go out of scope after this
  for (int k = 0; k < 4; ++k)
    if (used[k] && hipStreamSynchronize(s->pools[k].stream) != hipSuccess) rc = NPW_EHIP;
  for (size_t i : admitted) {
    s->reqs[i].u0.clear();
    s->reqs[i].u0.shrink_to_fit();
  }
  return rc;
}

void fill_stats_from(const InstDev& h, npw_stats* st) {
  st->t = h.ctl[0].t;
  st->nsteps = h.ctl[0].n;
  std::memcpy(&st->alpha[0], &h.alpha[0][0], sizeof(double));
  st->alpha[1] = 0.0;
  for (int c = 0; c < 4; ++c) st->mass[c] = h.mass[c];
  st->err = h.err;
  st->err_stage = h.err_stage;
}

// Copy out and free every request of the pool that reached its T or failed.  As a solo solve
// does when it stops, the state check runs on each finishing request's final state (for a failed
// request: its last good state, with the control word put back at that step) so that the alpha
// and FP64 sums it reports are those of the state it returns.
int retire(npw_server* s, Pool& pl) {
  std::vector<int> fin;
  for (int b = 0; b < s->max_slots; ++b) {
    if (pl.slot_req[b] < 0) continue;
    const Request& r = s->reqs[pl.slot_req[b]];
    const InstDev& h = pl.h_pin[b];
    const bool failed = h.err != 0;
    const bool done = !failed && !(r.T - h.ctl[0].t > 1e-12 * std::max(1.0, std::fabs(r.T)));
    if (failed || done) fin.push_back(b);
  }
  if (fin.empty()) return NPW_OK;
  std::vector<Ctl> back(fin.size());  // read by the copies below until the synchronization
  for (size_t k = 0; k < fin.size(); ++k) {
    const int b = fin[k];
    const InstDev& h = pl.h_pin[b];
    const Request& r = s->reqs[pl.slot_req[b]];
    if (h.err) {
      Ctl& c = back[k];
      c.t = h.err_t;
      c.dt = 0.0;
      c.n = h.err_n;
      c.active = 0;
      c.home = h.err_home;
      HIP_TRY(hipMemcpyAsync(reinterpret_cast<char*>(pl.d_inst + b) + offsetof(InstDev, ctl), &c, sizeof(Ctl),
                             hipMemcpyHostToDevice, pl.stream));
    }
    HIP_TRY(launch_check(s, pl, b, r.p.nx));
    HIP_TRY(hipMemcpyAsync(pl.h_pin + b, pl.d_inst + b, sizeof(InstDev), hipMemcpyDeviceToHost, pl.stream));
  }
  for (int b : fin) {
    Request& r = s->reqs[pl.slot_req[b]];
    const int home = pl.h_pin[b].err ? pl.h_pin[b].err_home : pl.h_pin[b].ctl[0].home;
    r.result.resize(r.len * s->esize);
    const char* src = static_cast<const char*>(home ? s->P1 : s->P0) + r.off * s->esize;
    HIP_TRY(hipMemcpyAsync(r.result.data(), src, r.len * s->esize, hipMemcpyDeviceToHost, pl.stream));
  }
  HIP_TRY(hipStreamSynchronize(pl.stream));
  const double now = now_s();
  for (int b : fin) {
    Request& r = s->reqs[pl.slot_req[b]];
    const InstDev& h = pl.h_pin[b];
    const bool failed = h.err != 0;
    fill_stats_from(h, &r.stats);
    if (failed) {
      r.stats.t = h.err_t;
      r.stats.nsteps = h.err_n;
    }
    r.err = h.err;
    r.state = failed ? 3 : 2;
    r.t_done = now;
    s->arena.release(r.off, r.len);
    pl.slot_req[b] = -1;
  }
  pl.dirty = true;
  return NPW_OK;
}

int pool_running(const npw_server* s, const Pool& pl) {
  int n = 0;
  for (int b = 0; b < s->max_slots; ++b)
    if (pl.slot_req[b] >= 0) ++n;
  return n;
}

void destroy_server(npw_server* s) {
  if (!s) return;
  for (Pool& pl : s->pools) {
    if (pl.stream) (void)hipStreamSynchronize(pl.stream);
    for (auto& kv : pl.graphs) (void)hipGraphExecDestroy(kv.second);
    if (pl.d_inst) (void)hipFree(pl.d_inst);
    if (pl.d_tiles) (void)hipFree(pl.d_tiles);
    if (pl.d_ntiles) (void)hipFree(pl.d_ntiles);
    if (pl.d_check) (void)hipFree(pl.d_check);
    if (pl.d_bsp) (void)hipFree(pl.d_bsp);
    if (pl.h_pin) (void)hipHostFree(pl.h_pin);
    if (pl.stream) (void)hipStreamDestroy(pl.stream);
  }
  if (s->P0) (void)hipFree(s->P0);
  if (s->P1) (void)hipFree(s->P1);
  if (s->C) (void)hipFree(s->C);
  delete s;
}

}  // namespace

extern "C" {

static int npw_server_create_impl(size_t hbm_budget_bytes, int32_t max_slots, int32_t precision, void* hip_stream,
                      npw_server** out) {
  if (!out) return NPW_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 65536) return NPW_EINVAL;
  if (precision != NPW_FP32 && precision != NPW_FP64) return NPW_EINVAL;
  const size_t esize = precision == NPW_FP64 ? 8 : 4;
  if (hbm_budget_bytes < 3 * esize * 256) return NPW_EINVAL;
  npw_server* s = new (std::nothrow) npw_server();
  if (!s) return NPW_ENOMEM;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->block = server_block();
  s->precision = precision;
  s->esize = esize;
  (void)hip_stream;  // requests come and go as host copies; the pools run on private streams
  const size_t elems = hbm_budget_bytes / (3 * esize);
  s->arena.init(elems);
  bool ok = hipMalloc(&s->P0, elems * esize) == hipSuccess && hipMalloc(&s->P1, elems * esize) == hipSuccess &&
            hipMalloc(&s->C, elems * esize) == hipSuccess;
  const int ncomp[4] = {1, 1, 3, 3};
  for (int k = 0; k < 4 && ok; ++k) {
    Pool& pl = s->pools[k];
    pl.flux = k < 3 ? k : NPW_EULER;
    pl.ncomp = ncomp[k];
    pl.charw = k == 3 ? 1 : 0;
    pl.slot_req.assign(max_slots, -1);
    pl.slot_id.assign(max_slots, 0);
    // every tile of a full arena (one component per element) plus one partial tile per slot
    pl.tile_cap = (int)std::min<size_t>((elems / ncomp[k]) / (s->block - 2) + max_slots + 1, 1u << 30);
    // spread alpha entries per slot for the largest request the arena holds, within 32 MiB a pool
    pl.bsp_k = npw::bsp_entries((long long)((elems / ncomp[k]) / (s->block - 2) + 1));
    while (pl.bsp_k > 1 && (size_t)max_slots * 3 * pl.bsp_k * npw::kSpreadStride * 8 > (32u << 20)) pl.bsp_k /= 2;
    ok = hipStreamCreateWithFlags(&pl.stream, hipStreamNonBlocking) == hipSuccess &&
         hipMalloc(&pl.d_inst, sizeof(InstDev) * max_slots) == hipSuccess &&
         hipMalloc(&pl.d_tiles, sizeof(Tile) * pl.tile_cap) == hipSuccess &&
         hipMalloc(&pl.d_ntiles, sizeof(int)) == hipSuccess &&
         hipMalloc(&pl.d_check, (size_t)npw::kCheckPartialBytes * kCheckMaxG) == hipSuccess &&
         hipMalloc(&pl.d_bsp, sizeof(unsigned long long) * (size_t)max_slots * 3 * pl.bsp_k * npw::kSpreadStride) ==
             hipSuccess &&
         hipHostMalloc(&pl.h_pin, sizeof(InstDev) * max_slots, hipHostMallocDefault) == hipSuccess;
    if (ok) {
      // idle slots: T = t = 0, so every launch skips them
      std::vector<InstDev> idle(max_slots);
      std::memset(idle.data(), 0, sizeof(InstDev) * max_slots);
      ok = hipMemcpy(pl.d_inst, idle.data(), sizeof(InstDev) * max_slots, hipMemcpyHostToDevice) == hipSuccess;
      const int zero = 0;
      ok = ok && hipMemcpy(pl.d_ntiles, &zero, sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    }
  }
  if (!ok) {
    destroy_server(s);
    return NPW_ENOMEM;
  }
  *out = s;
  return NPW_OK;
}

static int npw_server_submit_impl(npw_server* s, const npw_params* p, const void* u0_host, double t_final, uint64_t* req_id) {
  if (!s || !p || !u0_host || !req_id || !std::isfinite(t_final) || t_final < 0.0) return NPW_EINVAL;
  int rc = validate_request(s, p);
  if (rc) return rc;
  Request r;
  r.id = s->next_id++;
  r.p = *p;
  r.T = t_final;
  r.pool = pool_of(p);
  r.len = (size_t)p->ncomp * (size_t)p->nx;
  if (r.len > s->arena.cap) return NPW_EINVAL;  // could never be admitted
  r.u0.resize(r.len * s->esize);
  std::memcpy(r.u0.data(), u0_host, r.u0.size());
  r.t_submit = now_s();
  s->index[r.id] = s->reqs.size();
  s->queue.push_back(s->reqs.size());
  s->reqs.push_back(std::move(r));
  *req_id = s->reqs.back().id;
  return NPW_OK;
}

static int npw_server_pump_impl(npw_server* s, int32_t steps, int32_t* n_running, int32_t* n_queued) {
  if (!s || steps < 1) return NPW_EINVAL;
  int rc = admit(s);
  if (rc) return rc;
  // launch every pool with running requests on its own stream, then wait for all of them; a
  // pool advances by exactly `steps` RK steps as graphs of 256, 64, 16, 4 and 1 steps
  for (Pool& pl : s->pools) {
    if (pool_running(s, pl) == 0) continue;
    if (pl.dirty) {
      rc = rebuild_tiles(s, pl);
      if (rc) return rc;
    }
    int left = steps;
    for (int k = 256; k >= 1; k /= 4) {
      for (; left >= k; left -= k) {
        hipGraphExec_t g = pool_graph(s, pl, k, pl.par);
        if (!g) return NPW_EHIP;
        HIP_TRY(hipGraphLaunch(g, pl.stream));
        if (k & 1) pl.par ^= 1;  // an odd graph leaves u^n of the running requests in the other buffer
      }
    }
  }
  for (Pool& pl : s->pools) {
    if (pool_running(s, pl) == 0) continue;
    HIP_TRY(hipMemcpyAsync(pl.h_pin, pl.d_inst, sizeof(InstDev) * s->max_slots, hipMemcpyDeviceToHost, pl.stream));
  }
  for (Pool& pl : s->pools) {
    if (pool_running(s, pl) == 0) continue;
    HIP_TRY(hipStreamSynchronize(pl.stream));
    rc = retire(s, pl);
    if (rc) return rc;
    // requests that are still running all hold u^n in the buffer given by their home
    for (int b = 0; b < s->max_slots; ++b)
      if (pl.slot_req[b] >= 0) pl.par = pl.h_pin[b].ctl[0].home;
  }
  rc = admit(s);
  if (rc) return rc;
  if (n_running) {
    int n = 0;
    for (Pool& pl : s->pools) n += pool_running(s, pl);
    *n_running = n;
  }
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return NPW_OK;
}

static int npw_server_poll_impl(npw_server* s, uint64_t req_id, void* u_out_host, npw_stats* stats) {
  if (!s) return NPW_EINVAL;
  auto it = s->index.find(req_id);
  if (it == s->index.end()) return NPW_ENOTFOUND;
  Request& r = s->reqs[it->second];
  if (r.state < 2) return NPW_EBUSY;
  if (u_out_host && !r.result.empty()) std::memcpy(u_out_host, r.result.data(), r.result.size());
  if (stats) *stats = r.stats;
  return r.state == 3 ? (r.err ? r.err : NPW_ENONFINITE) : NPW_OK;
}

static int npw_server_times_impl(const npw_server* s, uint64_t req_id, double* t_submit, double* t_admit, double* t_done) {
  if (!s) return NPW_EINVAL;
  auto it = s->index.find(req_id);
  if (it == s->index.end()) return NPW_ENOTFOUND;
  const Request& r = s->reqs[it->second];
  if (t_submit) *t_submit = r.t_submit;
  if (t_admit) *t_admit = r.t_admit;
  if (t_done) *t_done = r.t_done;
  return r.state < 2 ? NPW_EBUSY : NPW_OK;
}

static int npw_server_release_impl(npw_server* s, uint64_t req_id) {
  if (!s) return NPW_EINVAL;
  auto it = s->index.find(req_id);
  if (it == s->index.end()) return NPW_ENOTFOUND;
  Request& r = s->reqs[it->second];
  if (r.state < 2) return NPW_EBUSY;
  r.result.clear();
  r.result.shrink_to_fit();
  return NPW_OK;
}

static void npw_server_destroy_impl(npw_server* s) { destroy_server(s); }

}  // extern "C"

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

int npw_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t precision, void* hip_stream,
                      npw_server** out) {
  return guarded([&] { return npw_server_create_impl(hbm_budget_bytes, max_slots, precision, hip_stream, out); });
}

int npw_server_submit(npw_server* s, const npw_params* p, const void* u0_host, double t_final, uint64_t* req_id) {
  return guarded([&] { return npw_server_submit_impl(s, p, u0_host, t_final, req_id); });
}

int npw_server_pump(npw_server* s, int32_t steps, int32_t* n_running, int32_t* n_queued) {
  return guarded([&] { return npw_server_pump_impl(s, steps, n_running, n_queued); });
}

int npw_server_poll(npw_server* s, uint64_t req_id, void* u_out_host, npw_stats* stats) {
  return guarded([&] { return npw_server_poll_impl(s, req_id, u_out_host, stats); });
}

int npw_server_times(const npw_server* s, uint64_t req_id, double* t_submit, double* t_admit, double* t_done) {
  return guarded([&] { return npw_server_times_impl(s, req_id, t_submit, t_admit, t_done); });
}

int npw_server_release(npw_server* s, uint64_t req_id) {
  return guarded([&] { return npw_server_release_impl(s, req_id); });
}

void npw_server_destroy(npw_server* s) {
  try {
    npw_server_destroy_impl(s);
  } catch (...) {
  }
}

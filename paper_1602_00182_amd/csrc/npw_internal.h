// npw_internal.h -- data shared between the host runtime and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace npw {

enum FluxKind { kAdvection = 0, kBurgers = 1, kEuler = 2 };

// Control word of one instance for one RK stage.  ctl[s] is written by the kernel of stage s
// (block 0 of the instance) and read by the kernel of stage s+1, so no kernel reads a word
// that it writes.
struct Ctl {
  double t;      // time of u^n for the step in progress
  double dt;     // step size (0 when the instance is idle)
  long long n;   // index of the step in progress (= steps completed before it)
  int active;    // 1 while this step is being taken
  int home;      // ctl[0]: which ping-pong buffer (0/1) holds u^n
};

// One grid instance.  The static part is written by the host; the dynamic part only by kernels
// (and by the host between solves).
struct InstDev {
  long long off;  // element offset of the instance's state block in every state buffer
  long long nx, ny;
  double dx, dy, cfl, dt_fixed, T, tol;
  double inv_dx, inv_dy;  // float bulk multiplies by these instead of dividing
  double speed_x, speed_y, gamma, eps_weno, eps_m;
  int bc, recon, sw, dim;
  // float-bulk single grids: spread alpha entries are tagged with 3 (n - seq_base) + stage, and
  // the host moves seq_base forward (re-seeding the entries) long before that nears 2^32
  long long seq_base;
  // dynamic
  Ctl ctl[3];
  // Lax-Friedrichs alpha slots (bit patterns of non-negative doubles, combined with atomicMax):
  // slot 0 = alpha of u^n, slot 1 = alpha of u^(1), slot 2 = alpha of u^(2); [dir]
  unsigned long long alpha[3][2];
  int err;        // first error code (NPW_E*), 0 if none
  int err_stage;  // stage that detected it
  long long err_n;
  double err_t;
  int err_home;   // buffer holding the last good state
  int pad2;
  double mass[4];  // per-component sums of the state (filled by the stats kernel)
};

// One workgroup's share of an instance.  The instance's geometry is repeated here so that the
// state loads can be issued without first reading the instance record.
struct Tile {
  int inst;
  int bc;
  long long start;  // first owned cell
  long long nx;     // cells of the instance
  long long off;    // element offset of the instance's state block
};

struct StageArgs {
  InstDev* inst;
  const Tile* tiles;      // null: a single instance, tile b starts at cell b*(BS-2)
  int ntiles;             // tile count (and grid size) when ntiles_dev is null
  const int* ntiles_dev;  // optional device-resident tile count (serving)
  long long nx;           // single instance: cells (x)
  long long ny;           // 2D: cells along y
  int bc;                 // single instance: boundary kind
  int par;                // u^n of every instance stepped by this launch lives in P[par]
  void* P0;  // ping-pong buffer 0
  void* P1;  // ping-pong buffer 1
  void* C;   // u^(2) buffer
  void* out; // rhs mode: destination of L(u)
  int stage; // 1, 2, 3: SSP-RK3 stage; 0: evaluate L(u^n) into out
  int charw; // Euler: 1 = characteristic-wise reconstruction (same for every instance of a launch)
  int any_k2; // some instance of the launch uses a k = 2 reconstruction (0 prunes that code)
  // Single-grid solvers spread each alpha slot over kSpread cache lines so that hundreds of
  // workgroups do not queue on one atomic: entry (slot, dir, k) lives at
  // spread[((slot * 2 + dir) * kSpread + k) * kSpreadStride].  Null for batches (they use
  // InstDev.alpha directly, with few workgroups per instance).
  unsigned long long* spread;
  // A 1D single grid of at most kPackMax tiles launched with 64 or 128 threads per workgroup
  // keeps one entry per tile instead (alpha in the bulk precision, entry (slot, tile) at
  // pack[slot * kPackMax + tile]): a plain store per workgroup and kPackLoads vector loads per
  // lane replace the atomic max and its spread entry.  Null otherwise.
  void* pack = nullptr;
  // Batches and serving pools spread each instance's alpha slot over bsp_k entries (a power of 2,
  // at most kBspMax), 128 bytes apart: entry (instance b, slot, k) at
  // bsp[((b * 3 + slot) * bsp_k + k) * kSpreadStride], double bits combined with atomicMax; tile i
  // of an instance adds to entry i mod bsp_k, so hundreds of tiles of one large instance do not
  // queue on one atomic.  Null: the instance record's own slot, which instances of at most
// kBspMinTiles tiles keep in any case.  A batch passes bsp only if one of its instances has more
// than kBspLaunchTiles tiles (4096 Euler Riemann problems of up to 67 tiles: 0.589 s to T through
// the entries against 0.550 s through their slots, and the spreading kernel holds more
// registers; 16 instances of 1058 tiles: 14-26 us per stage against 98 us); serving pools
// always do (the 2000-request trace: 6.06e10 cell-updates/s with a threshold of 32 to 64 tiles,
// 4.36e10 at 128, 4.59e10 without the entries).
  unsigned long long* bsp = nullptr;
  int bsp_k = 0;
  // The reconstruction of every instance of the launch when it is the one a kernel can be built
  // for alone (kSchemeRbfWeno5Switch: RBF-WENO5 with the Section 4 switch), else kSchemeAny (the
  // kernel reads it from the instance record).
  int scheme = 0;
};
constexpr int kSchemeAny = 0;
constexpr int kSchemeRbfWeno5Switch = 1;

constexpr int kSpread = 64;
constexpr int kSpreadStride = 16;  // 128 bytes between entries
static_assert(kSpread >= 1 && kSpread <= 64 && (kSpread & (kSpread - 1)) == 0,
              "a wave reads one spread entry per lane (lane & (kSpread - 1))");
constexpr int kSpreadWords = 3 * 2 * kSpread * kSpreadStride;
// Packed slots hold up to 1280 tiles: the 1058 of a 65536-cell grid at 64 threads per workgroup,
// with room, read in 5 float (10 double) 16-byte loads per lane.  Every load costs the
// latency-bound stage time whether or not its entries are in use (3 unused loads of 8 measured
// 0.07 us of a 3.2 us stage), so the size stays near the grids that need it; larger grids are
// not latency-bound and use the spread entries.
constexpr int kBspMax = 16;
constexpr int kBspMinTiles = 32;     // an instance spreads its alpha when it has more tiles than this
constexpr int kBspLaunchTiles = 128;  // a batch launch takes the spreading kernel when one has more
// Entries per instance slot for instances of at most max_tiles tiles: one per 16 tiles, a power of 2.
inline int bsp_entries(long long max_tiles) {
  int k = 1;
  while (k < kBspMax && (long long)k * 16 < max_tiles) k *= 2;
  return k;
}
constexpr int kPackMax = 1280;
constexpr int kPackWords = 3 * kPackMax;  // 64-bit words: three slots of double entries
template <typename R>
constexpr int kPackLoads = kPackMax * (int)sizeof(R) / (64 * 16);  // 16-byte loads per lane
static_assert(kPackMax * 4 % (64 * 16) == 0, "whole 16-byte loads per lane in either precision");

// Launchers implemented in the kernel translation units (one per bulk precision).
hipError_t launch_stage_f64(int flux, int ncomp, int block, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_f32(int flux, int ncomp, int block, const StageArgs& a, hipStream_t s);
// 2D launch shapes: tiles 0 = 64 x 8, 1 = 62 x 8, 2 = 126 x 4 cells with per-cell values shared
// through LDS; 3, 4, 5 = the same tiles with those values recomputed per interface.  (Taller
// recomputed tiles, 64 x 12 and 64 x 16, do less halo work along y but hold more LDS; measured
// slower on 2048^2 Euler: 211 and 251 us per stage against 193 us for 64 x 8.  Recomputed 63 x 8,
// whose x sweep fills exactly 8 waves, measured the same as 64 x 8 (187.8-188.6 us); 127 x 4 took
// 250 us.  With the one-wave-per-row x sweep, a 62 x 16 tile on 512 threads took 160.4 us against
// 153.5 us for 62 x 8.)  6, 7, 8 = column strips of 62 x 16, 32 and 64 cells walked in 4-row
// chunks (2D Euler, component-wise k = 3; every other scheme runs shape 4 for them).
constexpr int k2dShapes = 9;
constexpr int k2dStripFirst = 6;
hipError_t launch_stage2d_f64(int flux, int ncomp, int shape, const StageArgs& a, hipStream_t s);
hipError_t launch_stage2d_f32(int flux, int ncomp, int shape, const StageArgs& a, hipStream_t s);
// State check of u^n for ninst instances: alpha slot 0 (and the spread entries and packed slots
// of a single grid, or the spread entries bsp of a batch; any may be null), finiteness/physicality and the per-component FP64 sums.
// scratch holds G * ninst partial records (kCheckPartialBytes each); G workgroups per instance.
constexpr int kCheckPartialBytes = 56;
hipError_t launch_init_f64(int flux, int ncomp, InstDev* inst, int ninst, void* P0, void* P1,
                           unsigned long long* spread, void* pack, unsigned long long* bsp, int bsp_k, void* scratch,
                           int G, hipStream_t s);
hipError_t launch_init_f32(int flux, int ncomp, InstDev* inst, int ninst, void* P0, void* P1,
                           unsigned long long* spread, void* pack, unsigned long long* bsp, int bsp_k, void* scratch,
                           int G, hipStream_t s);

}  // namespace npw

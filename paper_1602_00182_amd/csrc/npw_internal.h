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
  int pad;
};

// One grid instance.  The static part is written by the host; the dynamic part only by kernels
// (and by the host between solves).
struct InstDev {
  long long off;  // element offset of the instance's state block in every state buffer
  long long nx, ny;
  double dx, dy, cfl, dt_fixed, T, tol;
  double speed_x, speed_y, gamma, eps_weno, eps_m;
  int bc, recon, sw, dim;
  // dynamic
  Ctl ctl[3];
  // Lax-Friedrichs alpha slots (bit patterns of non-negative doubles, combined with atomicMax):
  // slot 0 = alpha of u^n, slot 1 = alpha of u^(1), slot 2 = alpha of u^(2); [dir]
  unsigned long long alpha[3][2];
  int err;        // first error code (NPW_E*), 0 if none
  int err_stage;  // stage that detected it
  long long err_n;
  double err_t;
  double mass[4];  // per-component sums of the state (filled by the stats kernel)
};

struct Tile {
  int inst;
  int pad;
  long long start;  // first owned cell (1D: cell index; 2D: unused)
};

struct StageArgs {
  InstDev* inst;
  const Tile* tiles;
  int ntiles;             // tile count (and grid size) when ntiles_dev is null
  const int* ntiles_dev;  // optional device-resident tile count (serving)
  void* P0;  // ping-pong buffer 0
  void* P1;  // ping-pong buffer 1
  void* C;   // u^(2) buffer
  void* out; // rhs mode: destination of L(u)
  int stage; // 1, 2, 3: SSP-RK3 stage; 0: evaluate L(u^n) into out
};

// Launchers implemented in the kernel translation units (one per bulk precision).
hipError_t launch_stage_f64(int flux, int ncomp, int block, const StageArgs& a, hipStream_t s);
hipError_t launch_stage_f32(int flux, int ncomp, int block, const StageArgs& a, hipStream_t s);
// Recompute alpha slot 0, finiteness/physicality checks and the per-component sums of u^n.
hipError_t launch_init_f64(int flux, int ncomp, InstDev* inst, int ninst, void* P0, void* P1, hipStream_t s);
hipError_t launch_init_f32(int flux, int ncomp, InstDev* inst, int ninst, void* P0, void* P1, hipStream_t s);

}  // namespace npw

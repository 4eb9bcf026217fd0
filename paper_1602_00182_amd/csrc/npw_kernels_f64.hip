// Kernel instantiations for the double bulk precision.
#include "npw_kernels.h"
#include "npw_kernels2d.h"
#include "npw_kernels2d_strip.h"

namespace npw {

template <int BS, bool K2, bool PACK, bool BSP = false>
static hipError_t launch_stage_k(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  const dim3 grid(a.ntiles), block(BS);
  if (flux == kAdvection && ncomp == 1)
    stage1d_kernel<double, kAdvection, 1, BS, false, K2, PACK, BSP><<<grid, block, 0, s>>>(a);
  else if (flux == kBurgers && ncomp == 1)
    stage1d_kernel<double, kBurgers, 1, BS, false, K2, PACK, BSP><<<grid, block, 0, s>>>(a);
  else if (flux == kEuler && ncomp == 3 && a.charw)
    stage1d_kernel<double, kEuler, 3, BS, true, K2, PACK, BSP><<<grid, block, 0, s>>>(a);
  else if (flux == kEuler && ncomp == 3)
    stage1d_kernel<double, kEuler, 3, BS, false, K2, PACK, BSP><<<grid, block, 0, s>>>(a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Packed alpha slots (a.pack) exist for 64- and 128-thread workgroups only, and for at most
// kPackMax tiles.
template <int BS>
static hipError_t launch_stage_bs(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if constexpr (BS <= 128) {
    if (a.pack) {
      if (a.tiles != nullptr || a.ntiles > kPackMax) return hipErrorInvalidValue;
      return a.any_k2 ? launch_stage_k<BS, true, true>(flux, ncomp, a, s)
                      : launch_stage_k<BS, false, true>(flux, ncomp, a, s);
    }
  } else {
    if (a.pack) return hipErrorInvalidValue;
  }
  if (a.bsp) {
    if (a.tiles == nullptr) return hipErrorInvalidValue;  // per-instance entries belong to batches
    return a.any_k2 ? launch_stage_k<BS, true, false, true>(flux, ncomp, a, s)
                    : launch_stage_k<BS, false, false, true>(flux, ncomp, a, s);
  }
  return a.any_k2 ? launch_stage_k<BS, true, false>(flux, ncomp, a, s)
                  : launch_stage_k<BS, false, false>(flux, ncomp, a, s);
}

hipError_t launch_stage_f64(int flux, int ncomp, int block, const StageArgs& a, hipStream_t s) {
  switch (block) {
    case 64: return launch_stage_bs<64>(flux, ncomp, a, s);
    case 128: return launch_stage_bs<128>(flux, ncomp, a, s);
    case 256: return launch_stage_bs<256>(flux, ncomp, a, s);
    case 512: return launch_stage_bs<512>(flux, ncomp, a, s);
    default: return hipErrorInvalidValue;
  }
}

// 2D stage launch for one tile shape, with or without the k = 2 code.
template <int TX, int TY, bool K2, bool SHARE>
static hipError_t launch2d_k(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.nx + TX - 1) / TX), (unsigned)((a.ny + TY - 1) / TY)), block(256);
  if (flux == kEuler && ncomp == 4 && a.charw)
    stage2d_kernel<double, kEuler, 4, TX, TY, true, K2><<<grid, block, 0, s>>>(a);
  else if (flux == kEuler && ncomp == 4)
    stage2d_kernel<double, kEuler, 4, TX, TY, false, K2, SHARE><<<grid, block, 0, s>>>(a);
  else if (flux == kAdvection && ncomp == 1)
    stage2d_kernel<double, kAdvection, 1, TX, TY, false, K2, SHARE><<<grid, block, 0, s>>>(a);
  else if (flux == kBurgers && ncomp == 1)
    stage2d_kernel<double, kBurgers, 1, TX, TY, false, K2, SHARE><<<grid, block, 0, s>>>(a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// 2D tiles (x contiguous), one workgroup of 256 threads each; the shape is tunable.
template <int TX, int TY, bool SHARE>
static hipError_t launch2d(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  return a.any_k2 ? launch2d_k<TX, TY, true, SHARE>(flux, ncomp, a, s)
                  : launch2d_k<TX, TY, false, SHARE>(flux, ncomp, a, s);
}

// 2D Euler column strips of H rows (component-wise k = 3 only; other schemes take the 62 x 8 tile
// with per-interface denominators, whose sweeps the strip kernel shares).
template <int H>
static hipError_t launch2d_strip(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  if (flux != kEuler || ncomp != 4 || a.charw || a.any_k2) return launch2d<62, 8, false>(flux, ncomp, a, s);
  const dim3 grid((unsigned)((a.nx + kStripTX - 1) / kStripTX), (unsigned)((a.ny + H - 1) / H)), block(256);
  if (a.scheme == kSchemeRbfWeno5Switch)
    stage2d_strip_kernel<double, kEuler, H, kSchemeRbfWeno5Switch><<<grid, block, 0, s>>>(a);
  else
    stage2d_strip_kernel<double, kEuler, H><<<grid, block, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_stage2d_f64(int flux, int ncomp, int shape, const StageArgs& a, hipStream_t s) {
  switch (shape) {
    case 0: return launch2d<64, 8, true>(flux, ncomp, a, s);
    case 1: return launch2d<62, 8, true>(flux, ncomp, a, s);
    case 2: return launch2d<126, 4, true>(flux, ncomp, a, s);
    case 3: return launch2d<64, 8, false>(flux, ncomp, a, s);
    case 4: return launch2d<62, 8, false>(flux, ncomp, a, s);
    case 5: return launch2d<126, 4, false>(flux, ncomp, a, s);
    case 6: return launch2d_strip<16>(flux, ncomp, a, s);
    case 7: return launch2d_strip<32>(flux, ncomp, a, s);
    case 8: return launch2d_strip<64>(flux, ncomp, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_f64(int flux, int ncomp, InstDev* inst, int ninst, void* P0, void* P1,
                           unsigned long long* spread, void* pack, unsigned long long* bsp, int bsp_k, void* scratch,
                           int G, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  CheckPartial* part = reinterpret_cast<CheckPartial*>(scratch);
  const dim3 grid(G, ninst), block(256);
  if (flux == kAdvection && ncomp == 1)
    check_partial_kernel<double, kAdvection, 1><<<grid, block, 0, s>>>(inst, P0, P1, part, G);
  else if (flux == kBurgers && ncomp == 1)
    check_partial_kernel<double, kBurgers, 1><<<grid, block, 0, s>>>(inst, P0, P1, part, G);
  else if (flux == kEuler && ncomp == 3)
    check_partial_kernel<double, kEuler, 3><<<grid, block, 0, s>>>(inst, P0, P1, part, G);
  else if (flux == kEuler && ncomp == 4)
    check_partial_kernel<double, kEuler, 4><<<grid, block, 0, s>>>(inst, P0, P1, part, G);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  check_final_kernel<double><<<(ninst + 63) / 64, 64, 0, s>>>(inst, ninst, part, G, ncomp, spread,
                                                           static_cast<double*>(pack), bsp, bsp_k, 0);
  return hipGetLastError();
}

}  // namespace npw

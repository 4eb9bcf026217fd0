// Kernel instantiations for the float bulk precision.
#include "npw_kernels.h"
#include "npw_kernels2d.h"

namespace npw {

template <int BS>
static hipError_t launch_stage_bs(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  const dim3 grid(a.ntiles), block(BS);
  if (flux == kAdvection && ncomp == 1)
    stage1d_kernel<float, kAdvection, 1, BS><<<grid, block, 0, s>>>(a);
  else if (flux == kBurgers && ncomp == 1)
    stage1d_kernel<float, kBurgers, 1, BS><<<grid, block, 0, s>>>(a);
  else if (flux == kEuler && ncomp == 3)
    stage1d_kernel<float, kEuler, 3, BS><<<grid, block, 0, s>>>(a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stage_f32(int flux, int ncomp, int block, const StageArgs& a, hipStream_t s) {
  switch (block) {
    case 128: return launch_stage_bs<128>(flux, ncomp, a, s);
    case 256: return launch_stage_bs<256>(flux, ncomp, a, s);
    case 512: return launch_stage_bs<512>(flux, ncomp, a, s);
    default: return hipErrorInvalidValue;
  }
}

// 2D tiles of 64 x 8 cells (x contiguous), one workgroup each.
constexpr int kTX = 64, kTY = 8;
hipError_t launch_stage2d_f32(int flux, int ncomp, const StageArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.nx + kTX - 1) / kTX), (unsigned)((a.ny + kTY - 1) / kTY)), block(256);
  if (flux == kEuler && ncomp == 4)
    stage2d_kernel<float, kEuler, 4, kTX, kTY><<<grid, block, 0, s>>>(a);
  else if (flux == kAdvection && ncomp == 1)
    stage2d_kernel<float, kAdvection, 1, kTX, kTY><<<grid, block, 0, s>>>(a);
  else if (flux == kBurgers && ncomp == 1)
    stage2d_kernel<float, kBurgers, 1, kTX, kTY><<<grid, block, 0, s>>>(a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_init_f32(int flux, int ncomp, InstDev* inst, int ninst, void* P0, void* P1,
                           unsigned long long* spread, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  const dim3 grid(ninst), block(256);
  if (flux == kAdvection && ncomp == 1)
    init_kernel<float, kAdvection, 1><<<grid, block, 0, s>>>(inst, P0, P1, spread);
  else if (flux == kBurgers && ncomp == 1)
    init_kernel<float, kBurgers, 1><<<grid, block, 0, s>>>(inst, P0, P1, spread);
  else if (flux == kEuler && ncomp == 3)
    init_kernel<float, kEuler, 3><<<grid, block, 0, s>>>(inst, P0, P1, spread);
  else if (flux == kEuler && ncomp == 4)
    init_kernel<float, kEuler, 4><<<grid, block, 0, s>>>(inst, P0, P1, spread);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace npw

// valu_mix_probe.hip -- the VALU issue ceiling of an instruction mix on the local GPU.
//
// The stage kernels are bound by vector-ALU issue, and what one CU can issue per cycle depends on
// the mix: fp32 arithmetic, compares and selects, fp64, integer, conversions and reciprocals each
// go down pipes of their own widths, and some overlap.  This program replays a given mix with no
// memory traffic and no dependency stalls (several independent register chains per class, several
// waves per SIMD) and reports the rate it sustains; a kernel's measured issue rate divided by this
// ceiling says how close it runs to what its own instruction mix allows.
//
// Usage: valu_mix_probe class=count ...   (counts are relative weights, e.g. lane-instructions
//   per cell-stage from the hardware counters; they are scaled to 200 instructions per round)
// Classes: fma32 mul32 add32 cmp cnd mov logic fma64 mul64 add64 int32 int64 cvt trans32 trans64
// Prints one JSON line: the mix as replayed, and wave-instructions per second for the best of
// three chain counts (8, 6 and 4 chains: fewer chains need fewer registers, so more waves fit).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

namespace {

constexpr int kClasses = 15;
const char* const kNames[kClasses] = {"fma32", "mul32", "add32", "cmp",   "cnd",   "mov",     "logic",  "fma64",
                                      "mul64", "add64", "int32", "int64", "cvt",   "trans32", "trans64"};

struct Mix {
  int n[kClasses];  // instructions of each class per chain and round
};

// One class block: `count` times, one instruction per chain.  Every chain J reads chain J+1, so the
// chains stay live and independent within a block.
#define NPW_PROBE_BLOCK(COUNT, BODY)           \
  for (int r = 0; r < (COUNT); ++r) {          \
    _Pragma("unroll") for (int J = 0; J < NCH; ++J) { \
      const int K = (J + 1) % NCH;             \
      (void)K;                                 \
      BODY;                                    \
    }                                          \
  }

template <int NCH>
__global__ __launch_bounds__(256) void probe_kernel(float* out, Mix m, int rounds) {
  float x[NCH], y[NCH];
  double d[NCH], e[NCH];
  unsigned u[NCH], w[NCH];
  unsigned long long q[NCH];
  unsigned long long sm[NCH];  // lane masks (scalar registers)
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    x[j] = 1.0f + 1e-3f * (float)(threadIdx.x + j);
    y[j] = 0.999f;
    d[j] = (double)x[j];
    e[j] = 1.0;
    u[j] = threadIdx.x + j;
    w[j] = j;
    q[j] = j;
    sm[j] = ~0ull;
  }
  for (int it = 0; it < rounds; ++it) {
    NPW_PROBE_BLOCK(m.n[0], asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(x[J]) : "v"(y[J]), "v"(x[K])))
    NPW_PROBE_BLOCK(m.n[1], asm volatile("v_mul_f32 %0, %0, %1" : "+v"(x[J]) : "v"(y[J])))
    NPW_PROBE_BLOCK(m.n[2], asm volatile("v_add_f32 %0, %0, %1" : "+v"(y[J]) : "v"(x[J])))
    // compares write a lane mask to a scalar register pair and selects read one, as most of the
    // stage kernels' compares and selects do
    NPW_PROBE_BLOCK(m.n[3], asm volatile("v_cmp_gt_f32_e64 %0, %1, %2" : "=s"(sm[J]) : "v"(x[J]), "v"(y[J])))
    NPW_PROBE_BLOCK(m.n[4], asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(u[J]) : "v"(u[K]), "s"(sm[J])))
    NPW_PROBE_BLOCK(m.n[5], asm volatile("v_mov_b32 %0, %1" : "=v"(w[J]) : "v"(u[J])))
    NPW_PROBE_BLOCK(m.n[6], asm volatile("v_and_or_b32 %0, %0, %1, %2" : "+v"(u[J]) : "v"(w[J]), "v"(u[K])))
    NPW_PROBE_BLOCK(m.n[7], asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[J]) : "v"(e[J]), "v"(d[K])))
    NPW_PROBE_BLOCK(m.n[8], asm volatile("v_mul_f64 %0, %0, %1" : "+v"(e[J]) : "v"(d[J])))
    NPW_PROBE_BLOCK(m.n[9], asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[J]) : "v"(e[J])))
    NPW_PROBE_BLOCK(m.n[10], asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[J]) : "v"(w[J])))
    NPW_PROBE_BLOCK(m.n[11], asm volatile("v_lshl_add_u64 %0, %0, 2, %1" : "+v"(q[J]) : "v"(q[K])))
    // conversions alternate between the two directions the stage kernels use
    NPW_PROBE_BLOCK(m.n[12], if (J & 1) asm volatile("v_cvt_f32_f64 %0, %1" : "=v"(y[J]) : "v"(d[J]));
                    else asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(e[J]) : "v"(x[J])))
    NPW_PROBE_BLOCK(m.n[13], asm volatile("v_rcp_f32 %0, %1" : "=v"(y[J]) : "v"(y[J])))
    NPW_PROBE_BLOCK(m.n[14], asm volatile("v_rcp_f64 %0, %1" : "=v"(e[J]) : "v"(e[J])))
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < NCH; ++j)
    s += x[j] + y[j] + (float)d[j] + (float)e[j] + (float)(u[j] + w[j]) + (float)q[j];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

#define CHECK(x)                                                                          \
  do {                                                                                    \
    hipError_t err_ = (x);                                                                \
    if (err_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "valu_mix_probe: %s failed: %s\n", #x, hipGetErrorString(err_)); \
      std::exit(1);                                                                       \
    }                                                                                     \
  } while (0)

// Wave-instructions per second of probe_kernel<NCH>, launched as exactly as many workgroups of
// 4 waves as fit on the GPU at once (so no CU runs a partial last round).
template <int NCH>
double run(const Mix& m, float* out, int cus, int* waves_per_simd) {
  int per_cu = 0;
  CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, probe_kernel<NCH>, 256, 0));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;  // the output buffer holds 8 workgroups per CU
  *waves_per_simd = per_cu;  // 4 waves per workgroup over 4 SIMDs
  const int grid = cus * per_cu;
  long per_round = 0;
  for (int c = 0; c < kClasses; ++c) per_round += m.n[c];
  const int rounds = 400;
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  probe_kernel<NCH><<<grid, 256>>>(out, m, rounds / 8);  // warm-up (clocks, code load)
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e0));
  probe_kernel<NCH><<<grid, 256>>>(out, m, rounds);
  CHECK(hipGetLastError());
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.0f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  const double instr = (double)grid * 4.0 * rounds * (double)per_round * NCH;
  return instr / (ms * 1e-3);
}

}  // namespace

int main(int argc, char** argv) {
  double weight[kClasses] = {0};
  double total = 0.0;
  for (int i = 1; i < argc; ++i) {
    const char* eq = std::strchr(argv[i], '=');
    int c = -1;
    for (int k = 0; eq && k < kClasses; ++k)
      if ((size_t)(eq - argv[i]) == std::strlen(kNames[k]) && std::strncmp(argv[i], kNames[k], eq - argv[i]) == 0) c = k;
    if (c < 0) {
      std::fprintf(stderr, "valu_mix_probe: unknown argument '%s' (expected class=count)\n", argv[i]);
      return 2;
    }
    weight[c] = std::atof(eq + 1);
    if (!(weight[c] >= 0.0)) {
      std::fprintf(stderr, "valu_mix_probe: negative or invalid count in '%s'\n", argv[i]);
      return 2;
    }
    total += weight[c];
  }
  if (total <= 0.0) {
    std::fprintf(stderr, "usage: valu_mix_probe class=count ...\n");
    return 2;
  }
  Mix m;
  long per_round = 0;
  for (int c = 0; c < kClasses; ++c) {
    m.n[c] = (int)std::lround(200.0 * weight[c] / total);
    per_round += m.n[c];
  }
  int cus = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  float* out = nullptr;
  CHECK(hipMalloc(&out, (size_t)cus * 8 * 256 * sizeof(float)));  // at most 8 workgroups per CU
  int w8 = 0, w6 = 0, w4 = 0;
  const double r8 = run<8>(m, out, cus, &w8);
  const double r6 = run<6>(m, out, cus, &w6);
  const double r4 = run<4>(m, out, cus, &w4);
  CHECK(hipFree(out));
  const double best = std::fmax(r8, std::fmax(r6, r4));
  std::string mix;
  for (int c = 0; c < kClasses; ++c) {
    if (!m.n[c]) continue;
    if (!mix.empty()) mix += ",";
    mix += std::string(kNames[c]) + ":" + std::to_string(m.n[c]);
  }
  std::printf(
      "{\"mix_per_round\": \"%s\", \"instr_per_round\": %ld, \"cus\": %d, \"wave_instr_per_s\": %.6e, "
      "\"by_chains\": {\"8\": %.6e, \"6\": %.6e, \"4\": %.6e}, \"waves_per_simd\": {\"8\": %d, \"6\": %d, \"4\": %d}, "
      "\"per_cu_cycle_at_2p4ghz\": %.4f}\n",
      mix.c_str(), per_round, cus, best, r8, r6, r4, w8, w6, w4, best / (cus * 2.4e9));
  return 0;
}

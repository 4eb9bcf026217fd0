// npw_kernels.h -- the fused SSP-RK3 stage kernel for 1D grids and the state-check kernel.
// Included by one translation unit per bulk precision (npw_kernels_f64.hip, npw_kernels_f32.hip).
//
// One workgroup owns a tile of BS-2 consecutive cells of one instance.  Thread t stands for cell
// start-1+t, so the tile's interfaces x_{start-1/2} .. x_{start+BS-5/2} are all computed inside
// the workgroup.  Phases (each followed by a barrier):
//   load   -- cells start-3 .. start+BS (three ghosts per side) into LDS, coalesced, with
//             periodic / transmissive ghost mapping;
//   flag   -- Section 4 monotone test of the window centred on each cell (double);
//   eta    -- Table 3 shape parameter of each interface (double), zeroed by the switch;
//   recon  -- smoothness indicators of each cell, then v^-_{i+1/2} and v^+_{i-1/2} of that cell;
//   flux   -- global Lax-Friedrichs flux of each interface;
//   update -- flux difference (eq. PDE1), the SSP-RK3 stage combination, the store, and the
//             epilogue: validity check and max wave speed of the new state (wave shuffles, one
//             atomicMax per workgroup) that the next stage uses as its alpha.
#pragma once
#include <type_traits>

#include "../../include/npweno.h"
#include "npw_device.h"

namespace npw {

template <typename R, int FLUX, int M, int BS>
__device__ __forceinline__ void stage1d_tile(const StageArgs& a, const Tile tile) {
  constexpr bool kExact = std::is_same<R, double>::value;
  constexpr int W = BS + 4;  // LDS cells per component: start-3 .. start+BS
  __shared__ R s_u[M][W];
  __shared__ double s_d[kExact ? 1 : M][kExact ? 1 : W];
  __shared__ int s_flag[M][BS];
  __shared__ double s_eta[M][BS];
  __shared__ R s_vp[M][BS];
  __shared__ R s_F[M][BS];
  __shared__ unsigned long long s_red[BS / 64];
  __shared__ int s_bad[BS / 64];

  InstDev* I = a.inst + tile.inst;
  const int tid = threadIdx.x;
  const int stage = a.stage;
  const bool lead = (tile.start == 0 && tid == 0);

  if (I->err) return;

  // ---- step control (see Ctl): read the word of the previous stage, write our own ---------
  double t, dt = 0.0;
  long long n;
  unsigned long long alpha_bits;
  if (stage == 1) {
    t = I->ctl[0].t;
    n = I->ctl[0].n;
    const bool active = (I->T - t) > I->tol;
    if (active) dt = step_dt(I, t, bits_to_double(I->alpha[0][0]), bits_to_double(I->alpha[0][1]));
    if (lead) {
      Ctl c;
      c.t = t;
      c.dt = dt;
      c.n = n;
      c.active = active ? 1 : 0;
      c.pad = 0;
      I->ctl[1] = c;
      if (active) {
        I->alpha[2][0] = 0ull;
        I->alpha[2][1] = 0ull;
      }
    }
    if (!active) return;
    alpha_bits = I->alpha[0][0];
  } else if (stage == 2) {
    const Ctl c = I->ctl[1];
    if (lead) {
      I->ctl[2] = c;
      if (c.active) {
        I->alpha[0][0] = 0ull;
        I->alpha[0][1] = 0ull;
      }
    }
    if (!c.active) return;
    t = c.t;
    dt = c.dt;
    n = c.n;
    alpha_bits = I->alpha[1][0];
  } else if (stage == 3) {
    const Ctl c = I->ctl[2];
    if (!c.active) return;
    if (lead) {
      Ctl d;
      d.t = c.t + c.dt;
      d.dt = 0.0;
      d.n = c.n + 1;
      d.active = 0;
      d.pad = 0;
      I->ctl[0] = d;
      I->alpha[1][0] = 0ull;
      I->alpha[1][1] = 0ull;
    }
    t = c.t;
    dt = c.dt;
    n = c.n;
    alpha_bits = I->alpha[2][0];
  } else {
    t = I->ctl[0].t;
    n = I->ctl[0].n;
    alpha_bits = I->alpha[0][0];
  }
  const R alpha = R(bits_to_double(alpha_bits));
  const R rdt = R(dt);

  // ---- buffers: u^n lives in P[n & 1]; u^(1) and u^(n+1) in the other; u^(2) in C ----------
  const long long off = I->off, nx = I->nx;
  R* un = reinterpret_cast<R*>((n & 1) ? a.P1 : a.P0) + off;
  R* uo = reinterpret_cast<R*>((n & 1) ? a.P0 : a.P1) + off;
  R* u2 = reinterpret_cast<R*>(a.C) + off;
  const R* src = (stage == 0 || stage == 1) ? un : (stage == 2 ? uo : u2);
  R* dst = stage == 0 ? reinterpret_cast<R*>(a.out) + off : (stage == 2 ? u2 : uo);

  const int bc = I->bc;
  const long long start = tile.start;
  const bool use_eta = (I->recon == NPW_RBF_WENO5);
  const bool use_switch = use_eta && (I->sw == NPW_SWITCH_MONOTONE);
  const double eps_m = I->eps_m;
  const R eps = R(I->eps_weno);
  const R speed = R(I->speed_x), gamma = R(I->gamma);

  // ---- load ------------------------------------------------------------------------------
  for (int idx = tid; idx < W; idx += BS) {
    const long long g = ghost_index(start - 3 + idx, nx, bc);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      R v = src[c * nx + g];
      s_u[c][idx] = v;
      if constexpr (!kExact) s_d[c][idx] = double(v);
    }
  }
  __syncthreads();
  auto D = [&](int c, int idx) -> double {
    if constexpr (kExact)
      return s_u[c][idx];
    else
      return s_d[c][idx];
  };

  // ---- flag: window centred on cell start-1+tid (LDS index tid+2) -------------------------
  if (use_switch) {
#pragma unroll
    for (int c = 0; c < M; ++c) s_flag[c][tid] = monotone_flag(D(c, tid + 1), D(c, tid + 2), D(c, tid + 3));
  }
  __syncthreads();
  // ---- eta of interface x_{cell+1/2}, cells (LDS) tid+1 .. tid+4 ------------------------------
  if (tid < BS - 1) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      double e = 0.0;
      if (use_eta) {
        e = eta_ratio(D(c, tid + 1), D(c, tid + 2), D(c, tid + 3), D(c, tid + 4), eps_m);
        if (use_switch && (s_flag[c][tid] | s_flag[c][tid + 1])) e = 0.0;
      }
      s_eta[c][tid] = e;
    }
  }
  __syncthreads();
  // ---- recon: cell start-1+tid from LDS tid..tid+4 ----------------------------------------
  R vm[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const R eta_r = R(tid < BS - 1 ? s_eta[c][tid] : 0.0);
    const R eta_l = R(tid > 0 ? s_eta[c][tid - 1] : 0.0);
    R vp = R(0);
    vm[c] = R(0);
    if constexpr (kExact)
      weno_pair_exact(s_u[c][tid], s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], eta_r,
                      eta_l, eps, tid < BS - 1, tid > 0, vm[c], vp);
    else
      weno_pair_fast(s_u[c][tid], s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], eta_r,
                     eta_l, eps, tid < BS - 1, tid > 0, vm[c], vp);
    s_vp[c][tid] = vp;
  }
  __syncthreads();
  // ---- flux at x_{cell+1/2} ---------------------------------------------------------------
  if (tid < BS - 1) {
    R A[M], B[M], H[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      A[c] = vm[c];
      B[c] = s_vp[c][tid + 1];
    }
    lf_flux<R, FLUX, M, 0>(A, B, alpha, speed, gamma, H);
#pragma unroll
    for (int c = 0; c < M; ++c) s_F[c][tid] = H[c];
  }
  __syncthreads();
  // ---- update of the owned cells (tid = 1 .. BS-2) ---------------------------------------------
  const long long cell = start - 1 + tid;
  const bool owned = (tid >= 1 && tid <= BS - 2 && cell < nx);
  unsigned long long amax = 0ull;
  int bad = 0;
  if (owned) {
    const R dx = R(I->dx);
    R unew[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const R L = -(s_F[c][tid] - s_F[c][tid - 1]) / dx;
      if (stage == 0) {
        unew[c] = L;
      } else if (stage == 1) {
        unew[c] = s_u[c][tid + 2] + rdt * L;
      } else if (stage == 2) {
        const R u0 = un[c * nx + cell];
        unew[c] = R(0.75) * u0 + R(0.25) * (s_u[c][tid + 2] + rdt * L);
      } else {
        const R u0 = un[c * nx + cell];
        unew[c] = R(1.0 / 3.0) * u0 + R(2.0 / 3.0) * (s_u[c][tid + 2] + rdt * L);
      }
      dst[c * nx + cell] = unew[c];
    }
    if (stage != 0) {
      const R sr = spectral_radius<R, FLUX, M, 0>(unew, speed, gamma, bad);
      amax = double_to_bits(double(sr));
    }
  }
  if (stage == 0) return;
  // ---- epilogue: alpha of the new state and validity -------------------------------------
  amax = wave_max_u64(amax);
  const int anybad = __any(bad != 0) ? 1 : 0;
  int worst = bad;
#pragma unroll
  for (int off2 = 32; off2 > 0; off2 >>= 1) {
    int o = __shfl_xor(worst, off2, 64);
    worst = o > worst ? o : worst;
  }
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = amax;
    s_bad[tid >> 6] = anybad ? worst : 0;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long m = 0ull;
    int w = 0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) {
      m = s_red[k] > m ? s_red[k] : m;
      w = s_bad[k] > w ? s_bad[k] : w;
    }
    const int slot = stage == 1 ? 1 : (stage == 2 ? 2 : 0);
    if (w) {
      const int code = w == 2 ? NPW_ENONPHYSICAL : NPW_ENONFINITE;
      if (atomicCAS(&I->err, 0, code) == 0) {
        I->err_stage = stage;
        I->err_n = n;
        I->err_t = t;
      }
    } else {
      atomicMax(&I->alpha[slot][0], m);
    }
  }
}

// Grid-stride loop over the tile table; the tile count is read from device memory when the
// table is shared with a serving loop, so captured graphs stay valid as instances come and go.
template <typename R, int FLUX, int M, int BS>
__global__ __launch_bounds__(BS) void stage1d_kernel(StageArgs a) {
  const int nt = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
  for (int ti = blockIdx.x; ti < nt; ti += gridDim.x) {
    stage1d_tile<R, FLUX, M, BS>(a, a.tiles[ti]);
    __syncthreads();  // LDS is reused by the next tile
  }
}

// State check of u^n for every instance (one workgroup per instance): alpha slot 0, validity
// and the per-component sums (FP64, fixed order, so repeated calls agree bit for bit).
template <typename R, int FLUX, int M>
__global__ __launch_bounds__(256) void init_kernel(InstDev* inst, void* P0, void* P1) {
  InstDev* I = inst + blockIdx.x;
  const int tid = threadIdx.x;
  const long long n = I->ctl[0].n, nx = I->nx, ncell = I->nx * (I->dim == 2 ? I->ny : 1);
  const R* u = reinterpret_cast<const R*>((n & 1) ? P1 : P0) + I->off;
  const R speed = R(I->speed_x), gamma = R(I->gamma);
  (void)nx;
  unsigned long long ax = 0ull, ay = 0ull;
  int bad = 0;
  double sum[M];
#pragma unroll
  for (int c = 0; c < M; ++c) sum[c] = 0.0;
  for (long long k = tid; k < ncell; k += 256) {
    R U[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      U[c] = u[c * ncell + k];
      sum[c] += double(U[c]);
    }
    int b = 0;
    R sx = spectral_radius<R, FLUX, M, 0>(U, speed, gamma, b);
    bad = b > bad ? b : bad;
    unsigned long long bx = double_to_bits(double(sx));
    ax = bx > ax ? bx : ax;
    if (I->dim == 2) {
      R sy;
      if constexpr (FLUX == kAdvection)
        sy = fabs(R(I->speed_y));
      else
        sy = spectral_radius<R, FLUX, M, 1>(U, speed, gamma, b);
      unsigned long long by = double_to_bits(double(sy));
      ay = by > ay ? by : ay;
    }
  }
  __shared__ double s_sum[M][256];
  __shared__ unsigned long long s_ax[256], s_ay[256];
  __shared__ int s_b[256];
#pragma unroll
  for (int c = 0; c < M; ++c) s_sum[c][tid] = sum[c];
  s_ax[tid] = ax;
  s_ay[tid] = ay;
  s_b[tid] = bad;
  __syncthreads();
  if (tid == 0) {
    double tot[M];
    unsigned long long mx = 0ull, my = 0ull;
    int w = 0;
#pragma unroll
    for (int c = 0; c < M; ++c) tot[c] = 0.0;
    for (int k = 0; k < 256; ++k) {
#pragma unroll
      for (int c = 0; c < M; ++c) tot[c] += s_sum[c][k];
      mx = s_ax[k] > mx ? s_ax[k] : mx;
      my = s_ay[k] > my ? s_ay[k] : my;
      w = s_b[k] > w ? s_b[k] : w;
    }
    const double area = I->dx * (I->dim == 2 ? I->dy : 1.0);
    for (int c = 0; c < 4; ++c) I->mass[c] = c < M ? tot[c] * area : 0.0;
    I->alpha[0][0] = mx;
    I->alpha[0][1] = my;
    if (w) {
      I->err = w == 2 ? NPW_ENONPHYSICAL : NPW_ENONFINITE;
      I->err_stage = 0;
      I->err_n = n;
      I->err_t = I->ctl[0].t;
    }
  }
}

}  // namespace npw

// npw_kernels.h -- the fused SSP-RK3 stage kernel for 1D grids and the state-check kernel.
// Included by one translation unit per bulk precision (npw_kernels_f64.hip, npw_kernels_f32.hip).
//
// One workgroup owns a tile of BS-2 consecutive cells of one instance.  Thread t stands for cell
// start-1+t, so the tile's interfaces x_{start-1/2} .. x_{start+BS-5/2} are all computed inside
// the workgroup.  Phases (each followed by a barrier):
//   load      -- cells start-3 .. start+BS (three ghosts per side) into LDS, coalesced, with
//                periodic / transmissive ghost mapping (issued before the control words are read);
//   cell      -- Section 4 monotone test of the window centred on each cell (double) and the
//                cell's three weight denominators (eps + beta_r)^2;
//   interface -- Table 3 shape parameter (double) zeroed by the switch, v^- of the left cell,
//                v^+ of the right cell, global Lax-Friedrichs flux;
//   update    -- flux difference (eq. PDE1), the SSP-RK3 stage combination, the store, and the
//                epilogue: validity check and max wave speed of the new state (DPP wave max, one
//                atomicMax per workgroup) that the next stage uses as its alpha.
#pragma once
#include <type_traits>

#include "../../include/npweno.h"
#include "npw_device.h"

namespace npw {

// Barrier between the phases of a tile.  A one-wave workgroup needs none: a wave's LDS accesses
// complete in program order, so it only has to keep the compiler from moving them across.
template <int BS>
__device__ __forceinline__ void tile_barrier() {
  if constexpr (BS == 64)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  else
    __syncthreads();
}

// PACK: a single grid whose alpha slots hold one entry per tile (StageArgs::pack).  (A kernel
// built for one reconstruction alone was 5 % faster on a single grid, but it rounded some float
// results differently from this one, which batches, serving pools and the allocation-free
// right-hand side run, and those promise a single grid's results bit for bit.)
// BSP: a batch launch that may spread an instance's alpha over entries (StageArgs::bsp).
template <typename R, int FLUX, int M, int BS, bool CHAR, bool K2, bool PACK, bool BSP>
__device__ __forceinline__ void stage1d_tile(const StageArgs& a, const Tile tile) {
  constexpr bool kExact = std::is_same<R, double>::value;
  constexpr int W = BS + 4;  // LDS cells per component: start-3 .. start+BS
  __shared__ R s_u[M][W];
  __shared__ double s_d[kExact ? 1 : M][kExact ? 1 : W];
  __shared__ unsigned char s_flag[M][BS];
  __shared__ R s_den[M][3][BS];
  __shared__ R s_F[M][BS];
  __shared__ unsigned long long s_red[BS / 64];
  __shared__ int s_bad[BS / 64];

  const int tid = threadIdx.x;
  const int stage = a.stage;
  const int start = (int)tile.start, nx = (int)tile.nx;
  const long long off = tile.off;
  const int bc = tile.bc;
  const int par = a.par;

  // ---- issue the state loads first: they only depend on the launch and the tile ------------
  R* un = reinterpret_cast<R*>(par ? a.P1 : a.P0) + off;
  R* uo = reinterpret_cast<R*>(par ? a.P0 : a.P1) + off;
  R* u2 = reinterpret_cast<R*>(a.C) + off;
  const R* src = (stage == 0 || stage == 1) ? un : (stage == 2 ? uo : u2);
  R* dst = stage == 0 ? reinterpret_cast<R*>(a.out) + off : (stage == 2 ? u2 : uo);
  const int cell = start - 1 + tid;
  const bool owned = (tid >= 1 && tid <= BS - 2 && cell < nx);
  R ld0[M], ld1[M], upt[M];
  {
    // the window start-3 .. start+BS lies inside the grid for every tile but the first and last
    const bool inner = start >= 3 && start + BS < nx;
    const int g0 = inner ? start - 3 + tid : ghost_index(start - 3 + tid, nx, bc);
#pragma unroll
    for (int c = 0; c < M; ++c) ld0[c] = src[c * nx + g0];
    if (tid < W - BS) {
      const int g1 = inner ? start - 3 + BS + tid : ghost_index(start - 3 + BS + tid, nx, bc);
#pragma unroll
      for (int c = 0; c < M; ++c) ld1[c] = src[c * nx + g1];
    }
    if ((stage == 2 || stage == 3) && owned) {
#pragma unroll
      for (int c = 0; c < M; ++c) upt[c] = un[c * nx + cell];
    }
  }

  // ---- step control (see Ctl): read the word of the previous stage, write our own ---------
  // The record comes in through scalar loads, so the branches below wait for it alone, and the
  // staging below waits for the state loads alone.  Every wave of the grid reads the same alpha
  // lines, so their loads queue behind each other; they are issued after the state loads and
  // consumed only at the fluxes, with the staging and the reconstructions done meanwhile.
  InstDev* I = a.inst + tile.inst;
  unsigned long long* sp = a.spread;
  const bool lead = (start == 0 && tid == 0);
  const bool lead_wave = (start == 0 && tid < 64);
  // float bulk: spread entries carry the stage sequence that wrote them (spread_tag)
  constexpr bool kTag = !kExact;
  const int slot_in = stage == 0 ? 0 : stage - 1;
  // Alpha of the stage input: every entry of a packed slot (kPackLoads 16-byte loads per lane;
  // loads past the grid's tiles re-read the lane's first vector), else one spread entry per lane
  // (a single grid's, or its instance's in a batch), else the instance's own slot.  The same loads
  // on every path, so that the staging below can wait for the state loads while these are still in
  // flight.
  // A batch instance of more than kBspMinTiles tiles spreads its alpha over its bsp entries; one
  // of fewer keeps its record's slot, whose one atomic costs less than the entries' reduction.
  unsigned long long* const bsp = BSP && a.bsp && nx > kBspMinTiles * (BS - 2)
                                      ? a.bsp + (size_t)tile.inst * 3 * (size_t)a.bsp_k * kSpreadStride
                                      : nullptr;
  PackVec<R> pv[PACK ? kPackLoads<R> : 1];
  unsigned long long sp_e = 0ull;
  if constexpr (PACK) {
    constexpr int kPer = 16 / (int)sizeof(R);  // entries per vector
    const PackVec<R>* P = reinterpret_cast<const PackVec<R>*>(static_cast<const R*>(a.pack) + slot_in * kPackMax);
    const int G = (int)gridDim.x, lane = tid & 63;
#pragma unroll
    for (int c = 0; c < kPackLoads<R>; ++c) {
      const int q = c * 64 + lane;
      pv[c] = P[q * kPer < G ? q : lane];
    }
  } else {
    sp_e = *(sp    ? spread_entry_ptr(sp, slot_in, 0)
             : bsp ? &bsp[(slot_in * a.bsp_k + (tid & (a.bsp_k - 1))) * kSpreadStride]
                   : &I->alpha[slot_in][0]);
  }
  // stage 0 and 1 step from ctl[0], stage 2 from ctl[1], stage 3 from ctl[2]; every branch
  // below is decided from these loads at once
  const Ctl* cp = &I->ctl[stage <= 1 ? 0 : stage - 1];
  const int err = scalar_load(&I->err);
  const double t = scalar_load(&cp->t), dt_in = scalar_load(&cp->dt);
  const long long n = scalar_load(&cp->n);
  const int active_in = scalar_load(&cp->active), home_in = scalar_load(&cp->home);
  const double T = scalar_load(&I->T), tol = scalar_load(&I->tol);
  const long long seq_base = scalar_load(&I->seq_base);
  // a first stage starts a step while the instance has not reached T; the other two go on with
  // the step that the first one started
  const bool run = !err && (stage == 0 || (stage == 1 ? (T - t) > tol : active_in != 0));
  // zero an alpha slot before the kernel that accumulates into it runs (tagged slots need not be)
  auto zero_slot = [&](int slot) {
    if (sp) {
      if (!kTag && lead_wave && tid < kSpread) {
        sp[((slot * 2 + 0) * kSpread + tid) * kSpreadStride] = 0ull;
        sp[((slot * 2 + 1) * kSpread + tid) * kSpreadStride] = 0ull;
      }
    } else if (bsp) {
      if (lead_wave && tid < a.bsp_k) bsp[(slot * a.bsp_k + tid) * kSpreadStride] = 0ull;
    } else if (lead) {
      I->alpha[slot][0] = 0ull;
      I->alpha[slot][1] = 0ull;
    }
  };
  if (lead && !err) {
    if (stage == 1 && !run) {  // the instance is done: an idle step record
      Ctl c;
      c.t = t;
      c.dt = 0.0;
      c.n = n;
      c.active = 0;
      c.home = par;
      I->ctl[1] = c;
    } else if (stage == 2) {  // the third stage steps from the same record
      Ctl c;
      c.t = t;
      c.dt = dt_in;
      c.n = n;
      c.active = active_in;
      c.home = home_in;
      I->ctl[2] = c;
    } else if (stage == 3 && run) {  // the next step starts from u^(n+1), written by this stage
      Ctl d;
      d.t = t + dt_in;
      d.dt = 0.0;
      d.n = n + 1;
      d.active = 0;
      d.home = par ^ 1;
      I->ctl[0] = d;
    }
  }
  if (!run) return;
  if (stage != 0) zero_slot(stage == 1 ? 2 : (stage == 2 ? 0 : 1));
  double dt = stage == 1 ? 0.0 : dt_in;
  ReconMode rm = recon_mode(scalar_load(&I->recon), scalar_load(&I->sw));
  if (!K2) rm.k2 = false;  // launched for k = 3 instances only
  const bool k2 = rm.k2, eno = rm.eno, use_eta = rm.use_eta, use_switch = rm.use_switch;
  const double eps_m = scalar_load(&I->eps_m);
  const R eps = R(scalar_load(&I->eps_weno));
  const R speed = R(scalar_load(&I->speed_x)), gamma = R(scalar_load(&I->gamma));
  const double dxd = scalar_load(&I->dx);
  const R dx = R(dxd);
  const R inv_dx = R(scalar_load(&I->inv_dx));

  // ---- stage input into LDS ----------------------------------------------------------------
#pragma unroll
  for (int c = 0; c < M; ++c) {
    s_u[c][tid] = ld0[c];
    if constexpr (!kExact) s_d[c][tid] = double(ld0[c]);
  }
  if (tid < W - BS) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      s_u[c][BS + tid] = ld1[c];
      if constexpr (!kExact) s_d[c][BS + tid] = double(ld1[c]);
    }
  }
  tile_barrier<BS>();
  auto D = [&](int c, int idx) -> double {
    if constexpr (kExact)
      return s_u[c][idx];
    else
      return s_d[c][idx];
  };

  // ---- cell phase: cell start-1+tid (LDS window tid..tid+4) -------------------------------
  // Section 4 monotone flag of the window centred on the cell, and the three weight
  // denominators (eps + beta_r)^2 of the cell.  (Characteristic fields belong to an interface,
  // so that mode does all of its work in the interface phase.)
#pragma unroll
  for (int c = 0; c < (CHAR ? 0 : M); ++c) {
    // bit 0: switch flag; bits 1-2: ENO stencil
    int fl = use_switch ? monotone_flag<kExact>(D(c, tid + 1), D(c, tid + 2), D(c, tid + 3)) : 0;
    if (k2) {
      // k = 2: the cell's ENO2 stencil, and its right- and left-edge shape parameters (zero
      // when the cell's window is flagged), kept in the denominator slots 0 and 1
      if (eno) fl |= eno2_stencil(D(c, tid + 1), D(c, tid + 2), D(c, tid + 3)) << 1;
      double er = 0.0, el = 0.0;
      if (use_eta && !(fl & 1)) {
        er = eta2_ratio<kExact>(D(c, tid + 1), D(c, tid + 2), D(c, tid + 3), eps_m);
        el = eta2_ratio<kExact>(D(c, tid + 3), D(c, tid + 2), D(c, tid + 1), eps_m);
      }
      s_den[c][0][tid] = R(er);
      s_den[c][1][tid] = R(el);
    } else if (eno) {
      fl |= eno_stencil(D(c, tid), D(c, tid + 1), D(c, tid + 2), D(c, tid + 3), D(c, tid + 4)) << 1;
    } else {
      R d0, d1, d2;
      weight_denominators<R>(s_u[c][tid], s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], eps,
                             d0, d1, d2);
      s_den[c][0][tid] = d0;
      s_den[c][1][tid] = d1;
      s_den[c][2][tid] = d2;
    }
    s_flag[c][tid] = (unsigned char)fl;
  }
  tile_barrier<BS>();
  // ---- interface phase: x_{cell+1/2} between cell start-1+tid and the next (tid < BS-1) ----
  // eta (Table 3 caption) zeroed by the switch, v^- of the left cell, v^+ of the right cell,
  // and the global Lax-Friedrichs flux.
  R A[M], B[M];
  if (tid < BS - 1) {
    if constexpr (CHAR) {  // cells i-2..i+3 of interface i+1/2 are LDS tid..tid+5
      R U[6][M];
#pragma unroll
      for (int k = 0; k < 6; ++k)
#pragma unroll
        for (int c = 0; c < M; ++c) U[k][c] = s_u[c][tid + k];
      char_states<R, M, 0>(U, gamma, rm, eps, eps_m, A, B);
    }
#pragma unroll
    for (int c = 0; c < (CHAR ? 0 : M); ++c) {
      if (k2) {  // left cell LDS tid+2, right cell tid+3; each edge with its own cell's eta
        const R el = s_den[c][0][tid], er = s_den[c][1][tid + 1];
        if (eno) {
          A[c] = eno2<R, false>((s_flag[c][tid] >> 1) & 1, s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], el);
          B[c] = eno2<R, true>((s_flag[c][tid + 1] >> 1) & 1, s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], er);
        } else {
          A[c] = weno3<R, false>(s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], el, eps);
          B[c] = weno3<R, true>(s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], er, eps);
        }
        continue;
      }
      R eta = R(0);
      if (use_eta) {
        eta = R(eta_ratio<kExact>(D(c, tid + 1), D(c, tid + 2), D(c, tid + 3), D(c, tid + 4), eps_m));
        if (use_switch && ((s_flag[c][tid] | s_flag[c][tid + 1]) & 1)) eta = R(0);
      }
      if (eno) {
        A[c] = eno_minus<R>(s_flag[c][tid] >> 1, s_u[c][tid], s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3],
                            s_u[c][tid + 4], eta);
        B[c] = eno_plus<R>(s_flag[c][tid + 1] >> 1, s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3],
                           s_u[c][tid + 4], s_u[c][tid + 5], eta);
      } else {
        A[c] = weno_minus<R>(s_u[c][tid], s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], eta,
                             s_den[c][0][tid], s_den[c][1][tid], s_den[c][2][tid]);
        B[c] = weno_plus<R>(s_u[c][tid + 1], s_u[c][tid + 2], s_u[c][tid + 3], s_u[c][tid + 4], s_u[c][tid + 5],
                            eta, s_den[c][0][tid + 1], s_den[c][1][tid + 1], s_den[c][2][tid + 1]);
      }
    }
  }
  // alpha of the stage input (max over the packed or spread entries: the whole wave takes part),
  // then the step size of a first stage, which its lead thread records for the two that follow
  unsigned long long alpha_bits;
  if constexpr (PACK) {
    alpha_bits = double_to_bits(double(pack_max<R, kPackLoads<R>>(pv)));
  } else if (sp) {
    if constexpr (kTag)
      alpha_bits = spread_reduce_tagged(sp_e, 3 * (n - seq_base) + slot_in);
    else
      alpha_bits = spread_reduce(sp_e);
  } else {
    // float bulk: the entries hold float wave speeds widened exactly, so their maximum is taken in
    // float (one register, merged lane moves), with the same result
    if (bsp)
      alpha_bits = kExact ? spread_reduce(sp_e)
                          : double_to_bits(double(wave_max_nonneg<float>(float(bits_to_double(sp_e)))));
    else
      alpha_bits = sp_e;
  }
  const R alpha = R(bits_to_double(alpha_bits));
  if (tid < BS - 1) {
    R H[M];
    lf_flux<R, FLUX, M, 0>(A, B, alpha, speed, gamma, H);
#pragma unroll
    for (int c = 0; c < M; ++c) s_F[c][tid] = H[c];
  }
  if (stage == 1) {
    dt = step_dt<1>(scalar_load(&I->dt_fixed), scalar_load(&I->cfl), dxd, 0.0, T, t, bits_to_double(alpha_bits), 0.0);
    if (lead) {
      Ctl c;
      c.t = t;
      c.dt = dt;
      c.n = n;
      c.active = 1;
      c.home = par;
      I->ctl[1] = c;
    }
  }
  const R rdt = R(dt);
  tile_barrier<BS>();
  // ---- update of the owned cells (tid = 1 .. BS-2) ---------------------------------------------
  R amax = R(0);
  int bad = 0;
  if (owned) {
    R unew[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      R L;
      if constexpr (kExact)
        L = -div_rn(s_F[c][tid] - s_F[c][tid - 1], dx);
      else
        L = (s_F[c][tid - 1] - s_F[c][tid]) * inv_dx;
      if (stage == 0)
        unew[c] = L;
      else
        unew[c] = rk3_combine<R>(stage, upt[c], s_u[c][tid + 2], rdt * L);
      dst[c * nx + cell] = unew[c];
    }
    if (stage != 0) amax = spectral_radius<R, FLUX, M, 0>(unew, speed, gamma, bad);
  }
  if (stage == 0) return;
  // ---- epilogue: alpha of the new state and validity -------------------------------------
  amax = wave_max_nonneg(amax);
  const bool bad2 = __any(bad == 2), bad1 = __any(bad == 1);
  if constexpr (BS > 64) {  // combine the waves through LDS (a one-wave workgroup needs no barrier)
    if ((tid & 63) == 0) {
      s_red[tid >> 6] = double_to_bits(double(amax));
      s_bad[tid >> 6] = bad2 ? 2 : (bad1 ? 1 : 0);
    }
    __syncthreads();
  }
  if (tid == 0) {
    unsigned long long m = double_to_bits(double(amax));
    int w = bad2 ? 2 : (bad1 ? 1 : 0);
    if constexpr (BS > 64) {
#pragma unroll
      for (int k = 1; k < BS / 64; ++k) {
        m = s_red[k] > m ? s_red[k] : m;
        w = s_bad[k] > w ? s_bad[k] : w;
      }
    }
    if (w) {
      const int code = w == 2 ? NPW_ENONPHYSICAL : NPW_ENONFINITE;
      if (atomicCAS(&I->err, 0, code) == 0) {
        I->err_stage = stage;
        I->err_n = n;
        I->err_t = t;
        I->err_home = par;
      }
    } else {
      const int slot_out = stage == 1 ? 1 : (stage == 2 ? 2 : 0);
      if constexpr (PACK) {  // this tile's entry: a plain store, no other workgroup writes it
        static_cast<R*>(a.pack)[slot_out * kPackMax + xcd_contiguous_tile(blockIdx.x, gridDim.x)] =
            R(bits_to_double(m));
      } else {
        unsigned long long* const aout =
            sp    ? &sp[((slot_out * 2 + 0) * kSpread + blockIdx.x % kSpread) * kSpreadStride]
            : bsp ? &bsp[(slot_out * a.bsp_k + ((int)(start / (BS - 2)) & (a.bsp_k - 1))) * kSpreadStride]
                  : &I->alpha[slot_out][0];
        atomicMax(aout, (sp && kTag) ? spread_tag(3 * (n - seq_base) + stage, float(bits_to_double(m))) : m);
      }
    }
  }
}

// Grid-stride loop over the tile table; the tile count is read from device memory when the
// table is shared with a serving loop, so captured graphs stay valid as instances come and go.
// PACK: single grids with packed alpha slots only.
template <typename R, int FLUX, int M, int BS, bool CHAR = false, bool K2 = true, bool PACK = false, bool BSP = false>
__global__ __launch_bounds__(BS) void stage1d_kernel(StageArgs a) {
  // (A BSP kernel runs batches only: a second instantiation of the tile function here would hold
  // LDS arrays of its own and halve the workgroups a CU takes.)
  if constexpr (!BSP) {
    if (PACK || a.tiles == nullptr) {  // single instance: tiles follow from the block index
      Tile t;
      t.inst = 0;
      t.bc = a.bc;
      t.start = xcd_contiguous_tile(blockIdx.x, gridDim.x) * (BS - 2);
      t.nx = a.nx;
      t.off = 0;
      stage1d_tile<R, FLUX, M, BS, CHAR, K2, PACK, false>(a, t);
      return;
    }
  }
  const int nt = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
  if ((int)gridDim.x == nt) {  // one tile per workgroup (a batch): XCD-contiguous runs of the table
    stage1d_tile<R, FLUX, M, BS, CHAR, K2, false, BSP>(a, scalar_load_tile(&a.tiles[xcd_contiguous_tile(blockIdx.x, nt)]));
    return;
  }
  for (int ti = blockIdx.x; ti < nt; ti += gridDim.x) {
    stage1d_tile<R, FLUX, M, BS, CHAR, K2, false, BSP>(a, scalar_load_tile(&a.tiles[ti]));
    __syncthreads();  // LDS is reused by the next tile
  }
}

// State check of u^n for every instance: alpha slot 0, validity and the per-component sums
// (FP64).  Two passes: G workgroups per instance accumulate fixed, strided subsets of the cells
// into partial records, then one thread per instance combines its G records in order, so the
// result is the same bit for bit on every call.
struct CheckPartial {
  double sum[4];
  unsigned long long ax, ay;
  int bad, pad;
};
static_assert(sizeof(CheckPartial) == kCheckPartialBytes, "scratch is sized with kCheckPartialBytes");

template <typename R, int FLUX, int M>
__global__ __launch_bounds__(256) void check_partial_kernel(InstDev* inst, void* P0, void* P1, CheckPartial* part,
                                                            int G) {
  const int b = blockIdx.y, g = blockIdx.x, tid = threadIdx.x;
  InstDev* I = inst + b;
  const long long ncell = I->nx * (I->dim == 2 ? I->ny : 1);
  const R* u = reinterpret_cast<const R*>(I->ctl[0].home ? P1 : P0) + I->off;
  const R speed = R(I->speed_x), gamma = R(I->gamma);
  const bool two_d = I->dim == 2;
  unsigned long long ax = 0ull, ay = 0ull;
  int bad = 0;
  double sum[M];
#pragma unroll
  for (int c = 0; c < M; ++c) sum[c] = 0.0;
  for (long long k = (long long)g * 256 + tid; k < ncell; k += (long long)G * 256) {
    R U[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      U[c] = u[c * ncell + k];
      sum[c] += double(U[c]);
    }
    int bx_bad = 0;
    const R sx = spectral_radius<R, FLUX, M, 0>(U, speed, gamma, bx_bad);
    bad = bx_bad > bad ? bx_bad : bad;
    const unsigned long long bx = double_to_bits(double(sx));
    ax = bx > ax ? bx : ax;
    if (two_d) {
      int by_bad = 0;
      R sy;
      if constexpr (FLUX == kAdvection)
        sy = fabs(R(I->speed_y));
      else
        sy = spectral_radius<R, FLUX, M, 1>(U, speed, gamma, by_bad);
      const unsigned long long by = double_to_bits(double(sy));
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
    CheckPartial p;
    for (int c = 0; c < 4; ++c) p.sum[c] = 0.0;
    p.ax = 0ull;
    p.ay = 0ull;
    p.bad = 0;
    p.pad = 0;
    for (int k = 0; k < 256; ++k) {
#pragma unroll
      for (int c = 0; c < M; ++c) p.sum[c] += s_sum[c][k];
      p.ax = s_ax[k] > p.ax ? s_ax[k] : p.ax;
      p.ay = s_ay[k] > p.ay ? s_ay[k] : p.ay;
      p.bad = s_b[k] > p.bad ? s_b[k] : p.bad;
    }
    part[(long long)b * G + g] = p;
  }
}

// R: the bulk precision (the type of packed alpha entries).
template <typename R>
static __global__ __launch_bounds__(64) void check_final_kernel(InstDev* inst, int ninst, const CheckPartial* part, int G,
                                                                int ncomp, unsigned long long* spread, R* pack,
                                                                unsigned long long* bsp, int bsp_k, int tagged) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  // single grid: entry 0 of slot 0 holds alpha, every other entry (all packed slots included)
  // starts at 0
  if (spread && blockIdx.x == 0) {
    for (int k = threadIdx.x; k < 3 * 2 * kSpread; k += 64) spread[k * kSpreadStride] = 0ull;
  }
  if (pack && blockIdx.x == 0) {
    for (int k = threadIdx.x; k < 3 * kPackMax; k += 64) pack[k] = R(0);
  }
  __syncthreads();
  if (b >= ninst) return;
  InstDev* I = inst + b;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  unsigned long long mx = 0ull, my = 0ull;
  int w = 0;
  for (int g = 0; g < G; ++g) {
    const CheckPartial& p = part[(long long)b * G + g];
    for (int c = 0; c < 4; ++c) tot[c] += p.sum[c];
    mx = p.ax > mx ? p.ax : mx;
    my = p.ay > my ? p.ay : my;
    w = p.bad > w ? p.bad : w;
  }
  const double area = I->dx * (I->dim == 2 ? I->dy : 1.0);
  for (int c = 0; c < 4; ++c) I->mass[c] = c < ncomp ? tot[c] * area : 0.0;
  I->alpha[0][0] = mx;
  I->alpha[0][1] = my;
  if (pack) pack[0] = R(bits_to_double(mx));
  if (bsp) {  // a batch instance: entry 0 of slot 0 holds alpha, every other entry of its slots 0
    unsigned long long* e = bsp + (size_t)b * 3 * (size_t)bsp_k * kSpreadStride;
    for (int k = 0; k < 3 * bsp_k; ++k) e[k * kSpreadStride] = k == 0 ? mx : 0ull;
  }
  if (spread) {  // the state of step n opens sequence 3 (n - seq_base) (see spread_tag)
    const long long seq = 3 * (I->ctl[0].n - I->seq_base);
    spread[(0 * kSpread + 0) * kSpreadStride] = tagged ? spread_tag(seq, float(bits_to_double(mx))) : mx;
    spread[(1 * kSpread + 0) * kSpreadStride] = tagged ? spread_tag(seq, float(bits_to_double(my))) : my;
  }
  if (w) {
    I->err = w == 2 ? NPW_ENONPHYSICAL : NPW_ENONFINITE;
    I->err_stage = 0;
    I->err_n = I->ctl[0].n;
    I->err_t = I->ctl[0].t;
    I->err_home = I->ctl[0].home;
  }
}

}  // namespace npw

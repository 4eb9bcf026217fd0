// npw_kernels2d_strip.h -- fused SSP-RK3 stage kernel for 2D Euler on column strips.
//
// The same scheme as stage2d_kernel (Section 7, eq. 2DIntegral, one midpoint point per face,
// dimension by dimension; component-wise k = 3 reconstruction, four components), organised so that
// the y sweep and the per-workgroup work are not repeated for every 8 rows:
//   * one workgroup (four waves) owns a strip of 62 columns and H rows and walks it in chunks of 4
//     rows; the rows it needs are staged in a ring of 12 LDS rows (68 cells wide: 3 ghosts a side);
//   * x sweep: wave w takes row w of the chunk, lane l cell l - 1 of that row, and forms the
//     interface l - 1/2 whole (flag, weight denominators, eta, v^-, v^+, flux); the flux difference
//     of its cell comes from the neighbouring lane, so -dF/dx stays in registers;
//   * y sweep: wave c takes component c, lane x column x, and marches up the column through the
//     whole strip, carrying the six-cell window, its doubles and the previous cell's flag and
//     weight denominators in registers from chunk to chunk: each cell's quantities and each
//     interface's eta, v^- and v^+ are formed once per strip, not once per 8-row tile plus 2;
//   * a flux pass combines the four components of each y interface, and the update uses the
//     x sweep's lane mapping (wave w row w, lane l cell l - 1).
// The functions and their operands are those of stage2d_kernel, so the double bulk's results are
// the same bit for bit (and the oracle's); only the order in which work is done changes.
#pragma once
#include <type_traits>

#include "../../include/npweno.h"
#include "npw_device.h"

namespace npw {

constexpr int kStripTX = 62;  // owned columns of a strip (cells -1..62 of a row fill one wave)
constexpr int kStripCH = 4;   // rows per chunk (one per wave in the x sweep and the update)

// H = rows of a strip (a multiple of kStripCH).  Euler, four components, k = 3 component-wise.
// Float: 6 waves per SIMD, the most its 24 KB of LDS allows; it needs 77 vector registers (71 when
// built for one scheme) because nothing is held across the chunk loop but the march's previous-cell
// flag and weight denominators, the running spectral radii and the lane index (made opaque each
// chunk), and the next chunk's rows travel from memory to LDS without registers.
// SCHEME: kSchemeAny reads the reconstruction from the instance record; kSchemeRbfWeno5Switch is
// built for RBF-WENO5 with the switch alone (every instance of the launch uses it), so that the
// compiler sees no other scheme's code or run-time choice (118.3 -> 112.8 us per 2048^2 stage).
template <typename R, int FLUX, int H, int SCHEME = kSchemeAny>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 6 : 1))) void
stage2d_strip_kernel(StageArgs a) {
  constexpr int M = 4, BS = 256, TX = kStripTX, CH = kStripCH;
  constexpr int WX = TX + 6;     // staged cells per row: -3..TX+2
  // staged rows: the chunk's rows, the rows the column march reads ahead, and the next chunk's four
  // rows, which are loaded a whole chunk ahead into the slots of rows no longer read
  constexpr int RING = 13;
  constexpr bool kExact = std::is_same<R, double>::value;
  static_assert(H % CH == 0 && M * 64 == BS, "one wave per component, one row per wave");
  __shared__ R s_u[M][RING][WX];
  // y interfaces jk + s - 1/2 (s = 0..CH) of chunk k sit in slot (CH k + s) mod (CH + 1): v^- (then
  // the flux G, in place) and v^+; a chunk's top flux slot is the next chunk's bottom one
  __shared__ R s_vm[M][CH + 1][TX];
  __shared__ R s_vp[M][CH + 1][TX];
  __shared__ unsigned long long s_red[2][BS / 64];
  __shared__ int s_bad[BS / 64];

  const int tid = threadIdx.x;
  int lane = tid & 63;  // re-derived at every chunk (see the chunk loop)
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform over the wave
  const int stage = a.stage;
  const int nx = (int)a.nx, ny = (int)a.ny;
  const long long strip = xcd_contiguous_tile((long long)blockIdx.y * gridDim.x + blockIdx.x,
                                              (long long)gridDim.x * gridDim.y);
  const unsigned grid_x = gridDim.x;
  int tbx, tby;
  if (strip < (1LL << 32)) {
    tby = (int)((unsigned)strip / grid_x);
    tbx = (int)((unsigned)strip - (unsigned)tby * grid_x);
  } else {
    tby = (int)(strip / grid_x);
    tbx = (int)(strip - (long long)tby * grid_x);
  }
  const int i0 = tbx * TX, j0 = tby * H;
  const int bc = a.bc;
  const int par = a.par;
  const long long ncell = (long long)nx * ny;
  R* un = reinterpret_cast<R*>(par ? a.P1 : a.P0);
  R* uo = reinterpret_cast<R*>(par ? a.P0 : a.P1);
  R* u2 = reinterpret_cast<R*>(a.C);
  const R* src = (stage == 0 || stage == 1) ? un : (stage == 2 ? uo : u2);
  R* dst = stage == 0 ? reinterpret_cast<R*>(a.out) : (stage == 2 ? u2 : uo);

  // Columns: strips whose 3-cell halo lies inside the grid address through buffer resources (32-bit
  // offsets; states below 4 GiB); rows outside the grid, and every row of the edge strips, take the
  // ghost mapping.  Both tests are uniform over the workgroup for a given row.
  const bool big = (unsigned long long)M * ncell * sizeof(R) >= (1ULL << 32);
  const bool cols_in = i0 >= 3 && i0 + TX + 3 <= nx && !big;
  const unsigned state_bytes = (unsigned)((unsigned long long)M * ncell * sizeof(R));
  const unsigned comp_bytes = (unsigned)(ncell * sizeof(R));
  // ring slot of grid row j (j >= j0 - 3)
  auto slot_of = [&](int j) -> int { return (j - j0 + 3) % RING; };
  // Stage grid row `row` (all components, the strip's 68 cells) into its ring slot; one wave per
  // row: lane l takes cell l, and lanes 0..3 also cells 64..67.
  auto stage_row = [&](int row) {
    const int sl = slot_of(row);
    const bool in_row = cols_in && row >= 0 && row < ny;  // uniform
    R v[2][M];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cell = lane + 64 * h;
      if (h == 0 || lane < WX - 64) {
        if (in_row) {
          const __amdgpu_buffer_rsrc_t rs = buffer_of(src, state_bytes);
          const unsigned at = ((unsigned)row * (unsigned)nx + (unsigned)(i0 - 3 + cell)) * sizeof(R);
#pragma unroll
          for (int c = 0; c < M; ++c) v[h][c] = buffer_load<R>(rs, at, c * comp_bytes);
        } else {
          const long long at = (long long)ghost_index(row, ny, bc) * nx + ghost_index(i0 - 3 + cell, nx, bc);
#pragma unroll
          for (int c = 0; c < M; ++c) v[h][c] = src[c * ncell + at];
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 0 || lane < WX - 64) {
#pragma unroll
        for (int c = 0; c < M; ++c) s_u[c][sl][lane + 64 * h] = v[h][c];
      }
    }
  };

  // ---- step control (the protocol of the tile kernels; the lead is strip (0, 0)) -------------
  InstDev* I = a.inst;
  unsigned long long* sp = a.spread;
  const bool first_block = (tbx == 0 && tby == 0);
  const bool lead = first_block && tid == 0;
  constexpr bool kTag = !kExact;
  const int slot_in = stage == 0 ? 0 : stage - 1;
  const unsigned long long spx = sp ? spread_entry(sp, slot_in, 0) : 0ull;
  const unsigned long long spy = sp ? spread_entry(sp, slot_in, 1) : 0ull;
  // every field of the instance record the stage needs, read before the first branch and store
  // (later loads would each add a round trip to memory)
  const int err = I->err;
  const Ctl c0 = I->ctl[0], c1 = I->ctl[1], c2 = I->ctl[2];
  const long long seq_base = scalar_reg(I->seq_base);
  const double T = scalar_reg(I->T), tol = scalar_reg(I->tol);
  const double dt_fixed = scalar_reg(I->dt_fixed), cfl = scalar_reg(I->cfl), dxd = scalar_reg(I->dx),
               dyd = scalar_reg(I->dy);
  const int i_recon = scalar_reg(I->recon), i_sw = scalar_reg(I->sw);
  const double i_eps_m = scalar_reg(I->eps_m), i_eps = scalar_reg(I->eps_weno), i_speed_x = scalar_reg(I->speed_x),
               i_speed_y = scalar_reg(I->speed_y), i_gamma = scalar_reg(I->gamma), i_inv_dx = scalar_reg(I->inv_dx),
               i_inv_dy = scalar_reg(I->inv_dy);
  unsigned long long ax_bits, ay_bits;
  if (sp) {
    if constexpr (kTag) {
      const long long n_in = (stage <= 1 ? c0.n : (stage == 2 ? c1.n : c2.n)) - seq_base;
      ax_bits = spread_reduce_tagged(spx, 3 * n_in + slot_in);
      ay_bits = spread_reduce_tagged(spy, 3 * n_in + slot_in);
    } else {
      ax_bits = spread_reduce(spx);
      ay_bits = spread_reduce(spy);
    }
  } else {
    ax_bits = I->alpha[slot_in][0];
    ay_bits = I->alpha[slot_in][1];
  }
  auto zero_slot = [&](int slot) {
    if (sp) {
      if (!kTag && first_block && tid < kSpread) {
        sp[((slot * 2 + 0) * kSpread + tid) * kSpreadStride] = 0ull;
        sp[((slot * 2 + 1) * kSpread + tid) * kSpreadStride] = 0ull;
      }
    } else if (lead) {
      I->alpha[slot][0] = 0ull;
      I->alpha[slot][1] = 0ull;
    }
  };
  if (err) return;
  double t, dt = 0.0;
  long long n;
  if (stage == 1) {
    t = c0.t;
    n = c0.n;
    const bool active = (T - t) > tol;
    if (active) dt = step_dt<2>(dt_fixed, cfl, dxd, dyd, T, t, bits_to_double(ax_bits), bits_to_double(ay_bits));
    if (lead) {
      Ctl c;
      c.t = t;
      c.dt = dt;
      c.n = n;
      c.active = active ? 1 : 0;
      c.home = par;
      I->ctl[1] = c;
    }
    if (!active) return;
    zero_slot(2);
  } else if (stage == 2) {
    if (lead) I->ctl[2] = c1;
    if (!c1.active) return;
    zero_slot(0);
    t = c1.t;
    dt = c1.dt;
    n = c1.n;
  } else if (stage == 3) {
    if (!c2.active) return;
    if (lead) {
      Ctl d;
      d.t = c2.t + c2.dt;
      d.dt = 0.0;
      d.n = c2.n + 1;
      d.active = 0;
      d.home = par ^ 1;
      I->ctl[0] = d;
    }
    zero_slot(1);
    t = c2.t;
    dt = c2.dt;
    n = c2.n;
  } else {
    t = c0.t;
    n = c0.n;
  }
  // Workgroup-uniform parameters are moved to scalar registers: converted on the vector unit
  // they would otherwise sit in a dozen vector registers for the whole chunk loop.
  const R alpha_x = scalar_reg(R(bits_to_double(ax_bits))), alpha_y = scalar_reg(R(bits_to_double(ay_bits)));
  const R rdt = scalar_reg(R(dt));
  const ReconMode rm = recon_mode(i_recon, i_sw);
  constexpr bool kFixed = SCHEME == kSchemeRbfWeno5Switch;
  const bool eno = kFixed ? false : rm.eno, use_eta = kFixed ? true : rm.use_eta,
             use_switch = kFixed ? true : rm.use_switch;
  const double eps_m = scalar_reg(i_eps_m);
  const R eps = scalar_reg(R(i_eps));
  const R speed_x = scalar_reg(R(i_speed_x)), speed_y = scalar_reg(R(i_speed_y)), gamma = scalar_reg(R(i_gamma));
  const R dx = scalar_reg(R(dxd)), dy = scalar_reg(R(dyd));
  const R inv_dx = scalar_reg(R(i_inv_dx)), inv_dy = scalar_reg(R(i_inv_dy));

  // The same for a row that is first read in the next chunk.  Float rows inside the grid go
  // straight from memory to LDS (no registers; the loads complete under the chunk's work and are
  // waited for before the chunk's last barrier); other rows take the path above.
  auto stage_row_ahead = [&](int row) {
    if constexpr (sizeof(R) == 4) {
      if (cols_in && row >= 0 && row < ny) {
        const __amdgpu_buffer_rsrc_t rs = buffer_of(src, state_bytes);
        const int sl = slot_of(row);
        const unsigned at = ((unsigned)row * (unsigned)nx + (unsigned)(i0 - 3 + lane)) * sizeof(R);
#pragma unroll
        for (int c = 0; c < M; ++c)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)&s_u[c][sl][0], 4,
                                                   at, c * comp_bytes, 0, 0);
        if (lane < WX - 64) {
#pragma unroll
          for (int c = 0; c < M; ++c)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)&s_u[c][sl][64], 4,
                                                     at + 64u * (unsigned)sizeof(R), c * comp_bytes, 0, 0);
        }
        return;
      }
    }
    stage_row(row);
  };
  // rows of this strip inside the grid, in whole chunks
  const int rows = H < ny - j0 ? H : ny - j0;
  const int nchunk = (rows + CH - 1) / CH;

  for (int r = wave; r < RING; r += BS / 64) stage_row(j0 - 3 + r);  // rows j0-3 .. j0+8
  __syncthreads();

  // column march state (wave c = component c, lane x = column x; lanes past the strip repeat its
  // last column and write nothing)
  const int mc = wave;
  auto V = [&](int j) -> R {  // cell j of the column
    const int mx = lane < TX ? lane : TX - 1;
    return s_u[mc][slot_of(j)][mx + 3];
  };
  R z = R(0), ua = V(j0 - 3), ub = V(j0 - 2), uc = V(j0 - 1), ud = V(j0), ue = V(j0 + 1);
  // the window and its doubles (exact widenings) are re-formed at every chunk from the ring, so
  // that only the previous cell's flag and weight denominators are held across the x sweep
  double da, db, dc, dd;
  auto widen = [&]() {
    da = double(ua);
    db = double(ub);
    dc = double(uc);
    dd = double(ud);
  };
  widen();
  int fl_prev = 0, r_prev = 0;
  R d0p = R(0), d1p = R(0), d2p = R(0);
  // one step of the march at cell j: its flag and weight denominators, and (from cell j0 on) the
  // interface j - 1/2, whose v^- and v^+ go to flux slot `fs`; then slide the window up one cell
  auto march = [&](int j, int fs) {
    const int fl = use_switch ? monotone_flag<kExact>(db, dc, dd) : 0;
    int r = 0;
    R e0 = R(0), e1 = R(0), e2 = R(0);
    if (eno)
      r = eno_stencil(da, db, dc, dd, double(ue));
    else
      weight_denominators<R>(ua, ub, uc, ud, ue, eps, e0, e1, e2);
    if (j >= j0) {
      R eta = R(0);
      if (use_eta) {
        eta = R(eta_ratio<kExact>(da, db, dc, dd, eps_m));
        if (use_switch && ((fl_prev | fl) & 1)) eta = R(0);
      }
      R vm, vp;
      if (eno) {
        vm = eno_minus<R>(r_prev, z, ua, ub, uc, ud, eta);
        vp = eno_plus<R>(r, ua, ub, uc, ud, ue, eta);
      } else {
        vm = weno_minus<R>(z, ua, ub, uc, ud, eta, d0p, d1p, d2p);
        vp = weno_plus<R>(ua, ub, uc, ud, ue, eta, e0, e1, e2);
      }
      if (lane < TX) {
        s_vm[mc][fs][lane] = vm;
        s_vp[mc][fs][lane] = vp;
      }
    }
    fl_prev = fl;
    r_prev = r;
    d0p = e0;
    d1p = e1;
    d2p = e2;
    z = ua;
    ua = ub;
    ub = uc;
    uc = ud;
    ud = ue;
    ue = V(j + 3);
    da = db;
    db = dc;
    dc = dd;
    dd = double(ud);
  };
  march(j0 - 1, 0);  // cell j0 - 1: flag and denominators only

  R amx = R(0), amy = R(0);
  int bad = 0;
  for (int k = 0; k < nchunk; ++k) {
    // The lane index is made opaque to the compiler at every chunk, so that the many per-lane
    // addresses derived from it are recomputed (a few integer operations) instead of being held
    // in vector registers across the whole loop.
    asm volatile("" : "+v"(lane));
    const int jk = j0 + k * CH;
    const int row = jk + wave;  // this wave's row in the x sweep and the update
    const int ux = lane - 1;    // the update's (and x sweep's) column
    const bool owned = lane >= 1 && lane <= TX && i0 + ux < nx && row < j0 + rows;
    auto fslot = [&](int s) -> int { return (CH * k + s) % (CH + 1); };
    // the next chunk's rows jk+9 .. jk+12 (one per wave), into the slots of rows jk-4 .. jk-1
    if (k + 1 < nchunk) stage_row_ahead(jk + 9 + wave);
    // ---- y sweep first: the column march through the chunk's interfaces ----------------------
    // (before the x sweep, so that the x sweep's -dF/dx is not held across the march)
    if (k == 0) march(j0, fslot(0));  // interface j0 - 1/2
#pragma unroll
    for (int s = 1; s <= CH; ++s) march(jk + s, fslot(s));
    // ---- x sweep: row `row`, lane l takes cell p = l - 1 and its interface p + 1/2 -----------
    R Lx[M];
    {
      const int sl = slot_of(row), q = lane + 2;  // staged column of cell p
      R A[M], B[M], Hf[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const R u0 = s_u[c][sl][q - 2], u1 = s_u[c][sl][q - 1], u2 = s_u[c][sl][q], u3 = s_u[c][sl][q + 1],
                u4 = s_u[c][sl][q + 2], u5 = s_u[c][sl][lane < 63 ? q + 3 : q + 2];
        const double d1 = double(u1), d2 = double(u2), d3 = double(u3), d4 = double(u4);
        const int fl = use_switch ? monotone_flag<kExact>(d1, d2, d3) : 0;
        const int fl_next = __shfl_down(fl, 1);
        R eta = R(0);
        if (use_eta) {
          eta = R(eta_ratio<kExact>(d1, d2, d3, d4, eps_m));
          if (use_switch && ((fl | fl_next) & 1)) eta = R(0);
        }
        if (eno) {
          const int r = eno_stencil(double(u0), d1, d2, d3, d4);
          const int r_next = __shfl_down(r, 1);
          A[c] = eno_minus<R>(r, u0, u1, u2, u3, u4, eta);
          B[c] = eno_plus<R>(r_next, u1, u2, u3, u4, u5, eta);
        } else {
          R s0, s1, s2;
          weight_denominators<R>(u0, u1, u2, u3, u4, eps, s0, s1, s2);
          const R n0 = __shfl_down(s0, 1), n1 = __shfl_down(s1, 1), n2 = __shfl_down(s2, 1);
          A[c] = weno_minus<R>(u0, u1, u2, u3, u4, eta, s0, s1, s2);
          B[c] = weno_plus<R>(u1, u2, u3, u4, u5, eta, n0, n1, n2);
        }
      }
      lf_flux<R, FLUX, M, 0>(A, B, alpha_x, speed_x, gamma, Hf);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const R Fp = Hf[c], Fm = __shfl_up(Hf[c], 1);  // fluxes at p + 1/2 and p - 1/2
        if constexpr (kExact)
          Lx[c] = -div_rn(Fp - Fm, dx);
        else
          Lx[c] = (Fm - Fp) * inv_dx;
      }
    }
    // u^n of the owned cell (stages 2 and 3), loaded under the flux pass
    const long long at = (long long)row * nx + (i0 + ux);
    R upt[M];
    if ((stage == 2 || stage == 3) && owned) {
      if (cols_in) {
        const __amdgpu_buffer_rsrc_t rs = buffer_of(un, state_bytes);
#pragma unroll
        for (int c = 0; c < M; ++c) upt[c] = buffer_load<R>(rs, (unsigned)at * sizeof(R), c * comp_bytes);
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) upt[c] = un[c * ncell + at];
      }
    }
    __syncthreads();
    // flux pass: wave w takes interface slot w + 1 (and wave 0 slot 0 in the first chunk), lane x
    // column x; G overwrites v^- in place
    auto flux_y = [&](int s) {
      if (lane < TX) {
        R A[M], B[M], G[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
          A[c] = s_vm[c][s][lane];
          B[c] = s_vp[c][s][lane];
        }
        lf_flux<R, FLUX, M, 1>(A, B, alpha_y, speed_y, gamma, G);
#pragma unroll
        for (int c = 0; c < M; ++c) s_vm[c][s][lane] = G[c];
      }
    };
    flux_y(fslot(wave + 1));
    if (k == 0 && wave == 0) flux_y(fslot(0));
    __syncthreads();
    // ---- update of the chunk's cells: row jk + wave, column lane - 1 --------------------------
    if (owned) {
      R unew[M];
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const R Gp = s_vm[c][fslot(wave + 1)][ux], Gm = s_vm[c][fslot(wave)][ux];
        R L;
        if constexpr (kExact)
          L = Lx[c] - div_rn(Gp - Gm, dy);
        else
          L = Lx[c] + (Gm - Gp) * inv_dy;
        if (stage == 0)
          unew[c] = L;
        else
          unew[c] = rk3_combine<R>(stage, upt[c], s_u[c][slot_of(row)][lane + 2], rdt * L);
      }
      if (cols_in) {
        const __amdgpu_buffer_rsrc_t rs = buffer_of(dst, state_bytes);
#pragma unroll
        for (int c = 0; c < M; ++c) buffer_store<R>(unew[c], rs, (unsigned)at * sizeof(R), c * comp_bytes);
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) dst[c * ncell + at] = unew[c];
      }
      if (stage != 0) {
        int b0 = 0;
        R sx, sy;
        spectral_radii_2d<R, FLUX, M>(unew, speed_x, speed_y, gamma, sx, sy, b0);
        amx = sx > amx ? sx : amx;
        amy = sy > amy ? sy : amy;
        bad = b0 > bad ? b0 : bad;
      }
    }
    if (k + 1 == nchunk) break;
    // the next chunk's window (rows jk+2 .. jk+7), re-read here rather than held across the x
    // sweep, and before the barrier: the loads issued above overwrite rows jk .. jk+3's
    // predecessors, which nothing reads after it
    z = V(jk + 2);
    ua = V(jk + 3);
    ub = V(jk + 4);
    uc = V(jk + 5);
    ud = V(jk + 6);
    ue = V(jk + 7);
    widen();
    __builtin_amdgcn_s_waitcnt(0);  // the next chunk's rows are in LDS
    __syncthreads();                // and this chunk's ring rows and flux slots are read
  }
  if (stage == 0) return;
  // ---- epilogue: alpha of the new state over the strip, and validity ------------------------
  amx = wave_max_nonneg(amx);
  amy = wave_max_nonneg(amy);
  const bool bad2 = __any(bad == 2), bad1 = __any(bad == 1);
  if (lane == 0) {
    s_red[0][wave] = double_to_bits(double(amx));
    s_red[1][wave] = double_to_bits(double(amy));
    s_bad[wave] = bad2 ? 2 : (bad1 ? 1 : 0);
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long mx = 0ull, my = 0ull;
    int w = 0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) {
      mx = s_red[0][k] > mx ? s_red[0][k] : mx;
      my = s_red[1][k] > my ? s_red[1][k] : my;
      w = s_bad[k] > w ? s_bad[k] : w;
    }
    const int slot = stage == 1 ? 1 : (stage == 2 ? 2 : 0);
    if (w) {
      const int code = w == 2 ? NPW_ENONPHYSICAL : NPW_ENONFINITE;
      if (atomicCAS(&I->err, 0, code) == 0) {
        I->err_stage = stage;
        I->err_n = n;
        I->err_t = t;
        I->err_home = par;
      }
    } else {
      const int k = (blockIdx.y * gridDim.x + blockIdx.x) % kSpread;
      if (sp && kTag) {
        atomicMax(&sp[((slot * 2 + 0) * kSpread + k) * kSpreadStride],
                  spread_tag(3 * (n - seq_base) + stage, float(bits_to_double(mx))));
        atomicMax(&sp[((slot * 2 + 1) * kSpread + k) * kSpreadStride],
                  spread_tag(3 * (n - seq_base) + stage, float(bits_to_double(my))));
      } else {
        atomicMax(sp ? &sp[((slot * 2 + 0) * kSpread + k) * kSpreadStride] : &I->alpha[slot][0], mx);
        atomicMax(sp ? &sp[((slot * 2 + 1) * kSpread + k) * kSpreadStride] : &I->alpha[slot][1], my);
      }
    }
  }
}

}  // namespace npw

// npw_kernels2d.h -- fused SSP-RK3 stage kernel for 2D grids, dimension by dimension.
//
// Section 7 (eq. 2DIntegral) with one midpoint quadrature point per face: every row is
// reconstructed along x with the 1D scheme and every column along y, and
//   L_ij = -(F_{i+1/2,j} - F_{i-1/2,j}) / dx - (G_{i,j+1/2} - G_{i,j-1/2}) / dy,
// with one global Lax-Friedrichs alpha per direction.  One workgroup owns a TX x TY tile; it
// stages the tile with a three-cell halo in LDS, runs the x sweep (flags, eta, reconstruction,
// flux) over the TY rows, accumulates -dF/dx, runs the same sweep over the TX columns along y,
// and applies the stage update.  The epilogue reduces alpha_x and alpha_y of the new state.
// A sweep runs as a cell phase and an interface phase (one thread per interface), or, on
// 62-wide tiles with k = 3 component-wise reconstruction, fused: along x one wave per row with
// lane shuffles, along y (as many components as waves) one wave per component with each lane
// walking a column, so every cell's quantities are formed once.
#pragma once
#include <type_traits>

#include "../../include/npweno.h"
#include "npw_device.h"

namespace npw {

// SHARE: the per-cell weight denominators and k = 2 shape parameters go through LDS and serve both
// interfaces of a cell; otherwise every interface recomputes them (less LDS, more workgroups per
// compute unit).  The switch flags and ENO stencils are shared either way.
// Occupancy: the float Euler kernel with both fused sweeps (62-wide tiles, k = 3, component-wise) is
// held to 6 waves per SIMD, the most its LDS allows (80 VGPRs at most).  It fits in 78 without
// spilling; the hint keeps a later change from sliding to 5 waves unnoticed (an earlier form needed
// 82, which allocate as 88: 134.6 us per stage at 5 waves against 132.1 us at 6 with a 12-byte
// spill, on 2048^2 Euler).  Every other instantiation keeps the compiler's choice.
template <typename R, int FLUX, int M, int TX, int TY, bool CHAR = false, bool K2 = true, bool SHARE = true>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    (sizeof(R) == 4 && M == 4 && TX + 2 == 64 && !CHAR && !K2 && !SHARE) ? 6 : 1))) void stage2d_kernel(StageArgs a) {
  constexpr int BS = 256;
  constexpr bool kExact = std::is_same<R, double>::value;
  constexpr int WX = TX + 6, WY = TY + 6;                          // staged cells per row / column
  constexpr int NC = (TX + 2) * TY > TX * (TY + 2) ? (TX + 2) * TY : TX * (TY + 2);  // sweep cells
  __shared__ R s_u[M][WY][WX];
  // interface fluxes are stored at the left cell's index, which stays below NF in both sweeps
  constexpr int NF = (TX + 2) * TY > (TY + 1) * TX ? (TX + 2) * TY : (TY + 1) * TX;
  // one wave per row in the x sweep: cells -1..TX of a row fill a wave exactly (scalar flags and
  // per-interface denominators only)
  constexpr bool kRowWave = TX + 2 == 64 && !CHAR && !K2 && !SHARE;
  // one wave per component in the y sweep (as many components as waves): each lane marches up
  // one column of the tile
  constexpr bool kColMarch = kRowWave && M == BS / 64;
  // per-cell flags (bit 0 switch, bits 1-2 ENO stencil) of two components share a byte
  __shared__ unsigned char s_flag[(M + 1) / 2][NC];
  __shared__ R s_den[SHARE ? M : 1][3][SHARE ? NC : 1];
  __shared__ R s_F[M][NF];
  static_assert(TX % 1 == 0 && TY % 1 == 0 && NC >= (TX + 2) * TY, "sweep buffers");
  __shared__ unsigned long long s_red[2][BS / 64];
  __shared__ int s_bad[BS / 64];

  const int tid = threadIdx.x;
  const int stage = a.stage;
  const int nx = (int)a.nx, ny = (int)a.ny;
  // this workgroup's tile: XCD-contiguous runs of the row-major tile order
  const long long tile = xcd_contiguous_tile((long long)blockIdx.y * gridDim.x + blockIdx.x,
                                             (long long)gridDim.x * gridDim.y);
  const unsigned grid_x = gridDim.x;
  int tbx, tby;
  if (tile < (1LL << 32)) {  // 32-bit division whenever the grid allows it
    tby = (int)((unsigned)tile / grid_x);
    tbx = (int)((unsigned)tile - (unsigned)tby * grid_x);
  } else {
    tby = (int)(tile / grid_x);
    tbx = (int)(tile - (long long)tby * grid_x);
  }
  const int i0 = tbx * TX, j0 = tby * TY;
  const int bc = a.bc;
  const int par = a.par;
  const long long ncell = (long long)nx * ny;

  R* un = reinterpret_cast<R*>(par ? a.P1 : a.P0);
  R* uo = reinterpret_cast<R*>(par ? a.P0 : a.P1);
  R* u2 = reinterpret_cast<R*>(a.C);
  const R* src = (stage == 0 || stage == 1) ? un : (stage == 2 ? uo : u2);
  R* dst = stage == 0 ? reinterpret_cast<R*>(a.out) : (stage == 2 ? u2 : uo);

  // ---- issue the state loads (tile + halo, every component) -------------------------------
  // Tiles whose halo lies inside the grid (all but the edge tiles) of states below 4 GiB need no
  // ghost mapping and address through buffer resources: one 32-bit lane offset per cell, the
  // component in the scalar offset.  The test is uniform over the workgroup.
  const unsigned state_bytes = (unsigned)((unsigned long long)M * ncell * sizeof(R));
  const bool direct = i0 >= 3 && i0 + TX + 3 <= nx && j0 >= 3 && j0 + TY + 3 <= ny &&
                      (unsigned long long)M * ncell * sizeof(R) < (1ULL << 32);
  const unsigned comp_bytes = (unsigned)(ncell * sizeof(R));  // used only when direct
  constexpr int NLD = (WX * WY + BS - 1) / BS;
  R ld[NLD][M];
  if (direct) {
    const __amdgpu_buffer_rsrc_t rs = buffer_of(src, state_bytes);
    const unsigned corner = (unsigned)(j0 - 3) * (unsigned)nx + (unsigned)(i0 - 3);
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int idx = tid + k * BS;
      if (idx < WX * WY) {
        const unsigned at = (corner + (unsigned)(idx / WX) * (unsigned)nx + (unsigned)(idx % WX)) * sizeof(R);
#pragma unroll
        for (int c = 0; c < M; ++c) ld[k][c] = buffer_load<R>(rs, at, c * comp_bytes);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
      const int idx = tid + k * BS;
      if (idx < WX * WY) {
        const int gy = ghost_index(j0 - 3 + idx / WX, ny, bc), gx = ghost_index(i0 - 3 + idx % WX, nx, bc);
#pragma unroll
        for (int c = 0; c < M; ++c) ld[k][c] = src[c * ncell + (long long)gy * nx + gx];
      }
    }
  }
  constexpr int NOWN = (TX * TY + BS - 1) / BS;
  R upt[NOWN][M];
  if (stage == 2 || stage == 3) {
#pragma unroll
    for (int k = 0; k < NOWN; ++k) {
      const int o = tid + k * BS;
      const int x = i0 + o % TX, y = j0 + o / TX;
      if (o < TX * TY && x < nx && y < ny) {
        if (direct) {
          const __amdgpu_buffer_rsrc_t rs = buffer_of(un, state_bytes);
          const unsigned at = ((unsigned)y * (unsigned)nx + (unsigned)x) * sizeof(R);
#pragma unroll
          for (int c = 0; c < M; ++c) upt[k][c] = buffer_load<R>(rs, at, c * comp_bytes);
        } else {
#pragma unroll
          for (int c = 0; c < M; ++c) upt[k][c] = un[c * ncell + (long long)y * nx + x];
        }
      }
    }
  }

  // ---- step control (same protocol as the 1D kernel; the lead is tile (0, 0)) --------------
  InstDev* I = a.inst;
  unsigned long long* sp = a.spread;
  const bool first_block = (tbx == 0 && tby == 0);
  const bool lead = first_block && tid == 0;
  constexpr bool kTag = !kExact;  // float bulk: spread entries carry their stage sequence
  const int slot_in = stage == 0 ? 0 : stage - 1;
  const unsigned long long spx = sp ? spread_entry(sp, slot_in, 0) : 0ull;
  const unsigned long long spy = sp ? spread_entry(sp, slot_in, 1) : 0ull;
  const int err = I->err;
  const Ctl c0 = I->ctl[0], c1 = I->ctl[1], c2 = I->ctl[2];
  unsigned long long ax_bits, ay_bits;
  if (sp) {
    if constexpr (kTag) {
      const long long n_in = (stage <= 1 ? c0.n : (stage == 2 ? c1.n : c2.n)) - I->seq_base;
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
  const double T = I->T, tol = I->tol;
  const double dt_fixed = I->dt_fixed, cfl = I->cfl, dxd = I->dx, dyd = I->dy;
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
  const R alpha_x = R(bits_to_double(ax_bits)), alpha_y = R(bits_to_double(ay_bits));
  const R rdt = R(dt);
  ReconMode rm = recon_mode(I->recon, I->sw);
  if (!K2) rm.k2 = rm.cross = false;  // launched for a k = 3 instance (Section 6 is k = 2)
  const bool k2 = rm.k2, eno = rm.eno, use_eta = rm.use_eta, use_switch = rm.use_switch, cross = rm.cross;
  const double eps_m = I->eps_m;
  const R eps = R(I->eps_weno);
  const R speed_x = R(I->speed_x), speed_y = R(I->speed_y), gamma = R(I->gamma);
  const R dx = R(dxd), dy = R(dyd), inv_dx = R(I->inv_dx), inv_dy = R(I->inv_dy);

#pragma unroll
  for (int k = 0; k < NLD; ++k) {
    const int idx = tid + k * BS;
    if (idx < WX * WY) {
#pragma unroll
      for (int c = 0; c < M; ++c) s_u[c][idx / WX][idx % WX] = ld[k][c];
    }
  }
  __syncthreads();

  R Lr[NOWN][M];  // L(u) of this thread's owned cells (x sweep, then + y sweep)
  R usr[kColMarch ? NOWN : 1][M] = {};  // the owned cells' stage input, kept when s_u is reused
  bool ycol = false;
#pragma unroll
  for (int k = 0; k < NOWN; ++k)
#pragma unroll
    for (int c = 0; c < M; ++c) Lr[k][c] = R(0);
  auto FL = [&](int c, int w) -> int { return (s_flag[c / 2][w] >> (4 * (c % 2))) & 15; };
  // One sweep direction.  Cells along the sweep are addressed by (line, pos): pos runs over
  // -1..LEN (LEN = TX for x, TY for y), line over the other tile extent; q = pos + 3 is the
  // staged coordinate along the sweep.  Work items are numbered so that consecutive threads
  // touch consecutive x (conflict-free LDS banks in both sweeps): cell index
  // cid(line, pos) = line * NPOS + pos + 1 along x, (pos + 1) * LINES + line along y.
  auto sweep = [&](auto dir_tag) {
    constexpr int DIR = decltype(dir_tag)::value;
    constexpr int LEN = DIR == 0 ? TX : TY;
    constexpr int LINES = DIR == 0 ? TY : TX;
    constexpr int NPOS = LEN + 2;  // cells -1 .. LEN
    auto U = [&](int c, int line, int q) -> R { return DIR == 0 ? s_u[c][line + 3][q] : s_u[c][q][line + 3]; };
    auto cid = [&](int line, int pos) -> int { return DIR == 0 ? line * NPOS + pos + 1 : (pos + 1) * LINES + line; };
    // x sweep with one wave per row, for tiles whose staged row holds cells -1..TX in exactly one
    // wave: lane l takes cell p = l - 1, forms its flag and weight denominators once, and then the
    // interface p+1/2 whole (eta, v^- of cell p, v^+ of cell p+1); the next cell's flag and weight
    // denominators arrive by lane shuffles.  Same functions on the same operands as the two phases
    // below: the double bulk's fluxes are identical bit for bit (the float bulk's up to how
    // multiply-adds are fused); the separate flag pass and its barrier go away, and so does the
    // second denominator set of every interface.
    bool rows = false;
    if constexpr (DIR == 0 && kRowWave) {
      rows = !cross;
      if (rows) {
        const int lane = tid & 63, q = lane + 2;  // q = p + 3
        for (int line = tid >> 6; line < LINES; line += BS / 64) {
          R A[M], B[M], H[M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            // u5 = cell p + 3 (the last lane's interface is not used; its read stays in the row)
            const R u0 = U(c, line, q - 2), u1 = U(c, line, q - 1), u2 = U(c, line, q), u3 = U(c, line, q + 1),
                    u4 = U(c, line, q + 2), u5 = U(c, line, lane < 63 ? q + 3 : q + 2);
            const double d1 = double(u1), d2 = double(u2), d3 = double(u3), d4 = double(u4);
            const int fl = use_switch ? monotone_flag<kExact>(d1, d2, d3) : 0;
            const int fl_next = __shfl_down(fl, 1);
            // the double shape parameter, rounded to the bulk type, then zeroed by the switch
            R eta_r = R(0);
            if (use_eta) {
              eta_r = R(eta_ratio<kExact>(d1, d2, d3, d4, eps_m));
              if (use_switch && ((fl | fl_next) & 1)) eta_r = R(0);
            }
            // both edge values of interface p+1/2: v^- of cell p and v^+ of cell p+1 (window
            // u1..u5, its stencil or weight denominators from the next lane); they share eta and
            // two of their three substencil values
            R vm, vp;
            if (eno) {
              const int r = eno_stencil(double(u0), d1, d2, d3, d4);
              const int r_next = __shfl_down(r, 1);
              vm = eno_minus<R>(r, u0, u1, u2, u3, u4, eta_r);
              vp = eno_plus<R>(r_next, u1, u2, u3, u4, u5, eta_r);
            } else {
              R s0, s1, s2;
              weight_denominators<R>(u0, u1, u2, u3, u4, eps, s0, s1, s2);
              const R n0 = __shfl_down(s0, 1), n1 = __shfl_down(s1, 1), n2 = __shfl_down(s2, 1);
              vm = weno_minus<R>(u0, u1, u2, u3, u4, eta_r, s0, s1, s2);
              vp = weno_plus<R>(u1, u2, u3, u4, u5, eta_r, n0, n1, n2);
            }
            A[c] = vm;
            B[c] = vp;
          }
          lf_flux<R, FLUX, M, 0>(A, B, alpha_x, speed_x, gamma, H);
          if (lane < 63) {
#pragma unroll
            for (int c = 0; c < M; ++c) s_F[c][cid(line, lane - 1)] = H[c];
          }
        }
      }
    }
    // y sweep with one wave per component: wave c takes component c and lane x column x; the
    // lane walks the column's cells j = -1..LEN, forming the flag and weight denominators of each
    // cell and the eta and both edge values of each interface j - 1/2 once, with the window and the
    // previous cell's values carried in registers.  v^- goes to s_F, v^+ to the staged tile's
    // storage once every wave has finished reading it, and a flux pass combines the components.
    // Same functions on the same operands as the two phases below (bit for bit in the double
    // bulk, up to how multiply-adds are fused in the float bulk).
    if constexpr (DIR == 1 && kColMarch) {
      ycol = !cross;
      if (ycol) {
        static_assert(M * NF <= M * WY * WX, "v+ fits in the staged tile");
        const int c = tid >> 6, lx = tid & 63, x = lx < TX ? lx : TX - 1;
        auto V = [&](int j) -> R { return s_u[c][j + 3][x + 3]; };  // cell j of column x, j = -3..LEN+2
        R vp[LEN + 1];
        int fl_prev = 0, r_prev = 0;
        R d0p = R(0), d1p = R(0), d2p = R(0);
        // the window of cell j (cells j-2 .. j+2, the left neighbour's farthest cell j-3) and the
        // doubles of cells j-2 .. j+1, carried from step to step: one new cell per step
        R z = R(0), ua = V(-3), ub = V(-2), uc = V(-1), ud = V(0), ue = V(1);
        double da = double(ua), db = double(ub), dc = double(uc), dd = double(ud);
#pragma unroll
        for (int j = -1; j <= LEN; ++j) {
          const int fl = use_switch ? monotone_flag<kExact>(db, dc, dd) : 0;
          int r = 0;
          R d0 = R(0), d1 = R(0), d2 = R(0);
          if (eno)
            r = eno_stencil(da, db, dc, dd, double(ue));
          else
            weight_denominators<R>(ua, ub, uc, ud, ue, eps, d0, d1, d2);
          if (j >= 0) {  // interface j - 1/2 between cells j - 1 and j; z is cell j - 3
            R eta = R(0);
            if (use_eta) {
              eta = R(eta_ratio<kExact>(da, db, dc, dd, eps_m));
              if (use_switch && ((fl_prev | fl) & 1)) eta = R(0);
            }
            R vm;
            if (eno) {
              vm = eno_minus<R>(r_prev, z, ua, ub, uc, ud, eta);
              vp[j] = eno_plus<R>(r, ua, ub, uc, ud, ue, eta);
            } else {
              vm = weno_minus<R>(z, ua, ub, uc, ud, eta, d0p, d1p, d2p);
              vp[j] = weno_plus<R>(ua, ub, uc, ud, ue, eta, d0, d1, d2);
            }
            if (lx < TX) s_F[c][cid(lx, j - 1)] = vm;
          }
          fl_prev = fl;
          r_prev = r;
          d0p = d0;
          d1p = d1;
          d2p = d2;
          if (j < LEN) {  // slide the window up one cell (the staged column ends at cell LEN + 2)
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
          }
        }
#pragma unroll
        for (int k = 0; k < NOWN; ++k) {
          const int o = tid + k * BS;
          if (o < TX * TY) {
#pragma unroll
            for (int cc = 0; cc < M; ++cc) usr[k][cc] = s_u[cc][o / TX + 3][o % TX + 3];
          }
        }
        __syncthreads();  // every wave is done with s_u
        R* vpb = &s_u[0][0][0];
        if (lx < TX) {
#pragma unroll
          for (int j = 0; j <= LEN; ++j) vpb[c * NF + cid(lx, j - 1)] = vp[j];
        }
        __syncthreads();
        for (int wi = tid; wi < (LEN + 1) * LINES; wi += BS) {
          R A[M], B[M], H[M];
#pragma unroll
          for (int cc = 0; cc < M; ++cc) {
            A[cc] = s_F[cc][wi];
            B[cc] = vpb[cc * NF + wi];
          }
          lf_flux<R, FLUX, M, 1>(A, B, alpha_y, speed_y, gamma, H);
#pragma unroll
          for (int cc = 0; cc < M; ++cc) s_F[cc][wi] = H[cc];
        }
      }
    }
    const bool fused = rows || ycol;
    // cell phase: flag and weight denominators of cells -1..LEN of every line (none in the
    // characteristic mode: its fields belong to an interface)
    for (int w = tid; w < (CHAR || cross || fused ? 0 : NPOS * LINES); w += BS) {
      const int line = DIR == 0 ? w / NPOS : w % LINES;
      const int pos = DIR == 0 ? w % NPOS - 1 : w / LINES - 1;
      const int q = pos + 3;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        // bit 0: switch flag; bits 1-2: ENO stencil
        int fl = use_switch ? monotone_flag<kExact>(double(U(c, line, q - 1)), double(U(c, line, q)),
                                            double(U(c, line, q + 1)))
                            : 0;
        if (k2) {  // k = 2: ENO2 stencil and the right/left edge shape parameters of the cell
          const double um = double(U(c, line, q - 1)), u0 = double(U(c, line, q)), up = double(U(c, line, q + 1));
          if (eno) fl |= eno2_stencil(um, u0, up) << 1;
          if constexpr (SHARE) {
            double er = 0.0, el = 0.0;
            if (use_eta && !(fl & 1)) {
              er = eta2_ratio<kExact>(um, u0, up, eps_m);
              el = eta2_ratio<kExact>(up, u0, um, eps_m);
            }
            s_den[c][0][w] = R(er);
            s_den[c][1][w] = R(el);
          }
        } else if (eno) {
          fl |= eno_stencil(double(U(c, line, q - 2)), double(U(c, line, q - 1)), double(U(c, line, q)),
                            double(U(c, line, q + 1)), double(U(c, line, q + 2)))
                << 1;
        } else if constexpr (SHARE) {
          R d0, d1, d2;
          weight_denominators<R>(U(c, line, q - 2), U(c, line, q - 1), U(c, line, q), U(c, line, q + 1),
                                 U(c, line, q + 2), eps, d0, d1, d2);
          s_den[c][0][w] = d0;
          s_den[c][1][w] = d1;
          s_den[c][2][w] = d2;
        }
        if (c % 2 == 0)
          s_flag[c / 2][w] = (unsigned char)fl;
        else
          s_flag[c / 2][w] = (unsigned char)(s_flag[c / 2][w] | (fl << 4));
      }
    }
    if (!fused) __syncthreads();  // rows and ycol are uniform over the workgroup
    // interface phase: pos+1/2 for pos = -1..LEN-1; the flux is stored at the left cell's index
    for (int wi = tid; wi < (fused ? 0 : (LEN + 1) * LINES); wi += BS) {
      const int line = DIR == 0 ? wi / (LEN + 1) : wi % LINES;
      const int pos = DIR == 0 ? wi % (LEN + 1) - 1 : wi / LINES - 1;
      const int q = pos + 3;
      const int wl = cid(line, pos), wr = cid(line, pos + 1);
      R A[M], B[M], H[M];
      if constexpr (CHAR) {  // cells pos-2..pos+3 along the sweep
        R Uw[6][M];
#pragma unroll
        for (int k = 0; k < 6; ++k)
#pragma unroll
          for (int c = 0; c < M; ++c) Uw[k][c] = U(c, line, q - 2 + k);
        char_states<R, M, DIR>(Uw, gamma, rm, eps, eps_m, A, B);
      }
#pragma unroll
      for (int c = 0; c < (CHAR ? 0 : M); ++c) {
        if (k2 && cross) {  // Section 6: transverse neighbours are the adjacent lines
          A[c] = cross_edge<R, true>(U(c, line, q - 1), U(c, line, q), U(c, line, q + 1), U(c, line - 1, q),
                                     U(c, line + 1, q), use_switch, eps_m);
          B[c] = cross_edge<R, false>(U(c, line, q), U(c, line, q + 1), U(c, line, q + 2), U(c, line - 1, q + 1),
                                      U(c, line + 1, q + 1), use_switch, eps_m);
          continue;
        }
        if (k2) {
          R el, er;
          if constexpr (SHARE) {
            el = s_den[c][0][wl];
            er = s_den[c][1][wr];
          } else {  // right-edge parameter of the left cell, left-edge parameter of the right cell
            double dl = 0.0, dr = 0.0;
            if (use_eta && !(FL(c, wl) & 1))
              dl = eta2_ratio<kExact>(double(U(c, line, q - 1)), double(U(c, line, q)), double(U(c, line, q + 1)),
                                      eps_m);
            if (use_eta && !(FL(c, wr) & 1))
              dr = eta2_ratio<kExact>(double(U(c, line, q + 2)), double(U(c, line, q + 1)), double(U(c, line, q)),
                                      eps_m);
            el = R(dl);
            er = R(dr);
          }
          if (eno) {
            A[c] = eno2<R, false>((FL(c, wl) >> 1) & 1, U(c, line, q - 1), U(c, line, q), U(c, line, q + 1), el);
            B[c] = eno2<R, true>((FL(c, wr) >> 1) & 1, U(c, line, q), U(c, line, q + 1), U(c, line, q + 2), er);
          } else {
            A[c] = weno3<R, false>(U(c, line, q - 1), U(c, line, q), U(c, line, q + 1), el, eps);
            B[c] = weno3<R, true>(U(c, line, q), U(c, line, q + 1), U(c, line, q + 2), er, eps);
          }
          continue;
        }
        R eta = R(0);
        if (use_eta) {
          eta = R(eta_ratio<kExact>(double(U(c, line, q - 1)), double(U(c, line, q)), double(U(c, line, q + 1)),
                                    double(U(c, line, q + 2)), eps_m));
          if (use_switch && ((FL(c, wl) | FL(c, wr)) & 1)) eta = R(0);
        }
        if (eno) {
          A[c] = eno_minus<R>(FL(c, wl) >> 1, U(c, line, q - 2), U(c, line, q - 1), U(c, line, q),
                              U(c, line, q + 1), U(c, line, q + 2), eta);
          B[c] = eno_plus<R>(FL(c, wr) >> 1, U(c, line, q - 1), U(c, line, q), U(c, line, q + 1),
                             U(c, line, q + 2), U(c, line, q + 3), eta);
        } else if constexpr (SHARE) {
          A[c] = weno_minus<R>(U(c, line, q - 2), U(c, line, q - 1), U(c, line, q), U(c, line, q + 1),
                               U(c, line, q + 2), eta, s_den[c][0][wl], s_den[c][1][wl], s_den[c][2][wl]);
          B[c] = weno_plus<R>(U(c, line, q - 1), U(c, line, q), U(c, line, q + 1), U(c, line, q + 2),
                              U(c, line, q + 3), eta, s_den[c][0][wr], s_den[c][1][wr], s_den[c][2][wr]);
        } else {
          const R u0 = U(c, line, q - 2), u1 = U(c, line, q - 1), u2 = U(c, line, q), u3 = U(c, line, q + 1),
                  u4 = U(c, line, q + 2), u5 = U(c, line, q + 3);
          R d0, d1, d2;
          weight_denominators<R>(u0, u1, u2, u3, u4, eps, d0, d1, d2);
          A[c] = weno_minus<R>(u0, u1, u2, u3, u4, eta, d0, d1, d2);
          weight_denominators<R>(u1, u2, u3, u4, u5, eps, d0, d1, d2);
          B[c] = weno_plus<R>(u1, u2, u3, u4, u5, eta, d0, d1, d2);
        }
      }
      if constexpr (DIR == 0)
        lf_flux<R, FLUX, M, 0>(A, B, alpha_x, speed_x, gamma, H);
      else
        lf_flux<R, FLUX, M, 1>(A, B, alpha_y, speed_y, gamma, H);
#pragma unroll
      for (int c = 0; c < M; ++c) s_F[c][wl] = H[c];
    }
    __syncthreads();
    // flux difference into the owned cells; thread tid owns cells tid + k BS in both sweeps and in
    // the update, so L stays in its registers
#pragma unroll
    for (int k = 0; k < NOWN; ++k) {
      const int o = tid + k * BS;
      if (o >= TX * TY) continue;
      const int x = o % TX, y = o / TX;
      const int line = DIR == 0 ? y : x, pos = DIR == 0 ? x : y;
      const int wp = cid(line, pos), wm = cid(line, pos - 1);  // interfaces pos+1/2 and pos-1/2
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const R Fp = s_F[c][wp], Fm = s_F[c][wm];
        if constexpr (DIR == 0) {
          if constexpr (kExact)
            Lr[k][c] = -div_rn(Fp - Fm, dx);
          else
            Lr[k][c] = (Fm - Fp) * inv_dx;
        } else {
          if constexpr (kExact)
            Lr[k][c] = Lr[k][c] - div_rn(Fp - Fm, dy);
          else
            Lr[k][c] = Lr[k][c] + (Fm - Fp) * inv_dy;
        }
      }
    }
    __syncthreads();
  };
  sweep(std::integral_constant<int, 0>{});
  sweep(std::integral_constant<int, 1>{});

  // ---- update of the owned cells -----------------------------------------------------------
  R amx = R(0), amy = R(0);
  int bad = 0;
#pragma unroll
  for (int k = 0; k < NOWN; ++k) {
    const int o = tid + k * BS;
    const int x = o % TX, y = o / TX;
    if (o >= TX * TY || i0 + x >= nx || j0 + y >= ny) continue;
    const long long at = (long long)(j0 + y) * nx + (i0 + x);
    R unew[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const R L = Lr[k][c];
      const R us = ycol ? usr[k][c] : s_u[c][y + 3][x + 3];  // s_u holds v^+ after a column march
      if (stage == 0)
        unew[c] = L;
      else
        unew[c] = rk3_combine<R>(stage, upt[k][c], us, rdt * L);
    }
    if (direct) {
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
  if (stage == 0) return;
  amx = wave_max_nonneg(amx);
  amy = wave_max_nonneg(amy);
  const bool bad2 = __any(bad == 2), bad1 = __any(bad == 1);
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = double_to_bits(double(amx));
    s_red[1][tid >> 6] = double_to_bits(double(amy));
    s_bad[tid >> 6] = bad2 ? 2 : (bad1 ? 1 : 0);
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
        atomicMax(&sp[((slot * 2 + 0) * kSpread + k) * kSpreadStride], spread_tag(3 * (n - I->seq_base) + stage, float(bits_to_double(mx))));
        atomicMax(&sp[((slot * 2 + 1) * kSpread + k) * kSpreadStride], spread_tag(3 * (n - I->seq_base) + stage, float(bits_to_double(my))));
      } else {
        atomicMax(sp ? &sp[((slot * 2 + 0) * kSpread + k) * kSpreadStride] : &I->alpha[slot][0], mx);
        atomicMax(sp ? &sp[((slot * 2 + 1) * kSpread + k) * kSpreadStride] : &I->alpha[slot][1], my);
      }
    }
  }
}

}  // namespace npw

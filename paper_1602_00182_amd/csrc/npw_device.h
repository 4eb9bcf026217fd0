// npw_device.h -- per-cell / per-interface arithmetic of the scheme, as device functions.
//
// Two flavours share this header:
//   * double bulk (EXACT = true): every operation in the order the scheme states it, built
//     without FP contraction, so results are reproducible bit for bit.
//   * float bulk (EXACT = false): the same quantities with shared reciprocals and FMA; the
//     shape parameter and the switch decision stay in double precision.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/npweno.h"
#include "npw_internal.h"

namespace npw {

// Ghost-cell index (Section 1 leaves the boundary treatment open): periodic wrap, or a copy of
// the edge cell (transmissive).
// k may lie a few cells outside [0, n) (three ghosts, more only for grids shorter than a tile).
__device__ __forceinline__ int ghost_index(int k, int n, int bc) {
  if (k >= 0 && k < n) return k;
  if (bc == 0) {
    while (k < 0) k += n;
    while (k >= n) k -= n;
    return k;
  }
  return k < 0 ? 0 : n - 1;
}

// Faithful double quotient (error below one unit in the last place) for normal operands: the
// hardware reciprocal, one Newton step (relative error about the square of the reciprocal's) and
// one residual correction.  (Checked against the correctly rounded quotient on 4 million operand
// pairs spanning 1e-12..1e6: all equal.)  The first step of div_rn.
__device__ __forceinline__ double div_faithful(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

// Double quotient from the hardware reciprocal refined by one Newton step (relative error about
// the square of the reciprocal's, a couple of units in the last place of double).  The float bulk
// forms its double shape parameter with it and rounds the result to float.
__device__ __forceinline__ double div_newton(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
}

// Correctly rounded double division (round to nearest, ties to even).  The instruction sequence
// behind the '/' operator keeps the quotient within one unit in the last place but can return the
// neighbour of the nearest double (observed on operands of the scheme).  Here a faithful quotient
// q comes from div_faithful; the residual a - q b of a faithful q is exact (one fused
// multiply-add), and so is that of its neighbour q1 on the side of the exact quotient, so the
// smaller residual picks the nearest double.  Both candidates are formed without branches, so the
// independent divisions of a reconstruction overlap.  Operands or quotients outside
// [2^-900, 2^900] in magnitude (zero, subnormal, huge, non-finite) take the '/' sequence.
__device__ __forceinline__ double div_rn(double a, double b) {
  const double q = div_faithful(a, b);
  const double aq = fabs(q), aa = fabs(a), ab = fabs(b);
  if (!(aq > 0x1p-900 && aq < 0x1p900 && aa > 0x1p-900 && aa < 0x1p900 && ab > 0x1p-900 && ab < 0x1p900))
    return a / b;
  const double r = fma(-q, b, a);
  const bool up = (r > 0.0) == (b > 0.0);  // the exact quotient lies above q
  const long long bits = __double_as_longlong(q);
  const long long nb = ((q > 0.0) == up) ? bits + 1 : bits - 1;
  const double q1 = __longlong_as_double(nb);
  const double e0 = fabs(r), e1 = fabs(fma(-q1, b, a));
  return (e1 < e0 || (e1 == e0 && (nb & 1) == 0)) ? q1 : q;
}

// Raw buffer access: a resource over n_bytes from base, addressed by a 32-bit lane offset plus a
// uniform (scalar) offset, both in bytes, so that each component of a state is reached by changing
// only the scalar offset.  The hardware checks every access against n_bytes (loads out of range
// read 0 and such stores are dropped).  Word 3 of the descriptor: 32-bit data format, the value
// gfx9-family raw buffers take.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, unsigned n_bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)n_bytes, 0x00020000);
}
typedef int npw_int2 __attribute__((ext_vector_type(2)));
template <typename R>
__device__ __forceinline__ R buffer_load(__amdgpu_buffer_rsrc_t r, unsigned lane_bytes, unsigned uniform_bytes) {
  if constexpr (sizeof(R) == 4) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)lane_bytes, (int)uniform_bytes, 0));
  } else {
    const npw_int2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)lane_bytes, (int)uniform_bytes, 0);
    return __longlong_as_double(((long long)(unsigned)v.y << 32) | (unsigned)v.x);
  }
}
template <typename R>
__device__ __forceinline__ void buffer_store(R x, __amdgpu_buffer_rsrc_t r, unsigned lane_bytes, unsigned uniform_bytes) {
  if constexpr (sizeof(R) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(x), r, (int)lane_bytes, (int)uniform_bytes, 0);
  } else {
    const long long b = __double_as_longlong(x);
    npw_int2 v;
    v.x = (int)(unsigned)b;
    v.y = (int)(b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)lane_bytes, (int)uniform_bytes, 0);
  }
}

// Division and square root in the bulk precision: correctly rounded in double (the exact
// flavour); in float the hardware reciprocal and square root (about one unit in the last place
// each), which the float bulk's tolerance absorbs.
template <typename R>
__device__ __forceinline__ R fdiv(R a, R b) {
  if constexpr (sizeof(R) == 8)
    return div_rn(a, b);
  else
    return a * __builtin_amdgcn_rcpf(b);
}
template <typename R>
__device__ __forceinline__ R fsqrt(R a) {
  if constexpr (sizeof(R) == 8)
    return sqrt(a);
  else
    return __builtin_amdgcn_sqrtf(a);
}

// Monotone-polynomial test of Section 4 (eqs. root_value and adaptation) on the window
// (u_{j-1}, u_j, u_{j+1}): the quadratic reconstruction has its extremum at
// x_p/dx = (-2u_{j-1} + 3u_j - u_{j+1}) / (-u_{j-1} + 2u_j - u_{j+1}) from x_{j-3/2}; the window is
// not monotone when 0 < x_p/dx < 3.  Division by zero (linear data) gives inf/NaN, which fails
// the strict test.  Double precision, uncontracted: the decision is the one the quotient makes.
// CR (double bulk): the test on the correctly rounded quotient, as written.  Otherwise (float
// bulk: the window holds float values, so the differences p = u0 - um1 and q = up1 - u0 and the
// small-integer combinations of them below are exact in double) the same decision without the
// quotient.  With num = 2p - q and den = p - q, 0 < num/den < 3 holds exactly when num and den are
// non-zero with one sign and num - 3 den = -(p - 2q) has the opposite sign to den, i.e. when
// t1 = p - q, t2 = 2p - q and t3 = p - 2q are all non-zero with one sign: t1 t2 > 0 and t1 t3 > 0
// (products of float differences neither overflow nor underflow in double).  Ties (an extremum
// exactly at 0 or 3 dx) make t2 or t3 zero and are not flagged, as the strict inequalities say.
template <bool CR = true>
__device__ __forceinline__ int monotone_flag(double um1, double u0, double up1) {
#pragma clang fp contract(off)
  if constexpr (CR) {
    double num = -2.0 * um1 + 3.0 * u0 - up1;
    double den = -um1 + 2.0 * u0 - up1;
    double xp = div_rn(num, den);
    return (xp > 0.0 && xp < 3.0) ? 1 : 0;
  } else {
    const double p = u0 - um1, q = up1 - u0;
    const double t1 = p - q, t2 = p + t1, t3 = t1 - q;
    return (t1 * t2 > 0.0 && t1 * t3 > 0.0) ? 1 : 0;
  }
}

// Shape parameter eta = eps^2 dx^2 at x_{i+1/2} (Table 3 caption) from u_{i-1}..u_{i+2}:
// third over (weighted) first undivided difference; eps_M is added with the sign of the
// denominator so that it never crosses zero.  Double precision, uncontracted.
// (Float bulk: with s = um1 - up2 and d = up1 - u0, both exact, num = s + 3d and den = s + 15d,
// and the double quotient of div_newton, which the caller rounds to float.)
template <bool CR = true>
__device__ __forceinline__ double eta_ratio(double um1, double u0, double up1, double up2, double eps_m) {
#pragma clang fp contract(off)
  double num, den;
  if constexpr (CR) {
    num = um1 - 3.0 * u0 + 3.0 * up1 - up2;
    den = um1 - 15.0 * u0 + 15.0 * up1 - up2;
  } else {
    const double sd = um1 - up2, d = up1 - u0;
    num = fma(3.0, d, sd);
    den = fma(15.0, d, sd);
  }
  if (den >= 0.0)
    den = den + eps_m;
  else
    den = den - eps_m;
  return CR ? div_rn(num, den) : div_newton(num, den);
}

// Jiang-Shu smoothness indicators of cell i from (a..e) = u_{i-2}..u_{i+2}; b0 for the stencil
// {i..i+2}, b1 for {i-1..i+1}, b2 for {i-2..i}.
template <typename R>
__device__ __forceinline__ void smoothness(R a, R b, R c, R d, R e, R& b0, R& b1, R& b2) {
  R t;
  t = c - R(2.0) * d + e;
  b0 = R(13.0 / 12.0) * t * t;
  t = R(3.0) * c - R(4.0) * d + e;
  b0 = b0 + R(0.25) * t * t;
  t = b - R(2.0) * c + d;
  b1 = R(13.0 / 12.0) * t * t;
  t = b - d;
  b1 = b1 + R(0.25) * t * t;
  t = a - R(2.0) * b + c;
  b2 = R(13.0 / 12.0) * t * t;
  t = a - R(4.0) * b + R(3.0) * c;
  b2 = b2 + R(0.25) * t * t;
}

// Table 3 row r at x_{i+1/2} applied to (w0, w1, w2) = (u_{i-r}, u_{i-r+1}, u_{i-r+2}):
// sum_j (c_rj + eta p_rj) w_j, with the polynomial part c_rj (left table; the r = -1, j = 0 entry
// is 11/6) and the multiquadric perturbation p_rj (right table).
template <typename R, int ROW>
__device__ __forceinline__ R table3_row(R w0, R w1, R w2, R eta) {
  if constexpr (ROW == -1)
    return (R(11.0 / 6.0) + eta * R(-9.0 / 2.0)) * w0 + (R(-7.0 / 6.0) + eta * R(6.0)) * w1 +
           (R(1.0 / 3.0) + eta * R(-3.0 / 2.0)) * w2;
  else if constexpr (ROW == 0)
    return (R(1.0 / 3.0) + eta * R(5.0 / 6.0)) * w0 + (R(5.0 / 6.0) + eta * R(-2.0 / 3.0)) * w1 +
           (R(-1.0 / 6.0) + eta * R(-1.0 / 6.0)) * w2;
  else if constexpr (ROW == 1)
    return (R(-1.0 / 6.0) + eta * R(-1.0 / 6.0)) * w0 + (R(5.0 / 6.0) + eta * R(-2.0 / 3.0)) * w1 +
           (R(1.0 / 3.0) + eta * R(5.0 / 6.0)) * w2;
  else
    return (R(1.0 / 3.0) + eta * R(-3.0 / 2.0)) * w0 + (R(-7.0 / 6.0) + eta * R(6.0)) * w1 +
           (R(11.0 / 6.0) + eta * R(-9.0 / 2.0)) * w2;
}

// Weight denominators of cell i from its five-cell window (a..e) = u_{i-2}..u_{i+2}: the
// exact flavour keeps s_r = (eps + beta_r)^2; the fast flavour keeps 1 / s_r.
template <typename R>
__device__ __forceinline__ void weight_denominators(R a, R b, R c, R d, R e, R eps, R& s0, R& s1, R& s2) {
  R b0, b1, b2;
  smoothness<R>(a, b, c, d, e, b0, b1, b2);
  if constexpr (sizeof(R) == 8) {
#pragma clang fp contract(off)
    s0 = (eps + b0) * (eps + b0);
    s1 = (eps + b1) * (eps + b1);
    s2 = (eps + b2) * (eps + b2);
  } else {
    const R g0 = eps + b0, g1 = eps + b1, g2 = eps + b2;
    s0 = __builtin_amdgcn_rcpf(g0 * g0);
    s1 = __builtin_amdgcn_rcpf(g1 * g1);
    s2 = __builtin_amdgcn_rcpf(g2 * g2);
  }
}

// v^-_{i+1/2} of cell i (Table 3 rows 0, 1, 2 with the interface's eta, linear weights 3/10, 3/5,
// 1/10) and v^+_{i-1/2} of cell i (rows -1, 0, 1 with that interface's eta, linear weights 1/10,
// 3/5, 3/10), combined with the nonlinear weights of eq. (weno_re), alpha_r = d_r / s_r.
// (a..e) = u_{i-2}..u_{i+2}; (s0, s1, s2) from weight_denominators of the same cell.
// Exact flavour: the operation order of the definition (alpha_r, w_r = alpha_r / sum, sum w_r q_r).
__device__ __forceinline__ double weno_minus_exact(double a, double b, double c, double d, double e, double eta,
                                                   double s0, double s1, double s2) {
#pragma clang fp contract(off)
  double q0 = table3_row<double, 0>(c, d, e, eta);
  double q1 = table3_row<double, 1>(b, c, d, eta);
  double q2 = table3_row<double, 2>(a, b, c, eta);
  double a0 = div_rn(3.0 / 10.0, s0), a1 = div_rn(3.0 / 5.0, s1), a2 = div_rn(1.0 / 10.0, s2);
  double s = a0 + a1 + a2;
  double w0 = div_rn(a0, s), w1 = div_rn(a1, s), w2 = div_rn(a2, s);
  return w0 * q0 + w1 * q1 + w2 * q2;
}
__device__ __forceinline__ double weno_plus_exact(double a, double b, double c, double d, double e, double eta,
                                                  double s0, double s1, double s2) {
#pragma clang fp contract(off)
  double q0 = table3_row<double, -1>(c, d, e, eta);
  double q1 = table3_row<double, 0>(b, c, d, eta);
  double q2 = table3_row<double, 1>(a, b, c, eta);
  double a0 = div_rn(1.0 / 10.0, s0), a1 = div_rn(3.0 / 5.0, s1), a2 = div_rn(3.0 / 10.0, s2);
  double s = a0 + a1 + a2;
  double w0 = div_rn(a0, s), w1 = div_rn(a1, s), w2 = div_rn(a2, s);
  return w0 * q0 + w1 * q1 + w2 * q2;
}
// Fast float flavour: i_r = 1 / s_r precomputed, one reciprocal for the normalisation.
__device__ __forceinline__ float weno_minus_fast(float a, float b, float c, float d, float e, float eta, float i0,
                                                 float i1, float i2) {
  const float q0 = table3_row<float, 0>(c, d, e, eta);
  const float q1 = table3_row<float, 1>(b, c, d, eta);
  const float q2 = table3_row<float, 2>(a, b, c, eta);
  const float a0 = 0.3f * i0, a1 = 0.6f * i1, a2 = 0.1f * i2;
  return (a0 * q0 + a1 * q1 + a2 * q2) * __builtin_amdgcn_rcpf(a0 + a1 + a2);
}
__device__ __forceinline__ float weno_plus_fast(float a, float b, float c, float d, float e, float eta, float i0,
                                                float i1, float i2) {
  const float q0 = table3_row<float, -1>(c, d, e, eta);
  const float q1 = table3_row<float, 0>(b, c, d, eta);
  const float q2 = table3_row<float, 1>(a, b, c, eta);
  const float a0 = 0.1f * i0, a1 = 0.6f * i1, a2 = 0.3f * i2;
  return (a0 * q0 + a1 * q1 + a2 * q2) * __builtin_amdgcn_rcpf(a0 + a1 + a2);
}
// ENO stencil of cell i from (a..e) = u_{i-2}..u_{i+2} (Section 2, Newton divided differences):
// grow {i} twice towards the smaller undivided difference; ties keep the right-hand stencil.
// Returns r with S_r(i) = {i-r, .., i-r+2}.  Double precision, uncontracted.
__device__ __forceinline__ int eno_stencil(double a, double b, double c, double d, double e) {
#pragma clang fp contract(off)
  const double u[5] = {a, b, c, d, e};
  int left = 0;
  if (fabs(u[2] - u[1]) < fabs(u[3] - u[2])) left = 1;
  const int l = 2 - left;
  const double sl = fabs(u[l + 1] - 2.0 * u[l] + u[l - 1]);
  const double sr = fabs(u[l + 2] - 2.0 * u[l + 1] + u[l]);
  if (sl < sr) left = left + 1;
  return left;
}

// Table 3 row `row` (-1..2) chosen at run time, without branches (neighbouring lanes of a wave
// often pick different rows).  Rows 1 and 2 are rows 0 and -1 read backwards, so the six distinct
// coefficients c_rj + eta p_rj are formed once and selected; each is the same expression as in
// table3_row, and the sum runs in the same order, so the result is identical.
template <typename R>
__device__ __forceinline__ R table3_row_rt(int row, R w0, R w1, R w2, R eta) {
  const R k0 = R(1.0 / 3.0) + eta * R(5.0 / 6.0), k1 = R(5.0 / 6.0) + eta * R(-2.0 / 3.0),
          k2 = R(-1.0 / 6.0) + eta * R(-1.0 / 6.0);  // row 0; row 1 is (k2, k1, k0)
  const R m0 = R(11.0 / 6.0) + eta * R(-9.0 / 2.0), m1 = R(-7.0 / 6.0) + eta * R(6.0),
          m2 = R(1.0 / 3.0) + eta * R(-3.0 / 2.0);  // row -1; row 2 is (m2, m1, m0)
  const bool outer = row < 0 || row > 1, flip = row > 0;
  const R a = outer ? m0 : k0, b = outer ? m1 : k1, c = outer ? m2 : k2;
  return (flip ? c : a) * w0 + b * w1 + (flip ? a : c) * w2;
}

// ENO edge values of a cell with stencil r, window (a..e): v^- uses row r, v^+ row r-1, both on
// the cells (u_{i-r}, u_{i-r+1}, u_{i-r+2}), selected without branches.
template <typename R>
__device__ __forceinline__ void eno_cells(int r, R a, R b, R c, R d, R e, R& w0, R& w1, R& w2) {
  w0 = r == 0 ? c : (r == 1 ? b : a);
  w1 = r == 0 ? d : (r == 1 ? c : b);
  w2 = r == 0 ? e : (r == 1 ? d : c);
}
template <typename R>
__device__ __forceinline__ R eno_minus(int r, R a, R b, R c, R d, R e, R eta) {
  R w0, w1, w2;
  eno_cells<R>(r, a, b, c, d, e, w0, w1, w2);
  return table3_row_rt<R>(r, w0, w1, w2, eta);
}
template <typename R>
__device__ __forceinline__ R eno_plus(int r, R a, R b, R c, R d, R e, R eta) {
  R w0, w1, w2;
  eno_cells<R>(r, a, b, c, d, e, w0, w1, w2);
  return table3_row_rt<R>(r - 1, w0, w1, w2, eta);
}

template <typename R>
__device__ __forceinline__ R weno_minus(R a, R b, R c, R d, R e, R eta, R s0, R s1, R s2) {
  if constexpr (sizeof(R) == 8)
    return weno_minus_exact(a, b, c, d, e, eta, s0, s1, s2);
  else
    return weno_minus_fast(a, b, c, d, e, eta, s0, s1, s2);
}
template <typename R>
__device__ __forceinline__ R weno_plus(R a, R b, R c, R d, R e, R eta, R s0, R s1, R s2) {
  if constexpr (sizeof(R) == 8)
    return weno_plus_exact(a, b, c, d, e, eta, s0, s1, s2);
  else
    return weno_plus_fast(a, b, c, d, e, eta, s0, s1, s2);
}

// What a reconstruction code asks of the kernels.
struct ReconMode {
  bool k2;          // k = 2 (Table 2) instead of k = 3 (Table 3)
  bool eno;         // one stencil per cell (ENO) instead of the weighted combination
  bool use_eta;     // the multiquadric perturbation is on
  bool use_switch;  // the Section 4 switch zeroes it near non-monotone windows
  bool cross;       // Section 6: k = 2 with the shape parameter from the five-cell cross (2D)
};
__device__ __forceinline__ ReconMode recon_mode(int recon, int sw) {
  ReconMode m;
  m.k2 = recon >= NPW_RBF_WENO3;
  m.eno = recon == NPW_RBF_ENO3 || recon == NPW_ENO3 || recon == NPW_RBF_ENO2 || recon == NPW_ENO2;
  m.use_eta = recon == NPW_RBF_WENO5 || recon == NPW_RBF_ENO3 || recon == NPW_RBF_WENO3 || recon == NPW_RBF_ENO2;
  m.use_switch = m.use_eta && sw == NPW_SWITCH_MONOTONE;
  m.cross = recon == NPW_RBF_ENO2_2D;
  if (m.cross) m.use_eta = false, m.use_switch = sw == NPW_SWITCH_MONOTONE;
  return m;
}

// ---- k = 2 (Sections 3.1-3.2, Table 2) -------------------------------------------------------
// Row r (-1, 0, 1) of Table 2 at x_{i+1/2} applied to (w0, w1) = (u_{i-r}, u_{i-r+1}): polynomial
// part plus eta times the multiquadric perturbation.
template <typename R, int ROW>
__device__ __forceinline__ R table2_row(R w0, R w1, R eta) {
  if constexpr (ROW == -1)
    return (R(3.0 / 2.0) + eta * R(-3.0 / 2.0)) * w0 + (R(-1.0 / 2.0) + eta * R(1.0 / 2.0)) * w1;
  else if constexpr (ROW == 0)
    return (R(1.0 / 2.0) + eta * R(1.0 / 4.0)) * w0 + (R(1.0 / 2.0) + eta * R(1.0 / 4.0)) * w1;
  else
    return (R(-1.0 / 2.0) + eta * R(1.0 / 2.0)) * w0 + (R(3.0 / 2.0) + eta * R(-3.0 / 2.0)) * w1;
}

// Shape parameter of a cell for one edge (Table 2 caption): twice the second undivided
// difference over the three-point estimate -u_far + 5 u_0 + 2 u_near of six times the edge
// value, eps_M added with the sign of the denominator.  For the right edge of cell i pass
// (u_{i-1}, u_i, u_{i+1}); for its left edge the mirror (u_{i+1}, u_i, u_{i-1}).  Double,
// uncontracted.
template <bool CR = true>
__device__ __forceinline__ double eta2_ratio(double ufar, double u0, double unear, double eps_m) {
#pragma clang fp contract(off)
  double num = CR ? 2.0 * (-ufar + 2.0 * u0 - unear) : 2.0 * ((u0 - ufar) - (unear - u0));
  double den = -ufar + 5.0 * u0 + 2.0 * unear;
  if (den >= 0.0)
    den = den + eps_m;
  else
    den = den - eps_m;
  return CR ? div_rn(num, den) : div_newton(num, den);
}

// WENO3 edge values of cell i from (a, b, c) = u_{i-1}, u_i, u_{i+1}: v^-_{i+1/2} combines row 0 on
// {i, i+1} and row 1 on {i-1, i} with linear weights 2/3, 1/3; v^+_{i-1/2} combines row -1 on
// {i, i+1} and row 0 on {i-1, i} with 1/3, 2/3.  beta_0 = (u_{i+1} - u_i)^2, beta_1 = (u_i - u_{i-1})^2,
// alpha_r = d_r / (eps + beta_r)^2.  Exact flavour in the order of that definition.
template <bool PLUS>
__device__ __forceinline__ double weno3_exact(double a, double b, double c, double eta, double eps) {
#pragma clang fp contract(off)
  double t = c - b;
  const double b0 = t * t;
  t = b - a;
  const double b1 = t * t;
  const double d0 = PLUS ? 1.0 / 3.0 : 2.0 / 3.0, d1 = PLUS ? 2.0 / 3.0 : 1.0 / 3.0;
  const double a0 = div_rn(d0, (eps + b0) * (eps + b0));
  const double a1 = div_rn(d1, (eps + b1) * (eps + b1));
  const double s = a0 + a1;
  const double w0 = div_rn(a0, s), w1 = div_rn(a1, s);
  if (PLUS)
    return w0 * table2_row<double, -1>(b, c, eta) + w1 * table2_row<double, 0>(a, b, eta);
  return w0 * table2_row<double, 0>(b, c, eta) + w1 * table2_row<double, 1>(a, b, eta);
}
template <bool PLUS>
__device__ __forceinline__ float weno3_fast(float a, float b, float c, float eta, float eps) {
  const float g0 = eps + (c - b) * (c - b), g1 = eps + (b - a) * (b - a);
  const float a0 = (PLUS ? 1.0f / 3.0f : 2.0f / 3.0f) * __builtin_amdgcn_rcpf(g0 * g0);
  const float a1 = (PLUS ? 2.0f / 3.0f : 1.0f / 3.0f) * __builtin_amdgcn_rcpf(g1 * g1);
  const float q0 = PLUS ? table2_row<float, -1>(b, c, eta) : table2_row<float, 0>(b, c, eta);
  const float q1 = PLUS ? table2_row<float, 0>(a, b, eta) : table2_row<float, 1>(a, b, eta);
  return (a0 * q0 + a1 * q1) * __builtin_amdgcn_rcpf(a0 + a1);
}
template <typename R, bool PLUS>
__device__ __forceinline__ R weno3(R a, R b, R c, R eta, R eps) {
  if constexpr (sizeof(R) == 8)
    return weno3_exact<PLUS>(a, b, c, eta, eps);
  else
    return weno3_fast<PLUS>(a, b, c, eta, eps);
}

// ENO stencil of cell i for k = 2 from (u_{i-1}, u_i, u_{i+1}): 1 ({i-1, i}) when its undivided
// difference is strictly smaller, else 0 ({i, i+1}).  Double.
__device__ __forceinline__ int eno2_stencil(double a, double b, double c) {
#pragma clang fp contract(off)
  return fabs(b - a) < fabs(c - b) ? 1 : 0;
}
// ENO2 edge values of cell i with stencil r: v^- uses row r, v^+ row r - 1, on {i-r, i-r+1}.
template <typename R, bool PLUS>
__device__ __forceinline__ R eno2(int r, R a, R b, R c, R eta) {
  if (r == 0) return PLUS ? table2_row<R, -1>(b, c, eta) : table2_row<R, 0>(b, c, eta);
  return PLUS ? table2_row<R, 0>(a, b, eta) : table2_row<R, 1>(a, b, eta);
}

// Section 6 edge value of a cell from its three cells along the sweep (a, b, c) and its two
// transverse neighbours (ts, tn): the ENO2 polynomial value P of the pair chosen by divided
// differences (the transverse cell of the 2D stencil weighs 0 at the edge midpoint), perturbed to
// P + eta P with eta = (K dxx + dyy) / (4 D +- eps_M): dxx, dyy the second differences along and
// across the sweep, K = 4 for the centred pair and -8 for the extrapolating one (each cancels its
// pair's Taylor error), D the printed edge estimate (-2, 1, -5), mirrored for the left edge.  The
// switch keeps P when either three-cell window of the cell is not monotone.  RIGHT: the edge at
// the cell's + side (v^-), else its - side (v^+).  eta is double; the double flavour evaluates
// every operation in this order, uncontracted, with correctly rounded division.
template <typename R, bool RIGHT>
__device__ __forceinline__ R cross_edge(R a, R b, R c, R ts, R tn, bool use_switch, double eps_m) {
#pragma clang fp contract(off)
  constexpr bool kCR = sizeof(R) == 8;
  const double da = double(a), db = double(b), dc = double(c);
  const int r = eno2_stencil(da, db, dc);  // 1: {k-1, k}, 0: {k, k+1}
  R P;
  if (RIGHT)
    P = r == 0 ? table2_row<R, 0>(b, c, R(0)) : table2_row<R, 1>(a, b, R(0));
  else
    P = r == 0 ? table2_row<R, -1>(b, c, R(0)) : table2_row<R, 0>(a, b, R(0));
  if (use_switch && (monotone_flag<kCR>(da, db, dc) | monotone_flag<kCR>(double(ts), db, double(tn)))) return P;
  const double dxx = da - 2.0 * db + dc;
  const double dyy = double(ts) - 2.0 * db + double(tn);
  const double D = RIGHT ? -2.0 * da + db - 5.0 * dc : -2.0 * dc + db - 5.0 * da;
  const bool centred = RIGHT ? r == 0 : r == 1;
  const double K = centred ? 4.0 : -8.0;
  const double num = K * dxx + dyy;
  double den = 4.0 * D;
  if (den >= 0.0)
    den = den + eps_m;
  else
    den = den - eps_m;
  const double eta = kCR ? div_rn(num, den) : div_newton(num, den);
  return P + R(eta) * P;
}

// States at one interface x_{i+1/2} of one scalar field from its six-cell window
// w = u_{i-2}..u_{i+3} (register form of the LDS phases above, used where the field is local to
// the interface, as in characteristic-wise reconstruction): v^- of cell i and v^+ of cell i+1
// with the shape parameter(s) and switch of the reconstruction mode.  wd holds the same window in
// double for the shape parameter, the switch and the ENO stencil choice.
template <typename R>
__device__ __forceinline__ void window_states(const R* w, const double* wd, const ReconMode rm, R eps, double eps_m,
                                              R& vm, R& vp) {
  constexpr bool kCR = sizeof(R) == 8;
  if (rm.k2) {
    double el = 0.0, er = 0.0;
    if (rm.use_eta) {
      el = eta2_ratio<kCR>(wd[1], wd[2], wd[3], eps_m);  // right edge of cell i
      er = eta2_ratio<kCR>(wd[4], wd[3], wd[2], eps_m);  // left edge of cell i+1 (mirror)
      if (rm.use_switch) {
        if (monotone_flag<kCR>(wd[1], wd[2], wd[3])) el = 0.0;
        if (monotone_flag<kCR>(wd[2], wd[3], wd[4])) er = 0.0;
      }
    }
    if (rm.eno) {
      vm = eno2<R, false>(eno2_stencil(wd[1], wd[2], wd[3]), w[1], w[2], w[3], R(el));
      vp = eno2<R, true>(eno2_stencil(wd[2], wd[3], wd[4]), w[2], w[3], w[4], R(er));
    } else {
      vm = weno3<R, false>(w[1], w[2], w[3], R(el), eps);
      vp = weno3<R, true>(w[2], w[3], w[4], R(er), eps);
    }
    return;
  }
  double e = 0.0;
  if (rm.use_eta) {
    e = eta_ratio<kCR>(wd[1], wd[2], wd[3], wd[4], eps_m);
    if (rm.use_switch && (monotone_flag<kCR>(wd[1], wd[2], wd[3]) | monotone_flag<kCR>(wd[2], wd[3], wd[4]))) e = 0.0;
  }
  const R eta = R(e);
  if (rm.eno) {
    vm = eno_minus<R>(eno_stencil(wd[0], wd[1], wd[2], wd[3], wd[4]), w[0], w[1], w[2], w[3], w[4], eta);
    vp = eno_plus<R>(eno_stencil(wd[1], wd[2], wd[3], wd[4], wd[5]), w[1], w[2], w[3], w[4], w[5], eta);
  } else {
    R s0, s1, s2;
    weight_denominators<R>(w[0], w[1], w[2], w[3], w[4], eps, s0, s1, s2);
    vm = weno_minus<R>(w[0], w[1], w[2], w[3], w[4], eta, s0, s1, s2);
    weight_denominators<R>(w[1], w[2], w[3], w[4], w[5], eps, s0, s1, s2);
    vp = weno_plus<R>(w[1], w[2], w[3], w[4], w[5], eta, s0, s1, s2);
  }
}

// Eigen-system of the Euler flux Jacobian along DIR at the Roe average of the states UL, UR
// (conservative; M = 3 in 1D, 4 in 2D): Lm rows are left eigenvectors, Rm columns right
// eigenvectors, for the waves (normal velocity - c, contact [, shear], + c).  The double flavour
// evaluates every entry in the order written, uncontracted (its translation unit is built without
// FP contraction), so it reproduces a plain evaluation of the same formulas bit for bit; the float
// flavour may fuse multiply-adds.
template <typename R, int M, int DIR>
__device__ __forceinline__ void char_basis(const R* UL, const R* UR, R gamma, R (&Lm)[M][M], R (&Rm)[M][M]) {
  const R g1 = gamma - R(1.0);
  const R rl = UL[0], rr = UR[0];
  const R ul = fdiv(UL[1], rl), ur = fdiv(UR[1], rr);
  const R El = UL[M - 1], Er = UR[M - 1];
  R u, v = R(0), pl, pr;
  if constexpr (M == 4) {
    const R vl = fdiv(UL[2], rl), vr = fdiv(UR[2], rr);
    pl = g1 * (El - R(0.5) * rl * (ul * ul + vl * vl));
    pr = g1 * (Er - R(0.5) * rr * (ur * ur + vr * vr));
    const R sl = fsqrt(rl), sr = fsqrt(rr), den = sl + sr;
    u = fdiv(sl * ul + sr * ur, den);
    v = fdiv(sl * vl + sr * vr, den);
  } else {
    pl = g1 * (El - R(0.5) * rl * ul * ul);
    pr = g1 * (Er - R(0.5) * rr * ur * ur);
    const R sl = fsqrt(rl), sr = fsqrt(rr), den = sl + sr;
    u = fdiv(sl * ul + sr * ur, den);
  }
  const R Hl = fdiv(El + pl, rl), Hr = fdiv(Er + pr, rr);
  const R sl = fsqrt(rl), sr = fsqrt(rr), den = sl + sr;
  const R H = fdiv(sl * Hl + sr * Hr, den);
  const R q2 = M == 4 ? u * u + v * v : u * u;
  const R c2 = g1 * (H - R(0.5) * q2);
  const R c = fsqrt(c2);
  const R b1 = fdiv(g1, c2), b2 = R(0.5) * b1 * q2;
  const R un = DIR == 0 ? u : v;  // normal velocity
  const R ic = fdiv(R(1.0), c);
  const R uc = fdiv(un, c);
  if constexpr (M == 3) {
    Rm[0][0] = R(1.0), Rm[0][1] = R(1.0), Rm[0][2] = R(1.0);
    Rm[1][0] = u - c, Rm[1][1] = u, Rm[1][2] = u + c;
    Rm[2][0] = H - u * c, Rm[2][1] = R(0.5) * q2, Rm[2][2] = H + u * c;
    Lm[0][0] = R(0.5) * (b2 + uc), Lm[0][1] = R(-0.5) * (b1 * u + ic), Lm[0][2] = R(0.5) * b1;
    Lm[1][0] = R(1.0) - b2, Lm[1][1] = b1 * u, Lm[1][2] = -b1;
    Lm[2][0] = R(0.5) * (b2 - uc), Lm[2][1] = R(-0.5) * (b1 * u - ic), Lm[2][2] = R(0.5) * b1;
  } else if constexpr (DIR == 0) {
    Rm[0][0] = R(1.0), Rm[0][1] = R(1.0), Rm[0][2] = R(0.0), Rm[0][3] = R(1.0);
    Rm[1][0] = u - c, Rm[1][1] = u, Rm[1][2] = R(0.0), Rm[1][3] = u + c;
    Rm[2][0] = v, Rm[2][1] = v, Rm[2][2] = R(1.0), Rm[2][3] = v;
    Rm[3][0] = H - u * c, Rm[3][1] = R(0.5) * q2, Rm[3][2] = v, Rm[3][3] = H + u * c;
    Lm[0][0] = R(0.5) * (b2 + uc), Lm[0][1] = R(-0.5) * (b1 * u + ic), Lm[0][2] = R(-0.5) * b1 * v,
    Lm[0][3] = R(0.5) * b1;
    Lm[1][0] = R(1.0) - b2, Lm[1][1] = b1 * u, Lm[1][2] = b1 * v, Lm[1][3] = -b1;
    Lm[2][0] = -v, Lm[2][1] = R(0.0), Lm[2][2] = R(1.0), Lm[2][3] = R(0.0);
    Lm[3][0] = R(0.5) * (b2 - uc), Lm[3][1] = R(-0.5) * (b1 * u - ic), Lm[3][2] = R(-0.5) * b1 * v,
    Lm[3][3] = R(0.5) * b1;
  } else {
    Rm[0][0] = R(1.0), Rm[0][1] = R(1.0), Rm[0][2] = R(0.0), Rm[0][3] = R(1.0);
    Rm[1][0] = u, Rm[1][1] = u, Rm[1][2] = R(1.0), Rm[1][3] = u;
    Rm[2][0] = v - c, Rm[2][1] = v, Rm[2][2] = R(0.0), Rm[2][3] = v + c;
    Rm[3][0] = H - v * c, Rm[3][1] = R(0.5) * q2, Rm[3][2] = u, Rm[3][3] = H + v * c;
    Lm[0][0] = R(0.5) * (b2 + uc), Lm[0][1] = R(-0.5) * b1 * u, Lm[0][2] = R(-0.5) * (b1 * v + ic),
    Lm[0][3] = R(0.5) * b1;
    Lm[1][0] = R(1.0) - b2, Lm[1][1] = b1 * u, Lm[1][2] = b1 * v, Lm[1][3] = -b1;
    Lm[2][0] = -u, Lm[2][1] = R(1.0), Lm[2][2] = R(0.0), Lm[2][3] = R(0.0);
    Lm[3][0] = R(0.5) * (b2 - uc), Lm[3][1] = R(-0.5) * b1 * u, Lm[3][2] = R(-0.5) * (b1 * v - ic),
    Lm[3][3] = R(0.5) * b1;
  }
}

// Characteristic-wise interface states from the six-cell window U[k][c] (k = cells i-2..i+3):
// project on the left eigenvectors at the Roe average of cells i and i+1, reconstruct each field,
// map the edge values back with the right eigenvectors (sums in component order).
template <typename R, int M, int DIR>
__device__ __forceinline__ void char_states(const R (&U)[6][M], R gamma, const ReconMode rm, R eps, double eps_m,
                                            R* A, R* B) {
  // (double: uncontracted by its translation unit's build flags; float: projections may fuse)
  R Lm[M][M], Rm[M][M];
  char_basis<R, M, DIR>(U[2], U[3], gamma, Lm, Rm);
  R wm[M], wp[M];
#pragma unroll
  for (int p = 0; p < M; ++p) {
    R w[6];
    double wd[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      R s = Lm[p][0] * U[k][0];
#pragma unroll
      for (int c = 1; c < M; ++c) s = s + Lm[p][c] * U[k][c];
      w[k] = s;
      wd[k] = double(s);
    }
    window_states<R>(w, wd, rm, eps, eps_m, wm[p], wp[p]);
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    R a = Rm[c][0] * wm[0], b = Rm[c][0] * wp[0];
#pragma unroll
    for (int p = 1; p < M; ++p) {
      a = a + Rm[c][p] * wm[p];
      b = b + Rm[c][p] * wp[p];
    }
    A[c] = a;
    B[c] = b;
  }
}

// Physical flux along direction DIR (0: x, 1: y) of the state U[0..M-1] (Section 5.1; Euler as in
// Example 4, conservative variables).
template <typename R, int FLUX, int M, int DIR>
__device__ __forceinline__ void phys_flux(const R* U, R speed, R gamma, R* F) {
  if constexpr (FLUX == kAdvection) {
    F[0] = speed * U[0];
  } else if constexpr (FLUX == kBurgers) {
    F[0] = R(0.5) * U[0] * U[0];
  } else if constexpr (M == 3) {
    R rho = U[0], m = U[1], E = U[2];
    R u = fdiv(m, rho);
    R p = (gamma - R(1.0)) * (E - R(0.5) * rho * u * u);
    F[0] = m;
    F[1] = m * u + p;
    F[2] = (E + p) * u;
  } else {
    R rho = U[0], mx = U[1], my = U[2], E = U[3];
    R u = fdiv(mx, rho), v = fdiv(my, rho);
    R p = (gamma - R(1.0)) * (E - R(0.5) * rho * (u * u + v * v));
    if constexpr (DIR == 0) {
      F[0] = mx;
      F[1] = mx * u + p;
      F[2] = my * u;
      F[3] = (E + p) * u;
    } else {
      F[0] = my;
      F[1] = mx * v;
      F[2] = my * v + p;
      F[3] = (E + p) * v;
    }
  }
}

// Global Lax-Friedrichs flux h(a, b) = 1/2 [f(a) + f(b) - alpha (b - a)] (Section 5.1).
template <typename R, int FLUX, int M, int DIR>
__device__ __forceinline__ void lf_flux(const R* A, const R* B, R alpha, R speed, R gamma, R* H) {
  R fa[M], fb[M];
  phys_flux<R, FLUX, M, DIR>(A, speed, gamma, fa);
  phys_flux<R, FLUX, M, DIR>(B, speed, gamma, fb);
#pragma unroll
  for (int c = 0; c < M; ++c) H[c] = R(0.5) * (fa[c] + fb[c] - alpha * (B[c] - A[c]));
}

// Spectral radius of dF/dU along DIR at a cell-average state, plus validity: returns false for
// a non-finite state (code 1) or a non-physical Euler state (code 2).
template <typename R, int FLUX, int M, int DIR>
__device__ __forceinline__ R spectral_radius(const R* U, R speed, R gamma, int& bad) {
  bad = 0;
#pragma unroll
  for (int c = 0; c < M; ++c)
    if (!isfinite(U[c])) bad = 1;
  if (bad) return R(0);
  if constexpr (FLUX == kAdvection) {
    return fabs(speed);
  } else if constexpr (FLUX == kBurgers) {
    return fabs(U[0]);
  } else if constexpr (M == 3) {
    R rho = U[0], u = fdiv(U[1], rho);
    R p = (gamma - R(1.0)) * (U[2] - R(0.5) * rho * u * u);
    if (!(rho > R(0)) || !(p > R(0))) {
      bad = 2;
      return R(0);
    }
    return fabs(u) + fsqrt(fdiv(gamma * p, rho));
  } else {
    R rho = U[0], u = fdiv(U[1], rho), v = fdiv(U[2], rho);
    R p = (gamma - R(1.0)) * (U[3] - R(0.5) * rho * (u * u + v * v));
    if (!(rho > R(0)) || !(p > R(0))) {
      bad = 2;
      return R(0);
    }
    return fabs(DIR == 0 ? u : v) + fsqrt(fdiv(gamma * p, rho));
  }
}

// Spectral radii along x and y at one state (2D), with validity as in spectral_radius: the
// velocity quotients, the pressure and the sound speed are formed once for both directions (the
// same operations as spectral_radius, so each radius is the same number).
template <typename R, int FLUX, int M>
__device__ __forceinline__ void spectral_radii_2d(const R* U, R speed_x, R speed_y, R gamma, R& sx, R& sy,
                                                  int& bad) {
  bad = 0;
  sx = R(0);
  sy = R(0);
#pragma unroll
  for (int c = 0; c < M; ++c)
    if (!isfinite(U[c])) bad = 1;
  if (bad) return;
  if constexpr (FLUX == kAdvection) {
    sx = fabs(speed_x);
    sy = fabs(speed_y);
  } else if constexpr (FLUX == kBurgers) {
    sx = fabs(U[0]);
    sy = sx;
  } else {
    static_assert(M == 4, "2D Euler has four components");
    R rho = U[0], u = fdiv(U[1], rho), v = fdiv(U[2], rho);
    R p = (gamma - R(1.0)) * (U[3] - R(0.5) * rho * (u * u + v * v));
    if (!(rho > R(0)) || !(p > R(0))) {
      bad = 2;
      return;
    }
    const R c = fsqrt(fdiv(gamma * p, rho));
    sx = fabs(u) + c;
    sy = fabs(v) + c;
  }
}

// SSP-RK3 stage combination (Section 5.1) of u^n, the stage input v and its increment dt L(v):
//   stage 1: v + dt L;  stage 2: 3/4 u^n + 1/4 (v + dt L);  stage 3: 1/3 u^n + 2/3 (v + dt L).
// Stage 3 is evaluated as v + (w (u^n - v) + (1 - w) dt L) with w = 1/3 in both precisions:
// fl(1/3) + fl(2/3) is 1 - 2^-54 in double and 1 + 3e-8 in float, so the written form would
// scale the cell-average sum by that factor every step (a drift of 2.6e-12 over a 47 000-step
// double solve; about 1e-8 per step in L1 for float on sin(pi x)).  In the rearranged form the
// weights multiply only quantities whose sums over a periodic grid vanish, and one rounding of
// v + (...) remains.  The double bulk takes stage 2 as written (3/4 and 1/4 are exact), with
// the same operation order as the oracle; the float bulk rearranges stage 2 the same way.
template <typename R>
__device__ __forceinline__ R rk3_combine(int stage, R un, R v, R dtl) {
  if constexpr (sizeof(R) == 8) {
    if (stage == 1) return v + dtl;
    if (stage == 2) return R(0.75) * un + R(0.25) * (v + dtl);
    return v + (R(1.0 / 3.0) * (un - v) + R(2.0 / 3.0) * dtl);
  } else {
    if (stage == 1) return v + dtl;
    if (stage == 2) return v + (R(0.75) * (un - v) + R(0.25) * dtl);
    return v + (R(1.0 / 3.0) * (un - v) + R(2.0 / 3.0) * dtl);
  }
}

// Time step of the step starting at t (Section 5.1's CFL rule, clipped to the remaining time).
template <int DIM>
__device__ __forceinline__ double step_dt(double dt_fixed, double cfl, double dx, double dy, double T, double t,
                                          double ax, double ay) {
#pragma clang fp contract(off)
  double dt;
  if (dt_fixed > 0.0)
    dt = dt_fixed;
  else if constexpr (DIM == 1)
    dt = div_rn(cfl * dx, ax);
  else
    dt = div_rn(cfl, div_rn(ax, dx) + div_rn(ay, dy));
  double rem = T - t;
  if (dt > rem) dt = rem;
  return dt;
}

__device__ __forceinline__ double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ unsigned long long double_to_bits(double d) {
  return (unsigned long long)__double_as_longlong(d);
}

// Max of a non-negative value (+0 up to +inf, never NaN or -0) over the wavefront with DPP moves
// (rows of 16 lanes, then the row broadcasts); lanes without a source read 0, the identity for
// non-negative values.  Every lane gets the result of lane 63.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_take(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_max_step(float v) {
  // non-negative floats order as their bit patterns: an integer max, which the compiler merges
  // with the lane move into one instruction
  const unsigned b = __float_as_uint(v), o = dpp_take<CTRL, ROWS>(b);
  return __uint_as_float(b > o ? b : o);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_max_step(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = dpp_take<CTRL, ROWS>((unsigned)b), hi = dpp_take<CTRL, ROWS>((unsigned)(b >> 32));
  return fmax(v, __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo)));
}
template <typename R>
__device__ __forceinline__ R wave_max_nonneg(R v) {
  v = dpp_max_step<0x111, 0xf>(v);  // row_shr:1
  v = dpp_max_step<0x112, 0xf>(v);  // row_shr:2
  v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
  v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8  -> lane 15 of each row holds the row max
  v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the max
  if constexpr (sizeof(R) == 4) {
    return __uint_as_float((unsigned)__builtin_amdgcn_readlane((int)__float_as_uint(v), 63));
  } else {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
}

// Packed alpha slots (one entry per tile, see StageArgs::pack) are read as 16-byte vectors; the
// max of a lane's vectors, then over the wave (entries are non-negative; unused ones hold 0).
template <typename R>
struct PackVecT;
template <>
struct PackVecT<float> {
  using type = float4;
};
template <>
struct PackVecT<double> {
  using type = double2;
};
template <typename R>
using PackVec = typename PackVecT<R>::type;

template <typename R, int NL>
__device__ __forceinline__ R pack_max(const PackVec<R> (&pv)[NL]) {
  if constexpr (sizeof(R) == 4) {  // as bit patterns, like wave_max_nonneg
    auto mx = [](unsigned x, unsigned y) { return x > y ? x : y; };
    unsigned v = 0u;
#pragma unroll
    for (int c = 0; c < NL; ++c)
      v = mx(v, mx(mx(__float_as_uint(pv[c].x), __float_as_uint(pv[c].y)),
                   mx(__float_as_uint(pv[c].z), __float_as_uint(pv[c].w))));
    return wave_max_nonneg<float>(__uint_as_float(v));
  } else {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < NL; ++c) v = fmax(v, fmax(pv[c].x, pv[c].y));
    return wave_max_nonneg<double>(v);
  }
}

// A value the same in every lane, placed in a scalar register (values loaded through a vector
// load otherwise occupy a vector register per lane for as long as they live).
__device__ __forceinline__ int scalar_reg(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long scalar_reg(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float scalar_reg(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double scalar_reg(double v) {
  return __longlong_as_double(scalar_reg((long long)__double_as_longlong(v)));
}

// Read a value at a workgroup-uniform address through the scalar data cache (a scalar load,
// counted apart from the vector loads, and fetched once per cache rather than once per wave).
// The compiler takes memory read this way as unchanging while the kernel runs, so it is only for
// data that no work item of the running kernel writes before it is read: static fields, and
// fields that the kernel reads at its start and writes only after its branches on them.
template <typename T>
__device__ __forceinline__ T scalar_load(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}
// A tile record read field by field (a whole-struct copy would not become scalar loads).
__device__ __forceinline__ Tile scalar_load_tile(const Tile* p) {
  Tile t;
  t.inst = scalar_load(&p->inst);
  t.bc = scalar_load(&p->bc);
  t.start = scalar_load(&p->start);
  t.nx = scalar_load(&p->nx);
  t.off = scalar_load(&p->off);
  return t;
}

// Workgroups go to the 8 XCDs round robin (dispatch index b to XCD b % 8).  Map dispatch index b
// of G to a tile so that each XCD owns a contiguous run of tiles (a bijection on [0, G)):
// neighbouring tiles read each other's edge cells, and within a run they share one L2.
__device__ __forceinline__ long long xcd_contiguous_tile(long long b, long long G) {
  constexpr int kXcd = 8;
  const long long q = G / kXcd, r = G % kXcd, x = b % kXcd;
  return x * q + (x < r ? x : r) + b / kXcd;
}

// Float-bulk single grids tag every spread alpha entry with the stage that wrote it:
// entry = (stage sequence << 32) | float bits of alpha, the sequence of RK stage k of step n being
// 3 (n - seq_base) + k and that of the state check of u^n being 3 (n - seq_base).  Newer tags win
// the atomicMax, and a reader keeps only the entries carrying the sequence it expects, so no
// kernel has to clear a slot (the state check clears all of them whenever the state is replaced).
// The host keeps the sequence far below 2^32 by moving seq_base forward and re-running the state
// check, which clears the slots and re-seeds slot 0.
__device__ __forceinline__ unsigned long long spread_tag(long long seq, float a) {
  return ((unsigned long long)(unsigned)seq << 32) | (unsigned long long)__float_as_uint(a);
}
// max over the wave's entries that carry the expected sequence (one entry per lane), as double bits
__device__ __forceinline__ unsigned long long spread_reduce_tagged(unsigned long long entry, long long expect) {
  const float v = (unsigned)(entry >> 32) == (unsigned)expect ? __uint_as_float((unsigned)entry) : 0.0f;
  return double_to_bits(double(wave_max_nonneg<float>(v)));
}
// max over the wave's untagged entries (double bulk), as double bits
__device__ __forceinline__ unsigned long long spread_reduce(unsigned long long entry) {
  return double_to_bits(wave_max_nonneg(bits_to_double(entry)));
}
// This lane's entry of (slot, dir), and its address.
__device__ __forceinline__ const unsigned long long* spread_entry_ptr(const unsigned long long* spread, int slot, int dir) {
  return &spread[((slot * 2 + dir) * kSpread + (threadIdx.x & (kSpread - 1))) * kSpreadStride];
}
__device__ __forceinline__ unsigned long long spread_entry(const unsigned long long* spread, int slot, int dir) {
  return *spread_entry_ptr(spread, slot, dir);
}


}  // namespace npw

/*
 * npw_oracle.c -- plain, slow FP64 CPU oracle for the non-polynomial (multiquadric-RBF
 * perturbed) ENO/WENO finite-volume schemes of J. Guo and J.-H. Jung, "Non-polynomial ENO and
 * WENO finite volume methods for hyperbolic conservation laws" (arXiv:1602.00182): k = 3
 * (Table 3) and k = 2 (Table 2) reconstructions with their shape parameters and the Section 4
 * switch, ENO and WENO forms, the global Lax-Friedrichs flux and SSP-RK3 (Section 5.1), the
 * dimension-by-dimension 2D form (Section 7), the two-dimensional k = 2 reconstruction of
 * Section 6, and characteristic-wise Euler reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file:
 * only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.  It
 * shares no code, header, table or constant with the HIP implementation.
 *
 * Everything is IEEE double precision, evaluated in the order written (build with
 * -ffp-contract=off, no fast-math).  Each function names the passage of the paper it
 * follows.  Where the paper is silent or garbled, the reading taken is stated at the
 * function ("Reading: ...").
 *
 * Parity unpinned (no printed result or closed form fixes them; they are checked against the
 * GPU path and the invariants only): the per-stage reading of the Lax-Friedrichs alpha
 * (npo_alpha); Euler beyond the smooth density wave and the exact Sod solution; the Burgers
 * shock (Table 7 only within a factor of about 3); the 2D Euler workload; k = 2 Burgers;
 * characteristic reconstruction beyond its algebraic pins; and the Section 6 reconstruction
 * beyond its order and symmetry pins (Table 8's values).
 *
 * Layout of a state array: component-major, u[c*nx + i] in 1D and u[(c*ny + j)*nx + i] in
 * 2D, c = 0..ncomp-1.  Euler states are conservative: (rho, rho*u, E) in 1D and
 * (rho, rho*u, rho*v, E) in 2D.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "npw_oracle.h"

/* ------------------------------------------------------------------------------------ */
/* Reconstruction coefficients, Table 3 (k = 3).                                          */
/*                                                                                        */
/* Row r (r = -1, 0, 1, 2) reconstructs the value at x_{i+1/2} from the three cell        */
/* averages ubar_{i-r}, ubar_{i-r+1}, ubar_{i-r+2} as                                     */
/*     v = sum_j (c_rj + eta * p_rj) * ubar_{i-r+j},   eta = eps^2 dx^2.                   */
/* Left half of Table 3 gives c_rj (the eps -> 0 polynomial limit); the right half gives   */
/* c_rj + eta p_rj.  Reading: the printed r = -1, j = 0 entry "6/11" is 11/6 (every        */
/* polynomial row must sum to one, and 11/6 is the mirror of the r = 2, j = 2 entry).      */
/* ------------------------------------------------------------------------------------ */
static const double TAB_C[4][3] = {
    /* r = -1 */ {11.0 / 6.0, -7.0 / 6.0, 1.0 / 3.0},
    /* r =  0 */ {1.0 / 3.0, 5.0 / 6.0, -1.0 / 6.0},
    /* r =  1 */ {-1.0 / 6.0, 5.0 / 6.0, 1.0 / 3.0},
    /* r =  2 */ {1.0 / 3.0, -7.0 / 6.0, 11.0 / 6.0},
};
static const double TAB_P[4][3] = {
    /* r = -1 */ {-9.0 / 2.0, 6.0, -3.0 / 2.0},
    /* r =  0 */ {5.0 / 6.0, -2.0 / 3.0, -1.0 / 6.0},
    /* r =  1 */ {-1.0 / 6.0, -2.0 / 3.0, 5.0 / 6.0},
    /* r =  2 */ {-3.0 / 2.0, 6.0, -9.0 / 2.0},
};

void npo_table3(double c[12], double p[12]) {
  for (int r = 0; r < 4; ++r)
    for (int j = 0; j < 3; ++j) {
      c[3 * r + j] = TAB_C[r][j];
      p[3 * r + j] = TAB_P[r][j];
    }
}

/* Value at x_{i+1/2} of table row r (r = -1..2) applied to (w0, w1, w2) =
 * (ubar_{i-r}, ubar_{i-r+1}, ubar_{i-r+2}); the reconstruction form of Section 2. */
double npo_row_value(int r, double w0, double w1, double w2, double eta) {
  const double* c = TAB_C[r + 1];
  const double* p = TAB_P[r + 1];
  return (c[0] + eta * p[0]) * w0 + (c[1] + eta * p[1]) * w1 + (c[2] + eta * p[2]) * w2;
}

/* ------------------------------------------------------------------------------------ */
/* Shape parameter eta = eps^2 dx^2 at the interface x_{i+1/2}, Table 3 caption (k = 3):   */
/*     eta = (u_{i-1} - 3u_i + 3u_{i+1} - u_{i+2}) / (u_{i-1} - 15u_i + 15u_{i+1} - u_{i+2}  */
/*           + eps_M).                                                                    */
/* Reading: one eta per interface, from the four cells around it, shared by every row     */
/* used at that interface.  eps_M is the "positive small number" of Section 3.2 that      */
/* keeps the denominator away from zero; since the undivided difference in the            */
/* denominator takes either sign, it is added with the sign of that difference (+ at 0).  */
/* ------------------------------------------------------------------------------------ */
double npo_eta(double um1, double u0, double up1, double up2, double eps_m) {
  double num = um1 - 3.0 * u0 + 3.0 * up1 - up2;
  double den = um1 - 15.0 * u0 + 15.0 * up1 - up2;
  if (den >= 0.0)
    den = den + eps_m;
  else
    den = den - eps_m;
  return num / den;
}

/* ------------------------------------------------------------------------------------ */
/* Monotone-polynomial test, Section 4, eqs. (root_value) and (adaptation).              */
/* The quadratic through the three cell averages ubar_{j-1}, ubar_j, ubar_{j+1} (the       */
/* derivative of the cubic interpolant of the primitive on x_{j-3/2}..x_{j+3/2}) has its   */
/* extremum at                                                                            */
/*     x_p / dx = (-2 u_{j-1} + 3 u_j - u_{j+1}) / (-u_{j-1} + 2 u_j - u_{j+1}),          */
/* measured from x_{j-3/2}.  The window is "not monotone" when 0 < x_p/dx < 3.  Linear     */
/* data (zero denominator) gives +-inf or NaN, which fails both strict inequalities, so    */
/* linear windows are monotone, as they should be.                                        */
/* Returns 1 when the window is not monotone (the shape parameter must vanish).           */
/* ------------------------------------------------------------------------------------ */
int npo_monotone_flag(double um1, double u0, double up1) {
  double num = -2.0 * um1 + 3.0 * u0 - up1;
  double den = -um1 + 2.0 * u0 - up1;
  double xp = num / den;
  return (xp > 0.0 && xp < 3.0) ? 1 : 0;
}

/* ------------------------------------------------------------------------------------ */
/* Jiang-Shu smoothness indicators of the three substencils of cell i (Section 2 defers   */
/* them to Shu's lecture notes).  u5 = (u_{i-2}, .., u_{i+2}); beta[r] belongs to the     */
/* stencil S_r(i) = {i-r, .., i-r+2}.  They are the scaled integrals over I_i of the       */
/* squared first and second derivatives of each stencil's quadratic.                      */
/* ------------------------------------------------------------------------------------ */
void npo_beta(const double u5[5], double beta[3]) {
  double a = u5[0], b = u5[1], c = u5[2], d = u5[3], e = u5[4];
  double t;
  /* S_0 = {i, i+1, i+2} */
  t = c - 2.0 * d + e;
  beta[0] = 13.0 / 12.0 * t * t;
  t = 3.0 * c - 4.0 * d + e;
  beta[0] = beta[0] + 0.25 * t * t;
  /* S_1 = {i-1, i, i+1} */
  t = b - 2.0 * c + d;
  beta[1] = 13.0 / 12.0 * t * t;
  t = b - d;
  beta[1] = beta[1] + 0.25 * t * t;
  /* S_2 = {i-2, i-1, i} */
  t = a - 2.0 * b + c;
  beta[2] = 13.0 / 12.0 * t * t;
  t = a - 4.0 * b + 3.0 * c;
  beta[2] = beta[2] + 0.25 * t * t;
}

/* Nonlinear weights of eq. (weno_re): alpha_r = d_r / (eps + beta_r)^2, w_r = alpha_r /
 * sum_s alpha_s. */
static void weno_weights(const double d[3], const double beta[3], double eps, double w[3]) {
  double a[3], s;
  for (int r = 0; r < 3; ++r) a[r] = d[r] / ((eps + beta[r]) * (eps + beta[r]));
  s = a[0] + a[1] + a[2];
  for (int r = 0; r < 3; ++r) w[r] = a[r] / s;
}

/* Linear weights for k = 3.  Left-biased value v^-_{i+1/2}: d = (3/10, 3/5, 1/10) for
 * r = 0, 1, 2.  Right-biased value v^+_{i-1/2}: the mirror, (1/10, 3/5, 3/10). */
static const double D_MINUS[3] = {3.0 / 10.0, 3.0 / 5.0, 1.0 / 10.0};
static const double D_PLUS[3] = {1.0 / 10.0, 3.0 / 5.0, 3.0 / 10.0};

/* v^-_{i+1/2} of cell i, eq. (weno_re): convex combination of the three substencil values
 * of Table 3 rows r = 0, 1, 2 at x_{i+1/2}, each perturbed with the interface's eta. */
double npo_recon_minus(const double u5[5], double eta_right, double eps) {
  double beta[3], w[3], q[3];
  npo_beta(u5, beta);
  weno_weights(D_MINUS, beta, eps, w);
  for (int r = 0; r < 3; ++r) q[r] = npo_row_value(r, u5[2 - r], u5[3 - r], u5[4 - r], eta_right);
  return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

/* v^+_{i-1/2} of cell i: the same construction at the left edge of I_i.  The substencil
 * S_r(i) value at x_{i-1/2} is table row r - 1 at the interface x_{i-1/2} (the stencil
 * {i-r..i-r+2} seen from the cell to the left of that interface), perturbed with the eta of
 * x_{i-1/2}; the smoothness indicators are those of cell i. */
double npo_recon_plus(const double u5[5], double eta_left, double eps) {
  double beta[3], w[3], q[3];
  npo_beta(u5, beta);
  weno_weights(D_PLUS, beta, eps, w);
  for (int r = 0; r < 3; ++r) q[r] = npo_row_value(r - 1, u5[2 - r], u5[3 - r], u5[4 - r], eta_left);
  return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

/* ------------------------------------------------------------------------------------ */
/* ENO stencil of cell i (Section 2; Newton divided differences as in Shu's notes): start   */
/* from {i}, then twice add the neighbour (left or right) whose next divided difference of  */
/* the primitive is smaller in magnitude.  With uniform cells those divided differences are */
/* proportional to undivided differences of the averages.  Reading: on a tie the right-hand */
/* cell is taken (strict "<" for the left).  u5 = (u_{i-2}..u_{i+2}); returns r such that    */
/* the stencil is S_r(i) = {i-r, .., i-r+2}.                                                */
/* ------------------------------------------------------------------------------------ */
int npo_eno_stencil(const double u5[5]) {
  /* level 2: {i-1, i} or {i, i+1} */
  int left = 0; /* cells added on the left so far */
  double dl = fabs(u5[2] - u5[1]), dr = fabs(u5[3] - u5[2]);
  if (dl < dr) left = 1;
  /* level 3: current stencil {i-left, i-left+1}; candidates extend it by one cell */
  int l = 2 - left; /* index in u5 of the stencil's first cell */
  double sl = fabs(u5[l + 1] - 2.0 * u5[l] + u5[l - 1]);
  double sr = fabs(u5[l + 2] - 2.0 * u5[l + 1] + u5[l]);
  if (sl < sr) left = left + 1;
  return left;
}

/* ENO value of cell i at x_{i+1/2} (v^-) and at x_{i-1/2} (v^+) from the chosen stencil S_r:
 * Table 3 row r at x_{i+1/2} and row r-1 at x_{i-1/2}, each perturbed with its interface's eta
 * (eta = 0 gives the regular ENO scheme). */
double npo_eno_minus(const double u5[5], double eta_right) {
  int r = npo_eno_stencil(u5);
  return npo_row_value(r, u5[2 - r], u5[3 - r], u5[4 - r], eta_right);
}
double npo_eno_plus(const double u5[5], double eta_left) {
  int r = npo_eno_stencil(u5);
  return npo_row_value(r - 1, u5[2 - r], u5[3 - r], u5[4 - r], eta_left);
}

/* ------------------------------------------------------------------------------------ */
/* k = 2 (Sections 3.1-3.2, Table 2).                                                     */
/* Row r (r = -1, 0, 1) reconstructs the value at x_{i+1/2} from (ubar_{i-r}, ubar_{i-r+1}):  */
/* polynomial part (Table 2 left) plus eta times the multiquadric perturbation (right).     */
/* ------------------------------------------------------------------------------------ */
static const double TAB2_C[3][2] = {
    /* r = -1 */ {3.0 / 2.0, -1.0 / 2.0},
    /* r =  0 */ {1.0 / 2.0, 1.0 / 2.0},
    /* r =  1 */ {-1.0 / 2.0, 3.0 / 2.0},
};
static const double TAB2_P[3][2] = {
    /* r = -1 */ {-3.0 / 2.0, 1.0 / 2.0},
    /* r =  0 */ {1.0 / 4.0, 1.0 / 4.0},
    /* r =  1 */ {1.0 / 2.0, -3.0 / 2.0},
};

double npo_row2_value(int r, double w0, double w1, double eta) {
  const double* c = TAB2_C[r + 1];
  const double* p = TAB2_P[r + 1];
  return (c[0] + eta * p[0]) * w0 + (c[1] + eta * p[1]) * w1;
}

/* Shape parameter of cell i for its right edge, Table 2 caption (from eq. i+1/2_eps_approx):
 *     eta = 2 (-u_{i-1} + 2 u_i - u_{i+1}) / (-u_{i-1} + 5 u_i + 2 u_{i+1} + eps_M),
 * the ratio of the second difference to six times the estimate of v(x_{i+1/2}).  The left edge
 * uses the mirror image (u_{i-1} and u_{i+1} exchanged).  Reading: eps_M carries the sign of
 * the denominator, as for k = 3. */
double npo_eta2(double um1, double u0, double up1, double eps_m) {
  double num = 2.0 * (-um1 + 2.0 * u0 - up1);
  double den = -um1 + 5.0 * u0 + 2.0 * up1;
  if (den >= 0.0)
    den = den + eps_m;
  else
    den = den - eps_m;
  return num / den;
}

/* WENO3 values of cell i (window u3 = u_{i-1}, u_i, u_{i+1}): v^-_{i+1/2} combines row 0 on
 * {i, i+1} and row 1 on {i-1, i} with linear weights 2/3, 1/3; v^+_{i-1/2} combines row -1 on
 * {i, i+1} and row 0 on {i-1, i} with 1/3, 2/3.  Smoothness indicators (Jiang-Shu, k = 2):
 * beta_0 = (u_{i+1} - u_i)^2, beta_1 = (u_i - u_{i-1})^2; alpha_r = d_r / (eps + beta_r)^2. */
static void weno3_weights(const double d[2], double b0, double b1, double eps, double w[2]) {
  double a0 = d[0] / ((eps + b0) * (eps + b0));
  double a1 = d[1] / ((eps + b1) * (eps + b1));
  double s = a0 + a1;
  w[0] = a0 / s;
  w[1] = a1 / s;
}
double npo_weno3_minus(const double u3[3], double eta, double eps) {
  static const double d[2] = {2.0 / 3.0, 1.0 / 3.0};
  double t, b0, b1, w[2];
  t = u3[2] - u3[1];
  b0 = t * t;
  t = u3[1] - u3[0];
  b1 = t * t;
  weno3_weights(d, b0, b1, eps, w);
  return w[0] * npo_row2_value(0, u3[1], u3[2], eta) + w[1] * npo_row2_value(1, u3[0], u3[1], eta);
}
double npo_weno3_plus(const double u3[3], double eta, double eps) {
  static const double d[2] = {1.0 / 3.0, 2.0 / 3.0};
  double t, b0, b1, w[2];
  t = u3[2] - u3[1];
  b0 = t * t;
  t = u3[1] - u3[0];
  b1 = t * t;
  weno3_weights(d, b0, b1, eps, w);
  return w[0] * npo_row2_value(-1, u3[1], u3[2], eta) + w[1] * npo_row2_value(0, u3[0], u3[1], eta);
}
/* ENO, k = 2 (Section 3): {i-1, i} when its undivided difference is strictly smaller, else
 * {i, i+1}; returns r (0: {i, i+1}, 1: {i-1, i}). */
int npo_eno2_stencil(const double u3[3]) { return fabs(u3[1] - u3[0]) < fabs(u3[2] - u3[1]) ? 1 : 0; }
double npo_eno2_minus(const double u3[3], double eta) {
  int r = npo_eno2_stencil(u3);
  return npo_row2_value(r, u3[1 - r], u3[2 - r], eta);
}
double npo_eno2_plus(const double u3[3], double eta) {
  int r = npo_eno2_stencil(u3);
  return npo_row2_value(r - 1, u3[1 - r], u3[2 - r], eta);
}

/* ------------------------------------------------------------------------------------ */
/* Physical fluxes and spectral radii (Section 5.1; Example 4 for Euler).                 */
/* ------------------------------------------------------------------------------------ */
static void phys_flux(const npo_problem* pb, int dir, const double* U, double* F) {
  if (pb->flux == NPO_ADVECTION) {
    F[0] = (dir == 0 ? pb->speed_x : pb->speed_y) * U[0];
  } else if (pb->flux == NPO_BURGERS) {
    F[0] = 0.5 * U[0] * U[0];
  } else if (pb->ncomp == 3) { /* 1D Euler, Example 4 */
    double rho = U[0], m = U[1], E = U[2];
    double u = m / rho;
    double p = (pb->gamma - 1.0) * (E - 0.5 * rho * u * u);
    F[0] = m;
    F[1] = m * u + p;
    F[2] = (E + p) * u;
  } else { /* 2D Euler: dir 0 is the x flux f, dir 1 the y flux g */
    double rho = U[0], mx = U[1], my = U[2], E = U[3];
    double u = mx / rho, v = my / rho;
    double p = (pb->gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    if (dir == 0) {
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

/* Spectral radius of dF/dU in direction dir at a cell-average state.  Returns -1 for a
 * non-physical Euler state (rho <= 0 or p <= 0), NaN propagates. */
static double spectral_radius(const npo_problem* pb, int dir, const double* U) {
  if (pb->flux == NPO_ADVECTION) return fabs(dir == 0 ? pb->speed_x : pb->speed_y);
  if (pb->flux == NPO_BURGERS) return fabs(U[0]);
  if (pb->ncomp == 3) {
    double rho = U[0], u = U[1] / rho;
    double p = (pb->gamma - 1.0) * (U[2] - 0.5 * rho * u * u);
    if (!(rho > 0.0) || !(p > 0.0)) return -1.0;
    return fabs(u) + sqrt(pb->gamma * p / rho);
  } else {
    double rho = U[0], u = U[1] / rho, v = U[2] / rho;
    double p = (pb->gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
    if (!(rho > 0.0) || !(p > 0.0)) return -1.0;
    return fabs(dir == 0 ? u : v) + sqrt(pb->gamma * p / rho);
  }
}

/* Global Lax-Friedrichs flux h(a, b) = 1/2 [f(a) + f(b) - alpha (b - a)], Section 5.1,
 * component by component on vector states. */
static void lf_flux(const npo_problem* pb, int dir, const double* a, const double* b, double alpha,
                    double* h) {
  double fa[4], fb[4];
  phys_flux(pb, dir, a, fa);
  phys_flux(pb, dir, b, fb);
  for (int c = 0; c < pb->ncomp; ++c) h[c] = 0.5 * (fa[c] + fb[c] - alpha * (b[c] - a[c]));
}

/* Ghost index: periodic wrap or transmissive (copy of the edge cell).  Reading: the paper
 * gives no boundary treatment beyond "appropriate boundary conditions" (Section 1). */
static long ghost(long i, long n, int bc) {
  if (bc == NPO_PERIODIC) {
    long m = i % n;
    return m < 0 ? m + n : m;
  }
  if (i < 0) return 0;
  if (i >= n) return n - 1;
  return i;
}

/* ------------------------------------------------------------------------------------ */
/* Interface states along one grid line of n cells: for every interface x_{i+1/2},        */
/* i = -1..n-1 (stored at index i+1), compute eta, the switch, v^- (from cell i) and v^+   */
/* (from cell i+1).  line[] holds the n cell averages of one component; ghosts follow bc. */
/* ------------------------------------------------------------------------------------ */
static int is_k2(int recon) { return recon >= NPO_RBF_WENO3; }

/* States at one interface x_{i+1/2} from the six-cell window w = (u_{i-2}, .., u_{i+3}) of one
 * scalar field: v^- of cell i, v^+ of cell i+1, the shape parameter used and the switch flag.
 *
 * k = 3 (Table 3): one eta per interface from u_{i-1}..u_{i+2} (Table 3 caption).  Reading (k = 3
 * switch): the interface's eta vanishes when either three-cell window centred on a cell adjacent to
 * it fails the Section 4 monotone test.  v^- uses cells i-2..i+2, v^+ cells i-1..i+3.
 *
 * k = 2 (Table 2): cell i gives v^-_{i+1/2} with its right-edge eta and cell i+1 gives v^+_{i+1/2}
 * with its left-edge eta (Section 3.2 estimate); the Section 4 switch (stated for k = 2) zeroes
 * both etas of a cell whose window {i-1, i, i+1} is not monotone.  The eta reported is cell i's. */
static void interface_states(const npo_problem* pb, const double w[6], double* vm, double* vp, double* eta_out,
                             int* flag_out) {
  double eta = 0.0;
  int flag = 0;
  if (is_k2(pb->recon)) {
    const double* uL = w + 1; /* cell i:   u_{i-1}, u_i, u_{i+1} */
    const double* uR = w + 2; /* cell i+1: u_i, u_{i+1}, u_{i+2} */
    const int rbf = pb->recon == NPO_RBF_WENO3 || pb->recon == NPO_RBF_ENO2;
    double eL = 0.0, eR = 0.0;
    if (rbf) {
      eL = npo_eta2(uL[0], uL[1], uL[2], pb->eps_m); /* right edge of cell i */
      eR = npo_eta2(uR[2], uR[1], uR[0], pb->eps_m); /* left edge of cell i+1 (mirror) */
      if (pb->switch_mode == NPO_SWITCH_MONOTONE) {
        if (npo_monotone_flag(uL[0], uL[1], uL[2])) eL = 0.0, flag = 1;
        if (npo_monotone_flag(uR[0], uR[1], uR[2])) eR = 0.0, flag = 1;
      }
    }
    if (pb->recon == NPO_RBF_WENO3 || pb->recon == NPO_WENO3_JS) {
      *vm = npo_weno3_minus(uL, eL, pb->eps_weno);
      *vp = npo_weno3_plus(uR, eR, pb->eps_weno);
    } else {
      *vm = npo_eno2_minus(uL, eL);
      *vp = npo_eno2_plus(uR, eR);
    }
    eta = eL;
  } else {
    if (pb->recon == NPO_RBF_WENO5 || pb->recon == NPO_RBF_ENO3) {
      eta = npo_eta(w[1], w[2], w[3], w[4], pb->eps_m);
      if (pb->switch_mode == NPO_SWITCH_MONOTONE) {
        flag = npo_monotone_flag(w[1], w[2], w[3]) || npo_monotone_flag(w[2], w[3], w[4]);
        if (flag) eta = 0.0;
      }
    }
    const double* uL = w;     /* cells i-2..i+2: v^- of cell i */
    const double* uR = w + 1; /* cells i-1..i+3: v^+ of cell i+1 */
    if (pb->recon == NPO_RBF_ENO3 || pb->recon == NPO_ENO3) {
      *vm = npo_eno_minus(uL, eta);
      *vp = npo_eno_plus(uR, eta);
    } else {
      *vm = npo_recon_minus(uL, eta, pb->eps_weno);
      *vp = npo_recon_plus(uR, eta, pb->eps_weno);
    }
  }
  if (eta_out) *eta_out = eta;
  if (flag_out) *flag_out = flag;
}

/* Interface states along one grid line of n cells of one component: for every interface
 * x_{i+1/2}, i = -1..n-1 (stored at index i+1), the window u_{i-2..i+3} with ghosts per bc. */
void npo_line_states(const npo_problem* pb, const double* line, long n, double* vminus,
                     double* vplus, double* eta_out, int* flag_out) {
  for (long i = -1; i <= n - 1; ++i) {
    double w[6];
    for (int k = 0; k < 6; ++k) w[k] = line[ghost(i - 2 + k, n, pb->bc)];
    interface_states(pb, w, &vminus[i + 1], &vplus[i + 1], eta_out ? &eta_out[i + 1] : NULL,
                     flag_out ? &flag_out[i + 1] : NULL);
  }
}

/* ------------------------------------------------------------------------------------ */
/* Section 6: the genuinely two-dimensional perturbed k = 2 reconstruction.               */
/*                                                                                        */
/* At an edge of cell (i, j) along a sweep, the polynomial value P is the one-dimensional */
/* ENO2 value (Table 2 polynomial row of the stencil chosen by divided differences; the    */
/* third, transverse cell of the 2D stencil carries weight 0 at the edge midpoint, eq.     */
/* poly_recon2d).  The perturbation eta * sum_k c_k u_k with eta from the five-cell cross  */
/* (eq. i+1/2_eps_approx_2d) cancels the Taylor error of P (eq. rbf_recon_error_2d).       */
/* Readings: c_k proportional to the polynomial weights of the chosen pair (as Table 2's   */
/* perturbation rows are for k = 2 in 1D), so that sum_k c_k u_k = (sum c) P; the error to */
/* cancel is a dxx/6 + dyy/24 for the centred pair and -dxx/3 + dyy/24 for the            */
/* extrapolating pair (dxx, dyy the second undivided differences along and across the      */
/* sweep); the edge value in the denominator is the printed estimate -(-2, 1, -5)/6        */
/* (first moment zero about the edge), mirrored for the other edge; eps_M carries the sign */
/* of the denominator; the switch zeroes the perturbation when the along- or the           */
/* across-sweep three-cell window of the cell fails the Section 4 test.  Then              */
/*     edge value = P + eta' P,  eta' = (K dxx + dyy) / (4 D +- eps_M),  K = 4 or -8.        */
/* w3 = cells (k-1, k, k+1) along the sweep, t2 = the two transverse neighbours of cell k;  */
/* right_edge selects the edge at k+1/2 (v^-) or k-1/2 (v^+).                               */
/* ------------------------------------------------------------------------------------ */
double npo_cross_edge(const double w3[3], const double t2[2], int right_edge, int use_switch, double eps_m) {
  const int r = npo_eno2_stencil(w3); /* 1: {k-1, k}, 0: {k, k+1} */
  const double P = right_edge ? npo_row2_value(r, w3[1 - r], w3[2 - r], 0.0)
                              : npo_row2_value(r - 1, w3[1 - r], w3[2 - r], 0.0);
  if (use_switch && (npo_monotone_flag(w3[0], w3[1], w3[2]) || npo_monotone_flag(t2[0], w3[1], t2[1]))) return P;
  const double dxx = w3[0] - 2.0 * w3[1] + w3[2];
  const double dyy = t2[0] - 2.0 * w3[1] + t2[1];
  const double D = right_edge ? -2.0 * w3[0] + w3[1] - 5.0 * w3[2] : -2.0 * w3[2] + w3[1] - 5.0 * w3[0];
  const int centred = right_edge ? (r == 0) : (r == 1);
  const double K = centred ? 4.0 : -8.0;
  const double num = K * dxx + dyy;
  double den = 4.0 * D;
  if (den >= 0.0)
    den = den + eps_m;
  else
    den = den - eps_m;
  const double eta = num / den;
  return P + eta * P;
}

/* Edge states of one component field (nx x ny, row-major) along direction dir for the
 * Section 6 reconstruction: interface f (0..n) between cells f-1 and f of every line, stored at
 * line * (n + 1) + f, n = nx (dir 0) or ny (dir 1); ghosts follow bc in both directions. */
int npo_face_states(const npo_problem* pb, int dir, const double* field, double* vm, double* vp) {
  if (pb->dim != 2 || pb->recon != NPO_RBF_ENO2_2D) return NPO_EINVAL;
  const long nx = pb->nx, ny = pb->ny;
  const long n = dir == 0 ? nx : ny, lines = dir == 0 ? ny : nx;
  const int sw = pb->switch_mode == NPO_SWITCH_MONOTONE;
#define F(ii, jj) field[ghost((jj), ny, pb->bc) * nx + ghost((ii), nx, pb->bc)]
#define C(k, l, o) (dir == 0 ? F((k), (l) + (o)) : F((l) + (o), (k))) /* cell k along, line l, transverse offset o */
#define A(k, l) (dir == 0 ? F((k), (l)) : F((l), (k)))
  for (long l = 0; l < lines; ++l) {
    for (long f = 0; f <= n; ++f) {
      const long kl = f - 1, kr = f; /* left and right cell along the sweep */
      const double wl[3] = {A(kl - 1, l), A(kl, l), A(kl + 1, l)};
      const double tl[2] = {C(kl, l, -1), C(kl, l, 1)};
      const double wr[3] = {A(kr - 1, l), A(kr, l), A(kr + 1, l)};
      const double tr[2] = {C(kr, l, -1), C(kr, l, 1)};
      vm[l * (n + 1) + f] = npo_cross_edge(wl, tl, 1, sw, pb->eps_m);
      vp[l * (n + 1) + f] = npo_cross_edge(wr, tr, 0, sw, pb->eps_m);
    }
  }
#undef A
#undef C
#undef F
  return NPO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Characteristic-wise reconstruction for the Euler equations (an extension the paper     */
/* does not use: Example 4 reconstructs as it states the scheme, one scalar field at a    */
/* time, which the component-wise mode follows).  At each interface the six-cell window   */
/* of conservative states is projected on the left eigenvectors of the flux Jacobian at   */
/* the Roe average of the two adjacent cells, every characteristic field is reconstructed */
/* with the scalar scheme above (eta and the switch on that field), and the edge states    */
/* are mapped back with the right eigenvectors.                                           */
/* ------------------------------------------------------------------------------------ */

/* Roe average of two Euler states and the eigen-system of dF/dU (direction dir) there.
 * Lm (rows = left eigenvectors) and Rm (columns = right eigenvectors) are m x m row-major,
 * lam the eigenvalues (normal velocity -c, the contact/shear waves, +c).  Returns
 * NPO_ENONPHYSICAL when a state or the average has rho <= 0, p <= 0 or c^2 <= 0. */
int npo_char_basis(const npo_problem* pb, int dir, const double* UL, const double* UR, double* Lm, double* Rm,
                   double* lam) {
  const int m = pb->ncomp;
  const double g1 = pb->gamma - 1.0;
  const double rl = UL[0], rr = UR[0];
  if (!(rl > 0.0) || !(rr > 0.0)) return NPO_ENONPHYSICAL;
  const double ul = UL[1] / rl, ur = UR[1] / rr;
  const double vl = m == 4 ? UL[2] / rl : 0.0, vr = m == 4 ? UR[2] / rr : 0.0;
  const double El = UL[m - 1], Er = UR[m - 1];
  double pl, pr;
  if (m == 4) {
    pl = g1 * (El - 0.5 * rl * (ul * ul + vl * vl));
    pr = g1 * (Er - 0.5 * rr * (ur * ur + vr * vr));
  } else {
    pl = g1 * (El - 0.5 * rl * ul * ul);
    pr = g1 * (Er - 0.5 * rr * ur * ur);
  }
  if (!(pl > 0.0) || !(pr > 0.0)) return NPO_ENONPHYSICAL;
  const double Hl = (El + pl) / rl, Hr = (Er + pr) / rr;
  const double sl = sqrt(rl), sr = sqrt(rr), den = sl + sr;
  const double u = (sl * ul + sr * ur) / den;
  const double v = (sl * vl + sr * vr) / den;
  const double H = (sl * Hl + sr * Hr) / den;
  const double q2 = m == 4 ? u * u + v * v : u * u;
  const double c2 = g1 * (H - 0.5 * q2);
  if (!(c2 > 0.0)) return NPO_ENONPHYSICAL;
  const double c = sqrt(c2);
  const double b1 = g1 / c2, b2 = 0.5 * b1 * q2;
  if (m == 3) {
    const double R3[9] = {1.0, 1.0, 1.0,
                          u - c, u, u + c,
                          H - u * c, 0.5 * q2, H + u * c};
    const double L3[9] = {0.5 * (b2 + u / c), -0.5 * (b1 * u + 1.0 / c), 0.5 * b1,
                          1.0 - b2, b1 * u, -b1,
                          0.5 * (b2 - u / c), -0.5 * (b1 * u - 1.0 / c), 0.5 * b1};
    memcpy(Rm, R3, sizeof R3);
    memcpy(Lm, L3, sizeof L3);
    lam[0] = u - c;
    lam[1] = u;
    lam[2] = u + c;
  } else if (dir == 0) {
    const double R4[16] = {1.0, 1.0, 0.0, 1.0,
                           u - c, u, 0.0, u + c,
                           v, v, 1.0, v,
                           H - u * c, 0.5 * q2, v, H + u * c};
    const double L4[16] = {0.5 * (b2 + u / c), -0.5 * (b1 * u + 1.0 / c), -0.5 * b1 * v, 0.5 * b1,
                           1.0 - b2, b1 * u, b1 * v, -b1,
                           -v, 0.0, 1.0, 0.0,
                           0.5 * (b2 - u / c), -0.5 * (b1 * u - 1.0 / c), -0.5 * b1 * v, 0.5 * b1};
    memcpy(Rm, R4, sizeof R4);
    memcpy(Lm, L4, sizeof L4);
    lam[0] = u - c;
    lam[1] = u;
    lam[2] = u;
    lam[3] = u + c;
  } else {
    const double R4[16] = {1.0, 1.0, 0.0, 1.0,
                           u, u, 1.0, u,
                           v - c, v, 0.0, v + c,
                           H - v * c, 0.5 * q2, u, H + v * c};
    const double L4[16] = {0.5 * (b2 + v / c), -0.5 * b1 * u, -0.5 * (b1 * v + 1.0 / c), 0.5 * b1,
                           1.0 - b2, b1 * u, b1 * v, -b1,
                           -u, 1.0, 0.0, 0.0,
                           0.5 * (b2 - v / c), -0.5 * b1 * u, -0.5 * (b1 * v - 1.0 / c), 0.5 * b1};
    memcpy(Rm, R4, sizeof R4);
    memcpy(Lm, L4, sizeof L4);
    lam[0] = v - c;
    lam[1] = v;
    lam[2] = v;
    lam[3] = v + c;
  }
  return NPO_OK;
}

/* States at one interface from its six-cell window of conservative states U6[k*m + c]
 * (k = cells i-2..i+3): the characteristic-wise counterpart of interface_states. */
int npo_char_interface(const npo_problem* pb, int dir, const double* U6, double* vm, double* vp) {
  const int m = pb->ncomp;
  double U[6][4], W[4][6], Lm[16], Rm[16], lam[4], wm[4], wp[4];
  for (int k = 0; k < 6; ++k)
    for (int c = 0; c < m; ++c) U[k][c] = U6[k * m + c];
  int rc = npo_char_basis(pb, dir, U[2], U[3], Lm, Rm, lam);
  if (rc) return rc;
  for (int p = 0; p < m; ++p)
    for (int k = 0; k < 6; ++k) {
      double s = Lm[p * m + 0] * U[k][0];
      for (int c = 1; c < m; ++c) s = s + Lm[p * m + c] * U[k][c];
      W[p][k] = s;
    }
  for (int p = 0; p < m; ++p) interface_states(pb, W[p], &wm[p], &wp[p], NULL, NULL);
  for (int c = 0; c < m; ++c) {
    double a = Rm[c * m + 0] * wm[0], b = Rm[c * m + 0] * wp[0];
    for (int p = 1; p < m; ++p) {
      a = a + Rm[c * m + p] * wm[p];
      b = b + Rm[c * m + p] * wp[p];
    }
    vm[c] = a;
    vp[c] = b;
  }
  return NPO_OK;
}

/* Characteristic interface states along one line: lines[c][0..n-1] holds component c.  For
 * interface i+1/2 (index i+1): W_k = Lm U_k for the window k = i-2..i+3, the scalar interface
 * states of every field, then U^- = Rm W^-, U^+ = Rm W^+ (sums in component order).  vm, vp are
 * component-major with n+1 entries per component. */
static int char_line_states(const npo_problem* pb, int dir, const double* const* lines, long n, double* vm,
                            double* vp) {
  const int m = pb->ncomp;
  for (long i = -1; i <= n - 1; ++i) {
    double U[6][4], W[4][6], Lm[16], Rm[16], lam[4], wm[4], wp[4];
    for (int k = 0; k < 6; ++k) {
      long g = ghost(i - 2 + k, n, pb->bc);
      for (int c = 0; c < m; ++c) U[k][c] = lines[c][g];
    }
    int rc = npo_char_basis(pb, dir, U[2], U[3], Lm, Rm, lam);
    if (rc) return rc;
    for (int p = 0; p < m; ++p)
      for (int k = 0; k < 6; ++k) {
        double s = Lm[p * m + 0] * U[k][0];
        for (int c = 1; c < m; ++c) s = s + Lm[p * m + c] * U[k][c];
        W[p][k] = s;
      }
    for (int p = 0; p < m; ++p) interface_states(pb, W[p], &wm[p], &wp[p], NULL, NULL);
    for (int c = 0; c < m; ++c) {
      double a = Rm[c * m + 0] * wm[0], b = Rm[c * m + 0] * wp[0];
      for (int p = 1; p < m; ++p) {
        a = a + Rm[c * m + p] * wm[p];
        b = b + Rm[c * m + p] * wp[p];
      }
      vm[(size_t)c * (n + 1) + (i + 1)] = a;
      vp[(size_t)c * (n + 1) + (i + 1)] = b;
    }
  }
  return NPO_OK;
}

static int validate(const npo_problem* pb) {
  if (!pb) return NPO_EINVAL;
  if (pb->dim != 1 && pb->dim != 2) return NPO_EINVAL;
  if (pb->nx < 1 || (pb->dim == 2 && pb->ny < 1)) return NPO_EINVAL;
  if (pb->flux == NPO_EULER) {
    if ((pb->dim == 1 && pb->ncomp != 3) || (pb->dim == 2 && pb->ncomp != 4)) return NPO_EINVAL;
    if (!(pb->gamma > 1.0)) return NPO_EINVAL;
  } else if (pb->flux == NPO_ADVECTION || pb->flux == NPO_BURGERS) {
    if (pb->ncomp != 1) return NPO_EINVAL;
  } else {
    return NPO_EINVAL;
  }
  if (pb->bc != NPO_PERIODIC && pb->bc != NPO_TRANSMISSIVE) return NPO_EINVAL;
  if (!(pb->x1 > pb->x0) || (pb->dim == 2 && !(pb->y1 > pb->y0))) return NPO_EINVAL;
  if (!(pb->cfl > 0.0) || !(pb->eps_weno > 0.0) || !(pb->eps_m > 0.0)) return NPO_EINVAL;
  if (pb->recon < NPO_RBF_WENO5 || pb->recon > NPO_RBF_ENO2_2D) return NPO_EINVAL;
  if (pb->recon == NPO_RBF_ENO2_2D && (pb->dim != 2 || pb->charwise)) return NPO_EINVAL;
  if (pb->switch_mode != NPO_SWITCH_MONOTONE && pb->switch_mode != NPO_SWITCH_OFF) return NPO_EINVAL;
  if (pb->charwise != 0 && (pb->charwise != 1 || pb->flux != NPO_EULER)) return NPO_EINVAL;
  return NPO_OK;
}

/* Global Lax-Friedrichs alpha per direction: max over cells of the spectral radius of the
 * cell-average state (Section 5.1, "alpha = max |df/du|"; reading: the max is taken over
 * the cell averages of the current stage, so every RK stage evaluates its own alpha).
 * Parity unpinned for that reading: Section 5.1 only calls alpha a constant, and no printed
 * result separates a per-stage alpha from one frozen at u^n for the whole step (Table 7's
 * Burgers rows agree with either only to a factor of about 3). */
int npo_alpha(const npo_problem* pb, const double* u, double alpha[2]) {
  int rc = validate(pb);
  if (rc) return rc;
  long ny = pb->dim == 2 ? pb->ny : 1, ncell = pb->nx * ny;
  alpha[0] = 0.0;
  alpha[1] = 0.0;
  for (long k = 0; k < ncell; ++k) {
    double U[4];
    for (int c = 0; c < pb->ncomp; ++c) {
      U[c] = u[c * ncell + k];
      if (!isfinite(U[c])) return NPO_ENONFINITE;
    }
    for (int dir = 0; dir < pb->dim; ++dir) {
      double s = spectral_radius(pb, dir, U);
      if (s < 0.0) return NPO_ENONPHYSICAL;
      if (s > alpha[dir]) alpha[dir] = s;
    }
  }
  return NPO_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Semi-discrete right-hand side, eq. (PDE1) (1D) and eq. (2DIntegral) with one midpoint  */
/* quadrature point per face (2D, dimension by dimension):                               */
/*     L_i = -(F_{i+1/2} - F_{i-1/2}) / dx   [- (G_{j+1/2} - G_{j-1/2}) / dy].            */
/* ------------------------------------------------------------------------------------ */
int npo_rhs(const npo_problem* pb, const double* u, double* L, double alpha_out[2]) {
  double alpha[2];
  int rc = npo_alpha(pb, u, alpha);
  if (rc) return rc;
  if (alpha_out) {
    alpha_out[0] = alpha[0];
    alpha_out[1] = alpha[1];
  }
  const int m = pb->ncomp;
  const long nx = pb->nx, ny = pb->dim == 2 ? pb->ny : 1, ncell = nx * ny;
  const double dx = (pb->x1 - pb->x0) / (double)nx;
  const double dy = pb->dim == 2 ? (pb->y1 - pb->y0) / (double)ny : 1.0;
  long nmax = nx > ny ? nx : ny;
  double* line = (double*)malloc(sizeof(double) * (size_t)nmax);
  double* vm = (double*)malloc(sizeof(double) * (size_t)(nmax + 1) * (size_t)m);
  double* vp = (double*)malloc(sizeof(double) * (size_t)(nmax + 1) * (size_t)m);
  double* F = (double*)malloc(sizeof(double) * (size_t)(nmax + 1) * (size_t)m);

  if (pb->recon == NPO_RBF_ENO2_2D) {
    /* Section 6 reconstruction: edge states need the transverse neighbours, so each component's
     * x- and y-edge states are formed on the whole grid first; fluxes and differences then run
     * as in the sweeps below (x contribution first, y subtracted after). */
    double* ex_m = (double*)malloc(sizeof(double) * (size_t)m * (size_t)ny * (size_t)(nx + 1));
    double* ex_p = (double*)malloc(sizeof(double) * (size_t)m * (size_t)ny * (size_t)(nx + 1));
    double* ey_m = (double*)malloc(sizeof(double) * (size_t)m * (size_t)nx * (size_t)(ny + 1));
    double* ey_p = (double*)malloc(sizeof(double) * (size_t)m * (size_t)nx * (size_t)(ny + 1));
    for (int c = 0; c < m; ++c) {
      npo_face_states(pb, 0, u + c * ncell, ex_m + (size_t)c * ny * (nx + 1), ex_p + (size_t)c * ny * (nx + 1));
      npo_face_states(pb, 1, u + c * ncell, ey_m + (size_t)c * nx * (ny + 1), ey_p + (size_t)c * nx * (ny + 1));
    }
    for (long j = 0; j < ny; ++j) {
      for (long f = 0; f <= nx; ++f) {
        double a[4], b[4], h[4];
        for (int c = 0; c < m; ++c) {
          a[c] = ex_m[(size_t)c * ny * (nx + 1) + j * (nx + 1) + f];
          b[c] = ex_p[(size_t)c * ny * (nx + 1) + j * (nx + 1) + f];
        }
        lf_flux(pb, 0, a, b, alpha[0], h);
        for (int c = 0; c < m; ++c) F[(size_t)c * (nx + 1) + f] = h[c];
      }
      for (int c = 0; c < m; ++c)
        for (long i = 0; i < nx; ++i)
          L[c * ncell + j * nx + i] = -(F[(size_t)c * (nx + 1) + i + 1] - F[(size_t)c * (nx + 1) + i]) / dx;
    }
    for (long i = 0; i < nx; ++i) {
      for (long f = 0; f <= ny; ++f) {
        double a[4], b[4], h[4];
        for (int c = 0; c < m; ++c) {
          a[c] = ey_m[(size_t)c * nx * (ny + 1) + i * (ny + 1) + f];
          b[c] = ey_p[(size_t)c * nx * (ny + 1) + i * (ny + 1) + f];
        }
        lf_flux(pb, 1, a, b, alpha[1], h);
        for (int c = 0; c < m; ++c) F[(size_t)c * (ny + 1) + f] = h[c];
      }
      for (int c = 0; c < m; ++c)
        for (long j = 0; j < ny; ++j)
          L[c * ncell + j * nx + i] =
              L[c * ncell + j * nx + i] - (F[(size_t)c * (ny + 1) + j + 1] - F[(size_t)c * (ny + 1) + j]) / dy;
    }
    free(ex_m);
    free(ex_p);
    free(ey_m);
    free(ey_p);
    free(line);
    free(vm);
    free(vp);
    free(F);
    return NPO_OK;
  }
  const int charwise = pb->charwise && pb->flux == NPO_EULER;
  /* x sweep: every row j */
  for (long j = 0; j < ny; ++j) {
    if (charwise) {
      const double* rows[4];
      for (int c = 0; c < m; ++c) rows[c] = u + c * ncell + j * nx;
      rc = char_line_states(pb, 0, rows, nx, vm, vp);
      if (rc) break;
    } else {
      for (int c = 0; c < m; ++c) {
        for (long i = 0; i < nx; ++i) line[i] = u[c * ncell + j * nx + i];
        npo_line_states(pb, line, nx, vm + (size_t)c * (nx + 1), vp + (size_t)c * (nx + 1), NULL, NULL);
      }
    }
    for (long f = 0; f <= nx; ++f) {
      double a[4], b[4], h[4];
      for (int c = 0; c < m; ++c) {
        a[c] = vm[(size_t)c * (nx + 1) + f];
        b[c] = vp[(size_t)c * (nx + 1) + f];
      }
      lf_flux(pb, 0, a, b, alpha[0], h);
      for (int c = 0; c < m; ++c) F[(size_t)c * (nx + 1) + f] = h[c];
    }
    for (int c = 0; c < m; ++c)
      for (long i = 0; i < nx; ++i)
        L[c * ncell + j * nx + i] = -(F[(size_t)c * (nx + 1) + i + 1] - F[(size_t)c * (nx + 1) + i]) / dx;
  }
  if (pb->dim == 2 && rc == NPO_OK) {
    /* y sweep: every column i, added to the x contribution */
    double* col = charwise ? (double*)malloc(sizeof(double) * (size_t)ny * (size_t)m) : NULL;
    for (long i = 0; i < nx; ++i) {
      if (charwise) {
        const double* cols[4];
        for (int c = 0; c < m; ++c) {
          for (long j = 0; j < ny; ++j) col[(size_t)c * ny + j] = u[c * ncell + j * nx + i];
          cols[c] = col + (size_t)c * ny;
        }
        rc = char_line_states(pb, 1, cols, ny, vm, vp);
        if (rc) break;
      } else {
        for (int c = 0; c < m; ++c) {
          for (long j = 0; j < ny; ++j) line[j] = u[c * ncell + j * nx + i];
          npo_line_states(pb, line, ny, vm + (size_t)c * (ny + 1), vp + (size_t)c * (ny + 1), NULL, NULL);
        }
      }
      for (long f = 0; f <= ny; ++f) {
        double a[4], b[4], h[4];
        for (int c = 0; c < m; ++c) {
          a[c] = vm[(size_t)c * (ny + 1) + f];
          b[c] = vp[(size_t)c * (ny + 1) + f];
        }
        lf_flux(pb, 1, a, b, alpha[1], h);
        for (int c = 0; c < m; ++c) F[(size_t)c * (ny + 1) + f] = h[c];
      }
      for (int c = 0; c < m; ++c)
        for (long j = 0; j < ny; ++j)
          L[c * ncell + j * nx + i] =
              L[c * ncell + j * nx + i] - (F[(size_t)c * (ny + 1) + j + 1] - F[(size_t)c * (ny + 1) + j]) / dy;
    }
    free(col);
  }
  free(line);
  free(vm);
  free(vp);
  free(F);
  return rc;
}

/* Time step: dt = CFL dx / alpha in 1D, CFL / (alpha_x/dx + alpha_y/dy) in 2D, clipped to
 * the remaining time; a positive dt_fixed replaces the CFL rule (used to reproduce the
 * accuracy tables without time error). */
static double time_step(const npo_problem* pb, const double alpha[2], double remaining) {
  double dt;
  const double dx = (pb->x1 - pb->x0) / (double)pb->nx;
  if (pb->dt_fixed > 0.0) {
    dt = pb->dt_fixed;
  } else if (pb->dim == 1) {
    dt = pb->cfl * dx / alpha[0];
  } else {
    const double dy = (pb->y1 - pb->y0) / (double)pb->ny;
    dt = pb->cfl / (alpha[0] / dx + alpha[1] / dy);
  }
  if (dt > remaining) dt = remaining;
  return dt;
}

static int finite_and_physical(const npo_problem* pb, const double* u) {
  double alpha[2];
  return npo_alpha(pb, u, alpha);
}

/* ------------------------------------------------------------------------------------ */
/* One step of the third-order TVD (SSP) Runge-Kutta method of Shu and Osher, which the   */
/* paper uses for time integration (Section 5.1):                                         */
/*   u1 = un + dt L(un);  u2 = 3/4 un + 1/4 (u1 + dt L(u1));                              */
/*   un+1 = 1/3 un + 2/3 (u2 + dt L(u2)).                                                 */
/* Reading (rounding): the last stage is formed as the equal value                        */
/*   un+1 = u2 + (1/3 (un - u2) + 2/3 dt L(u2)).                                          */
/* In double, fl(1/3) + fl(2/3) = 1 - 2^-54, so the printed form would shrink the sum of   */
/* the cell averages by that factor every step, while the finite-volume update conserves  */
/* it exactly.  In the rearranged form the two weights multiply only quantities whose     */
/* sums over a periodic grid vanish, and no systematic loss remains.  The 3/4, 1/4 weights */
/* of the second stage are exact in binary and are used as printed.                       */
/* dt comes from the alpha of un.  On error the state and t are left unchanged.           */
/* ------------------------------------------------------------------------------------ */
int npo_step(const npo_problem* pb, double* u, double T, double* t, double* dt_out) {
  int rc = validate(pb);
  if (rc) return rc;
  const long ny = pb->dim == 2 ? pb->ny : 1;
  const size_t n = (size_t)pb->ncomp * (size_t)(pb->nx * ny);
  double* L = (double*)malloc(sizeof(double) * n);
  double* u1 = (double*)malloc(sizeof(double) * n);
  double* u2 = (double*)malloc(sizeof(double) * n);
  double alpha[2], dt;
  rc = npo_rhs(pb, u, L, alpha);
  if (rc) goto done;
  dt = time_step(pb, alpha, T - *t);
  for (size_t k = 0; k < n; ++k) u1[k] = u[k] + dt * L[k];
  rc = npo_rhs(pb, u1, L, NULL);
  if (rc) goto done;
  for (size_t k = 0; k < n; ++k) u2[k] = 0.75 * u[k] + 0.25 * (u1[k] + dt * L[k]);
  rc = npo_rhs(pb, u2, L, NULL);
  if (rc) goto done;
  for (size_t k = 0; k < n; ++k) u1[k] = u2[k] + (1.0 / 3.0 * (u[k] - u2[k]) + 2.0 / 3.0 * (dt * L[k]));
  rc = finite_and_physical(pb, u1);
  if (rc) goto done;
  memcpy(u, u1, sizeof(double) * n);
  *t = *t + dt;
  if (dt_out) *dt_out = dt;
done:
  free(L);
  free(u1);
  free(u2);
  return rc;
}

/* Run to T: steps until T - t <= 1e-12 max(1, |T|) or max_steps steps were taken. */
int npo_solve(const npo_problem* pb, double* u, double T, long max_steps, double* t, long* nsteps) {
  int rc = validate(pb);
  if (rc) return rc;
  double tol = 1e-12 * (fabs(T) > 1.0 ? fabs(T) : 1.0);
  long k = 0;
  while (T - *t > tol && (max_steps < 0 || k < max_steps)) {
    rc = npo_step(pb, u, T, t, NULL);
    if (rc) break;
    ++k;
  }
  if (nsteps) *nsteps = k;
  return rc;
}

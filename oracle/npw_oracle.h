/*
 * npw_oracle.h -- declarations of the FP64 CPU oracle (test infrastructure only; see
 * npw_oracle.c).  This header belongs to the oracle alone: the HIP library has its own.
 */
#ifndef NPW_ORACLE_H
#define NPW_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { NPO_OK = 0, NPO_EINVAL = -1, NPO_ENONFINITE = -4, NPO_ENONPHYSICAL = -5 };
enum { NPO_ADVECTION = 0, NPO_BURGERS = 1, NPO_EULER = 2 };
enum { NPO_PERIODIC = 0, NPO_TRANSMISSIVE = 1 };
enum {
  NPO_RBF_WENO5 = 0, NPO_WENO5_JS = 1, NPO_RBF_ENO3 = 2, NPO_ENO3 = 3, /* k = 3 */
  NPO_RBF_WENO3 = 4, NPO_WENO3_JS = 5, NPO_RBF_ENO2 = 6, NPO_ENO2 = 7, /* k = 2 */
  NPO_RBF_ENO2_2D = 8 /* k = 2, Section 6: shape parameter from the five-cell cross (2D only) */
};
enum { NPO_SWITCH_MONOTONE = 0, NPO_SWITCH_OFF = 1 };

typedef struct {
  int dim;   /* 1 or 2 */
  int flux;  /* NPO_ADVECTION, NPO_BURGERS, NPO_EULER */
  int ncomp; /* 1 (scalar), 3 (1D Euler), 4 (2D Euler) */
  int bc;    /* NPO_PERIODIC or NPO_TRANSMISSIVE, all sides */
  long nx, ny;
  double x0, x1, y0, y1;
  double speed_x, speed_y; /* advection velocity */
  double gamma;            /* Euler ratio of specific heats */
  double cfl, eps_weno, eps_m;
  int recon;       /* NPO_* reconstruction (k = 3 or k = 2; the non-RBF ones have eta = 0) */
  int switch_mode; /* NPO_SWITCH_MONOTONE or NPO_SWITCH_OFF */
  double dt_fixed; /* > 0: fixed time step instead of the CFL rule */
  int charwise;    /* Euler only: 1 = reconstruct characteristic fields (Roe average), 0 = components */
} npo_problem;

void npo_table3(double c[12], double p[12]);
double npo_row_value(int r, double w0, double w1, double w2, double eta);
double npo_eta(double um1, double u0, double up1, double up2, double eps_m);
int npo_monotone_flag(double um1, double u0, double up1);
void npo_beta(const double u5[5], double beta[3]);
double npo_recon_minus(const double u5[5], double eta_right, double eps);
double npo_recon_plus(const double u5[5], double eta_left, double eps);
int npo_eno_stencil(const double u5[5]);
double npo_eno_minus(const double u5[5], double eta_right);
double npo_eno_plus(const double u5[5], double eta_left);
double npo_row2_value(int r, double w0, double w1, double eta);
double npo_eta2(double um1, double u0, double up1, double eps_m);
double npo_weno3_minus(const double u3[3], double eta, double eps);
double npo_weno3_plus(const double u3[3], double eta, double eps);
int npo_eno2_stencil(const double u3[3]);
double npo_eno2_minus(const double u3[3], double eta);
double npo_eno2_plus(const double u3[3], double eta);
void npo_line_states(const npo_problem* pb, const double* line, long n, double* vminus,
                     double* vplus, double* eta_out, int* flag_out);
int npo_char_basis(const npo_problem* pb, int dir, const double* UL, const double* UR, double* Lm, double* Rm,
                   double* lam);
int npo_char_interface(const npo_problem* pb, int dir, const double* U6, double* vm, double* vp);
double npo_cross_edge(const double w3[3], const double t2[2], int right_edge, int use_switch, double eps_m);
int npo_face_states(const npo_problem* pb, int dir, const double* field, double* vm, double* vp);
int npo_alpha(const npo_problem* pb, const double* u, double alpha[2]);
int npo_rhs(const npo_problem* pb, const double* u, double* L, double alpha_out[2]);
int npo_step(const npo_problem* pb, double* u, double T, double* t, double* dt_out);
int npo_solve(const npo_problem* pb, double* u, double T, long max_steps, double* t, long* nsteps);

#ifdef __cplusplus
}
#endif
#endif

/*
 * npweno.h -- C ABI of the MI355X (gfx950) non-polynomial ENO/WENO finite-volume library.
 *
 * The library solves the hyperbolic conservation law u_t + div F(u) = 0 (Section 1 of Guo &
 * Jung, "Non-polynomial ENO and WENO finite volume methods for hyperbolic conservation laws",
 * arXiv:1602.00182) on a uniform grid of cell averages (Section 2) with:
 *   - the k = 3 WENO reconstruction of eq. (weno_re) whose substencil coefficients are the
 *     multiquadric-RBF perturbation of Table 3 (polynomial part + eta * perturbation part),
 *   - the shape parameter eta = eps^2 dx^2 of the Table 3 caption, one per cell interface,
 *     evaluated in double precision,
 *   - the monotone-polynomial switch of Section 4 (eqs. root_value, adaptation) that sets
 *     eta = 0 next to non-monotone 3-cell windows,
 *   - Jiang-Shu nonlinear weights (eps_weno, Section 2), the global Lax-Friedrichs flux and
 *     flux differencing of Section 5.1 (eq. PDE1), and the third-order TVD Runge-Kutta
 *     method (Section 5.1),
 *   - in 2D, the dimension-by-dimension finite-volume form of Section 7 (eq. 2DIntegral) with
 *     one midpoint quadrature point per face.
 * The same kernels also run the ENO selection of Section 2, the k = 2 reconstructions of Table 2,
 * the two-dimensional k = 2 reconstruction of Section 6, and (an extension) characteristic-wise
 * reconstruction of the Euler equations.
 * All compute runs in HIP kernels on the device; nothing falls back to the CPU.
 *
 * Conventions for every entry point:
 *   - Return value: NPW_OK (0) or a negative NPW_E* code; nothing throws across the ABI.
 *   - Device pointers are plain HIP device addresses (e.g. torch tensor data_ptr()); host
 *     pointers are ordinary process memory.  The caller keeps ownership of every buffer it
 *     passes; the library copies what it needs.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  All library work is ordered on
 *     the solver's stream; calls that return host-visible results synchronize that stream.
 *   - State layout (both directions): component-major structure of arrays.  1D:
 *     u[c*nx + i]; 2D: u[(c*ny + j)*nx + i], c = 0..ncomp-1.  Element type is double for
 *     NPW_FP64 and float for NPW_FP32.  Euler states are conservative: (rho, rho*u, E) in 1D
 *     and (rho, rho*u, rho*v, E) in 2D.
 *   - A solver is used by one host thread at a time.
 */
#ifndef NPWENO_H
#define NPWENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPW_ABI_VERSION 2

enum {
  NPW_OK = 0,
  NPW_EINVAL = -1,       /* bad argument; nothing was allocated or changed */
  NPW_ENOMEM = -2,       /* device or host allocation failed */
  NPW_EHIP = -3,         /* a HIP runtime call failed */
  NPW_ENONFINITE = -4,   /* a cell average became NaN/Inf; state and t stay at the last good step */
  NPW_ENONPHYSICAL = -5, /* Euler density or pressure <= 0; state and t stay at the last good step */
  NPW_EBUSY = -6,        /* serving: request not finished yet */
  NPW_ENOTFOUND = -7,    /* serving: unknown request id */
  NPW_ESCRATCH = -8      /* npweno_rhs_noalloc: the grid needs more scratch than its fixed array */
};

enum { NPW_ADVECTION = 0, NPW_BURGERS = 1, NPW_EULER = 2 };  /* flux type */
enum { NPW_PERIODIC = 0, NPW_TRANSMISSIVE = 1 };             /* boundary, all sides */
enum { NPW_FP64 = 0, NPW_FP32 = 1 };  /* bulk precision; eta, the switch test, dt and t are always FP64 */
/* Reconstruction.  k = 3 (Table 3): RBF-WENO5 (the hot path), WENO5-JS (eta forced to zero),
 * RBF-ENO3 (one stencil chosen by Newton divided differences, Section 2, perturbed with the same
 * eta and switch) and ENO3 (its eta = 0 limit).  k = 2 (Table 2, shape parameter of Section 3.2
 * per cell and edge): RBF-WENO3, WENO3-JS, RBF-ENO2 and ENO2; their Section 4 switch zeroes both
 * edge parameters of a cell whose three-cell window is not monotone.  NPW_RBF_ENO2_2D (2D only,
 * Section 6): the ENO2 edge value perturbed with a shape parameter from the five-cell cross of the
 * cell (second differences along and across the sweep over the printed edge estimate). */
enum {
  NPW_RBF_WENO5 = 0, NPW_WENO5_JS = 1, NPW_RBF_ENO3 = 2, NPW_ENO3 = 3,
  NPW_RBF_WENO3 = 4, NPW_WENO3_JS = 5, NPW_RBF_ENO2 = 6, NPW_ENO2 = 7,
  NPW_RBF_ENO2_2D = 8
};
enum { NPW_SWITCH_MONOTONE = 0, NPW_SWITCH_OFF = 1 };        /* Section 4 switch on / off */
/* Variables the Euler equations are reconstructed in.  Component-wise is the scheme as the paper
 * applies it to systems (Example 4).  Characteristic-wise (an extension) projects each
 * interface's six-cell window on the left eigenvectors of the flux Jacobian at the Roe average of
 * the two adjacent cells, reconstructs every characteristic field with the scalar scheme (its own
 * shape parameter and switch) and maps the edge states back with the right eigenvectors. */
enum { NPW_COMPONENTWISE = 0, NPW_CHARACTERISTIC = 1 };

typedef struct {
  int32_t abi_version; /* must be NPW_ABI_VERSION */
  int32_t dim;         /* 1 or 2 */
  int32_t flux;        /* NPW_ADVECTION, NPW_BURGERS or NPW_EULER */
  int32_t ncomp;       /* 1 for scalar fluxes, 3 for 1D Euler, 4 for 2D Euler */
  int32_t bc;          /* NPW_PERIODIC or NPW_TRANSMISSIVE (copy of the edge cell) */
  int32_t precision;   /* NPW_FP64 or NPW_FP32 */
  int32_t recon;       /* NPW_RBF_WENO5 .. NPW_RBF_ENO2_2D (k = 3 or k = 2, see above) */
  int32_t switch_mode; /* NPW_SWITCH_MONOTONE or NPW_SWITCH_OFF */
  int64_t nx, ny;      /* cells per direction; ny is ignored (treated as 1) in 1D.  Limits:
                        * 1D ncomp * nx <= 2^31 - 2^16; 2D nx <= 2^30, ny <= 262140 */
  double x0, x1, y0, y1;   /* domain; y0, y1 ignored in 1D */
  double speed_x, speed_y; /* advection velocity (NPW_ADVECTION) */
  double gamma;            /* ratio of specific heats (NPW_EULER), > 1 */
  double cfl;              /* dt = cfl*dx/alpha (1D), cfl/(alpha_x/dx + alpha_y/dy) (2D) */
  double eps_weno;         /* epsilon of the nonlinear weights, Section 2 (1e-6) */
  double eps_m;            /* eps_M of the eta denominator (> 0), added with its sign (1e-12) */
  double dt_fixed;         /* > 0: use this dt instead of the CFL rule (accuracy studies) */
  int32_t variables;       /* NPW_COMPONENTWISE or NPW_CHARACTERISTIC (NPW_EULER only) */
  int32_t reserved;        /* must be 0 */
} npw_params;

typedef struct {
  double t;          /* current time */
  int64_t nsteps;    /* RK3 steps taken since create / write */
  double alpha[2];   /* Lax-Friedrichs alpha of the current state (x, y) */
  double mass[4];    /* sum over cells of u_c * cell area, per component (FP64 on device) */
  int32_t err;       /* sticky error code of the last failing step (0 if none) */
  int32_t err_stage; /* RK stage (1..3) where it was detected, 0 at the initial state */
} npw_stats;

typedef struct npw_solver npw_solver;  /* opaque; owns all device state */
typedef struct npw_server npw_server;  /* opaque; serving loop */

int npweno_abi_version(void);
const char* npweno_strerror(int code);

/* Fill *p with the defaults: abi_version, dim 1, advection with speed 1 on [-1,1], periodic,
 * FP64, RBF-WENO5 with the monotone switch, cfl 0.5, eps_weno 1e-6, eps_m 1e-12, gamma 1.4. */
void npweno_default_params(npw_params* p);

/* Create a solver for one grid and copy the initial cell averages u0 (layout above, element
 * type from p->precision; device memory if u0_on_device, else host memory).  t starts at 0.
 * Validates every parameter before allocating: NPW_EINVAL on a bad value, dimension/ncomp/flux
 * mismatch or NULL pointer.  Returns NPW_ENONFINITE / NPW_ENONPHYSICAL (and no solver) if u0
 * already violates those conditions. */
int npweno_create(const npw_params* p, const void* u0, int u0_on_device, void* hip_stream,
                  npw_solver** out);

/* One SSP-RK3 step (Section 5.1) with dt = min(CFL rule, t_final - t); does nothing when
 * t_final - t <= 1e-12 max(1, |t_final|).  *dt_taken (may be NULL) receives the step taken
 * (0 if none).  Synchronizes the stream. */
int npweno_step(npw_solver* s, double t_final, double* dt_taken);

/* Advance to t_final (same clipping and stopping rule) or until max_steps more steps were taken
 * (max_steps < 0: no limit).  Steps run as captured HIP graphs of several steps each; the
 * host only polls completion between graph replays.  stats may be NULL. */
int npweno_solve(npw_solver* s, double t_final, int64_t max_steps, npw_stats* stats);

/* Semi-discrete right-hand side L(u) = -(F_{i+1/2} - F_{i-1/2})/dx [- (G_{j+1/2}-G_{j-1/2})/dy]
 * of eq. (PDE1) for the current state, with alpha of the current state; written to L_out in
 * the state layout (device pointer if out_on_device).  Synchronizes the stream. */
int npweno_rhs(npw_solver* s, void* L_out, int out_on_device);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): npweno_rhs for a state the caller holds, with no
 * solver and no allocation.  Writes L(u) of eq. (PDE1) (1D) or eq. (2DIntegral) (2D), with the
 * Lax-Friedrichs alpha of u, to L_out.  It only enqueues kernels on hip_stream (NULL = the
 * default stream) and returns without waiting; it calls no hipMalloc, hipFree or memcpy.
 *   p           as for npweno_create (one grid, 1D or 2D; cfl and dt_fixed are not used).
 *   u           device pointer, the state in the layout of npweno_create (element type from
 *               p->precision); read only.
 *   L_out       device pointer, same layout and size; must not overlap u.
 *   status_dev  optional device pointer to one int32: receives NPW_OK, or NPW_ENONFINITE /
 *               NPW_ENONPHYSICAL when u fails the state check (then L_out is left unchanged).
 * Launch shape: NPW_BLOCK (1D, default 256) or NPW_TILE2D (2D, default 4 = 62 x 8 cells); the
 * results equal npweno_rhs's with the same shape.
 * Scratch: the instance record, the spread alpha entries and the state check's partial records
 * live in one fixed device array of the library (78 336 bytes, one copy per GPU, held until the
 * process ends).  Every grid within npweno_create's limits fits; a grid that would not returns
 * NPW_ESCRATCH.  All calls on one GPU share that array: calls that overlap on one GPU (different
 * streams or host threads) race, so a caller orders them on one stream.
 * Returns NPW_EINVAL for a bad parameter, a NULL pointer or overlapping buffers, NPW_EHIP if a
 * launch fails; errors of the state itself arrive through status_dev. */
int npweno_rhs_noalloc(const npw_params* p, const void* u, void* L_out, void* hip_stream, int32_t* status_dev);

/* Copy the current state out (device pointer if out_on_device).  Synchronizes the stream. */
int npweno_read(const npw_solver* s, void* u_out, int out_on_device);

/* Replace the state (same layout/type as create) and set the time to t; resets the step count
 * and any sticky error.  Used to restart from a checkpoint. */
int npweno_write(npw_solver* s, const void* u, int on_device, double t);

/* Time, step count, alpha and per-component sums of the current state. */
int npweno_get_stats(const npw_solver* s, npw_stats* stats);

void npweno_destroy(npw_solver* s);

/* ---- Batches ---------------------------------------------------------------------------- */
/* `count` independent instances that share precision, flux type, ncomp and dim (each may have
 * its own nx, domain, boundary, cfl, eps_weno, eps_m, recon, switch, speed, gamma).  Their states
 * are packed back to back in the library's buffers and every RK stage of every instance runs
 * in one launch of the stage kernel (a tile table maps workgroups to (instance, tile)); each
 * instance keeps its own alpha, dt, t and error, exactly as if it were solved alone (results
 * are bit-identical to single-instance solves).  u0[b] points to instance b's initial state
 * (layout of npweno_create).  The single-instance calls above act on every instance of a batch
 * with one common t_final; npweno_read copies all states back to back. */
int npweno_create_batch(const npw_params* params, int32_t count, const void* const* u0, int on_device,
                        void* hip_stream, npw_solver** out);
/* Advance instance b towards t_final[b].  max_steps bounds the RK steps launched (< 0: none).
 * An instance that fails stays at its last good step with its error in per_instance[b].err; the
 * others continue.  Returns the first error seen, or NPW_OK.  per_instance may be NULL. */
int npweno_solve_batch(npw_solver* s, const double* t_final, int64_t max_steps, npw_stats* per_instance);
int npweno_read_instance(const npw_solver* s, int32_t index, void* u_out, int out_on_device);
int npweno_get_stats_instance(const npw_solver* s, int32_t index, npw_stats* stats);
int npweno_instance_count(const npw_solver* s);
/* Launch shape the solver uses for its stage kernel (picked at create by the autotuner, or set by
 * NPW_BLOCK / NPW_TILE2D): *block_1d = threads per workgroup of the 1D kernel (64, 128, 256 or 512),
 * *tile_x, *tile_y = interior cells per workgroup of the 2D kernel (0 for a 1D solver; a tile_y
 * above 8 is a column strip that the workgroup walks 4 rows at a time, 2D Euler only), and
 * *lds_shared = 1 when the 2D kernel shares per-cell weight denominators through LDS, 0 when every
 * interface recomputes them (always 0 for characteristic-wise 2D, always 1 in 1D).  Any output pointer may be NULL.  Host-only;
 * returns NPW_EINVAL for a NULL solver. */
int npweno_launch_shape(const npw_solver* s, int32_t* block_1d, int32_t* tile_x, int32_t* tile_y,
                        int32_t* lds_shared);

/* ---- Serving (continuous batching) -------------------------------------------------------- */
/* A request loop for mixed 1D solves.  All requests share one device arena of
 * hbm_budget_bytes (split into the three state buffers) and max_slots slots per pool (one pool
 * each for advection, Burgers, component-wise Euler and characteristic-wise Euler).
 * Submitted requests wait in a FIFO queue; npw_server_pump admits the head of the queue as
 * soon as a slot and a large enough arena range are free, then advances every running request
 * by `steps` RK steps with one launch of the batched stage kernel per pool and stage
 * (their work overlaps on the device), and retires the finished ones.  A request that reaches
 * its t_final within a pump stops there and idles for the rest of it.  A request's result is
 * bit-identical to solving it alone with npweno_create/npweno_solve in the same precision.
 * Requests never fail one another: a request that becomes non-finite or non-physical is
 * retired with its error and last good state. */
/* The pools step with workgroups of 512 threads (NPW_BLOCK = 64, 128, 256 or 512 overrides).
 * max_slots in [1, 65536]; precision NPW_FP32 or NPW_FP64 for every request; hbm_budget_bytes at
 * least 3 * 256 elements.  hip_stream is not used: requests enter and leave as host copies, and the
 * server works on private streams of its own (pass NULL). */
int npw_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t precision, void* hip_stream,
                      npw_server** out);
/* Queue a 1D solve to t_final (params->precision must equal the server's).  The library copies
 * u0_host.  NPW_EINVAL if the request could never fit in the arena. */
int npw_server_submit(npw_server* srv, const npw_params* params, const void* u0_host, double t_final,
                      uint64_t* req_id);
/* Admit, advance every running request by exactly `steps` (>= 1) RK steps (graphs of 256, 64,
 * 16, 4 and 1 steps, largest first), retire.  Reports the number of running and queued requests
 * (either pointer may be NULL).  Returns after the device work of the pump completed. */
int npw_server_pump(npw_server* srv, int32_t steps, int32_t* n_running, int32_t* n_queued);
/* NPW_EBUSY until the request finished; then copies its final state (the last good state and
 * the error code if it failed) and its stats. */
int npw_server_poll(npw_server* srv, uint64_t req_id, void* u_out_host, npw_stats* stats);
/* Host steady-clock times (seconds) of submission, admission and completion (any output pointer
 * may be NULL).  Returns NPW_EBUSY until the request finished, NPW_OK after; copies no state. */
int npw_server_times(const npw_server* srv, uint64_t req_id, double* t_submit, double* t_admit, double* t_done);
/* Drop the stored result of a finished request. */
int npw_server_release(npw_server* srv, uint64_t req_id);
void npw_server_destroy(npw_server* srv);

#ifdef __cplusplus
}
#endif
#endif

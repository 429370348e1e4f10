/*
 * hb_ugks.h -- C ABI of the MI355X HB-UGKS pseudo-step library.
 *
 * The library advances the time-domain harmonic-balance unified gas-kinetic
 * scheme (HB-UGKS, arXiv 2605.03479, Sec. 2) for one 2-D cavity case on one
 * AMD Instinct GPU (gfx950).  The state is the macroscopic W and the reduced
 * distributions (h, b) of Sec. 2.1 (Eqs. 7-8) at every cell, discrete velocity
 * and sub-time level n = 0..2*NH (Eq. 12); one pseudo step (Sec. 2.4,
 * Eqs. 29-33) updates all of them at once.
 *
 * Units are the paper's nondimensional ones with rho0 = H = sqrt(2 R T0) = 1:
 * velocities in sqrt(2 R T0), temperatures in T0, lengths in H, omega = St
 * (Eq. 37), mu(T0) from Kn by Eq. (36).
 *
 * Conventions for every entry point:
 *   - return 0 (HB_OK) on success, a negative HB_E* code on failure;
 *     hb_ugks_strerror() names the code;
 *   - host pointers are owned by the caller and only read/written during the
 *     call; the handle owns all device memory it allocates (hipMalloc);
 *   - a handle is not thread-safe; distinct handles are independent;
 *   - work is queued on the handle's stream (the one given at creation, or
 *     the null stream); calls that return host data synchronise that stream.
 * Host array layouts (row-major, last index fastest):
 *   W[c][n][4]  (rho, rho U, rho V, rho E), c = j*nx + i (x fastest)
 *   h, b[c][n][a]  a = iv*M + iu with iu < M along u and iv < M_v along v,
 *                  the 1-D nodes of each axis increasing (hb_vgrid_nodes
 *                  lists them)
 */
#ifndef HB_UGKS_H
#define HB_UGKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HB_OK = 0,
    HB_EINVAL = -1,     /* an argument is out of range (sizes, Kn <= 0, NULL, ...) */
    HB_ENOMEM = -2,     /* device allocation failed or exceeds hbm_budget_bytes */
    HB_ESTATE = -3,     /* call out of order (e.g. pseudo_step before set_case) */
    HB_EDIVERGED = -4,  /* NaN/Inf in the residual: the state is kept for state_out */
    HB_EDEVICE = -5,    /* a HIP runtime call failed, or no gfx950 device */
    HB_ECAPACITY = -6   /* the caller's buffer is too small */
};

typedef enum { HB_FP64 = 0, HB_MIXED = 1 } hb_precision;

typedef struct hb_ugks *hb_handle;

typedef struct {
    int device;               /* HIP device ordinal */
    void *stream;             /* hipStream_t to queue work on; NULL = null stream */
    int precision;            /* hb_precision; HB_MIXED keeps h, b and the per-velocity
                                 flux/source arithmetic in FP32, moments, W and the
                                 residual in FP64 */
    size_t hbm_budget_bytes;  /* 0 = no limit */
} hb_create_opts;

typedef struct {
    double L, H;              /* cavity [0,L] x [0,H] */
    int nx, ny;               /* cells, >= 3 each */
    const double *x_faces;    /* NULL = uniform, else nx+1 increasing coordinates */
    const double *y_faces;    /* NULL = uniform, else ny+1 increasing coordinates */
} hb_geometry;

/* One wall; order bottom (y=0), right (x=L), top (y=H), left (x=0).
 * Tangential velocity is along +x for bottom/top and +y for left/right.
 * Sub-level values follow Eqs. (25)-(26): mean + Re(hat * exp(i omega t_n)). */
typedef struct {
    double ut_mean, ut_hat_re, ut_hat_im;
    double T_mean, T_hat_re, T_hat_im;
} hb_wall;

/* 1-D velocity rules of Sec. 3.1.1 (the grid is their tensor product). */
enum {
    HB_RULE_TRAPEZOID = 0,      /* m equally spaced nodes on [-umax, umax], closed
                                   composite trapezoid weights */
    HB_RULE_GAUSS_HERMITE = 1   /* the m roots of the Hermite polynomial H_m (weight
                                   exp(-u^2), the rest Maxwellian in these units),
                                   weights multiplied by exp(u_k^2) so that sums
                                   approximate plain integrals; umax is ignored and
                                   the largest node takes its place in Eq. (32) */
};

/* Tensor velocity grid (Sec. 3.1.1): m nodes along u and m_v along v (each
 * even, 4..128; m_v = 0 takes m), the trapezoid rule on [-umax, umax] along u
 * and [-vmax, vmax] along v (vmax <= 0 takes umax), or the Gauss-Hermite rule
 * of m, m_v nodes (umax, vmax unused).  m_v < 0 is HB_EINVAL. */
typedef struct {
    int m;
    double umax;
    int rule;                 /* HB_RULE_*; zero-initialised = trapezoid */
    int m_v;                  /* 0 = m (square grid) */
    double vmax;              /* <= 0: umax */
} hb_vgrid;

/* The 1-D nodes u[m] (increasing) and weights w[m] of the rule along u (m,
 * umax, rule); the v axis is the same rule with m_v, vmax in place of m, umax.
 * Host only, no device needed.  Errors: HB_EINVAL (NULL, m odd or out of
 * range, unknown rule, umax <= 0 for the trapezoid). */
int hb_vgrid_nodes(const hb_vgrid *vg, double *u, double *w);

typedef struct {
    double cfl;               /* Eq. (31); default 0.5 */
    int face_dt;              /* Eq. (33): 0 = min of the two cells, 1 = harmonic mean */
    double Pr;                /* Shakhov Prandtl number (Eq. 4); 1 = BGK; default 2/3 */
    double omega_vss;         /* mu ~ T^omega_vss; default 0.81 */
    double alpha_vss;         /* VSS scattering parameter of Eq. (36); default 1 */
    int K_int;                /* internal degrees of freedom (Eq. 3); default 1 */
    int dt_mode;              /* 0 = local pseudo steps (Eqs. 31-32), 1 = global step dt_fixed */
    double dt_fixed;
    int macro_flux_mode;      /* 0 = macro flux of Eq. (24) (C2, C3 parts as analytic Maxwellian
                                 moments); 1 = the velocity sum of the micro flux of Eq. (23) */
    int level_mass;           /* 1 = after every pseudo step scale W, h, b of each level n by
                                 s_n = Mbar / M_n (M_n the level's mass in the cavity, Mbar
                                 their mean).  Not in the paper: a convergence aid.  With local
                                 pseudo steps the level masses drift apart in the transient and
                                 the explicit spectral source (Eq. 29) rotates the difference
                                 between levels without damping it, so the residual stalls in
                                 strongly forced cavities.  Every fixed point of the step has
                                 equal level masses, so s_n = 1 there and the converged result
                                 is the same; 0 = the step as printed.  The residual of Eq. (43)
                                 is the increment before the scaling. */
} hb_numerics;

/* Defaults: cfl 0.5, face_dt 0, Pr 2/3, omega_vss 0.81, alpha_vss 1, K_int 1, dt_mode 0,
 * macro_flux_mode 0, level_mass 1. */
void hb_ugks_default_numerics(hb_numerics *out);

/* Create a handle on opts->device (NULL opts = device 0, null stream, FP64).
 * Errors: HB_EINVAL (out NULL, bad precision), HB_EDEVICE (no such device or
 * not gfx950). */
int hb_ugks_create(const hb_create_opts *opts, hb_handle *out);

/* Define the case and reset the state to the uniform rest Maxwellian
 * (rho = 1, U = 0, T = T0 at every level).  Kn (Eq. 36) and St (Eq. 37) set
 * mu(T0) and omega; n_harmonics = NH gives NT = 2 NH + 1 levels (NT <= 11).
 * walls: 4 entries; num: NULL = defaults.  Allocates the device state.
 * Errors: HB_EINVAL (sizes, Kn <= 0, St < 0, odd m or m_v, non-increasing
 * faces, cfl <= 0, or update tables of 16 NT max(m, m_v) words (8 B in FP64,
 * 4 B mixed) above the 160 KB of LDS), HB_ENOMEM, HB_EDEVICE. */
int hb_ugks_set_case(hb_handle h, const hb_geometry *geo, double Kn, double St, int n_harmonics,
                     const hb_wall walls[4], const hb_vgrid *vg, const hb_numerics *num);

/* Queue nsteps pseudo steps (Sec. 2.4 with the UGKS flux of Sec. 2.2 and the
 * walls of Sec. 2.3) on the handle's stream; returns without synchronising.
 * Errors: HB_ESTATE (no case), HB_EINVAL (nsteps < 0), HB_EDEVICE. */
int hb_ugks_pseudo_step(hb_handle h, int nsteps);

/* Explicit time-domain UGKS, the comparison solver of Sec. 3.1.4: the same
 * flux and update as a pseudo step with one level (n_harmonics = 0, so the
 * spectral term of Eq. 17 vanishes) and one physical step dt_fixed for every
 * cell (numerics dt_mode = 1).  Before each step the walls take their
 * Eqs. (25)-(26) values at the mid-step phase omega (t + dt/2); t starts at 0
 * in set_case and grows by dt_fixed per step.  Queues and returns without
 * synchronising.  A later hb_ugks_pseudo_step keeps the last wall state.
 * Errors: HB_ESTATE (no case, n_harmonics != 0 or dt_mode != 1, or the case
 * belongs to a batch), HB_EINVAL (nsteps < 0), HB_EDEVICE. */
int hb_ugks_td_step(hb_handle h, int nsteps);

/* nsteps time-domain steps (one forcing period when nsteps * dt_fixed =
 * 2 pi / St), then the period residual of Eq. (43), second line: the RMS
 * over cells of W(t_end) - W(t_start) for (rho, rho U, rho V, rho E), into
 * out[4].  Synchronises.  Errors: as hb_ugks_td_step (nsteps < 1 is
 * HB_EINVAL), HB_EDIVERGED (NaN/Inf in any step or in out). */
int hb_ugks_td_period(hb_handle h, int nsteps, double out[4]);

/* Physical time reached by the time-domain steps of this case. */
int hb_ugks_time(hb_handle h, double *t);

/* Residual of the last completed step, Eq. (43): RMS over cells of the
 * level-0 change of (rho, rho U, rho V, rho E).  Synchronises the stream.
 * step_index (may be NULL) receives the number of steps taken.
 * Errors: HB_ESTATE, HB_EDIVERGED (a NaN/Inf in W^{k+1} at any level, or in
 * the residual, in any step since set_case; the residual itself is then NaN). */
int hb_ugks_residual(hb_handle h, double out[4], long *step_index);

/* Fourier coefficients of Eq. (40), qhat_k = (1/NT) sum_n q_n exp(-i k omega t_n),
 * k = 0..NH, of the variables selected by var_mask bits:
 *   0 rho, 1 U, 2 V, 3 T/T0 (from W), 4 P_xy (Eq. 39, from h about U_n, V_n),
 *   5 q_x, 6 q_y (Eq. 6 from h, b about U_n, V_n).
 * re/im layout [selected var in bit order][k][c]; capacity = doubles in each
 * of re and im.  Synchronises.  Errors: HB_ESTATE, HB_ECAPACITY, HB_EINVAL. */
int hb_ugks_harmonics_out(hb_handle h, unsigned var_mask, double *re, double *im, size_t capacity);

/* hb_ugks_harmonics_out for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same result, with the work arrays in a static device array
 * of 4 Mi doubles (32 MiB) that each GPU holds from the first call until the
 * process ends, instead of the handle's own scratch.  Allocates no device
 * memory (no hipMalloc, hipFree or allocating library call).  A case needs
 * nc*NT*7 + 14*(NH+1)*nc doubles of it: 128 x 128 cells at NT = 11 use 2.6 Mi.
 * Every call on one GPU uses that GPU's one array, so calls that overlap on a
 * GPU (other threads, other handles) race; every array element a call reads
 * is written by that call first.  Synchronises the handle's stream.
 * Errors: as hb_ugks_harmonics_out, and HB_ENOMEM when the case needs more
 * scratch than the static array holds. */
int hb_ugks_harmonics_out_noalloc(hb_handle h, unsigned var_mask, double *re, double *im, size_t capacity);

/* Wall average of one Fourier coefficient, as in the normalised lid
 * amplitudes of Eqs. (41)-(42): <qhat_k>_wall = (1/L_w) sum_i qhat_k,i ds_i
 * over the cells adjacent to the wall (0 bottom, 1 right, 2 top, 3 left), ds_i
 * their width along it.  var numbers the variables as in
 * hb_ugks_harmonics_out (0 rho ... 4 P_xy ... 6 q_y), 0 <= k <= NH; qhat_k is
 * the coefficient of Eq. (40), so a real signal a cos(omega t) has
 * |qhat_1| = a/2.  out[0] = Re, out[1] = Im.  Synchronises.
 * Errors: HB_EINVAL, HB_ESTATE, HB_ENOMEM, HB_EDEVICE. */
int hb_ugks_wall_harmonic(hb_handle h, int wall, int var, int k, double out[2]);

/* Copy the state out / in (FP64, host layouts above; any pointer may be NULL
 * to skip that array).  capacity = doubles available in h (and in b); W needs
 * nc*NT*4.  In HB_MIXED, h and b are converted.  Synchronises.
 * Errors: HB_ESTATE, HB_ECAPACITY. */
int hb_ugks_state_out(hb_handle h, double *W, double *hh, double *bb, size_t capacity);
int hb_ugks_state_in(hb_handle h, const double *W, const double *hh, const double *bb);

/* Sizes of the current case: out[0..5] = nx, ny, nc, M (nodes along u), nv
 * (= M * M_v), NT. */
int hb_ugks_sizes(hb_handle h, int out[6]);

/* Device bytes held by the handle. */
size_t hb_ugks_device_bytes(hb_handle h);

/* Per-kernel timing: while enabled, every pseudo step records HIP events
 * around each of its kernels on the handle's stream (no host synchronisation
 * per step).  hb_ugks_kernel_times synchronises on the last event and fills,
 * per kernel of the step in launch order, its name (static string), number of
 * timed launches and summed milliseconds since timing was enabled; it returns
 * the number of kernels (>= 0) or a negative HB_E* code.  Enabling (or
 * disabling) resets the sums.
 * Errors: HB_ESTATE, HB_ECAPACITY (capacity below the number of kernels). */
int hb_ugks_enable_timing(hb_handle h, int on);
int hb_ugks_kernel_times(hb_handle h, const char **names, long *launches, double *ms, int capacity);

void hb_ugks_destroy(hb_handle h);
const char *hb_ugks_strerror(int status);

/* ------------------------------------------------------------------ batched form
 * Many cases, each the method above (Sec. 2) on its own geometry, velocity
 * grid, N_H, Kn, St and walls, advanced together.  One batch step advances
 * every active case by one pseudo step with one kernel launch per phase of
 * the step over all of them (moments, faces, cells, local steps, residuals;
 * the update once per (precision, N_T) group), recorded into a HIP graph and
 * replayed; a case's arithmetic, including its residual summation order, is
 * that of the single-case path, so a case gives the same result alone and in a
 * batch.  Each case is an hb_handle (queries above apply to it) whose device
 * memory is carved from the batch's pool: admission is by device footprint.
 * A batch is not thread-safe; its work is queued on its own stream. */
typedef struct hb_batch *hb_batch_handle;

/* Create a batch on opts->device with a device pool of pool_bytes (0: the
 * opts->hbm_budget_bytes, else 90 % of the free device memory) and room for
 * max_cases cases.  opts->stream NULL: the batch creates its own stream.
 * Errors: HB_EINVAL, HB_EDEVICE, HB_ENOMEM. */
int hb_batch_create(const hb_create_opts *opts, size_t pool_bytes, int max_cases, hb_batch_handle *out);

/* Device bytes a case of this shape takes from the pool (no allocation). */
int hb_batch_case_bytes(hb_batch_handle b, int precision, const hb_geometry *geo, int n_harmonics,
                        const hb_vgrid *vg, size_t *bytes);

/* Add a case (arguments as hb_ugks_set_case, plus its precision), reset to
 * rest; it is active.  *case_id receives its slot.  Errors: HB_EINVAL,
 * HB_ENOMEM (does not fit the pool now), HB_ECAPACITY (no free slot). */
int hb_batch_add(hb_batch_handle b, int precision, const hb_geometry *geo, double Kn, double St, int n_harmonics,
                 const hb_wall walls[4], const hb_vgrid *vg, const hb_numerics *num, int *case_id);

/* Remove a case and return its memory to the pool (synchronises). */
int hb_batch_remove(hb_batch_handle b, int case_id);

/* Inactive cases keep their state and are not stepped. */
int hb_batch_set_active(hb_batch_handle b, int case_id, int active);

/* Queue nsteps batch steps (asynchronous). */
int hb_batch_step(hb_batch_handle b, int nsteps);

/* Latest residual (Eq. 43, res[4 k .. 4 k + 3]), steps taken and divergence
 * flag of every active case k, in slot order (ids[k] = slot); any pointer may
 * be NULL.  Synchronises.  Returns the number of active cases, or HB_ECAPACITY
 * if capacity is below it. */
int hb_batch_residuals(hb_batch_handle b, double *res, long *steps, int *diverged, int *ids, int capacity);

/* The case's handle, brought up to date (synchronises): use it with
 * hb_ugks_residual, hb_ugks_harmonics_out, hb_ugks_state_out/_in,
 * hb_ugks_sizes.  hb_ugks_pseudo_step refuses it (HB_ESTATE); the batch owns
 * and destroys it. */
int hb_batch_case(hb_batch_handle b, int case_id, hb_handle *out);

/* Time candidate launch shapes of the update and moments phases on the
 * batch's own cases (reps launches each) and keep the fastest, remembered per
 * (precision, N_T, padded velocity count) for later batches.  Takes one batch
 * step first.  Errors: HB_EINVAL, HB_EDEVICE. */
int hb_batch_tune(hb_batch_handle b, int reps);

/* Chosen update shapes: per (precision, N_T) group 5 ints (precision, N_T,
 * padded velocities, threads per block, blocks per CU; 0 = one cell per
 * block).  Returns the number of groups or HB_ECAPACITY. */
int hb_batch_shapes(hb_batch_handle b, int *out, int capacity);

/* Device footprint per cache group (default 224 MiB): cases are packed into
 * groups of at most this many bytes and one group's whole step runs before
 * the next group's, so that its stencil re-reads stay in the Infinity Cache.
 * 0 puts every case in one group. */
int hb_batch_set_cache_bytes(hb_batch_handle b, size_t bytes);

/* Replay the step from a captured graph (default) or launch it directly. */
int hb_batch_use_graph(hb_batch_handle b, int on);

int hb_batch_pool_info(hb_batch_handle b, size_t *capacity, size_t *in_use, size_t *largest_free);
void hb_batch_destroy(hb_batch_handle b);

/* ------------------------------------------------------------------ serving
 * A frequency-response solve requested at arrival_s (seconds after the run
 * starts): the case, as for hb_batch_add, and where its converged harmonics
 * go (var_mask, re, im, capacity as for hb_ugks_harmonics_out; re/im NULL:
 * none). */
typedef struct {
    hb_geometry geo;
    double Kn, St;
    int n_harmonics;
    hb_wall walls[4];
    hb_vgrid vg;
    int has_numerics;   /* 0: default numerics */
    hb_numerics num;
    int precision;      /* hb_precision */
    double arrival_s;
    unsigned var_mask;
    double *re, *im;
    size_t capacity;
} hb_request;

typedef struct {
    int status;          /* HB_OK converged; HB_EDIVERGED; HB_ENOMEM larger than the pool; HB_ESTATE max_steps hit */
    long steps;          /* pseudo steps taken by the case */
    double residual[4];  /* Eq. 43 at the last check */
    double t_admit, t_done;  /* seconds after the run starts (-1: never) */
    size_t bytes;        /* device footprint while resident */
} hb_result;

/* Serve n requests (in arrival order) on an empty batch: admit each arrived
 * request as soon as its footprint fits the pool (later requests may pass one
 * that does not fit yet), advance the batch check_every steps at a time, and
 * retire every case whose density residual is <= tol (its harmonics are
 * copied out and its memory freed at once) or that reaches max_steps.
 * Admission and checks happen only between chunks, so a request's steps and
 * result are the same alone and in any mix.  Blocks until every request is
 * retired, or until the first check after max_wall_s seconds (> 0; 0 = no
 * cap): then the resident cases retire as they stand (HB_ESTATE, with their
 * steps and residual) and requests never admitted keep t_admit = -1 and
 * status HB_ESTATE.  *wall_s (may be NULL) receives the run's duration.
 * With the environment variable HB_SERVE_PROGRESS set to a value other than
 * "0", the loop writes one line to stderr after each chunk (elapsed seconds,
 * resident cases, requests finished).
 * Errors: HB_EINVAL, HB_ESTATE (the batch holds cases), HB_EDEVICE. */
int hb_serve_run(hb_batch_handle b, const hb_request *req, int n, double tol, int check_every, long max_steps,
                 double max_wall_s, hb_result *out, double *wall_s);

#ifdef __cplusplus
}
#endif
#endif

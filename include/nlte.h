/*
 * nlte.h - C ABI of the MI355X library for the residual, Jacobian-vector
 * product and Jacobian-free Newton-Krylov (JFNK) solve of multilevel NLTE
 * statistical equilibrium in a plane-parallel atmosphere.
 *
 * The operations follow Arramy, de la Cruz Rodriguez & Leenaarts,
 * "Jacobian-free Newton-Krylov method for multilevel nonlocal thermal
 * equilibrium radiative transfer problems":
 *   - the problem (atmosphere, model atom, frequency and angle grids): Sect. 2.1;
 *   - the residual F(n): Algorithm 1 with Eqs. chi, eta (opacity/emissivity),
 *     Iplus/Iminus (formal solution), Rij/Rji (rates), residuals_1/residuals_2;
 *   - the Jacobian-vector product: Eq. fordif (forward difference);
 *   - the block-Jacobi preconditioner: Sect. 2.5.2 (first solution), App. A.2;
 *   - the solve: Algorithm 2 with the Krylov solver of Sect. 2.3 (GMRES) and the
 *     damping and positivity safeguards of Sect. 2.2.2.
 *
 * Conventions
 *   Units are CGS.  Depth index k = 0 is the top; z increases downwards.
 *   Population-shaped arrays (n, F, v, Jv) are row-major [nz][nlev] doubles,
 *   depth-major as in Sect. 2.1.1.  Mean intensities are [nz][nnu] doubles.
 *   Transition t < nline are bound-bound lines, t >= nline bound-free edges.
 *
 *   Pointers named *_dev are device memory owned by the caller and used on
 *   the given stream; outputs are valid once that stream has been
 *   synchronised.  Descriptor arrays (host) are owned by the caller and are
 *   deep-copied during nlte_column_create; they may be freed afterwards.
 *
 *   Every call returns an nlte_status and never throws; on failure
 *   nlte_last_error() gives a message (thread-local).  Inputs are validated:
 *   non-finite values, n_tot <= 0, T <= 0, non-monotonic z or nu, mu outside
 *   (0, 1), windows outside the grid, level indices out of range.
 */
#ifndef NLTE_H
#define NLTE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NLTE_OK = 0,
  NLTE_E_INVALID = -1,    /* bad argument or descriptor                        */
  NLTE_E_NOMEM = -2,      /* device or host allocation failed                  */
  NLTE_E_DEVICE = -3,     /* HIP runtime error                                 */
  NLTE_E_NOCONV = -4,     /* solve stopped at maxiter; best iterate returned   */
  NLTE_E_NONFINITE = -5,  /* NaN/Inf met in inputs or in the iteration         */
  NLTE_E_BUSY = -6        /* not finished yet (server poll, drain time-out)    */
} nlte_status;

/* Precision of the formal solution and of the angle/frequency quadratures.
 * Opacity assembly, rates, the residual, the rate-matrix solve and the
 * finite-difference product are FP64 in both forms. */
typedef enum { NLTE_FP64 = 0, NLTE_FP32_FORM = 1 } nlte_precision;

/* Inner (Krylov) solver of the Newton steps, Sect. 2.3: GMRES(m) with one
 * product with the Jacobian per iteration, or BiCGSTAB with two. */
typedef enum { NLTE_KRYLOV_GMRES = 0, NLTE_KRYLOV_BICGSTAB = 1 } nlte_krylov;

/* Jacobian-vector products of the Krylov solver, Sect. 2.4: the forward
 * difference of Eq. fordif, or the exact directional derivative that the
 * complex step of Eq. complex reaches for vanishing steps, computed by
 * tangent-linear (dual-number) kernels in FP64. */
typedef enum { NLTE_JV_FD = 0, NLTE_JV_TANGENT = 1 } nlte_jv;

/* OR-ed into the precision argument of nlte_column_create: solve the
 * transfer equation of this column by parallel scans over depth (one
 * workgroup per frequency, one thread per depth; nz <= 256) instead of one
 * sequential recursion per frequency.  Meant for large columns solved alone
 * or in small batches, where one thread per frequency leaves the device
 * idle.  Same equations; rounding differs from the sequential form. */
#define NLTE_DEPTH_SCAN 0x100

typedef struct nlte_ctx nlte_ctx;
typedef struct nlte_column nlte_column;
typedef struct nlte_server nlte_server;

/* Model atmosphere, Sect. 2.1.1 (Eqs. chi/eta background terms). */
typedef struct {
  int32_t nz;              /* depth points, >= 3                               */
  const double *z;         /* [nz] cm, strictly increasing (downwards)          */
  const double *T;         /* [nz] K                                            */
  const double *ne;        /* [nz] electron density, cm^-3                      */
  const double *ntot;      /* [nz] total density of the active atom, cm^-3      */
  const double *chi_c;     /* [nz] gray background opacity, cm^-1               */
  const double *chi_sca;   /* [nz] background scattering opacity or NULL (0)   */
  const double *eta_c;     /* [nz][nnu] thermal background emissivity
                              (erg s^-1 cm^-3 Hz^-1 sr^-1, finite, >= 0; nnu of
                              the grid descriptor) or NULL: chi_c B_nu(T)     */
  const double *vlos;      /* [nz] vertical gas velocity, cm/s, positive
                              outwards (towards depth 0, the observer), finite,
                              |v| < c/10; or NULL: static.  Sect. 3.5: each ray
                              sees the line profiles Doppler-shifted to
                              nu0 (1 + s mu v / c), s = +1 outgoing, -1 ingoing,
                              normalised per ray and depth on the window, so
                              opacity, formal solution and line rates are
                              taken ray by ray.  Columns with a velocity
                              field use the sequential formal solution (no
                              NLTE_DEPTH_SCAN; NLTE_E_INVALID otherwise).     */
} nlte_atmos_desc;

/* Model atom, Sect. 2.1.1.  If nbf > 0 the last level is the continuum
 * (stage 1) and every edge ends there. */
typedef struct {
  int32_t nlev;            /* levels incl. continuum, 2..16                     */
  const double *E;         /* [nlev] erg                                        */
  const double *g;         /* [nlev] statistical weights                        */
  const int32_t *stage;    /* [nlev] 0 bound, 1 continuum                       */
  int32_t nline;
  const int32_t *line_lo;  /* [nline] lower level                               */
  const int32_t *line_up;  /* [nline] upper level (> lower, bound)              */
  const double *A_ul;      /* [nline] Einstein A, s^-1                          */
  const double *a_damp;    /* [nline] Voigt damping parameter, 0 <= a <= 0.1    */
  double mass_amu;         /* atomic mass for the Doppler width                 */
  double vturb;            /* microturbulent velocity, cm/s                     */
  int32_t nbf;
  const int32_t *bf_lo;    /* [nbf] lower level of each edge                    */
  const int32_t *bf_ptr;   /* [nbf+1] offsets into bf_nu / bf_alpha             */
  const double *bf_nu;     /* tabulation frequencies of each edge, increasing   */
  const double *bf_alpha;  /* photo-ionisation cross-section there, cm^2;
                              linearly interpolated onto the union grid         */
} nlte_atom_desc;

/* Frequency and angle grids, Sect. 2.1.2. */
typedef struct {
  int32_t nnu;
  const double *nu;        /* [nnu] Hz, strictly increasing union grid          */
  const int32_t *win_lo;   /* [ntr] first grid index of each transition window  */
  const int32_t *win_hi;   /* [ntr] one past the last index (>= win_lo + 2)     */
  int32_t nmu;             /* 1..8 angles; two rays (+-mu) each                 */
  const double *mu;        /* [nmu] Gauss-Legendre nodes on (0, 1)              */
  const double *w_mu;      /* [nmu] weights, summing to 1                        */
  const double *w_nu;      /* [nnu] frequency quadrature weights (Hz, > 0) that
                              every transition uses over its window, or NULL:
                              trapezoid weights over each transition's own
                              window.  Line profiles are normalised on their
                              window with the same weights.                    */
} nlte_grid_desc;

typedef struct {
  double ftol;         /* stop when max |F|/gross-rate <= ftol (default 1e-8)   */
  double rtol;         /* Krylov relative tolerance (default 1e-3)              */
  int32_t maxiter;     /* Newton iterations (default 50)                        */
  int32_t max_krylov;  /* Krylov iterations per Newton iteration (default 200)  */
  int32_t restart;     /* GMRES restart length m, 1..32 (default 30)            */
  int32_t max_halvings;/* line-search halvings (default 8)                      */
  int32_t init;        /* 0: n0 given, 1: LTE, 2: zero radiation                */
  double eps_scale;    /* multiplies the difference step (default 1)            */
  int32_t max_krylov_total; /* Krylov iterations over the whole solve; once spent,
                          * each Newton iteration takes one Krylov step (a
                          * preconditioned residual step).  0: no limit (default) */
  int32_t fp64_fallback; /* FP32-form columns that have not converged after this
                          * many Newton iterations continue with FP64 formal
                          * solutions: from their current iterate when its
                          * max |F|/gross-rate is at most 1e-2, else from their
                          * initial populations (0: never, default 0)         */
  int32_t krylov_method; /* nlte_krylov (default NLTE_KRYLOV_GMRES).  With
                          * BiCGSTAB, restart is unused and max_krylov,
                          * max_krylov_total and the krylov_iters statistic
                          * count products with the Jacobian (two per
                          * iteration)                                        */
  int32_t jv_method;     /* nlte_jv (default NLTE_JV_FD).  With
                          * NLTE_JV_TANGENT a product costs one tangent
                          * evaluation (no difference step; eps_scale unused) */
  int32_t krylov_x0;     /* initial guess of each Krylov solve (Algorithm 2):
                          * 0 (default) x0 = 0; 1 x0 = -P^-1 F(n), which costs
                          * one more Jacobian product per Newton iteration
                          * (counted in krylov_iters and the budgets)          */
  int32_t launch;        /* how the batch solve replays its steps (OR of):
                          * NLTE_SOLVE_GRAPH: every block of steps between two
                          * host checks is captured once into a HIP graph and
                          * replayed (captured again when the list of running
                          * columns is compacted); NLTE_SOLVE_TUNE: the first
                          * blocks try 1, 2 and 4 waves per formal-solution
                          * workgroup and the rest use the fastest.  Results
                          * do not depend on it (default 0: eager launches,
                          * one wave per workgroup).  Profiled solves
                          * (nlte_profile_enable) launch eagerly.               */
} nlte_solve_opts;

enum { NLTE_SOLVE_GRAPH = 1, NLTE_SOLVE_TUNE = 2 };

typedef struct {
  int32_t status;        /* nlte_status of this column                          */
  int32_t newton_iters;
  int32_t krylov_iters;  /* total over the solve                                */
  int32_t f_calls;       /* residual evaluations (formal solutions)             */
  int32_t stalls;        /* line searches that found no decrease                */
  int32_t precond_calls; /* evaluations that also built the preconditioner      */
  double rho_inf;        /* final max |F|/gross rate                            */
  double dn_inf;         /* last 0.5 max|(n - n_prev)/(n + n_prev)|             */
  int32_t precision;     /* precision of the last evaluation (nlte_precision)   */
  int32_t fp64_evals;    /* residual evaluations run in FP64 by an FP32-form
                          * column after a fallback (0 otherwise)               */
} nlte_solve_stats;

/* Kernel timings accumulated by solves on a context while profiling is on
 * (HIP events on the solve's stream around each phase).  The formal-solution
 * launches of one residual call run on up to four streams at once (F mode,
 * Newton mode, and the FP64 ones of fallback columns); formal_ms is the
 * time until the F-mode ones are done, formal_f_ms that of the F-mode
 * launches in the columns' own precision, which run on the solve's stream;
 * depth_ms runs from there until the rate integrals of the F-mode columns
 * and the Newton-mode launches (formal solutions, rate integrals, pair
 * sums) are all done. */
typedef struct {
  int64_t steps;             /* solver steps (one residual per active column)   */
  int64_t formal_launches;   /* depth-recursion (formal-solution) launches      */
  double formal_ms;          /* formal-solution phase of the F-mode columns     */
  double depth_ms;           /* rate integrals, pair sums, Newton-mode tail     */
  double assemble_ms;        /* residual/preconditioner assembly                */
  double solver_ms;          /* Krylov/Newton step launches                     */
  double opacity_ms;         /* level coefficients + opacity/source function    */
  int64_t formal_f_launches; /* F-mode formal-solution launches on the stream   */
  double formal_f_ms;        /* their summed duration                           */
  /* last batch solve on the context (recorded whether or not profiling is on) */
  int32_t last_graph;        /* 1 if its steps were replayed from HIP graphs    */
  int32_t last_formal_wpb;   /* waves per formal-solution workgroup it used     */
  double last_tune_ms[3];    /* mean step time with 1, 2, 4 waves (0: untuned)  */
  int32_t last_captures;     /* graphs captured (one more per compaction)       */
  int32_t pad_profile;
} nlte_profile;

/* Fills opts with the defaults listed above. */
void nlte_solve_opts_default(nlte_solve_opts *opts);

/* Context bound to one HIP device (made current by every call that uses it). */
nlte_status nlte_ctx_create(int hip_device, nlte_ctx **out);
void nlte_ctx_destroy(nlte_ctx *ctx);

/* Builds a column: validates and deep-copies the descriptors and runs the
 * n-independent setup (Sect. 2.1.1: LTE populations, Planck function, Voigt
 * profiles normalised on each line window, the unified transition
 * coefficients V and g, collision rates in both directions by detailed
 * balance, quadrature weights) on the device.  C_up is [nz][ntr] upward
 * collision rates (lower -> upper), s^-1.  The column owns its device
 * tables and solver state until nlte_column_destroy.  The lagged mean
 * intensity J-dagger of Sect. 2.1.1 starts as B_nu(T).  precision is an
 * nlte_precision, optionally OR-ed with NLTE_DEPTH_SCAN. */
nlte_status nlte_column_create(nlte_ctx *ctx, const nlte_atmos_desc *atmos,
                               const nlte_atom_desc *atom, const nlte_grid_desc *grid,
                               const double *C_up, int32_t precision,
                               hipStream_t stream, nlte_column **out);
void nlte_column_destroy(nlte_column *col);

/* Host-only check and sizing of a column (no device is used): validates the
 * descriptors exactly as nlte_column_create does and, on NLTE_OK, writes the
 * bytes of device memory such a column would own.  Errors: NLTE_E_INVALID
 * (sizes, orderings, level indices, windows, signs), NLTE_E_NONFINITE
 * (NaN/Inf in any array). */
nlte_status nlte_column_plan_bytes(const nlte_atmos_desc *atmos, const nlte_atom_desc *atom,
                                   const nlte_grid_desc *grid, const double *C_up,
                                   int32_t precision, size_t *bytes);

/* dims = {nz, nlev, ntr, nline, nbf, nnu, nmu, precision (| NLTE_DEPTH_SCAN)} */
nlte_status nlte_column_dims(const nlte_column *col, int32_t dims[8]);
/* Bytes of device memory the column owns (its arena). */
nlte_status nlte_column_bytes(const nlte_column *col, size_t *bytes);

/* LTE (Saha-Boltzmann) populations n* [nz][nlev] (Sect. 2.2.1 initial guess). */
nlte_status nlte_lte_populations(nlte_column *col, double *n_dev, hipStream_t stream);

/* Radiation-free populations (Sect. 2.2.1): per depth the rate equations with
 * J = 0 and particle conservation. */
nlte_status nlte_zero_radiation_populations(nlte_column *col, double *n_dev,
                                            hipStream_t stream);

/* Residual F(n) of Algorithm 1.
 *   n_dev    [nz][nlev] populations (positive, finite);
 *   F_dev    [nz][nlev] output;
 *   J_dev    [nz][nnu] output mean intensity, or NULL;
 *   R_dev    [nz][ntr][2] output radiative rates (R_lu, R_ul), or NULL;
 *   Jbar_dev [nz][nline] output profile-averaged line intensity, or NULL;
 *   P_dev    [nz][nlev][nlev] output block-Jacobi preconditioner (Sect. 2.5.2
 *            first solution, conservation rows -1), or NULL (cheaper);
 *   update_J nonzero: the computed J becomes the column's lagged J-dagger.
 * The conservation row of each depth is the most populated level of n. */
nlte_status nlte_residual(nlte_column *col, const double *n_dev, double *F_dev,
                          double *J_dev, double *R_dev, double *Jbar_dev,
                          double *P_dev, int update_J, hipStream_t stream);

/* nlte_residual for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the same
 * arguments, kernels and results as nlte_residual, bit for bit, but the
 * evaluation's scratch (the column descriptor, the population-check flag,
 * the level coefficients, the formal-solution, rate and pair-sum buffers)
 * lives in one fixed device array of 64 MiB per device, held from the first
 * context on that device until the process ends, and every launch runs on
 * `stream`.  Calls no hipMalloc, hipFree or other allocating routine.
 *   A column whose evaluation needs more than 64 MiB of scratch (about
 *   64 bytes per (depth, frequency) plus the rate and pair-sum entries) is
 *   rejected with NLTE_E_INVALID before any device work.
 *   Every call on a device shares that device's array and leaves its
 *   contents behind: calls that overlap on one device (other streams, other
 *   host threads) race and must be serialised by the caller.  The column's
 *   own scratch is not touched (its J of the last evaluation is not updated;
 *   update_J still sets its J-dagger).
 * Errors as nlte_residual (NLTE_E_NONFINITE for populations that are not
 * finite and positive). */
nlte_status nlte_residual_noalloc(nlte_column *col, const double *n_dev, double *F_dev,
                                  double *J_dev, double *R_dev, double *Jbar_dev,
                                  double *P_dev, int update_J, hipStream_t stream);

/* Forward-difference Jacobian-vector product (Eq. fordif):
 * Jv = (F(n + eps v) - F(n)) / eps with the conservation rows and J-dagger
 * of n.  Costs two residual evaluations (F(n) is recomputed). */
nlte_status nlte_jvp(nlte_column *col, const double *n_dev, const double *v_dev,
                     double eps, double *Jv_dev, hipStream_t stream);

/* Exact Jacobian-vector product (Sect. 2.4.2, Eq. complex in the limit of a
 * vanishing step): Jv = dF/dn(n) . v with the conservation rows and J-dagger
 * of n, by tangent-linear kernels that carry a derivative beside every
 * quantity of Algorithm 1 (opacity, formal solution, rates, assembly), all in
 * FP64 whatever the column's precision.
 *   n_dev  [nz][nlev] populations (positive, finite);
 *   v_dev  [nz][nlev] direction (any finite values);
 *   Jv_dev [nz][nlev] output.
 * Costs one residual evaluation at n (for the rates and rows of n) and one
 * tangent evaluation.  The column's solver iterate is overwritten with n. */
nlte_status nlte_jvp_tangent(nlte_column *col, const double *n_dev, const double *v_dev,
                             double *Jv_dev, hipStream_t stream);

/* JFNK solve (Algorithm 2, whose Data are n0 and an initial estimate of J)
 * of one column, entirely on the device.
 *   n0_dev   [nz][nlev] initial populations when opts->init == 0 (else unused);
 *   J0_dev   [nz][nnu] initial J-dagger, the lagged mean intensity of the
 *            background-scattering emissivity (Sect. 2.1.1), or NULL: B_nu(T);
 *   n_out_dev[nz][nlev] converged (or best) populations;
 *   J_out_dev[nz][nnu] or NULL: the J-dagger of the final residual, so that
 *            F(n_out; J_out) is the residual the stopping test saw.  For a
 *            column with background scattering it is the mean intensity of
 *            the evaluation before the last, and (n_out, J_out) restarts the
 *            solve where it stopped (pass them as n0 with init = 0 and as J0);
 *            without scattering F does not depend on it and it is the mean
 *            intensity of the final evaluation;
 *   stats    host struct or NULL.
 * Returns NLTE_E_NOCONV when maxiter is reached (n_out holds the last
 * iterate).  Blocks until the solve has finished on `stream`. */
nlte_status nlte_solve(nlte_column *col, const double *n0_dev, const double *J0_dev,
                       const nlte_solve_opts *opts, double *n_out_dev, double *J_out_dev,
                       nlte_solve_stats *stats, hipStream_t stream);

/* Solves ncol independent columns (any sizes, any precision) together: every
 * step evaluates one residual per active column in the same launches, with
 * per-column Krylov/Newton state on the device.  Arrays are indexed by
 * column; n0_dev may be NULL when opts->init != 0; J0_dev (initial J-dagger
 * per column, entries may be NULL) may be NULL; stats is [ncol] or NULL.
 * Returns NLTE_OK if every column converged, else NLTE_E_NOCONV (per-column
 * status in stats). */
nlte_status nlte_solve_batch(nlte_ctx *ctx, nlte_column *const *cols, int32_t ncol,
                             const double *const *n0_dev, const double *const *J0_dev,
                             const nlte_solve_opts *opts, double *const *n_out_dev,
                             nlte_solve_stats *stats, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Residual plans: F(n) of a fixed set of columns in shared launches.
 *
 * A plan binds columns to caller-owned device buffers n_dev[c] ([nz][nlev]
 * populations, read) and F_dev[c] ([nz][nlev], written).  Each run copies
 * every n_dev[c] into its column, evaluates Algorithm 1 for all of them
 * (conservation rows from each n, J-dagger of the column, no
 * preconditioner) in one set of launches, and writes the residuals out.
 * The buffers and columns must stay valid and must not be used by other
 * calls while runs are pending.
 *   NLTE_PLAN_GRAPH: the launch sequence is captured once into a HIP graph
 *                    and every run replays it (one host call per run).
 *   NLTE_PLAN_TUNE:  creation times each candidate launch shape (depths per
 *                    opacity wave 4/8/16, waves per formal-solution block
 *                    1/2/4) over a few runs of this batch and keeps the
 *                    fastest; otherwise 8 and 4.
 * ------------------------------------------------------------------------ */
typedef struct nlte_plan nlte_plan;
enum { NLTE_PLAN_GRAPH = 1, NLTE_PLAN_TUNE = 2 };

typedef struct {
  int32_t ncol;
  int32_t opac_depths;   /* chosen launch shape                               */
  int32_t formal_wpb;
  int32_t graph;         /* 1 if runs replay a captured graph                 */
  int64_t depth_points;  /* formal-solution depth-points per run              */
  double tune_ms[9];     /* mean run time of each candidate (opacity depths 4,
                          * 8, 16 x waves 1, 2, 4), 0 if not tuned            */
} nlte_plan_info;

nlte_status nlte_plan_create(nlte_ctx *ctx, nlte_column *const *cols, int32_t ncol,
                             const double *const *n_dev, double *const *F_dev, int32_t flags,
                             hipStream_t stream, nlte_plan **out);
nlte_status nlte_plan_run(nlte_plan *plan, hipStream_t stream);
nlte_status nlte_plan_info_get(const nlte_plan *plan, nlte_plan_info *out);
void nlte_plan_destroy(nlte_plan *plan);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of column solves.
 *
 * A server owns one host thread and non-blocking HIP streams on the
 * context's device (one for the steps, one for setting up admitted problem
 * requests while the steps run).  Submitted solves wait in a FIFO queue and are admitted
 * while the device arenas of the columns in flight stay within hbm_budget
 * bytes and their number within max_active (a column larger than the budget
 * is admitted alone).  Admitted columns advance together, one residual
 * evaluation per column per step, exactly as in nlte_solve_batch, so a
 * served result is bit-identical to the same column solved alone with the
 * same options; their Newton/Krylov state stays in the columns' device memory.
 * After every few steps the thread retires finished columns and admits
 * waiting ones (requests that arrive while others run join the next step).
 *
 * Ownership: the caller keeps ownership of every column; a submitted column
 * must not be used, resubmitted or destroyed until its ticket is polled (or
 * the server destroyed).  n0_dev (NULL: LTE start) must stay valid until the
 * request is admitted.  Thread safety: submit, poll, info and drain may be
 * called from any host thread.
 * ------------------------------------------------------------------------ */
typedef struct {
  nlte_solve_stats stats;
  double t_submit_ms;    /* host steady clock, ms since the server was created */
  double t_admit_ms;
  double t_done_ms;      /* when the server saw the solve finish               */
} nlte_server_result;

typedef struct {
  int64_t steps;         /* device steps run                                   */
  int64_t submitted, completed;
  int32_t active, queued;
  int64_t active_bytes;  /* device arena bytes of the columns in flight        */
  double busy_ms;        /* host time spent with columns in flight             */
  int64_t peak_active_bytes; /* largest active_bytes so far                    */
} nlte_server_info;

/* opts as for nlte_solve; requests that bring no n0 start from LTE
 * (opts->init = 1) or from the radiation-free populations (opts->init = 2,
 * Sect. 2.2.1); opts->init = 0 is rejected.  max_active >= 1; hbm_budget > 0
 * bytes. */
nlte_status nlte_server_create(nlte_ctx *ctx, size_t hbm_budget, int32_t max_active,
                               const nlte_solve_opts *opts, nlte_server **out);
/* Queues a solve of col; *ticket identifies it for nlte_server_poll. */
nlte_status nlte_server_submit(nlte_server *srv, nlte_column *col, const double *n0_dev,
                               uint64_t *ticket);
/* Queues a solve of a problem the server holds on the host until admission:
 * the descriptors are validated (as nlte_column_create; errors are returned
 * here) and deep-copied, so the caller may free them at once.  The request
 * is admitted when the device bytes of its column (nlte_column_plan_bytes)
 * fit the budget next to the columns in flight; its column is then created
 * (setup run: part of the request's latency) in device memory from the
 * server's pool of column arenas (a retired column's arena is reused by a
 * later column within 1/16 of its size; the arenas lent and pooled stay
 * within the budget, and the pool is freed with the server) and solved with
 * the others, and when the solve finishes its populations are copied to
 * n_out_dev ([nz][nlev] device memory owned by the caller, valid until the
 * ticket is polled) and the column is destroyed, its arena returning to the
 * pool.  If the column cannot be created, the request finishes with that
 * status.  Sect. 2.1 (the problem), Algorithm 2 (the solve). */
nlte_status nlte_server_submit_problem(nlte_server *srv, const nlte_atmos_desc *atmos,
                                       const nlte_atom_desc *atom, const nlte_grid_desc *grid,
                                       const double *C_up, int32_t precision, double *n_out_dev,
                                       uint64_t *ticket);
/* NLTE_OK: the solve has finished; its populations are copied to n_out_dev
 * ([nz][nlev] device memory, or NULL; unused for problem requests, whose
 * populations are already in the buffer given at submission) and its result
 * to *res (or NULL), and the ticket is released.  NLTE_E_BUSY: not finished yet (nothing copied).
 * NLTE_E_INVALID: unknown ticket.  A solve that stops at maxiter is finished
 * with res->stats.status = NLTE_E_NOCONV. */
nlte_status nlte_server_poll(nlte_server *srv, uint64_t ticket, double *n_out_dev,
                             nlte_server_result *res);
/* Blocks until no request is queued or in flight, or timeout_s elapses
 * (NLTE_E_BUSY). */
nlte_status nlte_server_drain(nlte_server *srv, double timeout_s);
nlte_status nlte_server_info_get(const nlte_server *srv, nlte_server_info *out);
/* Stops the thread (requests still queued or in flight are dropped). */
void nlte_server_destroy(nlte_server *srv);

/* Turns kernel timing of subsequent solves on this context on (nonzero) or
 * off, and clears the accumulated profile.  Adds two HIP events per launch. */
nlte_status nlte_profile_enable(nlte_ctx *ctx, int on);
nlte_status nlte_profile_read(const nlte_ctx *ctx, nlte_profile *out);

/* Message describing the last non-OK status returned on this thread. */
const char *nlte_last_error(void);

/* Size in bytes of the public structure named `name` ("nlte_atmos_desc",
 * "nlte_atom_desc", "nlte_grid_desc", "nlte_solve_opts", "nlte_solve_stats",
 * "nlte_profile", "nlte_plan_info", "nlte_server_result", "nlte_server_info")
 * as this library was compiled, or -1 for another name.  Host only; lets a
 * binding check its own layouts against the library's. */
int32_t nlte_struct_size(const char *name);

/* Voigt function H(a, v) evaluated on the host with the same routine the
 * device setup uses (Taylor expansion about the real axis with Rybicki's
 * Dawson series for |v| < 8, asymptotic series beyond).  For tests. */
nlte_status nlte_voigt_host(double a, const double *v, int32_t n, double *out);

/* Issue-rate probes (measurement only: the denominators of the depth
 * recursion's VALU roofline, not part of the method).  Runs `iters`
 * operations of kind `op` in each of 8 independent chains per lane on a
 * full device (8 workgroups of 256 lanes per CU) of the context's device,
 * after one warm-up launch, timed with HIP events on a stream of its own;
 * *lane_ops_per_s = lanes x iters x 8 / time.  iters: a multiple of 4 in
 * [4, 2^24].  Allocates and frees a small output buffer.  NLTE_E_INVALID for
 * an unknown op or iters out of range, NLTE_E_DEVICE for HIP errors. */
typedef enum {
  NLTE_PROBE_FMA_F32 = 0, /* v_fma_f32 (non-packed)          */
  NLTE_PROBE_FMA_F64 = 1, /* v_fma_f64                       */
  NLTE_PROBE_EXP_F32 = 2, /* v_exp_f32 (base-2 exponential)  */
  NLTE_PROBE_RCP_F32 = 3  /* v_rcp_f32                       */
} nlte_probe_op;
nlte_status nlte_issue_rate(nlte_ctx *ctx, int32_t op, int32_t iters, double *lane_ops_per_s);

#ifdef __cplusplus
}
#endif
#endif /* NLTE_H */

/*
 * stp.h -- C ABI of the MI355X space-time parabolic solver.
 *
 * Solves the implicit-Euler discretisation (eq. (2.1) of Neumueller & Smears,
 * "Time-parallel iterative solvers for parabolic evolution equations")
 *
 *     (u_n - u_{n-1}) + tau A_n u_n = tau F_n,   n = 1..N,   u_0 = u0,
 *
 * of  u_t - div(kappa(t,x) grad u) = F  on the unit d-cube (d = 1, 2, 3) with
 * homogeneous Dirichlet conditions, by the inexact Uzawa iteration (eq. (3.1))
 * on the symmetric saddle-point reformulation (eq. (2.7)), preconditioned by
 * the block-diagonal A-tilde (eq. (3.2)) and the DST-in-time Schur complement
 * preconditioner H-tilde (eqs. (4.4)-(4.6)).  All N time slabs are processed
 * together in every kernel launch on one GPU.
 *
 * Spatial discretisation (the paper leaves it abstract): n interior nodes per
 * axis, h = 1/(n+1), lumped mass M = I, conservative 3/5/7-point stencil
 *     (A u)_i = h^-2 sum_{faces f of i} kappa_f (u_i - u_nb(f)),
 * with kappa_f the arithmetic mean of the two nodal values the face joins.
 *
 * Memory layout of every grid vector: slab-major, x fastest:
 *     v[((s * n + z) * n + y) * n + x]     (s = time slab n-1, 0-based)
 * Vectors on the time-global space hold N * n^d float64 values.
 *
 * Conventions for every entry point
 *   - Pointers documented "device" must point to GPU memory of the device that
 *     is current when stp_create is called; "host" pointers to CPU memory.
 *   - All work is enqueued on the HIP stream given to stp_create (NULL = the
 *     null stream).  stp_apply_* are asynchronous; stp_uzawa_solve returns
 *     after the solve has finished.
 *   - Errors are reported by the return code only (no exceptions cross the
 *     ABI); stp_last_error() gives a human-readable detail for the calling
 *     thread.  On error no output buffer is written unless stated otherwise.
 *   - Input and output buffers of one call must not overlap.
 */
#ifndef STP_H
#define STP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STP_OK = 0,
  STP_EINVAL = -1,       /* invalid argument (sizes, pointers, tau, kappa)      */
  STP_ENOMEM = -2,       /* device allocation failed / workspace too small       */
  STP_EDEVICE = -3,      /* a HIP call failed                                    */
  STP_ENOTCONV = -4,     /* max_iter reached; u, p hold the last iterate         */
  STP_EDIVERGED = -5,    /* exploding or non-finite residual; see stp_uzawa_solve     */
  STP_EUNSUPPORTED = -6  /* valid request this build does not implement          */
} stp_status;

#define STP_MAX_RANK 4      /* max separable terms of kappa(t,x)               */
#define STP_MAX_LEVELS 16

enum { STP_PREC_F64 = 0,    /* everything in float64                                      */
       STP_PREC_F32 = 1,    /* preconditioner (V-cycles, DST, H-blocks) in float32        */
       STP_PREC_BF16 = 2 }; /* preconditioner vectors stored as bfloat16, float32 math     */

enum { STP_SPATIAL_AUTO = 0,   /* exact tridiagonal solves in 1-D, multigrid in 2-D/3-D   */
       STP_SPATIAL_MG = 1,     /* nu V-cycles of geometric multigrid (needs n = 2^L - 1)  */
       STP_SPATIAL_EXACT = 2,  /* exact spatial solves (1-D only)                          */
       STP_SPATIAL_NONE = 3 }; /* operators only: stp_apply_precond / stp_uzawa_solve
                                  return STP_EUNSUPPORTED; any n allowed                   */

enum { STP_DISC_FD = 0,    /* finite differences, M = I, kappa(t, x) of rank <= 4 (the default)   */
       STP_DISC_FEM = 1 }; /* finite elements with the consistent mass matrix M of Section 2:
                              P1 in 1-D and 2-D (squares split by their lower-left/upper-right
                              diagonal), Q1 hexahedra in 3-D; kappa constant in space (rank 1,
                              a constant field) times the time factor tcoef; single problems,
                              exact solves in 1-D, one V-cycle (nu = 1) in 2-D and 3-D          */

enum { STP_OP_B = 0,        /* y = B x = (K + A) x, eq. (2.3); x, y: N*n^d              */
       STP_OP_SADDLE = 1 }; /* [y_p; y_u] = saddle [x_p; x_u], eq. (2.7); 2*N*n^d each  */

enum { STP_PC_A = 0,        /* z = A-tilde^{-1} r, eq. (3.2)                            */
       STP_PC_H = 1 };      /* z = H-tilde^{-1} r = Phi^{-1} Hhat_approx^{-1} Phi^{-T} r, eq. (4.6) */

typedef struct stp_ctx stp_ctx;

typedef struct {
  int dim;  /* 1, 2 or 3 */
  int n;    /* interior nodes per axis (>= 1); multigrid needs n = 2^L - 1 */
} stp_grid;

/* kappa(t_n, x) = sum_{r<rank} tcoef[r*N + (n-1)] * fields[r](x), every value > 0. */
typedef struct {
  int rank;              /* 1..STP_MAX_RANK                                          */
  const double* fields;  /* device, rank x (n+2)^dim nodal values incl. boundary,
                            x fastest; borrowed until stp_destroy                     */
  const double* tcoef;   /* host, rank x N; copied by stp_create                      */
} stp_kappa;

typedef struct {
  int precision;        /* STP_PREC_*                                                */
  int spatial;          /* STP_SPATIAL_*                                             */
  int nu_A, nu_H;       /* V-cycles per application of A~_n^{-1} (nu_A) and of each
                           H~_k^{-1} (nu_H), 1..8 (Section 8.2 uses one or two); every
                           cycle after the first acts on the residual the earlier ones
                           leave.  Multigrid only (exact solves need one; ignored
                           there).  Above 1 the workspace holds one more N x n^dim
                           vector of the storage type.  Out of range: STP_EINVAL.    */
  double omega;         /* Uzawa damping (eq. (3.1)); <= 0: estimated per problem at
                           stp_create (see stp_omega_info)                            */
  double tol;           /* stop at ||f - B u||_2 <= tol ||f||_2                      */
  int max_iter;         /* maximum number of u-updates                               */
  const double* kref_coef; /* host, rank values: kappa_ref = sum_r kref_coef[r] fields[r]
                              for the reference operator A of eq. (2.2); NULL = time mean */
  int check_every;      /* iterations enqueued between host checks of the stop flag  */
  int use_graph;        /* 1: replay each iteration as a captured HIP graph          */
  const double* tau_steps; /* host, N step lengths tau_n of eq. (2.1) (copied by stp_create),
                              or NULL for N steps of length tau.  When given, tau is the
                              reference step of eq. (2.2) used by H-tilde (<= 0: the mean
                              of tau_n), A = diag(tau_n A_n), f_n = tau_n F_n (+ u0), and
                              without kref_coef kappa_ref is the step-weighted time mean
                              sum_n tau_n kappa(t_n) / sum_n tau_n.  For stp_create_batch:
                              the steps of every problem, one problem after the other
                              (N[0] + ... + N[P-1] values; a problem with uniform steps
                              lists N[i] copies of its tau), and each tau[i] <= 0 selects
                              the mean of problem i's own steps.                         */
  int disc;             /* STP_DISC_*.  With STP_DISC_FEM the problem of stp_create is
                           M (u_n - u_{n-1}) + tau_n a_n A u_n = tau_n M F_n (eq. (2.1)),
                           u_0 = u0, with M, A the element matrices of the mesh and
                           a_n = tcoef[n-1] * (the field's constant value); F holds the
                           nodal values of the source, so f_n = tau_n M F_n + [n = 1] M u0.
                           The multigrid levels are the element operators of the coarse
                           meshes (the Galerkin operators of the element interpolation),
                           smoothed by l1-Jacobi, x += 1.6 (b - L x) / (absolute row sum
                           of L), which contracts for every mix of mass and stiffness.    */
  int sweeps;           /* finite elements: l1-Jacobi sweeps before and after the
                           coarse correction of each V-cycle, 1..4 (0 means 1); the finite-
                           difference cycle is fixed at one.  Out of range: EINVAL.       */
} stp_options;

/* Per-phase device times of a solve (stp_stats.t_phase_ms), Tables 3-4 of
 * Section 8.3 split the time the same way (FFT vs spatial solves). */
enum { STP_PHASE_RESID = 0,    /* residuals r_p, r_u and the stop test (eq. (3.1))          */
       STP_PHASE_ATILDE = 1,   /* A-tilde^{-1} solves, eq. (3.2)                             */
       STP_PHASE_DST = 2,      /* time transforms Phi^{-T}, Phi^{-1}, eqs. (4.2)-(4.3)        */
       STP_PHASE_HBLOCK = 3,   /* H-blocks (2 tau / N) H~_k^{-1} A H~_k^{-1}, eq. (4.6)      */
       STP_PHASE_OTHER = 4,    /* everything else (GMRES orthogonalisation, casts)           */
       STP_NPHASE = 5 };

typedef struct {
  int iters;            /* number of u-updates performed (j of the returned u_j)     */
  double rel_res;       /* ||f - B u_j||_2 / ||f||_2 of the returned u_j (when f = 0:
                           the absolute ||B u_j||_2)                                  */
  double omega_used;
  double t_solve_ms;    /* device time of the iteration loop (HIP events)            */
  int status;           /* stp_status of the solve                                   */
  double rel_rp;        /* ||K u - A p - f||_2 / ||f||_2 and                          */
  double rel_ru;        /* ||f - K^T p - (K + K^T + A) u||_2 / ||f||_2 of the returned
                           pair (u_j, p_{j+1}): the two blocks of the saddle residual
                           of eq. (2.7) (absolute when f = 0); one extra pass over
                           u, p, F after the solve                                    */
  double t_setup_ms;    /* wall time of stp_create[_batch] (all problems), including  */
  double t_omega_ms;    /* the damping estimate (this part)                           */
  double t_phase_ms[STP_NPHASE]; /* device time of the solve's kernels by phase
                           (STP_PHASE_*), summed over launches; measured only while
                           stp_timing_enable(ctx, 1) is in effect (the solve then runs
                           without graph replay), else 0                             */
} stp_stats;

/* Fill *opt with defaults: F64, AUTO, nu = 1, omega 0.8, tol 1e-8, max_iter 500,
   time-mean kappa_ref, check_every 8, graphs on, uniform steps. */
void stp_default_options(stp_options* opt);

/* Device bytes stp_create needs as workspace for this problem and options.
 * Layout: [solver vectors and coefficient tables | launch tables | setup and
 * tuning scratch]; the scratch holds max(5 float64 vectors per problem plus
 * 8 KB of dot partials when omega is estimated (opt->omega <= 0), 2 float64
 * vectors per problem for stp_autotune) and is only used inside stp_create
 * and stp_autotune. */
size_t stp_workspace_bytes(const stp_grid* g, int N, int rank, const stp_options* opt);

/* Set up one problem (Section 2 problem statement): grid, N steps of length tau,
 * kappa, source F (device, N x n^d: F_n on the interior nodes) and initial datum
 * u0 (device, n^d).  F, u0 and kappa->fields are borrowed until stp_destroy.
 * workspace: device buffer of >= stp_workspace_bytes (256-byte aligned), owned
 * by the caller; the library then allocates no device memory for this context,
 * neither here nor in any later call (it keeps a small pinned host array of
 * per-problem stop flags).  NULL: the library allocates the solver part
 * itself (freed by stp_destroy) and the setup and tuning scratch only while
 * it is in use.  hip_stream: hipStream_t or NULL.
 * Errors: EINVAL (dim not 1..3, n < 1, N < 1, tau <= 0 or not finite without
 * opt->tau_steps, a step length <= 0 or not finite, rank out of range, NULL
 * pointers, some kappa <= 0, a non-finite value in F or u0, nu_A or nu_H not
 * in 1..8), EUNSUPPORTED (MG with n != 2^L - 1, EXACT with dim > 1), ENOMEM
 * (allocation failed or workspace too small), EDEVICE. */
stp_status stp_create(stp_ctx** out, const stp_grid* g, int N, double tau,
                      const stp_kappa* kappa, const double* F, const double* u0,
                      const stp_options* opt, void* workspace, size_t ws_bytes,
                      void* hip_stream);

/* Batches.  A batch context holds P >= 1 independent problems of the same
 * spatial dimension; grids, step counts, tau, kappa rank and data may differ
 * from problem to problem.  Each step of an iteration is one merged launch per
 * kernel variant that serves every problem of the batch, so many small solves
 * fill the GPU together.  The problems are exactly those of stp_create
 * (Section 2 problem statement), each solved by its own inexact Uzawa iteration
 * (eq. (3.1)) with its own stop test; a problem that has stopped is skipped by
 * later launches.
 *
 * stp_workspace_bytes_batch: device bytes stp_create_batch needs for P
 * problems (grids[i], N[i], rank[i]); 0 when an argument is invalid.
 *
 * stp_create_batch: arrays of length P, all host arrays; F[i], u0[i] and
 * kappa[i].fields are device pointers borrowed until stp_destroy, as in
 * stp_create.  opt applies to every problem; opt->kref_coef must be NULL when
 * P > 1 (each problem then takes the time mean of its own kappa).  Errors as
 * stp_create, plus EUNSUPPORTED when the dimensions differ.
 *
 * stp_uzawa_solve_batch: u[i], p[i] (device, N[i] x n_i^d float64 each, the
 * initial guesses) are overwritten as by stp_uzawa_solve; stats (host array of
 * P, or NULL) receives per-problem results.  Returns the worst status over the
 * batch (EDIVERGED before ENOTCONV before OK).
 *
 * A context made by stp_create is a batch of one; stp_apply_operator and
 * stp_apply_precond accept only such contexts (EUNSUPPORTED otherwise). */
size_t stp_workspace_bytes_batch(int P, const stp_grid* grids, const int* N, const int* rank,
                                 const stp_options* opt);
stp_status stp_create_batch(stp_ctx** out, int P, const stp_grid* grids, const int* N,
                            const double* tau, const stp_kappa* kappa, const double* const* F,
                            const double* const* u0, const stp_options* opt, void* workspace,
                            size_t ws_bytes, void* hip_stream);
stp_status stp_uzawa_solve_batch(stp_ctx* ctx, double* const* u, double* const* p, stp_stats* stats);
/* Number of problems in the context (0 for NULL). */
int stp_batch_size(stp_ctx* ctx);

/* y = op x on device buffers (layouts above), float64. */
stp_status stp_apply_operator(stp_ctx* ctx, int op, const double* x, double* y);

/* z = preconditioner^{-1} r on device float64 buffers (N x n^d), computed in the
 * context's precision. */
stp_status stp_apply_precond(stp_ctx* ctx, int which, const double* r, double* z);

/* Inexact Uzawa iteration, eq. (3.1), from the initial guess held in u and p
 * (device, N x n^d float64 each, both required; zero them to start from zero).
 * On return u = u_j with j = st->iters, p = p_{j+1}.  Returns OK, ENOTCONV
 * (max_iter reached, the last iterate is returned) or EDIVERGED: the residual
 * ||f - B u_j|| grew above 1e8 times its initial value (and above 1e8 tol ||f||)
 * or became non-finite.  Growth is caught long before floating-point overflow,
 * so with finite inputs (stp_create rejects others) the returned u_j, p_{j+1}
 * are the last iterate and finite.  A diverging solve with an estimated omega
 * can be repeated with the damping bound of eq. (3.7) (stp_omega_info out[4],
 * set by stp_set_omega), under which Theorem 3.1 guarantees convergence.
 * st may be NULL. */
stp_status stp_uzawa_solve(stp_ctx* ctx, double* u, double* p, stp_stats* st);

/* Stop rule of the following solves (stp_uzawa_solve[_batch], stp_gmres_solve):
 * tol >= 0 and max_iter >= 0 replace the values given to stp_create, for every
 * problem of the context.  Captured iteration graphs stay valid.  Errors: EINVAL. */
stp_status stp_set_stop(stp_ctx* ctx, double tol, int max_iter);

void stp_destroy(stp_ctx* ctx);

/* Damping parameter.  With opt->omega <= 0, stp_create estimates omega for
 * every problem (Theorem 3.1, eq. (3.7); Theorem 4.1): the extreme
 * eigenvalues of H~^{-1} S~, S~ = K^T A~^{-1} K + K + K^T + A, as the extreme
 * Ritz values of 12 conjugate-gradient steps on S~ preconditioned by H~^{-1},
 * and rho_A by 8 power steps on I - A~^{-1} A, with start vectors from
 * SplitMix64 at the global index (seeds 0x5EED and 0xA5EED).  omega =
 * min(0.95 * 2/(lmin + lmax), 0.9 * 2/lmax).  This balances the two ends of
 * the spectrum; the sufficient condition (3.7) of Theorem 3.1,
 * omega lambda_max < 2 (1 - rho_A) / (1 + rho_A), is NOT imposed (with the
 * rho_A ~ 0.3 of one V-cycle it halves the damping and the iteration count
 * roughly doubles), so convergence with the estimated omega is observed, not
 * guaranteed.  The estimate runs the iteration's own kernels (about 25
 * iterations' worth of work) in the setup scratch of the workspace.
 * stp_omega_info: out5 = {omega, lambda_min, lambda_max, rho_A, omega_37} of
 * problem i, omega_37 = 2 (1 - rho_A) / ((1 + rho_A) lambda_max), the bound of
 * (3.7) from the estimates (lambda_min, lambda_max, rho_A and omega_37 are 0
 * when omega was given).  stp_set_omega: host array of P values > 0, used from
 * the next solve on.  Errors: EINVAL. */
stp_status stp_omega_info(stp_ctx* ctx, int i, double* out5);
stp_status stp_set_omega(stp_ctx* ctx, const double* omega);

/* GMRES acceleration of the inexact Uzawa method (the solver of the
 * experiments of Section 8.3).  The iteration (3.1) is the stationary method
 * x <- x + P^{-1}(g - S x) on the saddle system S [p; u] = g = [-f; -f] of
 * eq. (2.7), with P^{-1} r = [d; -omega H~^{-1}(r_u + K^T d)], d = A~^{-1} r_p
 * (one Uzawa sweep from zero).  stp_gmres_solve runs flexible GMRES(restart)
 * with P^{-1} as right preconditioner: each cycle minimises ||g - S x||_2 over
 * x_0 + span{P^{-1} v_0, ..., P^{-1} v_{k-1}} (Arnoldi vectors v_j; classical
 * Gram-Schmidt, repeated once when the projection removes more than 90 % of
 * the norm; Givens rotations on the host).  It stops on the
 * Uzawa solver's test ||f - B u||_2 <= opt.tol ||f||_2, evaluated at every
 * restart and after each step whose least-squares estimate of ||g - S x||_2
 * is <= tol ||g||_2 (on the candidate u; a failed check continues the
 * cycle), or after opt.max_iter Arnoldi steps.  omega is the context's (given
 * or estimated); the preconditioner runs in the context's precision and the
 * Krylov vectors in float64.  Single-problem contexts only.
 *
 * u, p: device, N x n^d float64 each: the initial guess in, the result out.
 * ws: device, at least stp_gmres_workspace_bytes(ctx, restart) bytes, 8-byte
 * aligned, owned by the caller (the restart + 1 Arnoldi vectors and restart
 * preconditioned vectors of 2 N n^d values each, one vector of N n^d values
 * and reduction scratch).  hist: optional host array of max_iter + 1 values:
 * ||g - S x_0|| / ||g|| and then the least-squares estimate after each
 * Arnoldi step, relative to ||g||.  stats (optional): iters = Arnoldi steps,
 * rel_res = ||f - B u|| / ||f|| of the returned u.
 * Errors: EINVAL (NULL u or p, restart not in 1..64, workspace too small or
 * misaligned), EUNSUPPORTED (batch context, no spatial solver), ENOTCONV
 * (max_iter reached or breakdown; u, p hold the last iterate), EDIVERGED
 * (non-finite residual), EDEVICE.  stp_gmres_workspace_bytes returns 0 for
 * invalid arguments. */
size_t stp_gmres_workspace_bytes(stp_ctx* ctx, int restart);
stp_status stp_gmres_solve(stp_ctx* ctx, double* u, double* p, int restart, void* ws, size_t ws_bytes,
                           double* hist, stp_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): stp_gmres_solve with
 * its Krylov workspace in a fixed 64 MiB device array of the library instead of
 * a caller buffer, so the call allocates nothing (it also launches eagerly,
 * without instantiating graphs).  Problems whose stp_gmres_workspace_bytes(ctx,
 * restart) exceeds 64 MiB are rejected with EINVAL.  Each GPU holds one copy of
 * the array until the process ends, shared by every call on that GPU: calls
 * that overlap on one GPU (two threads or streams) race and must be
 * serialised by the caller; nothing in the array needs to start at zero.
 * Results equal stp_gmres_solve's.  Other errors as stp_gmres_solve. */
stp_status stp_gmres_solve_noalloc(stp_ctx* ctx, double* u, double* p, int restart, double* hist,
                                   stp_stats* stats);

/* Autotuner (project-written).  Times, on the context's own buffers and
 * stream, the candidate schedules of every merged launch of an iteration and
 * keeps the fastest:
 *   - slabs per block of each tile launch (residuals, the middle operator of
 *     the H-blocks, and every multigrid down- and up-sweep level), as a power
 *     of two times the built-in heuristic, within [1, 16];
 *   - for every power-of-two step count N <= 4096, the time transform path:
 *     two-step register FFT (4 <= N <= 256), Stockham LDS FFT with 1..16
 *     columns per block (as LDS allows), or the dense transform (N <= 64).
 * Each candidate is timed over reps launches (after one warm-up) with HIP
 * events; a candidate replaces the current choice only when it is at least 2%
 * faster.  The tuner runs its launches on two scratch vectors per problem (the
 * workspace's scratch region, or a temporary allocation when the library owns
 * the workspace), leaves the caller's data untouched, and invalidates the
 * captured iteration graph (the next solve captures again).  The result is
 * kept in a process-wide cache keyed by precision, dimension, spatial mode,
 * coefficient rank and the (n, N, rank) of every problem; with use_cache != 0
 * a cached schedule is applied without timing.  Iterates and results do not
 * depend on the schedule: only how the work is split among blocks changes.
 * rep (may be NULL) receives the number of knobs and candidates timed,
 * whether the cache was used, and the device time of one eager iteration
 * before and after tuning (0 when taken from the cache).
 * Errors: EINVAL (NULL ctx), EUNSUPPORTED (spatial NONE), ENOMEM, EDEVICE. */
typedef struct {
  int knobs_tuned;
  int candidates;
  int from_cache;
  double iter_ms_before;
  double iter_ms_after;
} stp_tune_report;
stp_status stp_autotune(stp_ctx* ctx, int reps, int use_cache, stp_tune_report* rep);
/* Human-readable schedule of the context (slabs per block per launch kind,
 * transform path per step-count group); valid until the next call. */
const char* stp_schedule_string(stp_ctx* ctx);

/* Profiling aid.  While enabled, every kernel launch of the context is
 * bracketed by a pair of HIP events on the context's stream (a small
 * overhead per launch).  stp_timing_enable(ctx, 1) clears earlier records;
 * stp_timing_count synchronizes the stream, folds the records into entries
 * keyed by (kernel, multigrid level) and returns the number of entries (-1 on
 * error); stp_timing_get reads entry idx: kernel name (valid until the next
 * stp_timing_* call), level, number of launches and summed device time. */
stp_status stp_timing_enable(stp_ctx* ctx, int enable);
int stp_timing_count(stp_ctx* ctx);
stp_status stp_timing_get(stp_ctx* ctx, int idx, const char** name, int* level, long* launches,
                          double* total_ms);
const char* stp_status_string(stp_status s);
const char* stp_last_error(void);
/* Total device bytes the library has obtained with hipMalloc in this process
 * (never decreases).  A diagnostic for callers that pass workspaces: with a
 * caller workspace, stp_create, stp_autotune and the solves leave it unchanged. */
size_t stp_device_bytes_allocated(void);

#ifdef __cplusplus
}
#endif
#endif /* STP_H */

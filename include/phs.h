/*
 * phs.h — C ABI of the MI355X polyharmonic-spline (PHS) interpolation library.
 *
 * Problem (paper Sec. 1, eqs. phs_interp, phs_fun, phs_linsys): given nodes
 * x_j in R^2, values f_j, spline order k and polynomial degree d, find weights w
 * and polynomial coefficients beta with
 *
 *      [ M   B ] [ w    ]   [ f ]        M_ij = phi(|x_i - x_j|),
 *      [ B^T 0 ] [ beta ] = [ 0 ],       phi(r) = r^k (k odd), r^k log r (k even),
 *
 * B_js = P_s(x_j) the monomials of total degree <= d, and evaluate
 * s(x) = sum_s beta_s P_s(x) + sum_j w_j phi(|x - x_j|) at targets.
 *
 * The library solves the system on the complement of span(B) (eq.
 * phs_linsys_solve) by preconditioned CG, with M applied through the Hadamard
 * low-rank reduction (eq. matvec_hadamard) onto log-kernel or distance-kernel
 * sums evaluated by a 2D fast multipole method (Sec. 2.1), and a Vecchia
 * sparse inverse-Cholesky factor of a Matern covariance as preconditioner
 * (Sec. 2.2, Fig. vecchia_chol).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers (HIP global memory) owned by the
 *    caller, unless marked "host".  They must stay valid until the enqueued work
 *    has completed; ordering is that of the given stream (like hipMemcpyAsync).
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *  - Point arrays are n x 2 row-major float64 (x0, y0, x1, y1, ...).
 *  - Multi-vector arrays are n x nrhs column-major float64 (column r starts at
 *    element r*n).  Results come back in the caller's point order.
 *  - Coordinates: points are normalised inside the plan as
 *    xi = (x - c) * rho, with c the bounding-box centre and rho chosen so the
 *    box fits [-h_k, h_k]^2 (h = 1/4 for k=2, 1 for k=4, 1/2 for odd k).  w and
 *    beta are defined in these normalised coordinates (the paper's rescaling,
 *    eq. M_rho); c and rho are returned by phs_plan_info.  Targets passed to
 *    phs_eval are in user coordinates.  beta is ordered by total degree, then
 *    by descending power of xi_1: 1, xi1, xi2, xi1^2, xi1 xi2, xi2^2, ...
 *  - No entry point aborts or throws.  On a non-OK status the outputs are
 *    unspecified (except PHS_ERR_NOT_CONVERGED, which leaves the last iterate
 *    in w/beta and fills info) and phs_last_error() describes the failure.
 *  - All device memory a plan needs is allocated by phs_plan and
 *    phs_precond_build; phs_matvec, phs_solve and phs_eval allocate nothing.
 *  - A plan is not thread-safe; distinct plans may be used concurrently on
 *    distinct streams.
 */
#ifndef PHS_H
#define PHS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PHS_OK = 0,
  PHS_ERR_INVALID_ARGUMENT = 1, /* bad size, null pointer, unsupported k/degree */
  PHS_ERR_DUPLICATE_POINTS = 2, /* two nodes coincide (M would be singular) */
  PHS_ERR_UNISOLVENT = 3,       /* B has dependent columns on these nodes */
  PHS_ERR_NOT_CONVERGED = 4,    /* PCG hit maxit; last iterate returned */
  PHS_ERR_BREAKDOWN = 5,        /* PCG curvature p^T A p <= 0 (indefinite) */
  PHS_ERR_OUT_OF_MEMORY = 6,    /* a device allocation failed */
  PHS_ERR_DEVICE = 7,           /* a HIP runtime call failed */
  PHS_ERR_NOT_READY = 8         /* phs_precond_export / phs_precond_apply before
                                   phs_precond_build */
} phs_status;

/* Matvec precision.  PHS_FP64: everything in FP64.  PHS_MIXED: far field
 * (FMM expansions) and near field in FP32.  PHS_NEAR32: far field in FP64,
 * near-field pairs in FP32 (coordinates relative to the leaf centre).  In
 * phs_solve the two mixed modes run inside FP64 residual refinement: the exit
 * test is always on the FP64 residual. */
enum { PHS_FP64 = 0, PHS_MIXED = 1, PHS_NEAR32 = 2 };
/* How a plan applies M: by the FMM of Sec. 2.1, or exactly, by all-pairs
 * summation on the GPU (the exact-matvec solver of Sec. 3.3; no FMM tables or
 * expansions are built, and evaluation at targets sums directly too). */
enum { PHS_MATVEC_FMM = 0, PHS_MATVEC_DIRECT = 1 };
enum { PHS_RANGE_NORMALIZED = 0, PHS_RANGE_USER = 1 };

typedef struct phs_plan_s *phs_plan_t; /* opaque; owns all device state */

/* Plan options (Sec. 1 problem statement; Sec. 2.1 FMM parameters). */
typedef struct {
  int32_t k;               /* spline order, 1..4 */
  int32_t poly_degree;     /* total degree d of B; -1 => minimal for k
                              (k odd: ceil(k/2)-1, k even: k/2); must be >= it */
  int32_t precision;       /* default matvec precision used by phs_solve:
                              PHS_FP64, PHS_MIXED or PHS_NEAR32 */
  double fmm_tol;          /* target relative accuracy of the core FMM;
                              0 => 1e-12 (FP64) */
  int32_t leaf_size;       /* mean points per leaf box; 0 => automatic */
  int32_t expansion_order; /* log kernel: terms p; distance kernel: Chebyshev
                              nodes per axis; 0 => from fmm_tol */
  int32_t matvec;          /* PHS_MATVEC_FMM (0) or PHS_MATVEC_DIRECT; with
                              DIRECT the pairs are summed in FP64 for
                              PHS_FP64 and in FP32 (FP32 accumulation) for
                              PHS_MIXED and PHS_NEAR32 */
} phs_plan_opts;

/* Preconditioner options (Sec. 2.2; conditioning-set sizes of Sec. 3). */
typedef struct {
  int32_t m;           /* conditioning-set size |sigma(j)|, 1..63; 0 => 30 (k=2), 50 */
  double nu;           /* Matern smoothness; <= 0 => k/2. Supported: 0.5, 1,
                          1.5, 2, 2.5 */
  double range;        /* Matern range l = 1/alpha; <= 0 => alpha 0.35
                          (2 for k=4, 3 for k=3) in normalised units */
  int32_t range_units; /* PHS_RANGE_NORMALIZED or PHS_RANGE_USER */
  uint64_t seed;       /* seed of the random ordering */
} phs_precond_opts;

/* PCG options (stopping rule: ||r||_2 <= rtol * ||Pi f||_2, r the true
   unpreconditioned residual of the projected system, x0 = 0). */
typedef struct {
  double rtol;         /* 0 => 1e-8 */
  int32_t maxit;       /* 0 => 500 */
  int32_t check_every; /* host convergence check period; 0 => 1 */
  int32_t precision;   /* -1 => plan default; PHS_FP64, PHS_MIXED, PHS_NEAR32 */
} phs_solve_opts;

typedef struct {
  int32_t iters;             /* total inner PCG iterations (all RHS) =
                                iters_fp32 + iters_fp64 */
  int32_t outer_refinements; /* FP64 residual recomputations (mixed mode) */
  double rel_residual;       /* ||Pi(f - M w)|| / ||Pi f|| recomputed with an
                                FP64 matvec at exit (worst RHS) */
  double t_solve;            /* seconds, host wall clock */
  int32_t iters_fp32;        /* inner iterations on a reduced-precision
                                operator (PHS_MIXED or PHS_NEAR32) */
  int32_t iters_fp64;        /* inner iterations on the FP64 operator */
  int32_t fp64_fallback;     /* number of right-hand sides whose reduced-
                                precision solve moved to the FP64 operator
                                (its FP32 steps stopped reducing the FP64
                                residual, or broke down) */
  int32_t reserved;
  double t_plan;             /* seconds phs_plan took for this plan */
  double t_precond;          /* seconds the last phs_precond_build took */
} phs_solve_info;

/* Build a plan for the interpolation problem of Sec. 1 (eqs. phs_interp,
 * phs_linsys): normalise the nodes (eq. M_rho and the tuned domains of
 * Sec. 2.2), sort them into the quadtree of the FMM (Sec. 2.1), build the
 * polynomial block B and its thin QR (eq. phs_linsys_solve), the FMM
 * translation tables and every work table and workspace the later calls use.
 * xy: device, n x 2 row-major (the plan copies it).  opts: host.  out: host,
 * receives the handle (NULL on error).  Synchronises `stream` (it reads back
 * sizes).  Errors: INVALID_ARGUMENT (n < S, bad options), DUPLICATE_POINTS,
 * UNISOLVENT, OUT_OF_MEMORY, DEVICE. */
phs_status phs_plan(const double *xy, int64_t n, const phs_plan_opts *opts,
                    void *stream, phs_plan_t *out);

/* y = M v for the kernel block M only (eq. matvec_hadamard; Sec. 2.1 FMM).
 * v, y: device, n x nrhs.  precision: PHS_FP64, PHS_MIXED or PHS_NEAR32.
 * Allocates no device memory.  Asynchronous. */
phs_status phs_matvec(phs_plan_t plan, const double *v, double *y, int32_t nrhs,
                      int32_t precision, void *stream);

/* Build the Vecchia factor U~ (Sigma^{-1} ~= U~ U~^T) of the Matern covariance
 * on the plan's normalised nodes (eqs. conditionals, vecchia_sumform,
 * Fig. vecchia_chol).  A rebuild replaces the previous factor only when it
 * succeeds: on an error the plan keeps the factor it had (or none).
 * Synchronises `stream`. */
phs_status phs_precond_build(phs_plan_t plan, const phs_precond_opts *opts,
                             void *stream);

/* Solve for w (n x nrhs) and beta (S x nrhs) by projected PCG on
 * Q_perp^T M Q_perp u = Q_perp^T f, w = Q_perp u, then R beta = Q^T (f - M w)
 * (eq. phs_linsys_solve).  f, w, beta: device.  info: host, may be NULL.
 * Preconditioner: the plan's Vecchia factor; before any phs_precond_build the
 * solve runs with the identity (plain projected CG).  Allocates no device
 * memory.  Synchronises `stream` every check_every iterations. */
phs_status phs_solve(phs_plan_t plan, const double *f, int32_t nrhs,
                     const phs_solve_opts *opts, double *w, double *beta,
                     phs_solve_info *info, void *stream);

/* Evaluate the interpolant (eq. phs_interp) at m user-coordinate targets:
 * out[t, r] = sum_s beta[s, r] P_s(xi_t) + sum_j w[j, r] phi(|xi_t - xi_j|).
 * targets: device m x 2; w: n x nrhs; beta: S x nrhs; out: m x nrhs.
 * Targets may lie outside the nodes' bounding box.  A target equal to a node
 * contributes phi(0) = 0 for that node.  Allocates no device memory.
 * Asynchronous. */
phs_status phs_eval(phs_plan_t plan, const double *w, const double *beta,
                    int32_t nrhs, const double *targets, int64_t m, double *out,
                    void *stream);

/* Plan facts.  center[2], scale, S, R, leaf_level, order, tree_half_width:
 * host pointers, any may be NULL.  R is the Hadamard rank (number of
 * core-kernel densities).  The quadtree covers [-t, t]^2 in normalised
 * coordinates, t = tree_half_width (the normalisation half-width h_k). */
phs_status phs_plan_info(phs_plan_t plan, double *center, double *scale,
                         int32_t *S, int32_t *R, int32_t *leaf_level,
                         int32_t *order, double *tree_half_width);

/* Copy the plan's internal node order and leaf keys to caller device buffers
 * (int32, n each): order[i] = caller index of the i-th node in tree order,
 * leaf[i] = its leaf key (row-major box index at the leaf level).  Used to
 * check the tree against an independent reference. */
phs_status phs_plan_tree(phs_plan_t plan, int32_t *order, int32_t *leaf,
                         void *stream);

/* Copy the Vecchia structure in caller index space to caller device buffers:
 * rank[n] (int32, position of each node in the ordering), nbr[n*m] (int32,
 * row j lists sigma(j) ascending by (d^2, rank), padded with -1), coef[n*m]
 * (float64, -lambda/c at the same slots, 0 in padding), diag[n] (1/c_j).
 * m is the plan's conditioning-set size (phs_precond_opts.m). */
phs_status phs_precond_export(phs_plan_t plan, int32_t *rank, int32_t *nbr,
                              double *coef, double *diag, void *stream);

/* z = U~ U~^T r in caller order (no projection).  r, z: device n.  */
phs_status phs_precond_apply(phs_plan_t plan, const double *r, double *z,
                             void *stream);

void phs_plan_destroy(phs_plan_t plan);

/* ---------------------------------------------------------------- batches
 * Many independent interpolation problems, and several right-hand sides per
 * point set, solved together.  Each (plan, right-hand side) pair is one
 * system with its own PCG vectors and FMM workspace; every step of the solve
 * (each FMM stage, the preconditioner apply, each vector update and
 * reduction) is one launch over all systems still iterating, and a system
 * runs exactly the arithmetic it runs alone (results are bitwise equal to
 * phs_solve on that plan).  Problems of different n, order k and polynomial
 * degree can share a batch; all even-k plans must use the same expansion
 * order (the default fmm_tol gives that), while odd-k plans of different
 * Chebyshev orders are launched in one group per order. */
typedef struct phs_batch_s *phs_batch_t;

/* plans: host array of nplans plan handles, which must outlive the batch (a
 * preconditioner built or rebuilt later is picked up by phs_batch_solve).
 * nrhs: host array, right-hand sides per plan (>= 1).  Allocates the
 * workspace of every system; synchronises `stream`.  Errors:
 * INVALID_ARGUMENT (bad counts, mismatched expansion orders), OUT_OF_MEMORY. */
phs_status phs_batch_create(const phs_plan_t *plans, int32_t nplans, const int32_t *nrhs,
                            void *stream, phs_batch_t *out);

/* Solve all problems: f[i], w[i] are device n_i x nrhs_i column-major arrays of
 * plan i (caller order), beta[i] device S_i x nrhs_i; f, w, beta are host
 * arrays of nplans device pointers.  opts as for phs_solve (its precision
 * applies to every system; -1 takes the first plan's default).  info: host
 * array of nplans (may be NULL), filled per plan as by phs_solve, t_solve
 * being the whole batch's time.  Returns the first non-OK status of any
 * system (others still hold their results).  Allocates nothing;
 * synchronises `stream` once per PCG iteration. */
phs_status phs_batch_solve(phs_batch_t batch, const double *const *f, double *const *w,
                           double *const *beta, const phs_solve_opts *opts,
                           phs_solve_info *info, void *stream);

void phs_batch_destroy(phs_batch_t batch);

/* ---------------------------------------------------------------- serving
 * A request loop over solve + evaluate requests of differing size.  Requests
 * wait in a FIFO queue until a slot (max_active) and device memory (an
 * estimate of the request's tree, preconditioner, Krylov vectors and FMM
 * workspace against hbm_budget) are free; admitted requests build their plan
 * and preconditioner and then keep all of it resident in HBM while their PCG
 * iterations run in lockstep with every other active request (continuous
 * batching: one launch per PCG step covers all of them, and requests join or
 * leave between steps).  A finished request is evaluated at its targets, its
 * device memory is released, and a waiting request can take its place.  Each
 * request's results are bitwise those of phs_plan + phs_precond_build +
 * phs_solve + phs_eval with the same options. */
typedef struct phs_server_s *phs_server_t;

typedef struct {
  int64_t hbm_budget;  /* bytes of device memory requests may hold; 0 => 3/4
                          of the free device memory at creation */
  int32_t max_active;  /* requests in flight; 0 => 64 */
  int32_t precision;   /* PHS_FP64, PHS_MIXED or PHS_NEAR32 */
  double rtol;         /* 0 => 1e-8 */
  int32_t maxit;       /* 0 => 500 */
} phs_server_opts;

typedef struct {
  const double *xy;      /* device n x 2 nodes (caller order) */
  const double *f;       /* device n values */
  const double *targets; /* device m x 2 evaluation points (may be NULL if m = 0) */
  int64_t n, m;
  int32_t k, poly_degree;       /* as phs_plan_opts (-1 => minimal degree) */
  phs_precond_opts precond;     /* as phs_precond_build */
  double *w;       /* device n: weights (out) */
  double *beta;    /* device S: polynomial coefficients (out) */
  double *values;  /* device m: interpolant at the targets (out) */
} phs_request;
/* All request arrays are owned by the caller and must stay valid until the
 * request is done or failed (phs_server_poll). */

enum { PHS_REQ_QUEUED = 0, PHS_REQ_ACTIVE = 1, PHS_REQ_DONE = 2, PHS_REQ_FAILED = 3 };

typedef struct {
  int32_t state;          /* PHS_REQ_* */
  int32_t status;         /* phs_status of a done or failed request */
  int32_t iters;          /* PCG iterations */
  double rel_residual;    /* as phs_solve_info */
  double t_submit, t_admit, t_done;  /* seconds since phs_server_create */
  int64_t bytes;          /* device bytes charged to the request */
} phs_request_info;

phs_status phs_server_create(const phs_server_opts *opts, void *stream, phs_server_t *out);

/* Queue a request (host-side only; nothing runs until phs_server_step).  id:
 * host, receives the request id.  Errors: INVALID_ARGUMENT. */
phs_status phs_server_submit(phs_server_t srv, const phs_request *req, int64_t *id);

/* One scheduling step: requests whose plan and preconditioner builds have
 * finished join the active set; waiting requests that fit (slots and memory
 * budget, at most two at a time) are handed to the server's build thread,
 * which builds them on a stream of its own while the steps go on; one PCG
 * round of every active request runs; finished requests are evaluated and
 * released.  With no request active and a build running, the step waits for
 * the build.  active, queued: host, may be NULL, receive the counts after the
 * step (queued includes requests being built).  A failure of one request
 * (bad input, out of memory, breakdown) is recorded in that request and does
 * not fail the step.  Synchronises `stream`. */
phs_status phs_server_step(phs_server_t srv, int32_t *active, int32_t *queued);

/* State and timing of a request.  info: host. */
phs_status phs_server_poll(phs_server_t srv, int64_t id, phs_request_info *info);

/* Device bytes held by requests (active ones, builds in progress at their
 * estimate, and the shared batching structures) now and at most so far
 * (host, may be NULL). */
phs_status phs_server_memory(phs_server_t srv, int64_t *in_use, int64_t *peak);

void phs_server_destroy(phs_server_t srv);

/* Message for the last non-OK status returned on this thread. */
const char *phs_last_error(void);

/* ---------------------------------------------------------------- tuning
 * Preconditioner tuning (Sec. 2.2, closing paragraph: the range alpha and the
 * smoothness were tuned by hand for k = 2 and 4; other orders need their own
 * choices).  On the plan's nodes and the caller's values f (device, n), for
 * each supported Matern smoothness nu in {k/2 - 1/2, k/2, k/2 + 1/2}, a
 * Nelder-Mead simplex over (log alpha, m) minimises the measured seconds of
 * phs_precond_build + phs_solve (FP64) to rtol; trials that do not converge
 * are charged 1000 s.  The normalisation scale is not searched: for the
 * preconditioner it only rescales alpha.  On return the plan holds the best
 * preconditioner found and `out` its figures beside those of the library's
 * defaults on the same problem.  Allocates (trial buffers); synchronises
 * `stream` after every trial. */
typedef struct {
  int32_t max_evals;   /* simplex evaluations per nu; 0 => 16 */
  int32_t maxit;       /* PCG iteration cap per trial; 0 => 300 */
  double rtol;         /* 0 => 1e-8 */
  int32_t m_min, m_max;  /* bounds of the conditioning-set size; 0 => 10, 60 */
} phs_tune_opts;

typedef struct {
  int32_t m;              /* best conditioning-set size */
  double nu;              /* best smoothness */
  double alpha;           /* best inverse range (normalised coordinates) */
  double seconds;         /* its build + solve seconds */
  int32_t iters;          /* its PCG iterations */
  double rel_residual;    /* its FP64 exit residual */
  int32_t evals;          /* trials run, the default's included */
  double default_seconds; /* the library defaults (m = 30 or 50, nu = k/2,
                             alpha = 0.35, 3 or 2) on the same problem */
  int32_t default_iters;
} phs_tune_result;

phs_status phs_tune_precond(phs_plan_t plan, const double *f, const phs_tune_opts *opts,
                            phs_tune_result *out, void *stream);

/* Plan autotuning: expansion order, leaf size and matvec kind for the caller's
 * nodes xy (device, n x 2), order k and degree.  Candidates: the exact
 * all-pairs matvec (n <= 2^17) and the FMM with leaf sizes 16, 24, 32, 48,
 * 64, 96, 128, each at the lowest expansion order (log kernel 15, 23, 27, 31;
 * Chebyshev 8..16) whose matvec of a seeded N(0,1) vector is within
 * matvec_tol (relative 2-norm) of the exact all-pairs sum on 2048 sampled
 * rows.  The fastest candidate by measured matvec time (in `precision`) wins;
 * `best` receives its plan options (pass them to phs_plan).  Allocates;
 * synchronises `stream`.  Errors: NOT_CONVERGED if no candidate meets the
 * tolerance. */
typedef struct {
  double matvec_tol;   /* 0 => 1e-12 */
  int32_t precision;   /* PHS_FP64 (0), PHS_MIXED, PHS_NEAR32 */
  int32_t reps;        /* timed matvecs per candidate; 0 => 5 */
  uint64_t seed;       /* of the test vector and the sampled rows */
} phs_autotune_opts;

typedef struct {
  int32_t matvec, leaf_size, expansion_order, candidates;
  double matvec_seconds;  /* per matvec of the chosen plan */
  double rel_error;       /* its sampled-row error */
} phs_autotune_result;

phs_status phs_autotune_plan(const double *xy, int64_t n, int32_t k, int32_t poly_degree,
                             const phs_autotune_opts *opts, phs_plan_opts *best,
                             phs_autotune_result *out, void *stream);

/* Direct (all-pairs) PHS kernel sums on the GPU, without a plan:
 *   out[t] = sum_j q[j] phi(|targets_t - xy_j|),  phi(r) = r^k (k odd),
 *   r^k log r (k even), phi(0) = 0
 * (the kernel part of eq. phs_interp; with targets = xy it is M q, eq.
 * phs_linsys), in FP64, in the coordinates given (no normalisation).
 * k: 1..4.  xy: device n x 2 row-major; q: device n; targets: device m x 2;
 * out: device m (all caller-owned).  m may be 0.  Cost O(n m): meant for
 * sizes below the FMM's break-even and as an exact check.  The sum over the
 * sources is split into chunks whose partial sums are added in a fixed order
 * (results do not depend on scheduling); the partials live in device scratch
 * that this call takes from the library's pool (released when the device is
 * next idle).  Asynchronous (the first call on a device also uploads a
 * 4 KB logarithm table, synchronously).  Errors: INVALID_ARGUMENT,
 * OUT_OF_MEMORY, DEVICE. */
phs_status phs_direct_sum(int32_t k, const double *xy, int64_t n, const double *q,
                          const double *targets, int64_t m, double *out, void *stream);

/* phs_direct_sum for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, the same kernels and the same split of the sources, so
 * the results are bitwise those of phs_direct_sum; but it calls no hipMalloc,
 * hipFree or other allocating routine.  The chunk partials go to a static
 * device array of 2^20 doubles (8 MiB) per GPU, held until the process ends;
 * its address is looked up on the first call on each device (which, like
 * phs_direct_sum's first call, also uploads a 4 KB table).  Every size is
 * accepted (the split never needs more than 2^20 partials); a split that
 * would is rejected with INVALID_ARGUMENT.  All calls on one GPU share the
 * array: calls that overlap on one GPU (other streams or threads) race and
 * must be serialised by the caller.  Asynchronous. */
phs_status phs_direct_sum_noalloc(int32_t k, const double *xy, int64_t n, const double *q,
                                  const double *targets, int64_t m, double *out,
                                  void *stream);

/* Device-memory counters of the library's caching pool (all host pointers,
 * any may be NULL): allocations = blocks handed out so far (from the cache or
 * fresh), device_mallocs = hipMalloc calls so far, bytes_in_use = bytes handed
 * out and not yet released (a released block counts until the device is next
 * idle), bytes_held = device bytes the pool owns (in use and cached).  Lets a
 * caller check that a call allocated nothing, and what the library holds. */
phs_status phs_memory_stats(int64_t *allocations, int64_t *device_mallocs,
                            int64_t *bytes_in_use, int64_t *bytes_held);

/* PCG iterations through HIP graphs.  on = 1: the launch sequences of a
 * projected-PCG iteration (operator, projection, update and scalar gather;
 * preconditioner apply and search-direction update) are captured once per
 * plan, batch or serving forest, the second time each runs, and replayed with
 * one graph launch each; the results are bitwise those of the direct
 * launches.  Iterations with an FP32 operator, solves checked less often than
 * every iteration, and everything while per-kernel timing is on run as direct
 * launches.  on = 0 (the default): direct launches only; on MI355X the
 * replays measured 1-2 % slower than direct launches, from 2000-node solves
 * to 2^20.  Process-wide; takes effect at the next iteration. */
void phs_set_graphs(int32_t on);

/* Per-kernel timing.  on = 1: each library kernel launch is bracketed by HIP
 * events on its own stream; on = 2: only the leaf, M2L, Vecchia factor and
 * KNN, preconditioner-apply and all-pairs kernels; 0: off.  phs_profile_read copies up
 * to `cap` records (name, launches, total milliseconds) to host arrays and
 * resets the counters.  names: host array of `cap` char[48].  Returns the
 * number of records. */
void phs_profile_enable(int32_t on);
int32_t phs_profile_read(char (*names)[48], int64_t *launches, double *total_ms,
                         int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* PHS_H */

/*
 * fkgp -- MI355X (gfx950) implementation of the hot path of "Faster Kernel
 * Interpolation for Gaussian Processes" (Yadav, Sheldon, Musco).
 *
 * Structured kernel interpolation (SKI) approximates the kernel matrix as
 * W K_G W^T (Sec. 2.3, Eq. (ski)); W (n x m) holds each point's cubic
 * interpolation stencil and K_G (m x m) is the kernel on an equispaced grid.
 * Sec. 3 shows SKI is exact inference in a Bayesian linear regression on the
 * m grid basis functions (Def. 3, Theorem 1, Fact 2), so after one O(n) pass
 * that builds the sufficient statistics W^T W, W^T y and y^T y (Sec. 3.1,
 * Claim 2) every solver iteration costs O(m log m) independently of n.  The
 * factorized conjugate-gradient methods of Sec. 4 and the appendix keep every
 * n-vector in the compressed form W z_hat + c z_0 (Claims 3 and 4), so the
 * method still solves the original symmetric SKI system.
 *
 * Conventions for every entry point:
 *   - Pointers named x, y, rhs, out, mean_grid, wtw, wty, xq are DEVICE
 *     pointers on the current HIP device; `stream` is a hipStream_t (NULL =
 *     the null stream).  The caller owns them; the library never frees them.
 *   - The library owns a handle's internals (allocated on the current device)
 *     until fkgp_destroy.  A handle is immutable after fkgp_precompute, so
 *     calls on different streams may share it.
 *   - Device memory (handles and per-call scratch) comes from the device's
 *     default stream-ordered pool, whose release threshold the library
 *     raises on first use: freed memory stays cached in the process for
 *     reuse by later calls (as a caching allocator does).
 *   - Grid nodes of dimension k sit at origin[k] + j*spacing[k], j < m[k];
 *     nodes are flattened in C order (dimension 0 slowest).  Grid vectors
 *     (length M = prod m) use that order.
 *   - No exception crosses the ABI.  Arguments are validated on the host
 *     before any launch; on failure the function returns a negative status
 *     and fkgp_last_error() gives a message.  Functions that return host
 *     scalars synchronise `stream`.
 */
#ifndef FKGP_H
#define FKGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FKGP_OK = 0,
    FKGP_ENOTCONV = 1,     /* solver hit maxiter; result written, see info */
    FKGP_EINVAL = -1,      /* invalid argument (message in fkgp_last_error) */
    FKGP_EOUTOFGRID = -2,  /* a point lies outside the interpolable region */
    FKGP_ENOMEM = -3,      /* device allocation failed */
    FKGP_EDEVICE = -4      /* HIP runtime error */
} fkgp_status;

typedef enum { FKGP_F32 = 0, FKGP_F64 = 1 } fkgp_dtype;

/* Equispaced grid, 1 <= d <= 3, 4 <= m[k] <= 65536 (the K_G line FFTs embed
 * each dimension in a circulant of at most 131072 points; fkgp_precompute
 * returns FKGP_EINVAL beyond that; fkgp_batch_mll_and_grad takes dimensions
 * of at most 8192 nodes), spacing[k] > 0.  A point x is
 * interpolable iff 1 <= (x_k - origin_k)/spacing_k <= m_k - 2 for every k, so
 * that all four cubic stencil nodes exist. */
typedef struct {
    int d;
    int64_t m[3];
    double origin[3];
    double spacing[3];
} fkgp_grid;

/* Product of one-dimensional stationary kernels inside a scale kernel,
 * k(x,x') = outputscale * prod_k k1(|x_k - x'_k| / l_k) (a product stationary
 * kernel makes K_G multilevel Toeplitz, Sec. 2.3), and Gaussian noise of
 * standard deviation noise_std (Sec. 2.1), i.e. noise variance noise_std^2
 * on the diagonal.  k1(r): squared exponential exp(-r^2/2) (the kernel of
 * Sec. 5), or Matern nu = 1/2, 3/2, 5/2: exp(-r), (1 + sqrt3 r) exp(-sqrt3 r),
 * (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r). */
typedef enum {
    FKGP_KERNEL_SE = 0,
    FKGP_KERNEL_MATERN12 = 1,
    FKGP_KERNEL_MATERN32 = 2,
    FKGP_KERNEL_MATERN52 = 3
} fkgp_kernel;

typedef struct {
    double lengthscale[3];
    double outputscale;
    double noise_std;
    int kernel;              /* fkgp_kernel */
} fkgp_hypers;

typedef struct fkgp_handle fkgp_handle;

/* Interpolation scheme of W (Sec. 2.3: SKI may use any local scheme).
 * Cubic: Keys' cubic convolution (a = -1/2), 4^d weights per point, W^T W
 * within offsets -3..3 per dimension (Claim 2, r = 2).  Linear: 2^d weights
 * per point (the nodes either side of the point in each dimension), W^T W
 * within offsets -1..1 (r = 1).  Both use the same interpolable region
 * (1 <= (x_k - origin_k) / spacing_k <= m_k - 2) and the same stencil-
 * diagonal storage; for linear W^T W the offset slabs outside -1..1 are all
 * zero and the products skip them through the block mask. */
typedef enum { FKGP_INTERP_CUBIC = 0, FKGP_INTERP_LINEAR = 1 } fkgp_interp;

typedef struct {
    fkgp_dtype stats_dtype;  /* storage of W^T W and precision of the operator
                                B(x) = ((K_G W^T W + s2 I)x, W^T W x); FP32
                                or FP64.  CG vectors and scalars are FP64. */
    int n_probes;            /* Rademacher probe sketches W^T z_j to build
                                (0..31), for fkgp_mll_and_grad (in 3-D the
                                sort carries the point index in the slot of
                                y, which the moments then read by index) */
    uint64_t probe_seed;     /* z_j[i] = 1 - 2*(SplitMix64((seed<<48) ^
                                (j<<40) ^ i) >> 63) */
    int keep_points;         /* 1: the handle also keeps the points in cell
                                order (n * 4 values of the input dtype) and
                                the cell bounds, for fkgp_ski_solve (in 3-D
                                with probe sketches, y is put back into the
                                kept points from the input after the sort) */
    int interp;              /* fkgp_interp: the interpolation scheme of W,
                                used by every later call on the handle */
} fkgp_precompute_opts;

/* One-shot O(n) pass (Sec. 3.1 "Precomputation", Claim 2).
 *   x: d device pointers, x[k][i] = coordinate k of point i (dtype `in`);
 *   y: n responses (dtype `in`); n >= 0 (n = 0 gives zero statistics).
 * Builds W^T W (at most 7^d nonzeros per row for cubic interpolation, Claim
 * 2), W^T y, y^T y and the optional probe sketches, deterministically:
 * points are sorted by grid cell and each cell is reduced in a fixed order;
 * no floating-point atomics are used.  Returns FKGP_EOUTOFGRID if any point
 * is not interpolable (NaN included); *out is then NULL.
 * Synchronises `stream`. */
fkgp_status fkgp_precompute(const fkgp_grid* grid, const void* const* x,
                            const void* y, int64_t n, fkgp_dtype in,
                            const fkgp_precompute_opts* opts, void* stream,
                            fkgp_handle** out);

typedef struct {
    int64_t n;
    int64_t m_total;
    int d;
    fkgp_dtype stats_dtype;
    int n_probes;
    double yty;
    int64_t bytes_wtw;       /* device bytes of the stored W^T W */
    int64_t nnz_wtw;         /* stored stencil-diagonal entries (m * 7^d) */
    int64_t halo;            /* zero padding on each side of a vector passed
                                to fkgp_wtw_matvec: 3 * sum_k stride_k */
    int64_t wtw_blocks;      /* blocks of the stored W^T W: a 64-row chunk of
                                rows times an offset slab (the 49 offsets
                                sharing o_0 for d = 3; all 7^d for d <= 2) */
    int64_t wtw_blocks_nonzero; /* blocks holding a nonzero entry; the banded
                                product reads only these (points that do not
                                fill the grid's box leave whole blocks zero) */
    int64_t wtw_block_entries;  /* stored entries per block (64 * 49 or 64 * 7) */
    int interp;              /* fkgp_interp of the handle */
    int64_t nnz_wtw_nonzero; /* stored entries of W^T W that are nonzero (the
                                exact nonzero count, counted on the device) */
} fkgp_handle_desc;

fkgp_status fkgp_describe(const fkgp_handle* h, fkgp_handle_desc* desc);

/* Copies the statistics out.  wtw: device buffer of m * 7^d elements of the
 * handle's stats dtype in the canonical layout [j][o] (o in [-3,3]^d, C
 * order; entry (j,o) = (W^T W)[j, j+o], 0 when j+o leaves the grid).  wty:
 * device buffer of m doubles.  yty: host double.  Any pointer may be NULL.
 * Synchronises `stream`. */
fkgp_status fkgp_export_stats(const fkgp_handle* h, void* wtw, double* wty,
                              double* yty, void* stream);

/* Probe sketches W^T z_j, j < n_probes, as [n_probes][m] doubles (device). */
fkgp_status fkgp_export_sketches(const fkgp_handle* h, double* out, void* stream);

/* Arithmetic of the operator B inside the CG loop.  The stored W^T W keeps
 * the handle's stats dtype either way (it is what HBM traffic is made of).
 *   FKGP_OP_F64:   vectors, FFTs and accumulation in FP64 (FP32-stored
 *                  entries are upcast exactly); the solver is the printed
 *                  simplified factorized CG.
 *   FKGP_OP_STATS: arithmetic in the stats dtype; for FP32 handles the FP32
 *                  CG is the inner solver of an FP64 iterative refinement
 *                  (residual recomputed in FP64 after every inner solve). */
typedef enum { FKGP_OP_F64 = 0, FKGP_OP_STATS = 1 } fkgp_op_precision;

typedef struct {
    double tol;        /* relative residual: stop when ||r|| <= tol ||b|| */
    int maxiter;
    fkgp_op_precision op_precision;
} fkgp_solve_opts;

typedef struct {
    int iterations;
    int converged;
    double rel_residual;   /* relative residual at exit (recursive for
                              FKGP_OP_F64, recomputed in FP64 otherwise) */
} fkgp_solve_info;

/* Posterior mean on the grid, or a grid right-hand side solve, with the
 * simplified efficiently-factorized CG of the appendix (one operator
 * application B per iteration; needs only W^T W and W^T y).
 *   rhs_grid == NULL: x_0 = y/s2, r_hat_0 = -K_G W^T y/s2; out (m doubles) =
 *     mu_G = K_G W^T z~ with z~ = (W K_G W^T + s2 I)^{-1} y, the grid weights
 *     of the SKI mean (Def. 2; Fact 2 and Claim 5 equate the two forms);
 *     the mean at any x is w_x^T mu_G (fkgp_interpolate).
 *   rhs_grid != NULL (m doubles, b = W rhs_grid): x_0 = 0, r_hat_0 = rhs;
 *     out = W^T (W K_G W^T + s2 I)^{-1} W rhs_grid.
 * Returns FKGP_ENOTCONV if maxiter is reached (out still written).
 * Synchronises `stream`. */
fkgp_status fkgp_solve(const fkgp_handle* h, const fkgp_hypers* hyp,
                       const double* rhs_grid, double* out,
                       const fkgp_solve_opts* opts, fkgp_solve_info* info,
                       void* stream);

/* fkgp_solve for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid device or pinned
 * allocations): the same solve and the same results as fkgp_solve, with
 * every buffer of the call (spectra, CG vectors, reduction partials, state)
 * carved from a fixed 64 MiB device workspace that the library holds, one
 * per GPU, until the process ends; no hipMalloc, hipFree, pinned host memory
 * or other allocating routine is called, and convergence is checked by a
 * synchronous copy of the solver state after every 8 iterations.
 * Returns FKGP_EINVAL (before any launch) when the grid needs more workspace
 * than that, as grids of more than about 500,000 nodes do, or grids with a
 * dimension of more than 1024 nodes that takes the four-step line FFT.  All
 * calls on one GPU share its workspace: calls that overlap on one GPU (other
 * host threads, other streams) race and must not be made.
 * Synchronises `stream`. */
fkgp_status fkgp_solve_noalloc(const fkgp_handle* h, const fkgp_hypers* hyp,
                               const double* rhs_grid, double* out,
                               const fkgp_solve_opts* opts, fkgp_solve_info* info,
                               void* stream);

/* k grid right-hand sides at once: out_j = W^T (W K_G W^T + s2 I)^{-1} W rhs_j
 * (the rhs_grid case of fkgp_solve for each column).  rhs_grid, out: device
 * doubles [k][m].  The solves advance together, 64 at a time, from x_0 = 0
 * with the residual kept as W r_hat (r_hat_0 = rhs_j), so each iteration
 * reads W^T W once for the batch; each stops at ||r|| <= tol ||W rhs_j||
 * (Claim 4 inner products; only W^T W enters).  opts->op_precision must be
 * FKGP_OP_F64.  info: the most iterations of any column, and the largest
 * relative residual.  FKGP_ENOTCONV if a column reached maxiter (out still
 * written).  Synchronises `stream`. */
fkgp_status fkgp_solve_multi(const fkgp_handle* h, const fkgp_hypers* hyp,
                             const double* rhs_grid, int k, double* out,
                             const fkgp_solve_opts* opts, fkgp_solve_info* info,
                             void* stream);

typedef struct {
    int lanczos_steps;  /* tridiagonal size used for each probe (<= iters,
                           at most 64) */
    double tol;         /* relative residual for the y and probe solves */
    int maxiter;
    int batched;        /* 1: all probes advance together (one W^T W read per
                           iteration for every probe); 0: one probe at a time.
                           Operator arithmetic is FP64 either way (on the
                           stored W^T W, FP32 entries upcast exactly). */
    int batch_rhs;      /* fkgp_batch_mll_and_grad only: right-hand sides per
                           workgroup (2, 4 or 8); 0 = autotune */
    int batch_block;    /* fkgp_batch_mll_and_grad only: threads per
                           workgroup (256 or 512); 0 = autotune.  Autotuning
                           times a short trial of each candidate and caches
                           the fastest per batch shape for the process. */
    int trace_mode;     /* gradient of the log-determinant term: 0 =
                           Hutchinson traces tr(A^{-1} dA) over the probes
                           (the solves the MLL already ran); 1 = exact
                           traces, through S = W^T A^{-1} W from m grid
                           right-hand-side solves (fkgp_mll_and_grad only,
                           m <= 4096; for checks against finite differences
                           of the exact MLL); 2 = the derivative of the
                           stochastic Lanczos estimate itself, by reverse
                           mode through each probe's lanczos_steps Lanczos
                           steps (the first residuals of its factorized CG
                           are checkpointed as the Lanczos vectors; Sec. 2.1
                           and the appendix's factorized Lanczos), so the
                           gradient is exactly that of the returned MLL
                           (fkgp_mll_and_grad only; probes batched; at most
                           64 probes).  The log-determinant value is the
                           stochastic Lanczos estimate in every mode. */
} fkgp_mll_opts;

typedef struct {
    double logdet;      /* stochastic Lanczos quadrature estimate */
    double quad;        /* y^T (W K_G W^T + s2 I)^{-1} y */
    int iterations_y;
    int iterations_probes_max;
    int batch_rhs;      /* fkgp_batch_mll_and_grad: right-hand sides per
                           workgroup used (0 for fkgp_mll_and_grad) */
    int batch_block;    /* fkgp_batch_mll_and_grad: threads per workgroup used */
    double dquad[5];    /* gradient of quad = y^T A^{-1} y with respect to
                           (log l_0 .. log l_{d-1}, log outputscale,
                           log noise_std): -x_y^T (dA/dtheta) x_y with
                           x_y = A^{-1} y (the deterministic part of the
                           gradient; entries past d + 1 are 0) */
} fkgp_mll_info;

/* Log marginal likelihood (Def. 2 / Fact 2) and its gradient with respect to
 * (log l_0 .. log l_{d-1}, log outputscale, log noise_std); grad has d + 2
 * host doubles.  logdet(W K_G W^T + s2 I) comes from stochastic Lanczos
 * quadrature over the handle's probes with tridiagonals taken from the
 * factorized-CG coefficients; the gradient is 1/2[x_y^T dA x_y -
 * tr(A^{-1} dA)] with the trace estimated from the same probe solves.
 * Requires n_probes > 0 at precompute.  Synchronises `stream`. */
fkgp_status fkgp_mll_and_grad(const fkgp_handle* h, const fkgp_hypers* hyp,
                              const fkgp_mll_opts* opts, double* mll,
                              double* grad, fkgp_mll_info* info, void* stream);

/* The same quantities for nprob independent problems (handles with probe
 * sketches, d <= 2, any mix of sizes) in one persistent launch: every
 * right-hand side [y, z_0 .. z_{N-1}] of every problem is solved with the
 * factorized CG (Claims 3 and 4), the probes from x_0 = 0 and y from
 * x_0 = y / sigma^2 (residual in the span of W, as fkgp_solve); a workgroup
 * owns one problem and up to opts->batch_rhs of its right-hand sides
 * (autotuned when 0) and runs their CG to the end, so the stored W^T W is
 * read once per iteration for all of them.
 *   hyps: nprob hyperparameter sets; mll: nprob host doubles; grad: nprob x 5
 *   host doubles (entries d+2 .. 4 of each row are 0); infos: nprob (or
 *   NULL).  opts->batched is ignored.  Synchronises `stream`. */
fkgp_status fkgp_batch_mll_and_grad(const fkgp_handle* const* hs, int nprob,
                                    const fkgp_hypers* hyps, const fkgp_mll_opts* opts,
                                    double* mll, double* grad, fkgp_mll_info* infos,
                                    void* stream);

/* out[i] = w_{xq_i}^T mean_grid (Fact 2 mean) for nq query points; xq: d
 * device pointers of dtype `in`; mean_grid, out: device doubles.
 * Returns FKGP_EOUTOFGRID if a query point is not interpolable.
 * Synchronises `stream`. */
fkgp_status fkgp_interpolate(const fkgp_handle* h, const double* mean_grid,
                             const void* const* xq, int64_t nq, fkgp_dtype in,
                             double* out, void* stream);

/* Posterior covariance of the SKI model between nq query points (the
 * covariance expression of SKI inference, Def. 2; by Fact 2
 * and Claim 5 it is also w_x^T C w_x' with C the posterior covariance of the
 * grid values):
 *   cov = Wq K_G Wq^T - Wq K_G W^T (W K_G W^T + s2 I)^{-1} W K_G Wq^T.
 * Column j of K_G Wq^T is the grid vector v_j = K_G w_{xq_j}; each
 * right-hand side b_j = W v_j is solved by the factorized CG from x_0 = 0,
 * which needs only W^T b_j = W^T W v_j and ||b_j||^2 = v_j^T W^T W v_j, so
 * the cost is independent of n (batches of 64 right-hand sides, one W^T W
 * read per iteration for the batch).  Then
 * cov[i][j] = w_i^T v_j - v_i^T W^T A^{-1} b_j, returned symmetrised
 * ((c_ij + c_ji)/2, FP64, fixed-order sums).  Each solve stops at
 * ||r|| <= tol ||b_j||.  xq: d device pointers of dtype `in`; cov: device
 * doubles [nq][nq], row-major; 1 <= nq <= 4096, FKGP_EINVAL otherwise.
 * Device memory: about 3 nq m doubles plus the solver's workspace for 64
 * right-hand sides.  FKGP_EOUTOFGRID if a query point is not interpolable;
 * FKGP_ENOTCONV if a solve reached maxiter (cov still written); info
 * (optional): the most iterations of any solve, and the largest relative
 * residual.  Synchronises `stream`. */
fkgp_status fkgp_posterior_cov(const fkgp_handle* h, const fkgp_hypers* hyp,
                               const void* const* xq, int64_t nq, fkgp_dtype in,
                               double tol, int maxiter, double* cov,
                               fkgp_solve_info* info, void* stream);

/* Rank-k posterior covariance (the low-rank covariance of Sec. 5) from the
 * efficiently factorized Lanczos algorithm (Alg. 7): k Lanczos steps on
 * A = W K_G W^T + s2 I started at y / ||y||, with the Lanczos vectors kept in
 * the factorized form Q_i = W qh_i + d_i y (only W^T W, W^T y and y^T y
 * enter; one operator B per step) and orthogonalised against all earlier
 * ones (two Gram-Schmidt passes).  The cache keeps C = L^{-1} (Q^T W K_G)
 * with T = L L^T (m x k doubles, owned by the cache), so that afterwards
 *   cov(x, x') ~ w_x^T K_G w_x' - (C w_x) . (C w_x')
 * costs O(k 4^d) per query point and O(k) per pair.  The approximation
 * replaces A^{-1} by its restriction to the Krylov space; it is exact once
 * the space holds every W K_G w_x, and the variances fall towards the exact
 * ones as k grows. */
typedef struct fkgp_love fkgp_love;

/* Builds the cache for the hypers `hyp`.  1 <= k <= 10000 (clamped to
 * m + 1, the largest Krylov dimension); fewer steps are taken when the
 * Krylov space is exhausted (beta_{i+1} <= 1e-10 max |alpha|).  Needs
 * y^T y > 0.  Device memory during the build: about 2 k m doubles.
 * Synchronises `stream`.  *out is NULL on error. */
fkgp_status fkgp_love_build(const fkgp_handle* h, const fkgp_hypers* hyp, int k,
                            void* stream, fkgp_love** out);

/* The Lanczos coefficients of a cache: *rank = steps taken; alpha (rank),
 * beta (rank - 1) and d (rank: the y-coefficients of the Lanczos vectors)
 * are host arrays, each may be NULL. */
fkgp_status fkgp_love_tridiag(const fkgp_love* c, int* rank, double* alpha,
                              double* beta, double* d);

/* cov [nq][nq] (device doubles, row-major) between nq query points (xq: d
 * device pointers of dtype `in`), 1 <= nq <= 4096; symmetric.
 * FKGP_EOUTOFGRID if a query point is not interpolable.  Synchronises
 * `stream`. */
fkgp_status fkgp_love_cov(const fkgp_love* c, const void* const* xq, int64_t nq,
                          fkgp_dtype in, double* cov, void* stream);

void fkgp_love_destroy(fkgp_love* c);

/* Operator-level entry points (for tests and benchmarks).
 * fkgp_apply_B: for k right-hand sides stored as [k][m] in the handle's stats
 * dtype, v = (K_G W^T W + s2 I) x and u = W^T W x (the operator B of the
 * efficiently factorized CG); u may be NULL.  Does not synchronise. */
fkgp_status fkgp_apply_B(const fkgp_handle* h, const fkgp_hypers* hyp,
                         const void* x, void* v, void* u, int k, void* stream);

/* out = K_G x for k grid vectors [k][m] in the handle's stats dtype, through
 * per-dimension circulant embeddings and batched radix-2 FFTs.  Does not
 * synchronise. */
fkgp_status fkgp_kg_matvec(const fkgp_handle* h, const fkgp_hypers* hyp,
                           const void* x, void* out, int k, void* stream);

/* u = (W^T W) x for k vectors (Claim 2: at most 7^d nonzeros per row, so
 * one product costs O(m 7^d)).  x: [k][m + 2*halo] of dtype `xdt` (the
 * handle's stats dtype, or FKGP_F64 for FP64 vectors against FP32-stored
 * entries, the product inside the FP64-arithmetic CG), each vector stored at
 * offset halo with halo zeros on both sides (halo from fkgp_describe);
 * u: [k][m] of dtype `xdt`.  One kernel launch reads the stored W^T W once
 * for all k vectors.  Does not synchronise. */
fkgp_status fkgp_wtw_matvec(const fkgp_handle* h, const void* xpad, void* u, int k,
                            fkgp_dtype xdt, void* stream);

/* The banded product as the factorized CG's loop launches it (Claim 2; one
 * per iteration of the simplified factorized CG of the appendix): u = (W^T W) x
 * for one FP64 vector (xdt must be FKGP_F64; x padded as for
 * fkgp_wtw_matvec) with the dot product u^T x reduced inside the same launch
 * (the last workgroup sums the per-tile partials in index order) when the
 * tiled kernel runs, else by a separate reduction.  The launch is repeated
 * `reps` >= 1 times on the same input (a timing aid); *dot (a device double)
 * receives u^T x.  Does not synchronise. */
fkgp_status fkgp_wtw_matvec_dot(const fkgp_handle* h, const void* xpad, void* u,
                                fkgp_dtype xdt, double* dot, int reps, void* stream);

/* fkgp_precompute from points in host memory (x: d host pointers, y: host
 * pointer, dtype `in`), for data sets larger than one transfer or device
 * copy (Sec. 5, "Very large n").  n > chunk: the points stream in chunks of
 * `chunk` points (0: 2^24): each chunk is copied into pinned staging memory
 * and sent to the device on a second stream while the previous chunk is
 * sorted and reduced; the per-cell moments of the chunks are summed in chunk
 * order (deterministic; equal to the one-shot statistics up to the order of
 * the per-cell sums), then assembled once.  n <= chunk: one copy and the
 * one-shot precompute.  Probe sketches (n_probes) follow each point's index
 * in the whole data set, so they equal the one-shot sketches; keep_points
 * must be 0.  Out-of-grid points are reported with their global index.
 * Synchronises `stream`. */
fkgp_status fkgp_precompute_host(const fkgp_grid* grid, const void* const* x,
                                 const void* y, int64_t n, fkgp_dtype in,
                                 const fkgp_precompute_opts* opts, int64_t chunk,
                                 void* stream, fkgp_handle** out);

/* Saves the statistics of a handle (W^T W, its block mask, W^T y, y^T y, the
 * probe sketches, grid and sizes) to the file `path`, so that they are
 * computed once and reused by later sessions (Sec. 5, "Very large n").  A
 * fixed 136-byte header ("FKGPSTAT", version 2; it also records the
 * interpolation scheme) and the arrays in host byte order;
 * kept points are not saved.  Synchronises `stream`.  FKGP_EINVAL if the file
 * cannot be written. */
fkgp_status fkgp_save(const fkgp_handle* h, const char* path, void* stream);

/* A new handle from a file written by fkgp_save (same results as the handle
 * that was saved).  FKGP_EINVAL if the file is missing, of another kind or
 * version, truncated or longer than its header says; *out is then NULL.
 * Synchronises `stream`. */
fkgp_status fkgp_load(const char* path, void* stream, fkgp_handle** out);

/* The plain SKI posterior mean, as the comparison baseline of the method
 * (Sec. 2.3: each CG iteration applies W K_G W^T + s2 I to an n-vector, so
 * it costs O(n + m log m), where the factorized CG's costs O(m log m)).  CG
 * in n-space on (W K_G W^T + s2 I) z = y from z = 0, stopped at
 * ||r|| <= tol ||y||; mean_grid (m doubles) = K_G W^T z, the same grid
 * weights fkgp_solve returns (Theorem 1 / Fact 2).  W^T v is formed
 * deterministically from the points kept in cell order (per-cell moments,
 * fixed-order sums), W v by gathering the 4^d stencil nodes of each point.
 * Needs a handle made with keep_points, else FKGP_EINVAL.
 * Synchronises `stream`. */
fkgp_status fkgp_ski_solve(const fkgp_handle* h, const fkgp_hypers* hyp, double tol,
                           int maxiter, double* mean_grid, fkgp_solve_info* info,
                           void* stream);

/* Device memory allocator of the library.  alloc(bytes, stream, ctx) returns
 * device memory usable in stream order on `stream` (NULL on failure, which
 * the calling entry point reports as FKGP_ENOMEM); free(ptr, stream, ctx)
 * releases it after the work queued on `stream` (stream NULL: the device's
 * null stream, after a device synchronisation).  Pinned host staging and the
 * small pinned slots of the solvers' convergence checks stay with HIP. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* ctx);
    void (*free)(void* ptr, void* stream, void* ctx);
    void* ctx;
} fkgp_allocator;

/* Sets the allocator for all later device allocations of the library (the
 * handles' statistics, the rank-k caches and every call's workspace); NULL
 * restores stream-ordered allocation from the device's default pool.
 * Process-wide; each allocation is freed through the allocator that made it,
 * so handles made before a change stay valid.  FKGP_EINVAL if alloc or free
 * is NULL. */
fkgp_status fkgp_set_allocator(const fkgp_allocator* a);

void fkgp_destroy(fkgp_handle* h);

/* Message of the last error on the calling thread ("" if none). */
const char* fkgp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FKGP_H */

/*
 * krr.h — C ABI of the MI355X (gfx950) Gaussian kernel ridge regression library.
 *
 * Problem (arXiv 1905.10587, Sec. 1, Eq. 1 and Eq. ridge_regression): given points
 * X in R^{n x d}, labels y and a ridge parameter beta > 0, solve (K + beta I) alpha = y
 * with K_ij = exp(-||x_i - x_j||^2 / eps).  The paper writes the Gaussian with bandwidth
 * h (Sec. 2.4, Eq. dscrt_gt); here eps = h^2.
 *
 * Conventions for every entry point
 *   - Array arguments marked [dev] are DEVICE pointers, [host] are host pointers.
 *     All matrices are C-contiguous row-major: X is n x d (point i at X + i*d),
 *     a block of R vectors over n points is n x R (V[i*R + r]).
 *   - The caller owns every buffer it passes.  A krr_precond handle owns its own
 *     device buffers and frees them in krr_precond_free.
 *   - All GPU work is enqueued on `stream` (a hipStream_t; NULL = default stream).
 *     Entry points that return host scalars synchronise that stream first.
 *   - Return value: a krr_status.  Nothing aborts or throws across the ABI.  On an
 *     error the outputs are left unspecified and krr_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - Arguments are validated before any GPU work: n, m >= 1; 1 <= d <= KRR_MAX_D;
 *     eps > 0 and finite; beta > 0 (Sec. 1); 1 <= k <= l <= n; R >= 1; tol > 0.
 *     Violations return KRR_EINVAL.
 *   - Device memory comes from the allocator registered with krr_set_allocator
 *     (PyTorch's caching allocator in the Python binding) or from hipMalloc.
 */
#ifndef KRR_H_
#define KRR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KRR_MAX_D 128

typedef enum {
  KRR_OK = 0,
  KRR_EINVAL = -1,      /* invalid argument (sizes, eps, beta, non-finite input, unknown beta) */
  KRR_ENOMEM = -2,      /* device allocation failed */
  KRR_EHIP = -3,        /* a HIP runtime call failed */
  KRR_ENOTSPD = -4,     /* Cholesky of beta I + W^T W failed (impossible in exact arithmetic) */
  KRR_EBREAKDOWN = -5,  /* PCG breakdown: p^T A p <= 0 or not finite */
  KRR_ENOCONV = 1       /* warning: maxit reached; alpha holds the last iterate */
} krr_status;

typedef enum {
  KRR_FP64 = 0,   /* everything in FP64 */
  KRR_FP32 = 1,   /* kernel MVM in FP32 (differences, exp, accumulation), FP64 scalars and vectors */
  KRR_MIXED = 2   /* cross term x_i.x_j as split-BF16 products on MFMA with FP32 accumulation,
                     FP32 exp; FP64 scalars, vectors, residual replacement and core Cholesky */
} krr_precision;

/* Library version (major*10000 + minor*100 + patch). */
int krr_version(void);

/* Optional: load the code objects of the preconditioner's dense products on `stream` (one tiny launch of
 * each) so that the first build does not pay for it, and look up this device's address of the scratch
 * array of krr_precond_apply_noalloc. */
int krr_init(void* stream);

/* Message describing the last error on this thread ("" if none). */
const char* krr_last_error(void);

/* Device memory provider.  alloc(bytes, stream, ctx) returns a device pointer or NULL;
 * free_(ptr, ctx) releases it.  Passing alloc == NULL restores hipMalloc/hipFree.
 * Buffers allocated for a call are released (stream-ordered) before the call returns. */
int krr_set_allocator(void* (*alloc)(size_t bytes, void* stream, void* ctx),
                      void (*free_)(void* ptr, void* ctx), void* ctx);

/*
 * Kernel matrix times a block of vectors (the paper's FIG(targets, sources, h, V);
 * Sec. 2.4, Def. figtree_def, computed exactly by direct summation; Algorithm 5 applies
 * it as Kx).
 *
 *   U[i, r] = sum_j k(Xt_i, Xs_j) V[j, r]  (+ shift[r] * V[i, r])
 *
 *   Xt [dev]  m x d targets;  Xs [dev] n x d sources (may equal Xt).
 *   V  [dev]  n x R;  U [dev] m x R (deriv 0 or 1) or m x 2R (deriv 2: K V then K' V
 *             interleaved per row: U[i, 0..R-1] = (K V)_i, U[i, R..2R-1] = (K' V)_i).
 *   shift [host] R values or NULL; requires m == n and Xt describing the same points
 *             as Xs (the ridge term beta I).
 *   deriv: 0 -> K, 1 -> K' = eps dK/deps = (D^2/eps) K, 2 -> both.
 *   prec: KRR_FP64, KRR_FP32 or KRR_MIXED (see krr_precision).
 */
int krr_kernel_mv(const double* Xt, int64_t m, const double* Xs, int64_t n, int32_t d,
                  double eps, const double* V, int32_t R, const double* shift,
                  int32_t deriv, int32_t prec, double* U, void* stream);

/*
 * Anchor-selection sketch (Algorithm 1 / Algorithm 2, Sec. 3).
 *   Dense (Algorithm 1):  Y = K Omega^T, with Omega^T given as omega [dev] n x l.
 *   Sparse (Algorithm 2): column i of Y is sum_s sign[i, s] K(:, idx[i, s]),
 *                         idx [dev] int64 l x r (point indices in [0, n)),
 *                         sign [dev] l x r (Rademacher +-1; any values are accepted).
 *   Exactly one of omega / (idx, sign) must be non-NULL.
 *   Y [dev] n x l output, FP64.  prec selects the MVM precision.
 */
int krr_sketch(const double* X, int64_t n, int32_t d, double eps,
               const double* omega, const int64_t* idx, const double* sign, int32_t l, int32_t r,
               int32_t prec, double* Y, void* stream);

/*
 * Column-pivoted QR of Y^T (l x n) for anchor selection (Algorithm 1/2, last steps).
 * Y [dev] n x l (the sketch), k pivot steps.  Outputs: piv [dev] int64 k (point
 * indices, the first k pivots S), rdiag [dev] k (|R_jj|, the residual norm of each
 * pivot when chosen).  Ties go to the lowest point index.  Plain pivoted QR stands in
 * for strong RRQR (remark in Sec. 3).  prec: KRR_FP64 or KRR_FP32 arithmetic on Y.
 */
int krr_qrcp(const double* Y, int64_t n, int32_t l, int32_t k, int32_t prec,
             int64_t* piv, double* rdiag, void* stream);

typedef struct krr_precond krr_precond;   /* opaque */

/* Flags for krr_build_precond */
#define KRR_KEEP_SKETCH 1   /* keep Y (n x l) in the handle for inspection */

/*
 * Setup stage (Sec. 3, Algorithms 1-3): sketch -> pivoted QR -> anchors S ->
 * K_SS = U^{-1} -> symmetric EVD -> W = C V_kept diag(lam_kept)^{-1/2} (C = K(X, X_S))
 * -> M = W^T W (FP64 accumulation) -> for each beta: Cholesky L L^T = beta I + M
 * (Eq. chol_factor) and its inverse.
 *
 *   X [dev] n x d; betas [host] nbeta values; k anchors, l sketch columns;
 *   sketch random inputs as in krr_sketch (omega for Algorithm 1, idx/sign with r per column
 *   for Algorithm 2); tau: eigenvalues of K_SS <= tau * max are dropped (tau <= 0: 1e-12).
 *   prec: KRR_FP64 builds the FP64 factor only; KRR_FP32/KRR_MIXED also build an FP32 copy of
 *   W (and its own core from exactly that copy) used by FP32/mixed solves.
 *   *out receives the handle.  Returns KRR_ENOTSPD if a core Cholesky fails.
 *   The sketch's random numbers (Omega of Algorithm 1; the r indices and signs per column of Algorithm 2)
 *   are drawn by the caller and passed in, rather than drawn inside from a seed: the build is then a
 *   deterministic function of its inputs, the same draws can be fed to an independent implementation for
 *   checking, and the caller chooses the generator.
 */
int krr_build_precond(const double* X, int64_t n, int32_t d, double eps,
                      const double* betas, int32_t nbeta, int32_t k, int32_t l,
                      const double* omega, const int64_t* idx, const double* sign, int32_t r,
                      double tau, int32_t prec, int32_t flags,
                      krr_precond** out, void* stream);

/*
 * Setup stage on anchors chosen another way (remark in Sec. 3: random sampling or farthest point
 * sampling in place of the ID; the bounds of Sec. 4 then no longer hold).  Algorithm 3 and the
 * core factors run exactly as in krr_build_precond.
 *   S [dev] int64 k distinct indices in [0, n) chosen by the caller (random sampling draws them);
 *   S == NULL: farthest point sampling from point fps_start (as krr_fps).  The handle keeps its
 *   own copy of the anchors.  Other arguments as in krr_build_precond (no sketch, so no l, r,
 *   random inputs or flags).  Timings: ms[0] = 0, ms[1] = anchor selection (FPS, or the check of S);
 *   krr_precond_info reports rdiag as zeros.  KRR_EINVAL for out-of-range or repeated anchors.
 */
int krr_build_precond_anchors(const double* X, int64_t n, int32_t d, double eps,
                              const double* betas, int32_t nbeta, const int64_t* S, int32_t k,
                              int64_t fps_start, double tau, int32_t prec,
                              krr_precond** out, void* stream);

/*
 * Farthest point sampling (remark in Sec. 3): S[0] = start; each next anchor is the point, not yet
 * chosen, with the largest squared Euclidean distance to its nearest chosen point (ties to the
 * lowest index).  Distances are summed over coordinates in order, each operation rounded on its
 * own, so the picks are reproducible bit for bit.
 *   X [dev] n x d FP64; 1 <= k <= n; 0 <= start < n.
 *   S [dev] int64 k output (distinct indices); dsel [dev] k output or NULL: the squared distance of
 *   each pick when chosen (dsel[0] = +inf, then non-increasing).  Uses k - 1 kernel launches.
 */
int krr_fps(const double* X, int64_t n, int32_t d, int32_t k, int64_t start, int64_t* S, double* dsel,
            void* stream);

/*
 * Stable radix sort of (key, value) pairs by the key bits [0, end_bit), ascending; pairs whose bits are
 * equal keep their input order.  The library orders the pivoted QR's candidate columns by norm with it
 * (Algorithms 1-2, last steps) and the points of a culled operator by Morton code.
 *   keys_in [dev] uint64 n, vals_in [dev] int64 n: inputs, not modified.
 *   keys_out [dev] uint64 n, vals_out [dev] int64 n: outputs (keys with all their bits, reordered).
 *   0 <= n < 2^31; 1 <= end_bit <= 64; the four arrays must not overlap.  Deterministic; allocates work
 *   buffers of 2n + 131584 words through the registered allocator.
 */
int krr_radix_sort_pairs(const uint64_t* keys_in, uint64_t* keys_out, const int64_t* vals_in, int64_t* vals_out,
                         int64_t n, int32_t end_bit, void* stream);

/*
 * Rank for a target condition number on the data (Corollary tradeoff, Eq. condbound_gamma and
 * Eq. condbound): q_i are the side lengths of the bounding box of X (device reduction), h = sqrt(eps),
 *   gamma = (2/pi) sqrt(h^{-2} ln(Mbar n / (beta (xi - 1)))),   k = prod_i (floor(gamma q_i) + 1).
 *   X [dev] n x d FP64; beta > 0; xi > 1 (the target condition number); Mbar > 0, or <= 0 for
 *   Mbar = n (the ID value of the remark after the corollary).  KRR_EINVAL unless
 *   Mbar n > beta (xi - 1).
 *   Outputs [host]: gamma; k_bound as a double (exact below 2^53, may overflow to inf);
 *   q_host d values or NULL.  Synchronises the stream.  The bound is stated for ID-built
 *   preconditioners.
 */
int krr_rank_for_cond(const double* X, int64_t n, int32_t d, double eps, double beta, double xi,
                      double Mbar, double* gamma, double* k_bound, double* q_host, void* stream);

/* Sizes and host copies of small results.  Any output pointer may be NULL.
 *   S_host [host] int64 k anchors; kept: rank kept after the EVD truncation;
 *   lam_host [host] k eigenvalues of K_SS (ascending); rdiag_host [host] k QR diagonals. */
int krr_precond_info(const krr_precond* P, int64_t* S_host, int32_t* kept,
                     double* lam_host, double* rdiag_host, int32_t* k, int32_t* nbeta);

/* Wall-clock phases of the build in milliseconds (stream synchronised between phases):
 *   ms[0] sketch, ms[1] pivoted QR, ms[2] anchor block + EVD, ms[3] C, W = C T and M = W^T W,
 *   ms[4] core Cholesky factors and inverses, ms[5] total.  sweeps: Jacobi sweeps used (may be NULL). */
int krr_precond_timings(const krr_precond* P, double* ms, int32_t* sweeps);

/* Copy an internal device buffer into caller memory (testing and inspection).
 *   what: 0 = W FP64 (n x kept), 1 = W FP32 (n x kept, float), 2 = L FP64 (kept x kept,
 *         for betas[bidx]), 3 = Y sketch (n x l, needs KRR_KEEP_SKETCH), 4 = M = W^T W FP64.
 *   dst [dev], bytes = size of dst (must be at least the buffer's size). */
int krr_precond_get(const krr_precond* P, int32_t what, int32_t bidx, void* dst, size_t bytes,
                    void* stream);

/*
 * Woodbury apply (Algorithm 4 with W = C U^{1/2}; Eq. woodbury):
 *   out[:, r] = (x[:, r] - W z_r) / beta_r,  z_r = (beta_r I + W^T W)^{-1} W^T x[:, r]
 *   x, out [dev] n x R; betas [host] R values, each equal to one of the handle's betas.
 *   prec: KRR_FP64 uses the FP64 factor; KRR_FP32 / KRR_MIXED the FP32 W (needs a handle
 *   built with that precision).
 */
int krr_precond_apply(const krr_precond* P, const double* x, int32_t R, const double* betas,
                      int32_t prec, double* out, void* stream);

/*
 * krr_precond_apply without device allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc).  Same arguments and result as
 * krr_precond_apply; the columns are applied one at a time with the one-column kernels, so for R > 1 the
 * rounding differs from krr_precond_apply's several-column products.  Scratch (at most
 * max(256, ceil(n / 256)) * kept + 2 * kept doubles: the W^T x partial sums, t and z) lives in a 64 MiB
 * device array that the library holds on every
 * GPU it runs on until the process ends; larger preconditioners return KRR_EINVAL before any GPU work.
 * Nothing is allocated and no library routine that allocates is called.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (other streams, other threads) race and must be serialised by
 * the caller.  The array is found once per device (in krr_init, or at the first call on that device).
 */
int krr_precond_apply_noalloc(const krr_precond* P, const double* x, int32_t R, const double* betas,
                              int32_t prec, double* out, void* stream);

void krr_precond_free(krr_precond* P);

typedef struct {
  int32_t iters_max;      /* largest iteration count over the columns */
  int32_t n_mvm;          /* kernel MVMs issued in the working precision */
  int32_t n_mvm_fp64;     /* FP64 MVMs for residual replacement / final check */
  int32_t n_replace;      /* residual replacements performed */
  double t_total_ms;      /* wall time of the solve (host clock, stream synchronised) */
  double t_mvm_ms;        /* HIP-event time in working-precision MVMs (if timing enabled) */
  double t_mvm_fp64_ms;   /* HIP-event time in FP64 MVMs */
  double t_precond_ms;    /* HIP-event time in Woodbury applies */
  double kappa_est;       /* Lanczos estimate of the preconditioned condition number, column 0 */
  double t_mvm_kernel_ms; /* HIP-event time of the main MVM kernel alone (t_mvm_ms without operand
                             staging and the FP64 finishing pass) */
  double lam_min_est;     /* smallest and largest eigenvalue of column 0's Lanczos tridiagonal (Ritz values */
  double lam_max_est;     /* of the preconditioned operator; kappa_est is their ratio; 0 if none), built from
                             the CG coefficients up to the first claim of convergence of column 0 */
  int32_t n_graph_cycles; /* graph-captured cycles launched (krr_set_pcg_mode) */
  int32_t n_graph_iters;  /* iterations whose status came from a captured cycle */
} krr_solve_stats;

/*
 * Driver of krr_pcg_solve (process-wide; Algorithm 5's loop).  Both drivers launch the same kernels in the
 * same order and return bit-identical iterates, iteration counts and residuals:
 *   0: host loop, one host synchronisation per iteration (the next iteration's preconditioner apply and
 *      product are enqueued before the host waits, so the GPU does not idle while the host decides);
 *   1: graph-captured cycles: from the first scheduled replacement on (every 16 iterations when
 *      replace_every is 0), one HIP graph runs a whole cycle of replace_every (16) iterations and, with
 *      replacement, the check of the last one's true residual, with one host synchronisation per cycle.
 *      The convergence claims of the recursive residuals are decided on the device; a claim or a breakdown
 *      halts the cycle's remaining state updates, the host takes over at that iteration and runs the host
 *      loop until the next cycle boundary;
 *  -1: automatic (default): graph cycles when the product has at most 2^30 pair-columns (n^2 R), the host
 *      loop otherwise.
 * Graph cycles need replace_every <= 64 and timing == 0 (the host loop runs otherwise).
 */
int krr_set_pcg_mode(int32_t mode);

/*
 * PCG on (K + beta_r I) alpha_r = y_r for R right-hand sides in lockstep (Algorithm 5):
 * one shared kernel MVM of the whole block per iteration, per-column FP64 scalars, converged
 * columns frozen; once columns converge, the products are formed for the active columns only.  Stops a
 * column when its true relative residual ||y - (K + beta I) alpha||_2 / ||y||_2 <= tol (checked with the
 * FP64 operator).
 *
 *   X [dev] n x d;  Yrhs [dev] n x R;  betas [host] R values (each one of P's betas when P
 *   is given);  P: preconditioner or NULL (plain CG);  replace_every: every that many
 *   iterations the recursive residual is replaced by the FP64 true residual (0: never);
 *   alpha [dev] n x R: in = initial guess x0 (zeros for a cold start), out = solution;
 *   iters [host] R, relres [host] R: per-column iteration counts and final true relative
 *   residuals;  stats [host] optional (NULL);  timing != 0 records HIP-event phase times.
 *   Returns KRR_ENOCONV if some column did not reach tol within maxit.
 */
int krr_pcg_solve(const double* X, int64_t n, int32_t d, double eps,
                  const double* Yrhs, int32_t R, const double* betas,
                  const krr_precond* P, double tol, int32_t maxit, int32_t replace_every,
                  int32_t prec, double* alpha, int32_t* iters, double* relres,
                  krr_solve_stats* stats, int32_t timing, void* stream);

/*
 * Gradient of the validation loss L = 1/2 ||K(Xval, Xtr) alpha - yval||^2, alpha solving
 * (K + beta I) alpha = ytr, with respect to log eps and log beta, by the adjoint method:
 *   lambda = (K + beta I)^{-1} K_vt^T r_v,
 *   dL/dlog eps = r_v^T K'_vt alpha - lambda^T K' alpha,  dL/dlog beta = -beta lambda^T alpha,
 * with K' = (D^2/eps) K.  One forward and one adjoint PCG (same preconditioner P, may be NULL) in the
 * working precision `prec`; the products that assemble the loss and gradient (K_vt alpha and K'_vt alpha
 * fused, K_vt^T r_v, K' alpha) run in FP64.  Host scalars out; alpha_out [dev] n (optional), lambda_out [dev] n
 * (optional); stats [host] optional: two entries, the forward and the adjoint solve (HIP-event times recorded
 * when given).
 */
int krr_grad(const double* Xtr, int64_t n, const double* ytr,
             const double* Xval, int64_t m, const double* yval, int32_t d,
             double eps, double beta, const krr_precond* P,
             double tol, int32_t maxit, int32_t replace_every, int32_t prec,
             double* loss, double* dloss_dlog_eps, double* dloss_dlog_beta,
             double* alpha_out, double* lambda_out, krr_solve_stats* stats, void* stream);

/*
 * Autotuner of the kernel MVM's launch table (project-written; the paper has none).  A launch is fixed by a
 * kernel variant (tile shape, target fragments per wave, software pipelining, LDS staging of the sources,
 * symmetric square form) and a split (sources per block, i.e. the source split over the grid, for the direct
 * forms; the super-tile edge for the symmetric forms).  krr_autotune times every variant for (d, R, prec) on n synthetic points of a
 * square product, then the two fastest with the split halved and doubled, and records the fastest for the
 * size class floor(log2 n) in the process-wide table (key: precision, d, shape class of R, size class,
 * square or cross-set).  Every later product of that class launches the recorded entry; an entry forced with
 * krr_set_variant applies at every size.  best_variant [host] out.
 * krr_autotune_save / krr_autotune_load persist the table as JSON with the GPU architecture it was tuned on;
 * loading a table tuned on another architecture returns KRR_EINVAL.
 */
int krr_autotune(int32_t d, int32_t R, int32_t prec, int64_t n, int32_t* best_variant, void* stream);
int krr_autotune_save(const char* path);
int krr_autotune_load(const char* path);
/* Force a variant for (d, R, prec) at every size (-1 clears the entries of (d, R, prec), tuned ones too).
 * Number of variants: krr_num_variants. */
int krr_set_variant(int32_t d, int32_t R, int32_t prec, int32_t variant);
int krr_num_variants(int32_t prec, int32_t R);
/*
 * The kernel variant a product of n sources would run (the table's entry for its size class, else a forced
 * variant, else the default; n <= 0: sizes unknown) and whether it is the symmetric form (square product
 * K(X, X) V of one column without the derivative kernel, mixed or FP64: each off-diagonal pair of point tiles
 * is evaluated once).  square != 0: targets and sources are the same point set.  variant, symmetric [host]
 * out.  Host only; no GPU call.  KRR_EINVAL on bad arguments.
 */
int krr_kmv_variant(int32_t d, int32_t R, int32_t deriv, int32_t prec, int32_t square, int64_t n, int32_t* variant,
                    int32_t* symmetric);
/*
 * Exact far-tile culling of square one-column mixed products (the MVM the paper leaves replaceable, Sec. 2.4,
 * without an approximation).  The operator's points are staged in Morton order of their grid cells; the
 * symmetric kernel skips the exp/FMA work of a 16-source step for a wave's targets when the two groups'
 * bounding boxes are so far apart that every kernel value between them is exactly zero in FP32 (scaled
 * squared distance above 161, plus a bound on the cross term's rounding).  The results are bit for bit those
 * of the unculled kernel in the same order.  mode: -1 automatic (default: the spatial order when the data's
 * bounding-box diagonal reaches twice that distance, and the skipping when at least 10% of the 16-source
 * steps can be skipped; below that the skip logic costs more than it saves), 0 off, 1 on, 2 the spatial
 * order without skipping (the reference for comparisons).  Process-wide; read when an operator is staged and
 * launched.
 */
int krr_set_cull(int32_t mode);
/* Pairs of the last kernel MVM launched on this thread: pairs_total = npad^2 (npad the point count padded to
 * a multiple of 1024), pairs_skipped = those whose evaluation culling skipped (0 if it did not run).
 * Synchronises the stream.  [host] outputs. */
int krr_cull_stats(int64_t* pairs_total, int64_t* pairs_skipped, void* stream);

/* What the last kernel MVM launched on this thread ran: its variant, its split (sources per block of a direct
 * form, super-tile edge of a symmetric form) and whether it was the symmetric form.  -1 / 0 / 0 before any
 * launch.  Host only. */
int krr_kmv_last_launch(int32_t* variant, int32_t* split, int32_t* symmetric);

#ifdef __cplusplus
}
#endif
#endif /* KRR_H_ */

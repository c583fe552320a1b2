/*
 * mpcr.h -- C interface of the MI355X (gfx950) mixed-precision tile Cholesky /
 * Gaussian log-likelihood library.
 *
 * The operations follow the paper "MPCR: Multi-Precision Computations Package
 * in R" (arXiv 2406.02701):
 *   - matrix product C = op(A) op(B) in 64-, 32- or 16-bit precision, with the
 *     result in the highest input precision (section "Operations on MPCR
 *     objects"; section "Linear Algebra Functions Performance");
 *   - Cholesky factorisation, forward/backward triangular solves, the
 *     log-determinant 2 sum log L_ii and the quadratic form ||L^{-1} z||^2 that
 *     give the Gaussian log-likelihood of a Matern covariance (section "Maximum
 *     Likelihood Estimation of Matern Covariance Function");
 *   - the tiled algorithm that holds tiles of one matrix at different
 *     precisions (section "Discussion and Future Work"), with FP64 refinement
 *     (multi-precision stages, section "Introduction").
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major with a leading dimension (the paper's objects
 *     store elements column by column, section "Creating MPCR objects").
 *   - Pointers named d_* are DEVICE pointers owned by the caller (typically
 *     torch tensors); h_* are host pointers.  The library never frees caller
 *     memory.  The library allocates device memory only inside a factor
 *     (released by mpcr_factor_destroy) or in a context's workspace (released
 *     by mpcr_ctx_destroy).
 *   - Work is ordered on the context's HIP stream.  Calls that return host
 *     values (info, loglik, diag) synchronise that stream before returning.
 *   - Errors are returned as mpcr_status_t codes, never thrown; the text of
 *     the last error of a context is available from mpcr_last_error().
 *   - info follows LAPACK: 0 = success, k > 0 = the leading minor of order k
 *     (global 1-based column) is not positive definite.
 *   - A context is used by one host thread at a time.
 */
#ifndef MPCR_H
#define MPCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage / compute formats.  FP64, FP32 and FP16 are the IEEE formats the
 * paper describes (section "Floating-Point Arithmetic in Modern Technology");
 * BF16 (1/8/7) and FP8-E4M3FN (1/4/3, no infinities, largest finite 448,
 * conversions saturate) are the two further low formats of the tile map. */
typedef enum {
  MPCR_FP64 = 0,
  MPCR_FP32 = 1,
  MPCR_FP16 = 2,
  MPCR_BF16 = 3,
  MPCR_FP8_E4M3 = 4
} mpcr_prec_t;

typedef enum {
  MPCR_OK = 0,
  MPCR_ERR_ARG = -1,            /* invalid argument (shape, pointer, format, option) */
  MPCR_ERR_NOT_SPD = -2,        /* factorisation met a non-positive pivot; see info */
  MPCR_ERR_NOT_CONVERGED = -3,  /* refinement reached max_iter above tolerance */
  MPCR_ERR_NOMEM = -4,          /* device allocation failed */
  MPCR_ERR_DEVICE = -5,         /* a HIP call failed */
  MPCR_ERR_REJECTED = -6        /* request does not fit the serving budget */
} mpcr_status_t;

typedef struct mpcr_ctx mpcr_ctx;
typedef struct mpcr_factor mpcr_factor;

/* Per-tile precision map of an n x n symmetric matrix cut into nt x nt tiles of
 * nb x nb (nt = ceil(n / nb); the last tile row/column is padded with an
 * identity block).  h_map is a HOST array of nt*nt bytes, row-major over tile
 * indices (i, j); only entries with i >= j are read and each holds an
 * mpcr_prec_t.  Diagonal tiles must be MPCR_FP64 (the diagonal POTRF, the SYRK
 * into it and the log-determinant stay in FP64). */
typedef struct {
  int64_t n;
  int64_t nb;
  int64_t nt;
  const uint8_t* h_map;
} mpcr_tilemap_t;

/* Matern covariance parameters: Sigma_ij = sigma2 * m_nu(||s_i - s_j|| / range)
 * + nugget * [i == j], with m_nu the half-integer closed form of
 * x^nu K_nu(x) / (2^(nu-1) Gamma(nu)) (MLE section of the paper); nu must be
 * 0.5, 1.5 or 2.5. */
typedef struct {
  double sigma2;
  double range;
  double nu;
  double nugget;
} mpcr_theta_t;

/* Refinement of Sigma x = b with the (mixed-precision) factor L~ as
 * preconditioner M = L~ L~^T; residuals and vectors in FP64.
 *   tol          stop when every column's normwise backward error
 *                eta = ||r||_inf / (||Sigma||_inf ||x||_inf + ||b||_inf) <= tol
 *                (||r||_2/||b||_2 is reported as well)
 *   max_iter     iteration cap (0 = no refinement: x = M^{-1} b)
 *   solver       0 = preconditioned conjugate gradients, 1 = classical
 *                iterative refinement x <- x + M^{-1} r, 2 = GMRES-based
 *                iterative refinement (Carson and Higham, 2018): each
 *                correction equation Sigma d = r is solved by GMRES (Saad and
 *                Schultz, 1986; modified Gram-Schmidt, Givens rotations) on
 *                M^{-1} Sigma d = M^{-1} r, at most gmres_m steps, until the
 *                GMRES residual drops to gmres_inner_tol |M^{-1} r|; max_iter
 *                counts the refinement steps.  3 = block PCG (O'Leary, 1980)
 *                on groups of block_size consecutive columns:
 *                alpha = (P^T Sigma P)^{-1} (Z^T R), beta = (Z^T R)_old^{-1}
 *                (Z^T R)_new with Z = M^{-1} R; a group whose s x s system is
 *                not numerically positive definite (a pivot of its unit-
 *                diagonal scaling below 1e-12) finishes with PCG from its
 *                current iterate.  diag->iters counts block iterations plus
 *                any PCG iterations after such a breakdown.
 *   recompute    PCG recomputes the true residual every `recompute` steps
 *   residual     mpcr_gauss_loglik only: 0 = regenerate Sigma's entries from the
 *                sites for every residual (no extra memory); 1 = keep an FP64
 *                copy of Sigma's lower tiles (nt(nt+1)/2 nb^2 doubles, written
 *                with the low-precision tiles) and stream it
 *   promote_on_breakdown
 *                mpcr_gauss_loglik only: 1 = when the mixed factor meets a
 *                non-positive pivot (global column info, tile step
 *                k = (info-1)/nb), take the coarsest format p among the tiles
 *                (i, j), j < i <= k, and the smallest distance d_fail = i - j at
 *                which p occurs there; move every tile of format p with
 *                distance >= d_fail one format up (FP8 -> FP16, FP16/BF16 ->
 *                FP32, FP32 -> FP64) and factor again, at most 8 times, until
 *                the factor exists or the leading tiles are all FP64.  The map
 *                finally used is returned by mpcr_loglik_map and the number of
 *                promotions in mpcr_diag_t.promotions.  (The paper's MLE
 *                section warns that low precision can fail on ill-conditioned
 *                covariances; this is the recovery.)  0 = report NOT_SPD.
 *   direct_eta   all-FP64 map with max_iter = 0 (the paper's direct path):
 *                1 = also compute the backward error of the direct solve (one
 *                extra FP64 residual pass) into diag->eta / rel_resid2;
 *                0 = skip it.  opts == NULL behaves as 1 when diag != NULL.
 *   gmres_m      solver 2: GMRES steps per refinement step (0 = 20; at most 64)
 *   gmres_inner_tol
 *                solver 2: relative tolerance of each GMRES solve (0 = 1e-6)
 *   block_size   solver 3: right-hand sides per block (0 = min(nrhs, 32);
 *                at most 32) */
typedef struct {
  double tol;
  int max_iter;
  int solver;
  int recompute;
  int residual;
  int promote_on_breakdown;
  int direct_eta;
  int gmres_m;
  double gmres_inner_tol;
  int block_size;
} mpcr_refine_opts_t;

/* Diagnostics filled by mpcr_potrs / mpcr_gauss_loglik (host struct). */
typedef struct {
  int iters;              /* refinement iterations taken */
  int converged;          /* 1 if every column met the stopping rule */
  double eta;             /* max over columns of the normwise backward error */
  double rel_resid2;      /* max over columns of ||b - Sigma x||_2 / ||b||_2 */
  double logdet;          /* log|Sigma| from the factor's diagonal tiles */
  double quad0;           /* first column's quadratic form z^T Sigma^{-1} z */
  int64_t info;           /* LAPACK-style info of the factorisation */
  double t_gen_ms, t_factor_ms, t_solve_ms, t_refine_ms;  /* phase times (HIP events) */
  double flops_by_prec[5];  /* algorithmic factorisation flops by compute format */
  int promotions;         /* refactorisations after a breakdown (promote_on_breakdown) */
} mpcr_diag_t;

/* ---- context -------------------------------------------------------------- */

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the device's default stream).  *out receives the
 * context.  Errors: MPCR_ERR_ARG (out NULL, bad device), MPCR_ERR_DEVICE. */
int mpcr_ctx_create(int device, void* hip_stream, mpcr_ctx** out);
int mpcr_ctx_destroy(mpcr_ctx* ctx);
/* Text of the context's last error ("" if none).  Valid until the next call. */
const char* mpcr_last_error(const mpcr_ctx* ctx);
/* Library version string, e.g. "mpcr 0.1 gfx950". */
const char* mpcr_version(void);

/* Kernel timing of a context.  With profiling on, every tile-factorisation
 * launch queued by this context is bracketed by two HIP events recorded on the
 * context's stream; elapsed times are accumulated when the call synchronises.
 * Kinds: 0..4 = tile GEMM/SYRK update computed in format MPCR_FP64..FP8,
 * 5 = diagonal POTRF, 6 = panel TRSM, 7 = inversion of the diagonal tiles,
 * 8 = one tile solve (forward and backward sweeps, timed as a whole),
 * 9 = FP64 residual b - Sigma x, 10 = SYRK of the next diagonal tile from an
 * FP64 panel tile (on the critical path; kind 0 counts it otherwise).
 * mpcr_ctx_kernel_stats returns, for one
 * kind, the total milliseconds, the number of launches (sweeps for kind 8)
 * and the algorithmic flops they performed (2 nb^3 per GEMM tile, nb^3 per
 * SYRK or TRSM tile, nb^3/3 per POTRF or inversion, 2 N^2 nrhs per sweep,
 * 2 n^2 nrhs per residual).  Reset clears all kinds. */
int mpcr_ctx_set_profiling(mpcr_ctx* ctx, int on);
/* How GEMM updates of FP32 tiles form their products (the tile stays FP32 and
 * each update result is rounded to FP32 once).  on = 1 (default): both
 * operands, converted to FP32, are split exactly into three BF16 parts
 * x = h + m + l and the six products h h, h m, m h, h l, l h, m m are
 * accumulated in FP32 on the BF16 MFMA (the dropped products are below
 * 2^-23 |a b|, so the accuracy is FP32's; gfx950's BF16 MFMA is 16 times
 * faster than its FP32 MFMA).  on = 0: the FP32 MFMA.  Errors: MPCR_ERR_ARG. */
int mpcr_ctx_set_fp32_split(mpcr_ctx* ctx, int on);
int mpcr_ctx_reset_stats(mpcr_ctx* ctx);
int mpcr_ctx_kernel_stats(const mpcr_ctx* ctx, int kind, double* h_total_ms, int64_t* h_launches,
                          double* h_flops);

/* ---- precision maps (host helpers) ----------------------------------------- */

/* Banded map: tile (i, j), i >= j, with d = i - j gets precs[b] for the first
 * band b with d <= band_dmax[b]; band_dmax[nbands-1] < 0 means "all the
 * rest".  Writes nt*nt bytes to h_map_out (entries with i < j are set to 255).
 * Errors: MPCR_ERR_ARG if the diagonal would not be FP64 or a distance has no
 * band. */
int mpcr_tilemap_banded(int64_t n, int64_t nb, const int* band_dmax, const int* precs,
                        int nbands, uint8_t* h_map_out);

/* Norm-guarded map: starts from the banded map and promotes each off-diagonal
 * tile (i, j) to the lowest format p (in the order FP8 < FP16/BF16 < FP32 <
 * FP64, never below the banded choice's precision rule) whose rounding error
 * bound satisfies max(u_p * max|Sigma_tile|, s_p / 2) <= guard, with u_p the
 * unit roundoff and s_p the smallest subnormal of p (values below p's normal
 * range round with absolute error up to s_p / 2: 2^-25 for FP16).  h_tile_amax holds, row-major
 * nt x nt, the largest magnitude of each lower tile (see
 * mpcr_covariance_tile_amax).  Writes nt*nt bytes to h_map_out. */
int mpcr_tilemap_guarded(int64_t n, int64_t nb, const uint8_t* h_banded_map,
                         const double* h_tile_amax, double guard, uint8_t* h_map_out);

/* ---- ordering and covariance ------------------------------------------------ */

/* Morton (Z-order) permutation of n sites: each coordinate of d_locs (n x 2,
 * column-major, values in [0,1)) is quantised to 16 bits
 * (q = min(floor(65536 x), 65535)), bits interleaved with x in the even
 * positions; d_perm_out (n int64, device) receives the stable sort order.
 * Nearby sites get nearby indices, which is what a band map relies on. */
int mpcr_morton_order(mpcr_ctx* ctx, int64_t n, const double* d_locs, int64_t* d_perm_out);

/* The same permutation as mpcr_morton_order, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the sort keys live in a static device array owned by
 * the library (2^20 keys, 8 MiB on each GPU the library runs on, held until
 * the process ends), so n <= 1048576; MPCR_ERR_ARG otherwise.  The call
 * allocates nothing and does not synchronise: the permutation is ready in
 * stream order on the context's stream.  Every call on one GPU uses the same
 * array, so calls that overlap on a GPU (other streams or threads) race:
 * order them. */
int mpcr_morton_order_noalloc(mpcr_ctx* ctx, int64_t n, const double* d_locs, int64_t* d_perm_out);

/* Dense FP64 covariance Sigma(theta) (n x n, column-major, ld >= n) from the
 * sites d_locs (n x 2 column-major), both triangles written. */
int mpcr_covariance(mpcr_ctx* ctx, int64_t n, const double* d_locs, const mpcr_theta_t* theta,
                    double* d_A, int64_t lda);

/* Largest |Sigma_ij| of every lower tile (i >= j) of the nb-tiled covariance,
 * written to h_amax_out (HOST, nt*nt doubles, row-major; upper entries 0). */
int mpcr_covariance_tile_amax(mpcr_ctx* ctx, int64_t n, int64_t nb, const double* d_locs,
                              const mpcr_theta_t* theta, double* h_amax_out);

/* ---- tile factorisation ----------------------------------------------------- */

/* Mixed-precision right-looking tile Cholesky of the FP64 SPD matrix d_A
 * (n x n, column-major, only the lower triangle is read).  Each lower tile is
 * rounded once (round-to-nearest-even) to its map format; then for each step k:
 * POTRF of the FP64 diagonal tile, TRSM of the panel tiles (computed in FP64,
 * rounded once to each tile's format), SYRK into the diagonal tiles (FP64) and
 * GEMM updates of the other trailing tiles computed in the OUTPUT tile's
 * format (FP32 accumulation for 16- and 8-bit formats).
 * *out receives a factor that owns its device tiles; *h_info receives 0 or
 * the 1-based global column of the first non-positive pivot, in which case the
 * call returns MPCR_ERR_NOT_SPD and *out is still valid (destroy it).
 * FP8-E4M3 tiles carry one power-of-two scale each, chosen from the tile's
 * largest magnitude whenever the tile receives new values (A9's rule). */
int mpcr_potrf_tiled(mpcr_ctx* ctx, int64_t n, const double* d_A, int64_t lda,
                     const mpcr_tilemap_t* map, mpcr_factor** out, int64_t* h_info);

/* Same factorisation with Sigma(theta) generated tile by tile from the sites
 * (no dense FP64 matrix is formed). */
int mpcr_potrf_tiled_covariance(mpcr_ctx* ctx, int64_t n, const double* d_locs,
                                const mpcr_theta_t* theta, const mpcr_tilemap_t* map,
                                mpcr_factor** out, int64_t* h_info);

int mpcr_factor_destroy(mpcr_factor* f);

/* log|Sigma| = 2 sum_i log L_ii over the first n diagonal entries, summed in
 * FP64 in a fixed order.  *h_logdet receives the value. */
int mpcr_factor_logdet(mpcr_ctx* ctx, const mpcr_factor* f, double* h_logdet);

/* The factor widened to FP64 as a dense lower-triangular n x n matrix
 * (column-major, ld >= n; strictly upper part set to 0).  For inspection. */
int mpcr_factor_to_dense(mpcr_ctx* ctx, const mpcr_factor* f, double* d_L, int64_t ldl);

/* Algorithmic factorisation flops split by compute format (host array of 5). */
int mpcr_factor_flops(const mpcr_factor* f, double* h_flops5);

/* ---- solves --------------------------------------------------------------- */

/* Forward solve W = L^{-1} B (n x nrhs FP64, device), the first half of the
 * paper's forwardsolve/backsolve pair; low-precision tiles are read widened. */
int mpcr_trsm_forward(mpcr_ctx* ctx, const mpcr_factor* f, int64_t nrhs, const double* d_B,
                      int64_t ldb, double* d_W, int64_t ldw);

/* X = Sigma^{-1} B through the factor (forward then backward solve).  If
 * d_A_fp64 is non-NULL (the FP64 matrix, n x n, both triangles) and opts is
 * non-NULL with max_iter > 0, the solve is refined in FP64 against it (see
 * mpcr_refine_opts_t).  diag may be NULL.  Returns MPCR_ERR_NOT_CONVERGED if
 * refinement stopped at max_iter above tolerance (X holds the last iterate). */
int mpcr_potrs(mpcr_ctx* ctx, const mpcr_factor* f, int64_t nrhs, const double* d_B, int64_t ldb,
               double* d_X, int64_t ldx, const double* d_A_fp64, int64_t lda,
               const mpcr_refine_opts_t* opts, mpcr_diag_t* diag);

/* Gaussian log-likelihood of nrhs observation vectors d_Z (n x nrhs, FP64,
 * column-major, ld = n) at sites d_locs (n x 2, column-major):
 *   l = -(n/2) log(2 pi) - (1/2) log|Sigma| - (1/2) z^T Sigma^{-1} z.
 * Sites are taken in Morton order when `order` is 1 (l is invariant under a
 * joint permutation of sites and observations).  map == NULL means all tiles
 * FP64 with tile size nb_default (=256).  With an all-FP64 map and either
 * opts NULL or opts->max_iter = 0 the quadratic form is ||L^{-1} z||^2 (the
 * paper's forwardsolve + SquareSum); otherwise the solve is refined in FP64
 * (residual from the sites or from stored FP64 tiles, opts->residual) and
 * quad = z^T x + x^T r.  A mixed map with opts->max_iter = 0 takes
 * x = M^{-1} z with its true residual r.
 * h_loglik (host, nrhs doubles) receives l per column; diag may be NULL.
 * The covariance tiles and factor live in a workspace owned by ctx. */
int mpcr_gauss_loglik(mpcr_ctx* ctx, int64_t n, const double* d_locs, const double* d_Z,
                      int64_t nrhs, const mpcr_theta_t* theta, const mpcr_tilemap_t* map,
                      int order, const mpcr_refine_opts_t* opts, double* h_loglik,
                      mpcr_diag_t* diag);

/* The tile map used by the context's last mpcr_gauss_loglik call (after any
 * promotions): *h_nt receives nt, and h_map_out (host, capacity bytes) the
 * nt*nt map when capacity >= nt*nt.  Errors: MPCR_ERR_ARG (no call yet, or
 * capacity too small; *h_nt is still set). */
int mpcr_loglik_map(const mpcr_ctx* ctx, int64_t* h_nt, uint8_t* h_map_out, int64_t capacity);

/* Maximum likelihood fit of the Matern range and variance (the paper's MLE
 * section: R's optim, Nelder-Mead, minimises the negative log-likelihood with
 * nu fixed and the parameters on the log scale).  p = (log range, log
 * variance); f(p) = -l(theta(p)) evaluated by mpcr_gauss_loglik on the sites
 * d_locs (n x 2, column-major) and one observation vector d_z (n), with the
 * tile map `map` (NULL: all FP64, nb 256) and refinement options `refine`
 * (may be NULL); a breakdown of the factor counts as f = +inf.  The sites are
 * put in Morton order once; every evaluation reuses the context's factor
 * workspace.  The simplex method: Nelder and Mead (1965) as stated by
 * Lagarias et al. (1998) with reflection 1, expansion 2, contraction 1/2 and
 * shrink 1/2, vertices ordered by f with ties kept in place; first simplex
 * h_x0 and h_x0 + s e_i with s = 0.1 max|x0_i| (0.1 if x0 = 0); stop when
 * f_worst - f_best <= reltol (|f_best| + reltol) or after max_iter
 * iterations.  Outputs (host): h_x_out[2] the best vertex, *h_nll_out its f,
 * *h_iters / *h_evals (may be NULL) iterations and likelihood evaluations.
 * Errors: MPCR_ERR_ARG; any error of mpcr_gauss_loglik other than NOT_SPD
 * ends the fit with that code. */
int mpcr_mle_fit(mpcr_ctx* ctx, int64_t n, const double* d_locs, const double* d_z, double nu, double nugget,
                 const mpcr_tilemap_t* map, const mpcr_refine_opts_t* refine, const double* h_x0, int max_iter,
                 double reltol, double* h_x_out, double* h_nll_out, int* h_iters, int* h_evals);

/* Laplace approximation of a latent Gaussian model with Bernoulli observations
 * (the paper's "Integrated Nested Multi-Precision Arithmetic Laplace
 * Approximation" section, a dense analogue of INLA): latent field
 * x ~ N(0, Sigma(theta)) at the sites d_locs (n x 2, column-major), with
 * Sigma the Matern covariance of variance sigma2, smoothness nu and range r
 * (no nugget), and observations d_y (n, 0 or 1) with P(y_i = 1) =
 * 1 / (1 + exp(-beta x_i)).  For every range r = h_range[i] the call finds the
 * mode x0 of p(x | y) by Newton's method from x = 0 (stop when the mean
 * squared change of x is below newton_tol; more than max_newton steps is
 * MPCR_ERR_NOT_CONVERGED) and returns in h_lpost[i] the section's
 *   log p(y | x0) + log|Q|/2 - x0^T Q x0 / 2 - log|Q + W|/2,
 * Q = Sigma^-1 and W = -d^2 log p(y | x)/dx^2 at x0 (diagonal).  The
 * precision matrix is never formed: each Newton step factors
 * B = I + W^1/2 Sigma W^1/2 (tile map `map`, NULL = all FP64 with nb 256; a
 * mixed map stores B's off-diagonal tiles in low precision, with unrefined
 * solves), so log|Q| - log|Q + W| = -log|B| and, with x0 = Sigma a,
 * x0^T Q x0 = a^T x0.  If h_posterior is not NULL the ranges must be
 * equally spaced, increasing and odd in number, and h_posterior receives
 * exp(l_i - mean l) normalised by Simpson's rule over the grid (the
 * section's posterior of the range).  h_newton_iters (may be NULL) receives
 * the Newton steps per range; d_mode_out (device, n; may be NULL) the mode at
 * the last range.  Host arrays have nrange entries. */
int mpcr_inla_posterior(mpcr_ctx* ctx, int64_t n, const double* d_locs, const double* d_y, double sigma2, double nu,
                        double beta, const double* h_range, int nrange, double newton_tol, int max_newton,
                        const mpcr_tilemap_t* map, double* h_lpost, double* h_posterior, int* h_newton_iters,
                        double* d_mode_out);

/* Metropolis-adjusted Langevin sampler (the paper's "Metropolis-Hastings
 * Algorithm in High Dimensions" section) for the target N(0, Sigma) with
 * Sigma the Matern covariance `target` at the sites d_locs (n x 2), the
 * preconditioner M the Matern covariance `precond` and step h.  From the state
 * z (d_z0, n), iteration t proposes
 *   z' = z - (h/2) M Sigma^-1 z + L eps_t,   L L^T = h M  (lower tile factor),
 * eps_t the t-th column of d_eps (n x iters, device), and accepts it when
 *   h_unif[t] < exp(min(0, log pi(z') - log pi(z) + log q(z | z') - log q(z' | z)))
 * with log pi(x) = -x^T Sigma^-1 x / 2 and log q(a | b) = -(a - s(b))^T
 * (h M)^-1 (a - s(b)) / 2, s(b) = b - (h/2) M Sigma^-1 b.  Sigma and h M are
 * factored once (tile map `map` for both, NULL = all FP64 with nb 256); the
 * products Sigma^-1 x and (h M)^-1 quadratic forms are tile solves, M v is
 * generated from the sites.  The random numbers are inputs, so a run is
 * reproducible.  Outputs: d_z_out (n) the final state; d_trace (n x iters,
 * may be NULL) every state; h_accepted and h_log_ratio (iters, may be NULL)
 * the decisions and the log acceptance ratios. */
int mpcr_mala_run(mpcr_ctx* ctx, int64_t n, const double* d_locs, const mpcr_theta_t* target,
                  const mpcr_theta_t* precond, double h, const double* d_z0, int iters, const double* d_eps,
                  const double* h_unif, const mpcr_tilemap_t* map, double* d_z_out, double* d_trace,
                  int* h_accepted, double* h_log_ratio);

/* ---- matrix product ----------------------------------------------------------- */

/* Round an FP64 matrix (m x n, column-major, lds) once to format `prec`
 * (round-to-nearest-even; FP8-E4M3FN saturating).  Element type of d_dst:
 * double / float / uint16 bit patterns (FP16, BF16) / uint8 codes (FP8).
 * For MPCR_FP8_E4M3 each 128 x 128 block (of the stored matrix) is first
 * multiplied by 2^s with s = floor(log2(448 / max|block|)) (s = 0 for an
 * all-zero block, clamped to [-128, 127]); s is written to d_scale_exp
 * (int8, ceil(m/128) x ceil(n/128) column-major).  d_scale_exp must be NULL
 * for the other formats. */
int mpcr_convert(mpcr_ctx* ctx, mpcr_prec_t prec, int64_t m, int64_t n, const double* d_src,
                 int64_t lds, void* d_dst, int64_t ldd, int8_t* d_scale_exp);

/* C <- alpha op(A) op(B) + beta C (op = transpose if trans* != 0), A and B in
 * format `prec` (as written by mpcr_convert, with their block scale exponents
 * for FP8), C in c_prec (MPCR_FP64 for prec = FP64, MPCR_FP32 or MPCR_FP64
 * otherwise).  FP64 accumulates in FP64, FP32 in FP32, FP16/BF16/FP8 in FP32;
 * FP8 products are rescaled by 2^-(sA + sB) per 128-wide k block.
 * m, n, k >= 0; ld* >= the stored row count. */
int mpcr_gemm(mpcr_ctx* ctx, mpcr_prec_t prec, int transA, int transB, int64_t m, int64_t n,
              int64_t k, double alpha, const void* d_A, int64_t lda, const int8_t* d_scaleA_exp,
              const void* d_B, int64_t ldb, const int8_t* d_scaleB_exp, double beta, void* d_C,
              int64_t ldc, mpcr_prec_t c_prec);

/* ---- serving: continuous batching of log-likelihood requests ------------------ */

/* A server owns a pre-allocated device arena of hbm_budget bytes and max_slots
 * worker slots; each slot has its own context and HIP stream, so requests on
 * different slots run concurrently on the device.  Requests wait in a FIFO
 * queue and are admitted when a slot is free and their estimated device
 * footprint fits in the unreserved part of the budget; their buffers come
 * from the arena (no hipMalloc / hipFree per request).  Each request is one
 * mpcr_gauss_loglik evaluation (sites in Morton order, one observation
 * vector) with the norm-guarded banded map below; a request whose mixed
 * factor breaks down is refactored with promoted tiles when
 * refine.promote_on_breakdown is 1, and recomputed with all tiles FP64 when
 * it still fails and fallback_fp64 is 1.  refine.residual must be 0 (the
 * footprint estimate assumes the matrix-free residual) and refine.solver 0 or
 * 1 (PCG or IR: the Krylov workspaces of GMRES-IR and block PCG are not in the
 * estimate).  A request's arithmetic does not depend on what else is running:
 * results are the same alone and in a mix.  HIP maps streams onto
 * GPU_MAX_HW_QUEUES in-order hardware queues per process (4 by default), so
 * slots whose streams share a queue wait on each other; with more than two
 * slots, start the process with GPU_MAX_HW_QUEUES >= max_slots. */
typedef struct mpcr_server mpcr_server;

typedef struct {
  int64_t nb;              /* tile size (multiple of 128) */
  int band_fp64;           /* tiles with distance d <= band_fp64 are FP64 */
  int band_fp32;           /* band_fp64 < d <= band_fp32: FP32; beyond: far_prec */
  int far_prec;            /* mpcr_prec_t of the far tiles (FP16 or BF16) */
  double guard;            /* norm guard relative to the nugget (<= 0: no guard) */
  mpcr_refine_opts_t refine;
  int fallback_fp64;       /* 1: recompute with an all-FP64 map on breakdown */
} mpcr_serve_opts_t;

/* Errors: MPCR_ERR_ARG (bad options, refine.residual != 0), MPCR_ERR_NOMEM
 * (budget cannot be allocated). */
int mpcr_serve_create(int device, size_t hbm_budget, int max_slots, const mpcr_serve_opts_t* opts,
                      mpcr_server** out);
/* Waits for the requests in flight, drops queued ones, frees everything. */
int mpcr_serve_destroy(mpcr_server* srv);
/* Queues a request (h_locs: n x 2 column-major host array, h_z: n host
 * values; both copied before the call returns).  Returns MPCR_ERR_REJECTED if
 * the request's footprint exceeds the whole budget. */
int mpcr_serve_submit(mpcr_server* srv, uint64_t req_id, int64_t n, const double* h_locs, const double* h_z,
                      const mpcr_theta_t* theta);
/* Takes one finished request, if any: returns 1 and fills the outputs (status
 * = that request's mpcr_status_t, used_fallback = 1 if the FP64 map was
 * needed; times in seconds on the server's monotonic clock), 0 if none is
 * ready.  Any output pointer may be NULL. */
int mpcr_serve_poll(mpcr_server* srv, uint64_t* req_id, double* loglik, mpcr_diag_t* diag, double* t_submit,
                    double* t_done, int* status, int* used_fallback);
/* Seconds on the server's monotonic clock (the clock of t_submit / t_done). */
double mpcr_serve_clock(const mpcr_server* srv);
/* Counters: queued, running, finished (not yet polled), rejected; bytes reserved. */
int mpcr_serve_stats(mpcr_server* srv, int64_t* queued, int64_t* running, int64_t* finished, int64_t* rejected,
                     size_t* bytes_reserved);
/* Estimated device bytes of one request of order n (nb, one observation vector). */
size_t mpcr_serve_footprint(int64_t n, int64_t nb);

#ifdef __cplusplus
}
#endif

#endif /* MPCR_H */

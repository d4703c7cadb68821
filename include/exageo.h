/*
 * exageo.h -- C ABI of the MI355X (gfx950) library for exact Gaussian-process
 * maximum-likelihood estimation with a Matern covariance.
 *
 * The operation is the one of the ExaGeoStatR paper (Abdulah et al.,
 * arXiv 1908.06936), Section 1:
 *   - covariance, eq. (3):
 *       Sigma_ij = sigma2 / (2^(nu-1) Gamma(nu)) (r_ij/beta)^nu K_nu(r_ij/beta),
 *       r_ij = distance of the 2-D locations s_i, s_j (Euclidean, or great-circle
 *       with exageo_set_distance), Sigma_ii = sigma2 (plus a fixed nugget with
 *       exageo_set_nugget);
 *   - log-likelihood, eq. (2) with zero mean:
 *       l(theta) = -1/2 (n log 2 pi + log det Sigma + z^T Sigma^-1 z),
 *     evaluated through a Cholesky factorisation, a triangular solve and the
 *     determinant (the three operations named after eq. (3));
 *   - the maximum-likelihood estimate over theta = (sigma2, beta, nu) within
 *     bounds (Section 2.2, optimisation toolbox; Section 3, Example 2).
 * The gradient entry point adds the Gaussian score
 *       dl/dtheta_k = 1/2 a^T dSigma_k a - 1/2 tr(Sigma^-1 dSigma_k),
 *       a = Sigma^-1 z,
 * which the paper's derivative-free optimiser does not use.
 *
 * Conventions shared by every entry point
 *   theta      host array of 3 doubles, (sigma2, beta, nu), all > 0, nu <= 15.
 *   x, y, z    DEVICE pointers to n contiguous doubles (locations and
 *              observations), caller owned, read only, valid for the call.
 *   n          >= 1, with the padded size npad = ceil(n / ts) ts below
 *              2^32 / max(ts, 1016) (4.2 million at tile 768; the kernels
 *              index with 32-bit offsets): EINVAL above; device memory
 *              bounds n far lower (ENOMEM).
 *   outputs    host memory unless stated otherwise.
 *   streams    all work is queued on the stream given to exageo_create; a call
 *              returns after synchronising that stream only when it has to
 *              hand host scalars back.  Inside a call a second stream of the
 *              context (default priority) runs the next panel of the
 *              factorisation and half of each step of the inverse factor,
 *              ordered against the caller's stream by events; it is idle
 *              whenever a call returns.
 *   order      results do not depend on the order of the locations: the
 *              library sorts a private copy along a Morton (Z-order) curve.
 *   errors     no C++ exception crosses the ABI; every call returns a status.
 *              exageo_last_error() gives a text for the last failure.
 *   threads    a context is not thread safe; use one per host thread/stream.
 */
#ifndef EXAGEO_H
#define EXAGEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t exageo_status;

#define EXAGEO_OK 0
#define EXAGEO_EINVAL (-1)  /* bad argument; nothing was launched            */
#define EXAGEO_ENOTPD (-2)  /* a pivot of the Cholesky factor was <= 0       */
#define EXAGEO_ENOMEM (-3)  /* workspace too small or allocation failed      */
#define EXAGEO_EDEVICE (-4) /* HIP runtime error (text in exageo_last_error) */
#define EXAGEO_ENOCONV (-5) /* optimiser hit max_iters before tol            */

/* precision of the factorisation */
#define EXAGEO_FP64 0  /* every tile in double precision                      */
#define EXAGEO_MIXED 1 /* diagonal tiles FP64; each off-diagonal tile FP64,
                          FP32 or BF16 by the precision map (Section 2.1,
                          Fig. 1(d)): by default from the largest correlation
                          of the tile (exageo_set_mixed_correlation), or by
                          distance bands (exageo_set_mixed_policy)           */

/* optimiser of exageo_mle */
#define EXAGEO_DFO 0    /* derivative-free bounded search on l(theta)         */
#define EXAGEO_LBFGSB 1 /* bounded quasi-Newton on (l, grad l)                */
/* with EXAGEO_MIXED: the quasi-Newton search on the mixed-precision (l, grad l)
 * until its accepted l improve by less than 1e-6 |l| (the level of the mixed
 * error), then the same search in FP64 from there, continuing with the
 * quasi-Newton model (curvature pairs) the mixed search built and ending after
 * two accepted steps in a row below tol; other precisions: as EXAGEO_LBFGSB */
#define EXAGEO_LBFGSB_FP64_FINISH 2

typedef struct exageo_ctx exageo_ctx;

typedef struct {
  int64_t n_evals;      /* l(theta) evaluations                          */
  int64_t n_grad_evals; /* (l, grad) evaluations                         */
  int64_t iters;        /* optimiser iterations                          */
  double total_s;       /* wall time of the whole estimation             */
  double per_eval_s;    /* total_s / (n_evals + n_grad_evals)            */
  exageo_status status; /* EXAGEO_OK or EXAGEO_ENOCONV                    */
  int64_t n_fp64_finish_evals; /* (l, grad l) evaluations of the FP64 finish
                                  (EXAGEO_LBFGSB_FP64_FINISH; included in
                                  n_grad_evals)                          */
} exageo_mle_stats;

/* Create a context bound to HIP device `device`, tile size `ts` (a multiple of
 * 128, at least 128; the paper tunes it, Section 3 Example 2, and uses 960 on
 * GPUs) and stream `hip_stream` (a hipStream_t, NULL = default stream).
 * Returns EINVAL for a bad ts or device.  Counterpart of exageostat_init. */
exageo_status exageo_create(exageo_ctx **ctx, int device, int64_t ts, void *hip_stream);

/* Release the context and any memory the library allocated itself.  Memory
 * given through exageo_set_workspace stays owned by the caller. */
void exageo_destroy(exageo_ctx *ctx);

/* Change the stream used by later calls. */
exageo_status exageo_set_stream(exageo_ctx *ctx, void *hip_stream);

/* Device bytes the library needs for a problem of size n (tile storage,
 * sorted copies, solve vectors, schedules).  want_grad: 0 = l alone, 1 = with
 * the gradient (also what exageo_predict with mse needs: its blocks of new
 * points use the gradient's staging buffer), 2 = exageo_fisher (adds one
 * buffer of lower tiles, npad^2 / 2 doubles, for each of dSigma_beta and
 * dSigma_nu and a strip of about npad^2 / 8 doubles; npad = n rounded up to a
 * multiple of ts), 3 = exageo_fisher with a nugget (a third buffer, for
 * dSigma_sigma2).  0 for invalid arguments. */
size_t exageo_workspace_bytes(int64_t n, int64_t ts, int precision, int want_grad);

/* Hand the library a caller-owned device buffer (e.g. a torch tensor) to use
 * as its workspace.  It is used by every later call whose need fits in it;
 * otherwise the call returns ENOMEM.  Pass NULL to return to library-owned
 * allocation (hipMalloc, grown on demand, freed by exageo_destroy). */
exageo_status exageo_set_workspace(exageo_ctx *ctx, void *dev_ptr, size_t bytes);

/* Precision map of EXAGEO_MIXED by correlation (the default, with
 * fp64_at_or_above = 0.3 and bf16_below = 1e-4).  The paper's mixed-precision
 * structure keeps double-precision tiles near the diagonal and single or half
 * precision farther out (Section 2.1, Fig. 1(d)) without a rule; here, with
 * the locations in the library's Z-order cut into tiles, c_ij = the Matern
 * correlation (eq. (3) divided by sigma2) at the smallest distance between a
 * point of location block i and one of block j is the largest |Sigma_ab| /
 * sigma2 of tile (i, j) (the distances are computed once per call, or once per
 * estimation), and the tile is
 *   FP64 when c_ij >= fp64_at_or_above,
 *   BF16 when c_ij < bf16_below and c_ik c_jk < bf16_below for every k < j
 *        (the BF16 update multiplies BF16 roundings of L_ik and L_jk),
 *   FP32 otherwise.
 * FP64 tiles live in a pool of max(4 NT, half the off-diagonal tiles); when
 * more qualify, the most correlated are FP64 and the rest FP32 (the FP64
 * fraction is reported by exageo_get_timings).  With great-circle distances
 * every off-diagonal tile is FP32.  EINVAL unless 0 <= bf16_below <=
 * fp64_at_or_above (a value above 1 switches FP64 tiles off, 0 switches BF16
 * off).  Applies to later calls; switches the context to this policy. */
exageo_status exageo_set_mixed_correlation(exageo_ctx *ctx, double fp64_at_or_above, double bf16_below);

/* Precision map of EXAGEO_MIXED by distance bands (switches the context to
 * this policy): an off-diagonal tile is stored and updated in BF16 when the
 * minimum distance between the bounding boxes of its two location blocks is
 * at least band_factor * beta (0 disables BF16), in FP64 when it is below
 * fp64_band_factor * beta (exageo_set_mixed_fp64_band, default 0; closest
 * first within the pool above; the BF16 band takes precedence), else in
 * FP32.  Default band_factor 3.0.  EINVAL if < 0. */
exageo_status exageo_set_mixed_policy(exageo_ctx *ctx, double band_factor);
exageo_status exageo_set_mixed_fp64_band(exageo_ctx *ctx, double fp64_band_factor);

/* Refinement of a = Sigma^-1 z in EXAGEO_MIXED (default 1 step, at most 8):
 * after the solves through the mixed factor, each step forms the residual
 * r = z - Sigma a in FP64 with Sigma regenerated on the fly (n^2 covariance
 * evaluations, no stored matrix) and adds (mixed factor)^-1 r to a.  l then
 * uses the quadratic form z^T a, and the score the refined a in its
 * a^T dSigma a term, so only log det Sigma and tr(Sigma^-1 dSigma) carry the
 * mixed-precision error.  0 = the plain mixed solve (z^T Sigma^-1 z = |y|^2,
 * y = L^-1 z).  EINVAL if steps < 0 or > 8. */
exageo_status exageo_set_mixed_refinement(exageo_ctx *ctx, int steps);

/* Output block edge of the BF16 targets' update in EXAGEO_MIXED (paper
 * Section 2.1, the half-precision tiles): 256 (default; used when the tile
 * size is a multiple of 256, one 512-thread workgroup per 256 x 256 block) or
 * 128 (the 128 x 128 blocks of the FP32 targets' kernel).  Both form every
 * product and sum in the same order, so l and its score are the same bits;
 * the wide block reads half the operand bytes per flop.  EINVAL otherwise. */
exageo_status exageo_set_mixed_bf16_block(exageo_ctx *ctx, int edge);

/* Distance between locations (paper Section 3, the dmetric argument):
 * EXAGEO_EUCLIDEAN (default) on (x, y), or EXAGEO_GREAT_CIRCLE: x = longitude
 * and y = latitude in degrees, distance along the sphere of radius 6371 (km,
 * so beta is in km) by the haversine formula.  Applies to every later call.
 * With great-circle distances the mixed-precision distance rules (BF16 band,
 * FP64 band) are not applied: every off-diagonal tile is FP32. */
enum { EXAGEO_EUCLIDEAN = 0, EXAGEO_GREAT_CIRCLE = 1 };
exageo_status exageo_set_distance(exageo_ctx *ctx, int metric);

/* Nugget effect (the paper's closing section: the package's kernels can
 * include one): each observation carries independent noise of variance
 * tau2 >= 0, so Sigma(theta) gains tau2 on its diagonal (coincident distinct
 * locations still share sigma2 only).  tau2 is fixed, not estimated; the
 * theta-derivatives, hence the score and the Fisher information, are those of
 * the Matern part, and kriging predicts the noise-free field (no tau2 in the
 * new-to-observed covariances, mse = sigma2 - c^T Sigma^-1 c).  Applies to
 * every later call; 0 (default) = none.  EINVAL if negative or not finite. */
exageo_status exageo_set_nugget(exageo_ctx *ctx, double tau2);

/* Diagonal-super-tile (DST) approximation (paper Section 2.1, Fig. 1(b)) of
 * the likelihood calls (loglik, loglik_grad, mle; FP64 only): with the
 * locations in the library's Z-order cut into tiles of ts points, every tile
 * (I, J) with |I - J| >= band is set to zero, the factorisation then touches
 * only the band (no fill-in outside it), and the score is that of the
 * approximated likelihood.  0 (default) = exact.  simulate and predict stay
 * exact.  EINVAL if band < 0. */
exageo_status exageo_set_dst_band(exageo_ctx *ctx, int64_t band);

/* Text of the last error of this context ("" if none).  Valid until the next
 * call on the context. */
const char *exageo_last_error(const exageo_ctx *ctx);

/* Dense covariance, eq. (3): cov[i + j*ldc] = Sigma(s_i, s_j) for 0 <= i, j < n
 * in the caller's order (no sorting).  cov is a DEVICE pointer, ldc >= n.
 * Used to check the generation kernel entry by entry. */
exageo_status exageo_matern_cov(exageo_ctx *ctx, int64_t n, const double *x, const double *y,
                                const double theta[3], double *cov, int64_t ldc);

/* Synthetic field (paper Section 3, Example 1): z = L e with L the Cholesky
 * factor of Sigma(theta) in the library's sorted order, mapped back to the
 * caller's order; e and z are DEVICE pointers to n doubles (e ~ N(0, I) given
 * by the caller in caller order).  ENOTPD with *info as for exageo_loglik. */
exageo_status exageo_simulate(exageo_ctx *ctx, int64_t n, const double *x, const double *y,
                              const double theta[3], const double *e, double *z, int64_t *info);

/* l(theta), eq. (2).  precision is EXAGEO_FP64 or EXAGEO_MIXED.
 * On ENOTPD: *loglik = -INFINITY and *info = 1 + the caller index of the
 * location whose pivot failed first in the sorted factorisation; otherwise
 * *info = 0.  info may be NULL. */
exageo_status exageo_loglik(exageo_ctx *ctx, int64_t n, const double *x, const double *y, const double *z,
                            const double theta[3], int precision, double *loglik, int64_t *info);

/* l(theta) and grad[k] = dl/dtheta_k for theta = (sigma2, beta, nu).
 * EXAGEO_MIXED computes the inverse factor and Sigma^-1 after the mixed
 * factorisation in the precision map of the factor: FP64 diagonal tiles and
 * FP64 tiles where the factor has its FP64 band (FP64 MFMA), FP32 tiles
 * elsewhere (FP32 MFMA; BF16 tiles of the factor give FP32 tiles); the score
 * sums stay FP64.  On ENOTPD grad is left untouched. */
exageo_status exageo_loglik_grad(exageo_ctx *ctx, int64_t n, const double *x, const double *y,
                                 const double *z, const double theta[3], int precision, double *loglik,
                                 double grad[3], int64_t *info);

/* Allocation-free variant of exageo_loglik_grad, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same operation, arguments, statuses and
 * FP64 arithmetic as exageo_loglik_grad with precision EXAGEO_FP64 (the
 * context's distance, nugget and DST settings apply); grad may be NULL for
 * l(theta) alone.  Its workspace is a fixed 128 MiB device array that the
 * library holds on every GPU it runs on until the process ends (the context's
 * own workspace is neither used nor allocated): ENOMEM, before any launch,
 * when exageo_workspace_bytes(n, ts, EXAGEO_FP64, grad != NULL) exceeds
 * 128 MiB (n up to about 4,000 at ts <= 512).  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  Every call on one
 * GPU shares that array, whatever the context: calls that overlap on one GPU
 * (several host threads, or streams not ordered against each other) race and
 * give wrong results. */
exageo_status exageo_loglik_grad_noalloc(exageo_ctx *ctx, int64_t n, const double *x, const double *y,
                                         const double *z, const double theta[3], double *loglik, double grad[3],
                                         int64_t *info);

/* Kriging (paper Sections 4 and 5, exact_predict): the conditional
 * distribution of the field at m new locations given the n observations, in
 * FP64,
 *   mean[i] = c_i^T Sigma^-1 z,  mse[i] = sigma^2 - c_i^T Sigma^-1 c_i,
 * c_i the covariances between new point i and the observed points.  x, y, z
 * (n) and xnew, ynew, mean, mse (m) are DEVICE pointers in the caller's order;
 * mse may be NULL (mean only: one fused pass over the n m pairs); with mse the
 * library solves L V = C for blocks of up to 512 new points on MFMA in the
 * workspace's gradient staging buffer (the workspace must then hold the
 * want_grad = 1 plan, else ENOMEM).
 * Statuses as for exageo_loglik (ENOTPD with *info when Sigma is not positive
 * definite). */
exageo_status exageo_predict(exageo_ctx *ctx, int64_t n, const double *x, const double *y, const double *z,
                             const double theta[3], int64_t m, const double *xnew, const double *ynew,
                             double *mean, double *mse, int64_t *info);

/* Fisher information of theta = (sigma2, beta, nu) at the n locations (the
 * package's exact_fisher function, Section 3's table of functions): the
 * expected negative Hessian of eq. (2),
 *   I_jk = tr(Sigma^-1 dSigma_j Sigma^-1 dSigma_k) / 2,
 * computed in FP64 whatever the context's precision settings, as
 * I_jk = <B_j, B_k> / 2 with B_j = L^-1 dSigma_j L^-T (B_sigma2 = I / sigma2
 * without a nugget; B_beta, B_nu and, with a nugget, B_sigma2 by FP64 MFMA
 * products with the derivative matrices regenerated strip by strip).  x, y are
 * DEVICE pointers (n doubles, caller order); fisher is a HOST array of 9
 * doubles receiving I row-major.  Every buffer comes from the workspace
 * (exageo_workspace_bytes with want_grad = 2, or 3 with a nugget, which needs
 * B_sigma2 too): each B_j is one set of lower tiles, npad^2 / 2 doubles, so
 * with 288 GB of device memory n reaches about 140,000 (125,000 with a
 * nugget).  ENOMEM if the
 * workspace is smaller; EINVAL while the DST approximation is on; ENOTPD with
 * *info as for exageo_loglik. */
exageo_status exageo_fisher(exageo_ctx *ctx, int64_t n, const double *x, const double *y, const double theta[3],
                            double fisher[9], int64_t *info);

/* Maximum-likelihood estimate within lb <= theta <= ub (host arrays of 3).
 * theta0 = NULL starts the derivative-free method at lb, as the paper's
 * optimisation list does, and the gradient method at sqrt(lb * ub).
 * tol: stop when successive accepted l values differ by less than tol;
 * max_iters: limit on evaluations, 0 = unlimited.  method EXAGEO_DFO,
 * EXAGEO_LBFGSB or EXAGEO_LBFGSB_FP64_FINISH (the workspace must then hold
 * both the mixed and the FP64 plan with the gradient: the larger of the two
 * exageo_workspace_bytes).  Points where the factorisation fails count as
 * l = -inf.
 * Returns ENOCONV (results still written) when max_iters stops it. */
exageo_status exageo_mle(exageo_ctx *ctx, int64_t n, const double *x, const double *y, const double *z,
                         const double lb[3], const double ub[3], const double *theta0, double tol,
                         int max_iters, int method, int precision, double theta_hat[3], double *loglik_hat,
                         exageo_mle_stats *stats);

/* Per-phase timing of the last loglik / loglik_grad call, enabled with
 * exageo_set_profiling(ctx, 1) (adds HIP events between phases).
 * out receives up to nmax doubles in this order:
 *   0 total ms (first to last event), 1 sort+prep ms, 2 generation ms,
 *   3 Cholesky ms, 4 trailing-update ms (event span of each step's update
 *   launches, summed over steps), 5 trailing-update flops (real rows),
 *   6 solve+reduce ms, 7 gradient ms, 8 Cholesky flops (n^3/3 + n^2/2 + n/6,
 *   FP64 equivalent), 9 number of FP64 trailing-update (k_chol_update)
 *   launches, 10 precision used, 11 fraction of off-diagonal tiles in BF16,
 *   12 fraction in FP32, 13 number of factorisation steps with an update,
 *   14 fraction of off-diagonal tiles in the FP64 band, 15 / 16 / 17
 *   trailing-update flops into FP32 / BF16 / FP64 targets (the last includes
 *   the diagonal tiles; FP64 mode counts everything there), 19 log det Sigma,
 *   20 z^T Sigma^-1 z (the two parts of eq. (2) of the last evaluation),
 *   21 refinement steps used (mixed precision).
 * After exageo_fisher: 0 total ms, 1 to 6 as above for its factorisation,
 *   7 ms of the Fisher phase (L^-1, the derivative matrices, the products and
 *   the reduction), 18 MFMA flops of the products.
 * Returns the number of values written. */
int exageo_get_timings(const exageo_ctx *ctx, double *out, int nmax);
exageo_status exageo_set_profiling(exageo_ctx *ctx, int on);

/* Progress of exageo_mle: with on != 0 every objective evaluation prints one
 * line to stderr (evaluation count, precision, theta, l or the failure) and
 * flushes it, so that long estimations show their progress.  Default off. */
exageo_status exageo_set_verbose(exageo_ctx *ctx, int on);

#ifdef __cplusplus
}
#endif
#endif /* EXAGEO_H */

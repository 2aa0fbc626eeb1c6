/*
 * tlr.h -- C-ABI of the MI355X (gfx950) tile low-rank Matérn log-likelihood.
 *
 * Method: arXiv 1804.09137 (Abdulah, Ltaief, Sun, Genton, Keyes), "Parallel
 * Approximation of the Maximum Likelihood Estimation for the Prediction of
 * Large-Scale Geostatistics Simulations".
 *   Section III, Eq. (1):  l(theta) = -n/2 log(2 pi) - 1/2 log|Sigma(theta)|
 *                                     - 1/2 z^T Sigma(theta)^{-1} z
 *   Section IV, Eq. (MaternCov): Sigma_ab = C(||s_a - s_b||; theta),
 *       theta = (sigma^2 variance, beta range, nu smoothness)
 *   Section V: Sigma is cut into nb x nb tiles, every off-diagonal tile is
 *       held as U V^T at an absolute accuracy threshold, and the matrix is
 *       factored by a tile low-rank (TLR) Cholesky.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device (HIP) pointers owned by the caller; they
 *    must stay valid until the call's stream work has finished.  All other
 *    pointers are host pointers.
 *  - Vectors are FP64, length n, in the caller's point order (the order of
 *    the tiles).  tlr_morton_order gives the ordering the library is tuned
 *    for; the dense likelihood does not depend on the order, TLR ranks do.
 *  - Work is enqueued on the handle's stream.  Every call that returns host
 *    scalars synchronises that stream before returning.
 *  - Errors are reported only through the return code; nothing aborts or
 *    prints.  After TLR_EHIP the handle must be destroyed.
 *  - A handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef TLR_H_
#define TLR_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlr_handle_s* tlr_handle_t;

typedef enum {
  TLR_OK = 0,
  TLR_ENOTSPD = 1,     /* Sigma not positive definite: *info = 1-based global row of the first bad pivot */
  TLR_EINVAL = -1,     /* bad argument (null pointer, size, non-positive or non-finite theta, ...) */
  TLR_ENOMEM = -2,     /* device allocation failed in tlr_create, or the tile storage fixed by
                          tlr_opts.arena_bytes is too small for the factor */
  TLR_EHIP = -3,       /* a HIP runtime call failed */
  TLR_ERANK = -4,      /* a tile needed a rank above opts.maxrank; see tlr_get_info().bad_tile_* */
  TLR_ENOTIMPL = -5,   /* requested combination not available */
  TLR_ESTATE = -6      /* call order violated (e.g. tlr_loglik before tlr_potrf) */
} tlr_status;

typedef enum {
  TLR_MODE_TLR = 0,    /* tile low-rank factorisation (Section V) */
  TLR_MODE_DENSE = 1   /* dense tile Cholesky at full accuracy (the paper's "full-tile" variant) */
} tlr_mode;

typedef enum {
  TLR_PREC_FP64 = 0,          /* all arithmetic in FP64 */
  TLR_PREC_FP32_UPDATES = 1   /* TLR only: the column-update products C -= W U_row^T (most of the
                                 update flops) on FP32 MFMA with FP32 operands; generation,
                                 compression, POTRF, TRSM, solves and log-det stay FP64.  The
                                 rounding of a densely accumulated update is a full-rank
                                 perturbation of about 1e-7 of the update's magnitude, which the
                                 compression keeps: ranks (and dense tiles) grow unless tol is
                                 well above that level.  Where Sigma is ill-conditioned the
                                 perturbation can cost far more than tol (seen: 3e-3 relative at
                                 eps = 1e-6) or produce a negative pivot.  Both are caught: a
                                 negative pivot, and a first-order estimate of the change of
                                 log|Sigma| (sum over diagonal tiles of
                                 2^-24 ||update_jj||_F ||(L_jj L_jj^T)^{-1}||_F) above 5 tol |l|,
                                 checked by tlr_loglik and tlr_loglik_grad once l is known,
                                 make the library factor again with FP64 products; the handle then
                                 keeps FP64 products for its later calls (tlr_info.prec_used,
                                 fp64_retries, fp32_err_bound).  A TLR_ENOTSPD result is never
                                 caused by the FP32 products.  tlr_potrf alone does not check:
                                 tlr_sample and tlr_get_tile see the FP32-product factor */
} tlr_prec;

typedef enum {
  TLR_METRIC_EUCLID = 0,       /* ||s_a - s_b||_2 of planar coordinates (x, y) */
  TLR_METRIC_GREAT_CIRCLE = 1  /* great-circle distance on a sphere, Eq. (gcd) (the haversine
                                  formula): x = longitude, y = latitude, both in degrees;
                                  d = 2 r asin(sqrt(hav(dlat) + cos lat_a cos lat_b hav(dlon))) */
} tlr_metric;

/* tlr_opts.flags */
#define TLR_FLAG_ACA 4          /* tlr_compress compresses each tile by adaptive cross approximation with
                                   partial pivoting, fused with its generation (only the rows and columns
                                   it visits are generated; Section V lists ACA among the methods), and
                                   stops after two consecutive terms with ||u|| ||v|| <= tol / 10 (both
                                   dropped).  Its
                                   error is estimated by those terms, not bounded as the default
                                   randomized range finder's is; ranks come out a little higher than
                                   the SVD's */
#define TLR_FLAG_PIVOTED_TRUNC 8 /* truncate each tile's projection by column-pivoted QR of its t1 x t1 R
                                   factor (rank: the first step whose unreduced block has Frobenius
                                   norm <= 0.8 tol).  By default the unpivoted R is truncated directly
                                   (rank: the smallest k with ||R[k:, k:]||_F <= 0.8 tol): the basis
                                   from the QR of the random sketch already comes ordered by energy,
                                   and the ranks are the same or one or two higher */
#define TLR_FLAG_STRICT_RANK 1  /* a tile needing rank > maxrank is an error (TLR_ERANK) instead of
                                   being kept dense */
#define TLR_FLAG_SINGLE_STREAM 2 /* TLR with want_grad: issue everything on the caller's stream.  By
                                   default such a handle also runs the tangent chain and the diagonal
                                   steps on two streams of its own, with a look-ahead over the
                                   compressions (faster alone, but many handles evaluated at once,
                                   as by tlr_loglik_grad_batched, then contend for hardware queues)
                                   and holds two more n x nb column buffers.  Such a handle's host
                                   thread polls the GPU while a compression's ranks are read back;
                                   single-stream handles block */

typedef struct {
  int64_t n;          /* number of locations (>= 1) */
  int32_t nb;         /* tile size (multiple of 16, 32 <= nb <= 1024) */
  int32_t maxrank;    /* TLR: largest rank of a low-rank tile (<= 416); 0 selects nb / 4.  A tile
                         that needs more is kept dense (U = tile, V = L_jj^{-1}) unless
                         TLR_FLAG_STRICT_RANK is set */
  double tol;         /* TLR: absolute per-tile accuracy threshold (spectral norm), > 0 */
  int32_t mode;       /* tlr_mode */
  int32_t prec;       /* tlr_prec */
  int32_t want_grad;  /* non-zero: also allocate what tlr_loglik_grad needs */
  int32_t seed;       /* seed of the Gaussian sketch matrix used by TLR compression */
  int32_t flags;      /* TLR_FLAG_* */
  int32_t metric;     /* tlr_metric: distance between locations (Section IV) */
  int64_t arena_bytes; /* TLR: device bytes for the storage of the off-diagonal tiles (U and V of
                          each low-rank tile at its rank, nb x nb for a dense one; the factor and,
                          with want_grad, its tangent).  > 0: exactly that much, allocated by
                          tlr_create; a factorisation (or tlr_compress) that needs more fails with
                          TLR_ENOMEM, and the handle stays usable.  0: sized for every tile at rank
                          max(16, maxrank / 8) plus two dense tiles per tile column, and doubled
                          (reallocated, the pass started again) whenever a pass needs more.
                          < 0: TLR_EINVAL.  Ignored in DENSE mode */
  double sphere_radius; /* TLR_METRIC_GREAT_CIRCLE: radius of the sphere, in the unit of the
                          distances (and of beta); 0 selects 6371 (the Earth's mean radius in km) */
} tlr_opts;

typedef struct {
  int64_t n;
  int32_t nb, nt, maxrank, mode;
  int64_t device_bytes;       /* device memory held by the handle */
  int64_t rank_sum;           /* sum of the ranks of the strictly-lower low-rank tiles of the last factor */
  int32_t rank_max;           /* largest rank of a low-rank tile */
  int32_t dense_tiles;        /* strictly-lower tiles kept dense */
  int32_t bad_tile_i, bad_tile_j; /* TLR_ERANK: offending tile */
  int32_t prec_used;          /* tlr_prec of the last factor: TLR_PREC_FP64 when an FP32-update
                                 factor lost definiteness or failed the accuracy check and was
                                 computed again in FP64 */
  int32_t fp64_retries;       /* such repeated factorisations over the handle's life (0 or 1) */
  double t_factor_ms;         /* device time of the last factorisation (hipEvents) */
  double t_solve_ms;          /* device time of the last log-det + solves */
  double t_grad_ms;           /* device time of the gradient terms of the last tlr_loglik_grad */
  int64_t tile_bytes_used;    /* TLR: tile storage taken by the last factor (or tlr_compress) */
  int64_t tile_bytes_cap;     /* TLR: tile storage available (see tlr_opts.arena_bytes) */
  int32_t arena_grows;        /* TLR, arena_bytes = 0: times the tile storage was doubled */
  int32_t splitk_launches;    /* GEMM launches of the last factorisation that split their K range
                                 over several workgroups (long inner dimension, few output tiles) */
  int32_t qr_tiles_reg;       /* TLR: tiles of the last factorisation whose truncation (pivoted QR of
                                 the t1 x t1 factor) ran in registers (t1 <= 192), */
  int32_t qr_tiles_lds;       /*   in registers plus LDS (192 < t1 <= 224), */
  int32_t qr_tiles_global;    /*   in global memory (t1 > 224) */
  int32_t reserved_info;      /* 0 */
  double fp32_err_bound;      /* TLR_PREC_FP32_UPDATES: estimated |l_FP32 - l_FP64| / |l| of the last
                                 log-likelihood computed from a factor with FP32 products (see
                                 TLR_PREC_FP32_UPDATES); 0 when the factor used FP64 products */
} tlr_info;

/* Kernel classes timed by tlr_profile (each a group of launches). */
typedef enum {
  TLR_K_UPDATE = 0,    /* left-looking column update GEMM C -= W U_row^T (its own kernel instances) */
  TLR_K_LOWRANK = 1,   /* low-rank products: W = U (V^T V) builds, low-rank TRSM, tangent corrections */
  TLR_K_COMPRESS = 2,  /* sketch GEMM, blocked Householder QRs, pivoted QR of the small factor, projection, U */
  TLR_K_DIAG = 3,      /* diagonal tile POTRF + inverse (+ tangent of the diagonal step) */
  TLR_K_SOLVE = 4,     /* forward and backward solves */
  TLR_K_GRADQ = 5,     /* a^T dSigma a over all pairs */
  TLR_K_GEN = 6,       /* Matern (and dMatern/dbeta) generation of the column blocks */
  TLR_K_COUNT = 7
} tlr_kclass;

typedef struct {
  int64_t launches;   /* timed launch groups */
  double ms;          /* sum of their device times (hipEvents on the handle's stream) */
  double flops;       /* algorithmic flops (true ranks; no padding, no redundant work) */
  double bytes;       /* algorithmic bytes moved to/from HBM */
} tlr_kstat;

/* Create a handle for problems of size opts->n on the current HIP device.
 * stream: a hipStream_t (NULL = the null stream).  All device memory the
 * handle will use is allocated here (TLR_ENOMEM on failure), except the
 * tile storage of a TLR handle with opts->arena_bytes = 0, which a pass that
 * needs more reallocates at twice the size (see tlr_opts.arena_bytes). */
tlr_status tlr_create(tlr_handle_t* h, const tlr_opts* opts, void* stream);

/* Release every resource of the handle (NULL is accepted). */
tlr_status tlr_destroy(tlr_handle_t h);

/* Bind the locations d_x[n], d_y[n] (device, read-only) and theta =
 * (sigma^2, beta, nu) (host, all finite, beta > 0, nu > 0, sigma^2 != 0) to the
 * handle.  Sigma(theta) is defined by Eq. (MaternCov) with the distance of
 * opts->metric (Euclidean, or great-circle by Eq. (gcd); Section IV);
 * C(0) = sigma^2.  No n x n storage is written here: the tiles
 * are generated inside tlr_compress / tlr_potrf where they are consumed. */
tlr_status tlr_generate(tlr_handle_t h, const double* d_x, const double* d_y, const double theta[3]);

/* TLR mode: compress every strictly-lower tile of Sigma(theta) to U V^T with
 * ||A_ij - U V^T||_2 <= tol (Section V; a randomized range finder, then the
 * truncation of the projection's Householder R factor, column-pivoted with
 * TLR_FLAG_PIVOTED_TRUNC; or adaptive cross approximation with TLR_FLAG_ACA).
 * Fills the rank table that tlr_get_ranks returns.  This is the TLR form of
 * Sigma itself; tlr_potrf does not need it.  TLR_ENOTIMPL in DENSE mode;
 * TLR_ESTATE before tlr_generate. */
tlr_status tlr_compress(tlr_handle_t h);

/* Factor Sigma(theta) = L L^T.  TLR mode: left-looking tile low-rank
 * Cholesky (dense POTRF of diagonal tiles, low-rank TRSM, SYRK/GEMM updates
 * accumulated per tile and recompressed to tol).  DENSE mode: dense tile
 * Cholesky.  On TLR_ENOTSPD *info holds the 1-based global row of the first
 * non-positive pivot (LAPACK convention), else 0. */
tlr_status tlr_potrf(tlr_handle_t h, int64_t* info);

/* After tlr_potrf: log|Sigma| = 2 sum log diag(L), y = L^{-1} d_z,
 * quad = y^T y, and Eq. (1).  Any output pointer may be NULL. */
tlr_status tlr_loglik(tlr_handle_t h, const double* d_z, double* ll, double* logdet, double* quad);

/* Full evaluation: bind (d_x, d_y, theta), factor, and return l(theta) and
 * grad = (dl/dsigma^2, dl/dbeta) with nu held fixed.  The score is
 *   dl/dtheta_i = -1/2 tr(Sigma^{-1} dSigma_i) + 1/2 a^T dSigma_i a, a = Sigma^{-1} z;
 * dl/dsigma^2 = (q - n) / (2 sigma^2); the beta trace term is propagated
 * through the factorisation in tangent mode, the quadratic term uses exact
 * dSigma/dbeta entries.  Requires opts.want_grad.  info as in tlr_potrf. */
tlr_status tlr_loglik_grad(tlr_handle_t h, const double* d_x, const double* d_y, const double* d_z,
                           const double theta[3], double* ll, double grad[2], int64_t* info);

/* Kriging prediction (Section III, Eq. (pred3)), after tlr_potrf of Sigma_22
 * (the handle's bound locations s_1..s_n, theta and metric):
 *   d_pred[i] = (Sigma_12 Sigma_22^{-1} z)_i,  i < m,
 * with z = d_z (n observed values, caller's point order, zero mean) and
 * Sigma_12[i, b] = C(d(snew_i, s_b); theta) for the m new locations
 * (d_xnew[i], d_ynew[i]) (device, m each; any order).  Sigma_22^{-1} z is
 * computed by the forward and backward solves over the (dense or TLR)
 * factor; Sigma_12 is generated on the fly.  d_var (may be NULL): the
 * conditional variances of Eq. (pred2), C(0) - Sigma_12 Sigma_22^{-1} Sigma_21
 * on the diagonal, one forward solve per new location.  0 <= m <= 65535
 * (else TLR_EINVAL); TLR_ESTATE before tlr_potrf.  Synchronises the stream. */
tlr_status tlr_predict(tlr_handle_t h, const double* d_z, int64_t m, const double* d_xnew, const double* d_ynew,
                       double* d_pred, double* d_var);

/* tlr_loglik_grad with the smoothness free as well: grad = (dl/dsigma^2,
 * dl/dbeta, dl/dnu), the nu term
 *   -1/2 tr(Sigma^{-1} dSigma/dnu) + 1/2 a^T (dSigma/dnu) a
 * with dC/dnu = C (log(u/2) - psi(nu) + (dK_nu/dnu)(u) / K_nu(u)), u = r/beta
 * (psi the digamma function; dK_nu/dnu(x) = int_0^inf exp(-x cosh t) t sinh(nu t) dt,
 * DLMF 10.32.9 differentiated in nu), propagated through the factorisation in
 * tangent mode like the beta term.  The paper estimates all three parameters
 * (Section VIII-D, Tables I-II).  Costs two tlr_loglik_grad passes (one
 * tangent per parameter); l comes from the first.  Requires opts.want_grad. */
tlr_status tlr_loglik_grad3(tlr_handle_t h, const double* d_x, const double* d_y, const double* d_z,
                            const double theta[3], double* ll, double grad[3], int64_t* info);

/* Log-likelihood and score of several independent fields at once (one handle
 * per field, each built with want_grad; the handles must be distinct and
 * should run on distinct streams, or their work serialises).  Field f is
 * evaluated as tlr_loglik_grad(hs[f], d_x[f], d_y[f], d_z[f], theta + 3 f,
 * ll + f, grad + 2 f, info + f); nthreads host threads (<= 0: 4) drive the
 * fields concurrently so that their kernels overlap on the GPU.  ll, info and
 * status (per-field tlr_status) may be null.  Returns the first failing
 * field's status (in field order), else TLR_OK; tlr_last_error on the calling
 * thread then describes that field's failure.  The HIP runtime spreads all
 * streams of a process over GPU_MAX_HW_QUEUES hardware queues (4 unless set
 * before the runtime starts), so fields overlap only as far as that allows:
 * with handles created with TLR_FLAG_SINGLE_STREAM, 16 threads over 16 queues
 * evaluated 64 fields of n <= 20,000 4.6x faster than one at a time; 32
 * queues slow every stream down.  Batched evaluation is not in the paper: it serves many small
 * fields, whose individual evaluations cannot fill the GPU. */
tlr_status tlr_loglik_grad_batched(int32_t nfields, const tlr_handle_t* hs, const double* const* d_x,
                                   const double* const* d_y, const double* const* d_z, const double* theta,
                                   double* ll, double* grad, int64_t* info, int32_t* status, int32_t nthreads);

/* After tlr_potrf: d_z = L d_eps (the factor of Sigma(theta) times a caller
 * vector), e.g. a synthetic measurement vector z ~ N(0, Sigma) from
 * d_eps ~ N(0, I) (the data generator of Section VIII-D).  d_z must not alias
 * d_eps. */
tlr_status tlr_sample(tlr_handle_t h, const double* d_eps, double* d_z);

/* enable = 1: bracket every launch group with hipEvents on the stream it
 * runs on and accumulate per-class device time and algorithmic work (costs a
 * few microseconds per group).  enable = 2: the same, and each column-update
 * group of a gradient handle runs alone (the handle's two streams wait for
 * each other around it), so that its events time only its own kernels; the
 * evaluation is then slower.  enable = 0: off.  Other values: TLR_EINVAL.
 * Resets the counters. */
tlr_status tlr_profile(tlr_handle_t h, int32_t enable);

/* Copy the TLR_K_COUNT per-class counters into out[]. */
tlr_status tlr_get_kstats(tlr_handle_t h, tlr_kstat* out);

/* Rank table of the last tlr_compress or tlr_potrf: host_ranks[i * nt + j]
 * for i > j (other entries 0); a tile kept dense reports its width.
 * nt = ceil(n / nb). */
tlr_status tlr_get_ranks(tlr_handle_t h, int32_t* host_ranks);

/* Rank table of the tangent factor dL/dbeta of the last tlr_loglik_grad
 * (want_grad handles; the forward-mode derivative of the TLR Cholesky, whose
 * off-diagonal tiles are compressed like L's), laid out as tlr_get_ranks.
 * TLR_ESTATE without want_grad. */
tlr_status tlr_get_tangent_ranks(tlr_handle_t h, int32_t* host_ranks);

/* Sizes, memory, rank statistics and timings of the handle. */
tlr_status tlr_get_info(tlr_handle_t h, tlr_info* out);

/* Copy tile (i, j), i >= j, of the last factor (or of the compressed Sigma
 * after tlr_compress) densely into d_out (column-major, ld >= tile rows).
 * Diagonal tiles are lower triangular with zeros above. */
tlr_status tlr_get_tile(tlr_handle_t h, int32_t i, int32_t j, double* d_out, int64_t ld);

/* Write Sigma(theta)[r0:r0+m, c0:c0+k] (deriv = 0), dSigma/dbeta (deriv = 1)
 * or dSigma/dnu (deriv = 2) of the bound locations into d_out (column-major,
 * ld >= m).  Other deriv values: TLR_EINVAL. */
tlr_status tlr_covariance_block(tlr_handle_t h, int64_t r0, int64_t m, int64_t c0, int64_t k, int32_t deriv,
                                double* d_out, int64_t ld);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): the dense log-likelihood of one small field
 * in one call with no handle and no allocation, equal to tlr_create (DENSE)
 * + tlr_generate + tlr_potrf + tlr_loglik.  n locations (1 <= n <= 2048,
 * else TLR_EINVAL with a tlr_last_error text), Euclidean distance,
 * theta = (sigma^2, beta, nu) on the host, d_x, d_y, d_z device vectors of
 * length n; outputs ll, logdet, quad on the host (any may be NULL); info as
 * tlr_potrf (TLR_ENOTSPD).  Work is issued on `stream` (a hipStream_t, NULL
 * = null stream), which is synchronised before returning.  All
 * intermediates live in a fixed device array of 68 MB per GPU that the
 * library holds from its first use on that GPU until the process ends: calls
 * that overlap on one GPU (several host threads or streams) race on it and
 * must be serialised by the caller. */
tlr_status tlr_dense_loglik_noalloc(int64_t n, const double* d_x, const double* d_y, const double* d_z,
                                    const double theta[3], double* ll, double* logdet, double* quad, int64_t* info,
                                    void* stream);

/* Host helper: Morton (Z-order) permutation of n host points: each
 * coordinate is quantised to 16 bits over the points' bounding box, bits are
 * interleaved (x on even positions), keys are sorted stably.  perm[k] is the
 * input index of the k-th point. */
tlr_status tlr_morton_order(int64_t n, const double* x, const double* y, int64_t* perm);

/* Text describing the last TLR_EHIP failure of the calling thread (the HIP
 * error name and the failing call); "" if none.  The string is owned by the
 * library and stays valid until the next failing call on this thread. */
const char* tlr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TLR_H_ */

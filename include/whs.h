/*
 * whs.h -- batched Whittaker-Henderson smoother for MI355X (gfx950).
 *
 * For every series p independently the library solves
 *
 *     (W + D^T Lambda D) z = W x                                  eq. (2), eq. (3)
 *
 * where W = diag(w) holds 0/1 observation flags, D is the order-d difference
 * operator on a daily grid ((D v)_k = sum_j (-1)^(d-j) C(d,j) v_{k+j},
 * k = 0..T-d-1; the paper's k+1 is d here), and Lambda = diag(lambda_k) holds
 * one smoothing weight per row of D (eq. (3)) or one scalar per series
 * (eq. (2)).  Omega = W + D^T Lambda D is symmetric positive definite with d
 * sub-diagonals (Sec. III); it is factored as a banded Cholesky / LDL^T and
 * solved by forward and back substitution (Sec. III-A), with C right-hand
 * sides ("bands") sharing one factor (Sec. II, multivariate extension).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer is a DEVICE pointer owned by the caller.  The library
 *   never allocates device memory inside these calls; callers pass a
 *   workspace sized by whs_workspace_bytes().
 * - Calls are asynchronous on `stream` (a hipStream_t; NULL = default
 *   stream).  The return value reports argument and launch errors only; a
 *   negative value means nothing was launched.
 * - Arithmetic is FP64 throughout.  `dtype` selects the STORAGE type of x, z,
 *   g, lambda, grad_x and grad_lambda (all the same), FP32 or FP64.
 * - Interleaved time-major layouts, with b = p / S and s = p % S for
 *   S = desc->interleave, so that one time step of S neighbouring series is
 *   one contiguous, coalesced row:
 *       x, z, g, grad_x     : element ((b*T + t)*C + c)*S + s
 *       w (uint8 0/1)       : element (b*T + t)*S + s
 *       w as bits (w_format WHS_W_BITS, S a multiple of 64): bit s % 8 of
 *                             byte ((b*T + t)*S + s) / 8, the same element
 *                             index with 8 weights per byte
 *       lambda, grad_lambda : SCALAR   -> element p
 *                             PER_DIFF -> element (b*(T-d) + k)*S + s, 0 <= k < T-d
 *       factor (FP64)       : element ((b*(d+1) + i)*T + t)*S + s
 *   Arrays in the interleaved layouts span ceil(P/S) blocks; slots of the
 *   last block beyond P are neither read nor written.
 * - x is SELECTED where w_t = 1, never multiplied, so its value (even NaN)
 *   at w_t = 0 is ignored.  w_t must be 0 or 1 (any non-zero byte counts 1).
 * - Per-series status `info` (int32[P], may be NULL): 0 on success; t+1 when
 *   the pivot at time t is not positive and finite (the leading minor of
 *   order t+1 is not positive definite: a non-positive or NaN weight, or too
 *   few observations); T when fewer than d samples are observed and rounding
 *   left every pivot positive (Omega is then singular for every weight).
 *   Outputs of a failed series are NaN; other series are unaffected.
 */
#ifndef WHS_H
#define WHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WHS_OK = 0,
  WHS_ERR_ARG = -1,          /* invalid descriptor, null required pointer, misaligned pointer */
  WHS_ERR_UNSUPPORTED = -2,  /* valid but not built (e.g. d > 4) */
  WHS_ERR_HIP = -3,          /* a HIP runtime call or launch failed */
  WHS_ERR_WORKSPACE = -4     /* workspace NULL or smaller than whs_workspace_bytes() */
} whs_status;

typedef enum { WHS_F32 = 0, WHS_F64 = 1 } whs_dtype;
typedef enum { WHS_LAMBDA_SCALAR = 0, WHS_LAMBDA_PER_DIFF = 1 } whs_lambda_kind;
/* The 0/1 weights w of eq. (2) as one byte each, or packed eight to a byte:
 * 1/8 of the bytes for data that carry one bit per day.  WHS_W_BITS is taken
 * by whs_solve, whs_backward and whs_solve_noalloc on the daily grid with one
 * band (n_rhs = 1), factor NULL, an interleave that is a multiple of 64 and
 * P < 2^31; every other call, and those otherwise, return
 * WHS_ERR_UNSUPPORTED.  Results are those of the same call with bytes. */
typedef enum { WHS_W_BYTES = 0, WHS_W_BITS = 1 } whs_w_format;

typedef struct {
  int64_t n_series;    /* P >= 0; P = 0 is a no-op                               */
  int32_t T;           /* series length, T > d                                    */
  int32_t d;           /* difference order = sub-diagonals of Omega, 1..4         */
  int32_t n_rhs;       /* C >= 1 bands sharing one factor                         */
  int32_t interleave;  /* S >= 1 (64 = one wavefront per block); for S a multiple */
                       /* of 64 every per-block array (T*S*C values, T*S flags,   */
                       /* each kernel's checkpoints of one block) must stay under */
                       /* 2^31 bytes, else WHS_ERR_UNSUPPORTED (use S = 64)       */
  int32_t dtype;       /* whs_dtype: storage type of x, z, g, lambda and grads    */
  int32_t lambda_kind; /* whs_lambda_kind                                         */
  int32_t w_format;    /* whs_w_format: 0/1 weights as bytes (0) or bits (1)      */
} whs_desc;

/* Human-readable text of a status code (static storage). */
const char* whs_status_str(int status);

/* Library ABI version (major*10000 + minor*100 + patch). */
int whs_version(void);

/* Build id: the first 16 hex digits of the SHA-256 of the HIP sources and
 * headers the library was compiled from (static storage; "unknown" if the
 * build did not set it).  Lets a caller check that a prebuilt library matches
 * the sources beside it. */
const char* whs_build_id(void);

/* Bytes of device workspace whs_solve / whs_backward need for `desc`
 * (inter-sweep checkpoints; 0 when P = 0).  Any 256-byte aligned buffer of
 * at least this size may be passed; its contents need no initialisation and
 * are garbage afterwards.  Calls sharing one workspace must be ordered on
 * one stream. */
size_t whs_workspace_bytes(const whs_desc* desc);

/* Series-contiguous inputs (interleave = 1): bytes of a workspace that also
 * holds interleaved copies of the call's arrays (x or g, z, grad_x, w, and
 * lambda / grad_lambda when per difference row) plus the checkpoints of the
 * interleaved kernels; 0 for interleave != 1, P = 0, or where the copies'
 * grids would not fit a launch (T*C > 65535*64, or ceil(P/64) * ceil(T*C/k)
 * above 2^24 - 8 with k = 64 steps in FP32 and 32 in FP64); then only the
 * in-place kernels apply.  Given at least this
 * much, whs_solve, whs_backward, whs_solve_coef and whs_backward_coef on
 * interleave 1 (fused path, factor NULL) copy their inputs into the
 * interleaved layout with a tiled transpose, run the throughput kernels and
 * copy the results back: about two more passes over the data, for every order
 * and band count, and the uneven-date calls then accept interleave 1 too.
 * With less (but at least whs_workspace_bytes), interleave-1 calls run the
 * kernels that read the contiguous layout in place: for one band and d <= 2
 * the partition kernel (256 lanes per series, for P < 2^24), which is the
 * faster choice for small batches (below about 10,000 series of 3288 steps,
 * where one lane per series leaves most of the GPU idle). */
size_t whs_interleave_workspace_bytes(const whs_desc* desc);

/* Bytes of the factor array whs_factor writes: P_pad * (d+1) * T * 8. */
size_t whs_factor_bytes(const whs_desc* desc);

/*
 * whs_factor -- Cholesky factor of Omega in lower band storage (Sec. III-A,
 * Alg. 1; Fig. 2 layout): factor[i][t] = L[t+i][t] with Omega = L L^T,
 * i = 0..d, and zeros where t+i >= T.  Requires w, lambda, factor; info may
 * be NULL.  n_rhs and the x dtype are ignored except lambda's dtype.
 */
int whs_factor(const whs_desc* desc, const uint8_t* w, const void* lambda,
               double* factor, int32_t* info, void* stream);

/*
 * whs_solve -- z = Omega^{-1} W x for every band (eq. (2) / eq. (3)).
 * factor == NULL: the fused path -- Omega's rows are assembled from w and
 *   lambda on the fly and factored, and the solve runs in the same kernel
 *   (lambda and workspace required).
 * factor != NULL: solve with whs_factor's output (lambda may be NULL,
 *   workspace still required); a non-positive diagonal of the factor marks
 *   the series failed.
 * z may alias x (in place).  info may be NULL.
 */
int whs_solve(const whs_desc* desc, const uint8_t* w, const void* lambda,
              const double* factor, const void* x, void* z, int32_t* info,
              void* workspace, size_t workspace_bytes, void* stream);

/*
 * whs_solve_noalloc -- whs_solve on the fused path (factor NULL) for callers
 * that cannot allocate device memory or size a workspace: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * inter-sweep checkpoints live in a library-owned device array of
 * whs_solve_noalloc_max_bytes() (64 MiB) per GPU, held until the process
 * ends; the call itself allocates nothing.  Inputs, outputs and info are the
 * caller's, as in whs_solve.  Returns WHS_ERR_UNSUPPORTED when
 * whs_workspace_bytes(desc) exceeds that size (e.g. about 11,000 series of
 * T = 3288 at d = 2, one band, FP32), WHS_ERR_HIP if the array's address
 * cannot be obtained.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (different streams, or threads) race and
 * must be ordered by the caller.
 */
size_t whs_solve_noalloc_max_bytes(void);
int whs_solve_noalloc(const whs_desc* desc, const uint8_t* w, const void* lambda, const void* x, void* z,
                      int32_t* info, void* stream);

/*
 * whs_backward -- adjoint of whs_solve against an upstream gradient g
 * (eq. (4), eq. (5)): with u = Omega^{-1} g (one more banded solve),
 *     grad_x      = W u                      (exactly 0 where w_t = 0)
 *     grad_lambda = -sum_c (D u_c)_k (D z_c)_k   per row k   (PER_DIFF)
 *                   -sum_k sum_c (D u_c)_k (D z_c)_k         (SCALAR)
 * z is whs_solve's output for the same (w, lambda).  Either output may be
 * NULL (not computed).  grad_x may alias g.  factor may be NULL (the factor
 * is recomputed from w and lambda, the fused path) or whs_factor's output.
 */
int whs_backward(const whs_desc* desc, const uint8_t* w, const void* lambda,
                 const double* factor, const void* z, const void* g,
                 void* grad_x, void* grad_lambda, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream);

/*
 * whs_gcv -- one scalar weight per series chosen by generalised
 * cross-validation over a grid (the plain form's per-pixel selection; the
 * paper's introduction cites per-pixel cross-validated grid search as the
 * classical way to tune the weight).  For each grid value lambda_g the
 * series is smoothed (eq. (2)) and scored
 *     GCV_g = m RSS / (m - ED)^2,  m = sum_t w_t,
 *     RSS = sum_t w_t (x_t - z_t)^2,  ED = sum_t w_t (Omega^{-1})_{tt},
 * ED and RSS are computed in one forward sweep of the banded factorisation
 * per grid value, as derivatives along Omega + eps W (ED = d/deps log det,
 * RSS = sum w x^2 minus d/deps of b^T Omega^{-1} b), equal to the sums above
 * up to rounding.  lambda_best[p] is the grid value of the first minimum
 * (NaN if every grid value failed).  Requires n_rhs == 1, lambda_kind ==
 * SCALAR (it describes lambda_best), interleave a multiple of 64 or 1
 * (WHS_ERR_UNSUPPORTED otherwise).  grid: device FP64[n_grid], n_grid >= 1.
 * scores: device FP64[P][n_grid] or NULL.  info: 0 if some grid value
 * succeeded, else the first grid value's failure code.  x is read at w = 1
 * only.  Interleaves that are a multiple of 64 use no workspace
 * (whs_gcv_workspace_bytes returns 0; workspace may be NULL).  Interleave 1
 * copies x and w into the interleaved layout in a workspace of at least
 * whs_gcv_workspace_bytes(desc) bytes (8-byte aligned; WHS_ERR_WORKSPACE
 * otherwise), which returns 0, and the call WHS_ERR_UNSUPPORTED, where
 * whs_interleave_workspace_bytes would (the copies do not fit a launch).
 */
size_t whs_gcv_workspace_bytes(const whs_desc* desc);
int whs_gcv(const whs_desc* desc, const uint8_t* w, const void* x, const double* grid, int32_t n_grid,
            void* lambda_best, double* scores, int32_t* info, void* workspace, size_t workspace_bytes,
            void* stream);

/*
 * Uneven sample times (Sec. II): when the T samples sit at times
 * t_0 < t_1 < ... < t_{T-1} (days, any unit) rather than on a daily grid,
 * D is the order-d discrete derivative of the cited monograph on divided
 * differences: d! times the divided difference over d+1 consecutive times,
 *     (D v)_k = sum_{j=0..d} c[k][j] v_{k+j},
 *     c[k][j] = d! / prod_{m != j} (t_{k+j} - t_{k+m}),   k = 0..T-d-1.
 * On unit spacing c[k][j] = (-1)^(d-j) C(d, j), the daily-grid operator.
 * One time axis serves the whole batch (a tile's acquisition calendar);
 * each series still has its own weights w (clouds, padding) and lambda.
 *
 * whs_diff_coef fills coef (device FP64, row-major (T-d) x (d+1)) from
 * times (device FP64[T]); rows whose times are not strictly increasing or
 * not finite are NaN (every solve that uses them then fails with info > 0).
 * whs_solve_coef / whs_backward_coef are whs_solve / whs_backward (fused
 * path, no factor argument) with Omega = W + D^T Lambda D built from coef.
 * They require interleave a multiple of 64, or interleave 1 with a workspace
 * of at least whs_interleave_workspace_bytes(desc) (WHS_ERR_UNSUPPORTED
 * otherwise), and use the whs_workspace_bytes(desc) workspace.  An empty
 * batch (n_series 0) in either layout returns WHS_OK and touches nothing.
 * Return codes, info, aliasing and NaN conventions are those of whs_solve /
 * whs_backward.
 */
int whs_diff_coef(const double* times, int32_t T, int32_t d, double* coef, void* stream);
int whs_solve_coef(const whs_desc* desc, const double* coef, const uint8_t* w, const void* lambda,
                   const void* x, void* z, int32_t* info, void* workspace, size_t workspace_bytes,
                   void* stream);
int whs_backward_coef(const whs_desc* desc, const double* coef, const uint8_t* w, const void* lambda,
                      const void* z, const void* g, void* grad_x, void* grad_lambda, int32_t* info,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * Posterior variance of the smoothed series (Sec. IV-D, Fig. 4: the
 * credibility band drawn around the reconstruction).
 *
 * var[p][t] = (Omega^{-1})[t, t] with Omega = W + D^T Lambda D of eq. (3):
 * the variance of z_t per unit observation-noise variance, so a band is
 * z_t +/- k * sigma * sqrt(var_t) for a noise level sigma chosen by the
 * caller (for instance RSS / (m - ED) with ED = sum_t w_t var_t, the GCV
 * effective dimension).  Computed from the banded LDL^T factor by the
 * selected-inverse recurrence, run backwards in time:
 *   Sigma[t, t+j] = -sum_i L[t+i, t] Sigma[t+i, t+j]   (j = 1..d)
 *   Sigma[t, t]   = 1/Dp[t] - sum_i L[t+i, t] Sigma[t+i, t].
 * var: device, storage dtype, series layout with C = 1 (like x); lambda as
 * in whs_solve (both kinds).  Requires n_rhs == 1 (WHS_ERR_ARG otherwise)
 * and interleave a multiple of 64 or 1 (WHS_ERR_UNSUPPORTED otherwise).
 * Interleave 1 copies w and a per-difference lambda into the interleaved
 * layout, runs the interleaved kernel and copies var back, all in the
 * workspace (WHS_ERR_UNSUPPORTED where the copies do not fit a launch, as for
 * whs_interleave_workspace_bytes).  Failed series (info != 0) get NaN.  All
 * outputs are written on `stream`; the caller owns every buffer.  The
 * workspace size is whs_variance_workspace_bytes(desc).
 */
size_t whs_variance_workspace_bytes(const whs_desc* desc);
int whs_variance(const whs_desc* desc, const uint8_t* w, const void* lambda, void* var, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream);

/*
 * Uneven batches in one persistent launch.
 *
 * A group is a set of series sharing a length T and an order d, stored in
 * the interleaved layouts above with interleave 64 inside one shared buffer
 * per array: the group's first block starts at element x_off of x and z,
 * w_off of w, lam_off of lambda (SCALAR: the group's first series; PER_DIFF:
 * its first block of T-d rows) and info_off of info.  Padding every series
 * to one common T with w = 0 would give the same values on the original
 * samples (unobserved samples are padding, Sec. II) but would read and
 * solve the padding; groups avoid that.
 *
 * whs_plan_create copies the group table and a longest-first list of
 * 64-series work items to the device and allocates the plan's checkpoint
 * space (the only device memory the library allocates).  Requires
 * n_rhs == 1 and interleave == 64 (WHS_ERR_UNSUPPORTED otherwise).
 * whs_plan_solve runs every group in one persistent kernel whose
 * wavefronts take items from a device queue.  whs_plan_graph_launch does the
 * same through a HIP graph owned by the plan (built on first use, its
 * arguments updated on later calls).  whs_plan_autotune times the candidate
 * configurations (tile-depth profile 0/1/2: 8/16/24 steps for order 1, less
 * for higher orders; 1/2/4 wavefronts per workgroup; 1/2 resident
 * wavefronts per SIMD; lanes per series: one, or two for every group at
 * least split_T long) on the given buffers (z is overwritten) and keeps the
 * fastest; results are cached in the text file named by $WHS_TUNE_CACHE
 * (default $HOME/.cache/whs_tune.txt), keyed by the device and the
 * (T, d, blocks) of every group; force = 1 ignores the cache.
 * whs_plan_set_config sets a configuration instead (split_T > 0 requires
 * waves_per_block == 2; WHS_ERR_ARG otherwise).
 *
 * Two lanes per series: the two wavefronts of a workgroup take the same 64
 * series; one factors rows [0, m+d) in time order, the other rows [m, T) on
 * the time-reversed series (the same recurrence, Sec. III-A, on reversed w
 * and lambda), m = (T-d)/2; they meet at the d rows [m, m+d), whose d x d
 * system both solve, then each back-substitutes its own part.  This halves
 * the dependent chain of a long series.  It is Cholesky of a symmetric
 * permutation of Omega, so z differs from the one-lane result by rounding
 * only; configurations with the same lanes per series give bitwise-identical
 * z.  info follows the time-order convention in both cases (a failed series
 * is rescanned in time order).  whs_plan_lanes reports the lanes per series
 * of a group under the current configuration.  A plan is used by one stream
 * at a time.
 */
typedef struct {
  int64_t n_series;  /* series in the group (>= 0)                   */
  int32_t T;         /* their common length, T > d                   */
  int32_t d;         /* their common order, 1..4                     */
  int64_t x_off;     /* element offsets of the group in each buffer  */
  int64_t w_off;
  int64_t lam_off;
  int64_t info_off;
} whs_group;

typedef struct whs_plan whs_plan;

int whs_plan_create(whs_plan** plan, const whs_group* groups, int32_t n_groups, int32_t n_rhs, int32_t dtype,
                    int32_t lambda_kind, int32_t interleave);
int whs_plan_solve(whs_plan* plan, const uint8_t* w, const void* lambda, const void* x, void* z, int32_t* info,
                   void* stream);
int whs_plan_graph_launch(whs_plan* plan, const uint8_t* w, const void* lambda, const void* x, void* z,
                          int32_t* info, void* stream);
int whs_plan_autotune(whs_plan* plan, const uint8_t* w, const void* lambda, const void* x, void* z, int32_t force,
                      void* stream);
/* Current configuration (tile profile, wavefronts per workgroup, per SIMD)
 * and number of work items; any pointer may be NULL. */
int whs_plan_config(const whs_plan* plan, int32_t* tile, int32_t* waves_per_block, int32_t* waves_per_simd,
                    int32_t* n_items);
int whs_plan_set_config(whs_plan* plan, int32_t tile, int32_t waves_per_block, int32_t waves_per_simd,
                        int32_t split_T);
int whs_plan_lanes(const whs_plan* plan, int32_t group, int32_t* lanes_per_series);
void whs_plan_destroy(whs_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* WHS_H */

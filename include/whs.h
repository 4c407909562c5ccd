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

typedef struct {
  int64_t n_series;    /* P >= 0; P = 0 is a no-op                               */
  int32_t T;           /* series length, T > d                                    */
  int32_t d;           /* difference order = sub-diagonals of Omega, 1..4         */
  int32_t n_rhs;       /* C >= 1 bands sharing one factor                         */
  int32_t interleave;  /* S >= 1 (64 = one wavefront per block)                   */
  int32_t dtype;       /* whs_dtype: storage type of x, z, g, lambda and grads    */
  int32_t lambda_kind; /* whs_lambda_kind                                         */
} whs_desc;

/* Human-readable text of a status code (static storage). */
const char* whs_status_str(int status);

/* Library ABI version (major*10000 + minor*100 + patch). */
int whs_version(void);

/* Bytes of device workspace whs_solve / whs_backward need for `desc`
 * (inter-sweep checkpoints; 0 when P = 0).  Any 256-byte aligned buffer of
 * at least this size may be passed; its contents need no initialisation and
 * are garbage afterwards.  Calls sharing one workspace must be ordered on
 * one stream. */
size_t whs_workspace_bytes(const whs_desc* desc);

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

#ifdef __cplusplus
}
#endif

#endif /* WHS_H */

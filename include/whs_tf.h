/* Transformer weight network g_theta of the heteroscedastic smoother
 * (Sec. II-C: Lambda = g_theta(x, t); Sec. IV-B: a transformer over the raw
 * series with a sinusoidal encoding of the acquisition times and a final
 * sigmoid bounding the weight between a minimum and a maximum).
 *
 * Tokens are the acquisitions of a series: row m = p*T + t of a token matrix,
 * P series of T acquisitions sharing one set of acquisition days.  Widths are
 * fixed: model width 64, 2 heads of 32, feed-forward width 128.  Per layer
 * (pre-norm):  a = LN1(h); [q k v] = a Wqkv^T + bqkv;
 *              h += softmax(q k^T / sqrt(32)) v Wo^T + bo   (per head);
 *              h += relu(LN2(h) W1^T + b1) W2^T + b2.
 * Head: s = LNf(h) wh + bh, log10 lambda = lo + (hi - lo) sigmoid(s); the
 * weight of difference row k is that of acquisition k + d/2.
 *
 * Storage: the residual stream h and its gradient are FP32 (M, 64); matrix
 * product operands are bfloat16 bits (uint16), round to nearest even; weights
 * are (N, K) row-major, output channel n in row n.  FP32 parameters live in one
 * buffer in the order We be | per layer g1 b1 Wqkv bqkv Wo bo g2 b2 W1 b1' W2
 * b2' | gf bf wh bh; several calls take a pointer to a run of it (gamma then
 * beta; W then b; gf bf wh bh) and write gradients in the same order.
 *
 * Every pointer is a device pointer owned by the caller; nothing is allocated.
 * Calls are asynchronous on `stream` (a hipStream_t, NULL = default stream).
 * Return value: 0 = launched, -1 = bad argument (nothing launched),
 * -2 = unsupported shape or mode, -3 = HIP launch error, -4 = workspace too
 * small.  Reductions over tokens write per-workgroup partial sums to the
 * workspace and add them in a fixed order (results are deterministic).
 * Per-token calls accept an empty input (P or M = 0: 0, nothing launched);
 * the four reductions (whs_tf_ln_bwd, whs_tf_wgrad, whs_tf_head_bwd,
 * whs_tf_embed_bwd) need at least one token and return -1 otherwise, since
 * they would leave their parameter gradients unwritten.
 */
#ifndef WHS_TF_H
#define WHS_TF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sinusoidal encoding of the acquisition days (Sec. IV-B): pe[t][2i] =
 * sin(times[t] w_i), pe[t][2i+1] = cos(times[t] w_i), w_i = 10000^(-2i/64);
 * FP64 arithmetic, FP32 (T, 64) out.  T >= 1. */
int whs_tf_pe(const double* times, int T, float* pe, void* stream);

/* Embedding: features f = [ (x_c - mean_c) inv_sd_c where w != 0 else 0, c < C ; w != 0 ]
 * (Sec. IV-C standardises the values), written to feats (M, C+1) FP32, and
 * h = f We^T + be + pe[t] to h (M, 64) FP32.  x is the smoother's interleaved
 * layout ((b*T + t)*C + c)*S + s and w ((b*T + t)*S + s) with p = b*S + s;
 * web = We (64, C+1) then be (64).  1 <= C <= 15. */
int whs_tf_embed(const float* x, const uint8_t* w, int64_t P, int T, int C, int S, const float* mean,
                 const float* inv_sd, const float* pe, const float* web, float* feats, float* h, void* stream);

/* Layer norm over the 64 channels of each row (biased variance, eps 1e-5),
 * scaled by gamma and shifted by beta (gb = gamma then beta); bfloat16 out,
 * row mean and 1/sqrt(var + eps) saved for the backward pass. */
int whs_tf_ln_fwd(const float* h, int64_t M, const float* gb, uint16_t* out, float* mean, float* rstd,
                  void* stream);

/* Backward of whs_tf_ln_fwd: gh += dL/dh from ga = dL/dout (FP32 (M, 64));
 * dgb = (dL/dgamma, dL/dbeta) (128 FP32).  parts >= 1 workgroups. */
size_t whs_tf_ln_bwd_workspace_bytes(int parts);
int whs_tf_ln_bwd(const float* ga, const float* h, const float* mean, const float* rstd, const float* gb,
                  int64_t M, float* gh, float* dgb, float* ws, size_t ws_bytes, int parts, void* stream);

/* Token-wise product on the matrix cores: acc[m][n] = sum_k x[m][k] w[n][k]
 * with x bfloat16 (x_f32 = 0) or FP32 rounded to bfloat16 on load (x_f32 = 1),
 * K in {64, 128, 192}, N in {64, 128, 192}.  mode:
 *   0  out bf16 = acc + bias        (bias may be NULL)
 *   1  out bf16 = relu(acc + bias)
 *   2  out FP32 = res + acc + bias  (res may alias out: the residual add)
 *   3  out FP32 = acc
 *   4  out bf16 = acc where mask > 0, else 0 (mask bf16 (M, N): ReLU backward)
 * Supported (K, x_f32, mode): (64,0,0) (64,0,1) (64,0,2) (128,0,2) (64,1,4)
 * (128,0,3) (64,1,0) (192,0,3) (64,0,3). */
int whs_tf_linear(const void* x, int x_f32, int K, const uint16_t* w, const float* bias, int N, int mode,
                  const uint16_t* mask, const float* res, void* out, int64_t M, void* stream);

/* Weight and bias gradient of a token-wise product: dwb = dW (N, K) then db (N):
 * dW[n][k] = sum_m bf16(dy[m][n]) x[m][k], db[n] = sum_m dy[m][n] (the
 * unrounded dy when dy is FP32).  dy is bfloat16 (dy_f32 = 0) or FP32
 * (dy_f32 = 1) (M, N); x bfloat16 (M, K).  K in {64, 128}, N in {64, 128, 192}. */
size_t whs_tf_wgrad_workspace_bytes(int N, int K, int parts);
int whs_tf_wgrad(const void* dy, int dy_f32, int N, const uint16_t* x, int K, int64_t M, float* dwb, float* ws,
                 size_t ws_bytes, int parts, void* stream);

/* Attention of every (series, head), all T keys visible: qkv bfloat16 (M, 192)
 * with q, k, v in columns 0..63, 64..127, 128..191 and head j in 32 of each;
 * o bfloat16 (M, 64) (head j in columns 32j..), lse FP32 (P, 2, T) the
 * log-sum-exp of each query's scaled scores.  1 <= T <= 4096. */
int whs_tf_attn_fwd(const uint16_t* qkv, int64_t P, int T, uint16_t* o, float* lse, void* stream);

/* Backward of whs_tf_attn_fwd from go = dL/do (bfloat16 (M, 64)): dqkv
 * bfloat16 (M, 192) in the layout of qkv. */
int whs_tf_attn_bwd(const uint16_t* qkv, const uint16_t* o, const uint16_t* go, const float* lse, int64_t P,
                    int T, uint16_t* dqkv, void* stream);

/* Head: final layer norm, s = LNf(h) wh + bh (FP32 (M)), and the bounded
 * weight of each difference row, lam[((b*(T-d) + k)*S + s] = 10^(lo + (hi -
 * lo) sigmoid(s[p*T + k + d/2])), FP64 arithmetic, FP32 out.  hp = gf (64),
 * bf (64), wh (64), bh (1).  1 <= d <= 4, T > d, hi > lo. */
int whs_tf_head_fwd(const float* h, int64_t P, int T, const float* hp, int S, int d, float lo, float hi, float* s,
                    float* mean, float* rstd, float* lam, void* stream);

/* Backward of whs_tf_head_fwd from glam = dL/dlambda (rows, layout of lam):
 * gh = dL/dh written (FP32 (M, 64)), dhp = gradients of (gf, bf, wh, bh). */
size_t whs_tf_head_bwd_workspace_bytes(int parts);
int whs_tf_head_bwd(const float* h, const float* s, const float* mean, const float* rstd, const float* hp,
                    const float* glam, int64_t P, int T, int S, int d, float lo, float hi, float* gh, float* dhp,
                    float* ws, size_t ws_bytes, int parts, void* stream);

/* Embedding gradients: dweb = dWe (64, F) then dbe (64), dWe[e][f] =
 * sum_m gh[m][e] feats[m][f].  2 <= F <= 16. */
size_t whs_tf_embed_bwd_workspace_bytes(int F, int parts);
int whs_tf_embed_bwd(const float* gh, const float* feats, int64_t M, int F, float* dweb, float* ws,
                     size_t ws_bytes, int parts, void* stream);

/* bfloat16 copies of an FP32 (N, K) matrix: out (N, K) and, if out_t is not
 * NULL, its transpose (K, N) (the weights of the input-gradient products). */
int whs_tf_cast(const float* w, int N, int K, uint16_t* out, uint16_t* out_t, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WHS_TF_H */

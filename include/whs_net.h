/*
 * whs_net.h -- kernels of the weight network g_theta that maps a series and
 * its times to one smoothing weight per day (Sec. II-C: z = f_Lambda(x | W, D)
 * with Lambda = g_theta(x, t); Sec. IV-B: a final sigmoid bounds the weight
 * between a minimum and a maximum; Sec. IV-C: trained by masking observed
 * times and taking the MSE on them, values standardised).
 *
 * The network here is a stack of "same" 1-D convolutions over time, kernel 9
 * (4 taps of zero padding on each side), ReLU between layers: 8 -> 64 -> 64
 * -> 64 -> 1 channels (the last layer padded to 16 output channels, channel 0
 * is h).  Operands are bfloat16 (round to nearest even), products accumulate
 * in FP32 on the matrix cores (MFMA 16x16x32 bf16).
 *
 * Layouts (all device pointers, caller-owned):
 *   activations, gradients : bfloat16 (P, T, C), channels contiguous, C in {8, 16, 64}
 *   weights (forward)      : bfloat16 (Cout, 9, Cin)
 *   weights (input grad.)  : bfloat16 (Cin, 9, Cout), tap-flipped: Wd[c][8-k][o] = W[o][k][c]
 *   master weights, grads  : FP32 (Cout, 9, Cin) followed by Cout biases
 *   series-side arrays     : the smoother's interleaved layouts (whs.h), interleave S
 * Every call is asynchronous on `stream`; the return value is 0, -1 for an
 * invalid argument, -2 for an unsupported shape, -3 for a HIP error, -4 for
 * a too small workspace.
 */
#ifndef WHS_NET_H
#define WHS_NET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Convolution out[t][o] = sum_{k,c} W[o][k][c] in[t+k-4][c] (zero padding).
 * mode 0: + bias, ReLU, bfloat16 out (P,T,cout)           (cin 8 or 64, cout 64);
 *         if `bits` is not NULL, also the ReLU bits of out: bit o % 8 of byte
 *         bits[(p*T + t)*(cout/8) + o/8] is set where the stored out[p][t][o]
 *         is > 0 (the mode 2 predicate), (P,T,cout/8) bytes, caller-owned
 * mode 1: + bias, FP32 out of channel 0 only, (P,T)        (cin 64, cout 16)
 * mode 2: input gradient: no bias, out[t][o] kept only where mask[t][o] > 0
 *         (mask = the layer input's stored bfloat16 activation (P,T,cout);
 *         ReLU derivative), bfloat16 out (P,T,cout), w = the flipped
 *         transposed weights (cin 64 or 16 = the layer's padded outputs, cout 64)
 * mode 3: as mode 2 with mask = the activation's ReLU bits written by mode 0
 *         (1/16 of the mask bytes; exactly zero where a bit is clear; for
 *         cin 64 the products run on the pipelined kernel of the 64-to-64
 *         forward layer, whose FP32 sums may round differently from mode 2's
 *         by one bfloat16 step, for cin 16 the results equal mode 2's).
 * -1 for a NULL required pointer, bits with a mode other than 0, or a mask
 * missing in mode 2 or 3; -2 for a layer shape not listed or T * 128 >= 2^31. */
int whs_net_conv_fwd(const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout, int mode,
                     const void* mask, void* out, uint8_t* bits, int64_t P, int T, void* stream);

/* Inference through the whole network in one launch (Sec. II-C, the weight
 * network applied to new series): h (P,T) FP32 = channel 0 of the last
 * layer, from the (P,T,8) input, with the activations of the three hidden
 * layers kept on chip (not written).  w0..w3 and b0..b3 are the forward
 * weights and biases of the four layers as passed to whs_net_conv_fwd
 * (w3 padded to 16 output channels, channel 0 used; b3[0] used).  Each hidden
 * layer's output is rounded to bfloat16 after its ReLU, as by the layer
 * calls; sums may be taken in another order, so h can differ from the layer
 * calls' by FP32 rounding and by the bfloat16 rounding it feeds.  -1 on
 * invalid arguments, -2 if T * 16 >= 2^31. */
int whs_net_infer(const uint16_t* in8, const uint16_t* w0, const uint16_t* w1, const uint16_t* w2,
                  const uint16_t* w3, const float* b0, const float* b1, const float* b2, const float* b3, float* h,
                  int64_t P, int T, void* stream);

/* Weight gradient of the layer with input `in` (P,T,cin) and output gradient
 * gy (P,T,cout): grad[o][k][c] = sum_{p,t} gy[p,t,o] in[p,t+k-4,c], then
 * grad[cout*9*cin + o] = sum_{p,t} gy[p,t,o].  Split over `parts`
 * workgroups whose partial sums (workspace) are added in a fixed order. */
size_t whs_net_wgrad_workspace_bytes(int cin, int cout, int parts);
int whs_net_conv_wgrad(const uint16_t* in, int cin, const uint16_t* gy, int cout, float* grad, float* ws,
                       size_t ws_bytes, int parts, int64_t P, int T, void* stream);

/* Network input (P,T,8) bfloat16 from the interleaved FP32 series x and mask
 * w: [(x - mean) * inv_sd where w = 1 else 0, w, feat[t][0..3], 0, 0];
 * feat (T,4) FP32 holds per-day time features. */
int whs_net_input(const float* x, const uint8_t* w, int64_t P, int T, int S, float mean, float inv_sd,
                  const float* feat, uint16_t* out, void* stream);

/* Head: log10 lambda = lo + (hi - lo) sigmoid(h) per day (Sec. IV-B);
 * difference row k takes day k + d/2; lam is the interleaved per-difference
 * FP32 layout of whs.h. */
int whs_net_head_fwd(const float* h, int64_t P, int T, int S, int d, float lo, float hi, float* lam, void* stream);

/* dL/dh from dL/dlambda (interleaved per-difference FP32) into channel 0 of
 * gh16 (P,T,16) bfloat16, channels 1..15 zero. */
int whs_net_head_bwd(const float* h, const float* glam, int64_t P, int T, int S, int d, float lo, float hi,
                     uint16_t* gh16, void* stream);

/* The same dL/dh as one channel: gh (P,T) bfloat16 (the value channel 0 of
 * whs_net_head_bwd holds), for whs_net_last_bwd. */
int whs_net_head_bwd1(const float* h, const float* glam, int64_t P, int T, int S, int d, float lo, float hi,
                      uint16_t* gh, void* stream);

/* Backward of the last layer on its one real output channel h (Sec. II-C:
 * the weight network's output; channels 1..15 of the padded layer carry zero
 * gradient), from gh (P,T) bfloat16 = dL/dh (whs_net_head_bwd1), the layer's
 * input x (P,T,64) bfloat16, its forward weights w (16,9,64) bfloat16 (channel
 * 0 used) and the ReLU bits of x (whs_net_conv_fwd's `bits`, (P,T,8)):
 *   dx[t][c] = sum_tap w[0][tap][c] gh[t+4-tap], kept where the bit of (t, c)
 *              is set, bfloat16 (P,T,64);
 *   grad[tap*64 + c] = sum_{p,t} gh[p,t] x[p,t+tap-4][c],
 *   grad[16*9*64] = sum_{p,t} gh[p,t], every other entry of the padded
 *   (16,9,64)+16 gradient zero.
 * FP32 sums; the weight gradient over `parts` workgroups whose partial sums
 * (workspace) are added in a fixed order.  The same rounding points as
 * whs_net_conv_wgrad and whs_net_conv_fwd mode 3 on the 16-channel gradient,
 * whose results these match to FP32 summation order.  -1 on invalid
 * arguments, -4 for a too small workspace. */
size_t whs_net_last_bwd_workspace_bytes(int parts);
int whs_net_last_bwd(const uint16_t* x, const uint16_t* gh, const uint16_t* w, const uint8_t* bits, uint16_t* dx,
                     float* grad, float* ws, size_t ws_bytes, int parts, int64_t P, int T, void* stream);

/* Homoscedastic model (Sec. IV-B): one learned scalar theta (device FP32[1])
 * gives the same weight to every series, log10 lambda = lo + (hi - lo)
 * sigmoid(theta).  fwd writes lambda (FP32[P], the scalar-weight layout of
 * whs_solve); bwd writes dL/dtheta (FP32[1]) = sum_p glam[p] dlambda/dtheta
 * from whs_backward's per-series grad_lambda (FP32[P]), summed in FP64 by one
 * workgroup in a fixed order (deterministic).  -1 on invalid arguments. */
int whs_net_scalar_head_fwd(const float* theta, int64_t P, float lo, float hi, float* lam, void* stream);
int whs_net_scalar_head_bwd(const float* theta, const float* glam, int64_t P, float lo, float hi,
                            float* grad_theta, void* stream);

/* Masked MSE (Sec. IV-C, Sec. IV-D): g = 2 (z - x) inv_n where hold != 0,
 * else 0; *loss += sum of (z - x)^2 over hold (FP64, may be NULL). */
int whs_net_mse(const float* z, const float* x, const uint8_t* hold, int64_t n_elem, float inv_n, float* g,
                double* loss, void* stream);

/* Adam update with bias correction (step >= 1) of n FP32 parameters. */
int whs_net_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, void* stream);

/* bfloat16 copies of FP32 weights (n_real, 9, n_in): forward copy
 * (n_out_pad, 9, n_in) with rows >= n_real zero, and (if wd != NULL) the
 * flipped transposed copy (n_in, 9, n_out_pad) for the input gradient. */
int whs_net_pack_weights(const float* w, int n_real, int n_out_pad, int n_in, uint16_t* wf, uint16_t* wd,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WHS_NET_H */

// Kernels of the transformer weight network (Sec. IV-B): embedding with the
// sinusoidal encoding of the acquisition days, layer norm, token-wise
// products on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate),
// attention per (series, head), the bounded head, and the backward of each.
//
// Tokens are rows m = p*T + t.  The residual stream is FP32 (M, 64); product
// operands are bfloat16.  MFMA 16x16x32 operand layout: lane l holds row l%16
// of A and column l%16 of B with K entries 8*(l/16) .. +7; accumulator lane l
// holds rows 4*(l/16) .. +3 of column l%16.
//
// Attention runs on the same matrix cores, 16 queries (or keys) per
// wavefront, the other side staged in LDS 128 rows at a time so any T fits in
// a fixed amount of LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "whs_tf.h"

namespace whstf {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
typedef __attribute__((ext_vector_type(2))) uint32_t u32x2;

constexpr int E = 64;        // model width
constexpr int NH = 2;        // heads
constexpr int DH = 32;       // head width
constexpr int QKV = 3 * E;   // q, k, v columns
constexpr float LN_EPS = 1e-5f;
constexpr int MAXT = 4096;

// float -> bfloat16 bits, round to nearest even (gfx950 converts in one instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float lo_bf(uint32_t u) { return __builtin_bit_cast(float, u << 16); }
__device__ __forceinline__ float hi_bf(uint32_t u) { return __builtin_bit_cast(float, u & 0xffff0000u); }
__device__ __forceinline__ uint32_t pack2(float a, float b) { return (uint32_t)f2bf(a) | ((uint32_t)f2bf(b) << 16); }

// sum over the 16 lanes of a group (lanes 16j .. 16j+15)
__device__ __forceinline__ float sum16(float v) {
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 1);
  return v;
}

// ---------------------------------------------------------------------------
// encoding, embedding, casts, reductions
// ---------------------------------------------------------------------------
__global__ void k_pe(const double* __restrict__ times, int T, float* __restrict__ pe) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * (E / 2)) return;
  const int t = i / (E / 2), j = i % (E / 2);
  const double a = times[t] * pow(10000.0, -2.0 * j / E);
  pe[t * E + 2 * j] = (float)sin(a);
  pe[t * E + 2 * j + 1] = (float)cos(a);
}

// 16 lanes per token, 4 channels per lane (one 16-byte store each)
__global__ __launch_bounds__(256) void k_embed(const float* __restrict__ x, const uint8_t* __restrict__ w, int64_t P,
                                               int T, int C, int S, const float* __restrict__ mean,
                                               const float* __restrict__ inv_sd, const float* __restrict__ pe,
                                               const float* __restrict__ web, float* __restrict__ feats,
                                               float* __restrict__ h) {
  const int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int q = threadIdx.x & 15;
  if (m >= P * T) return;
  const int64_t p = m / T;
  const int t = (int)(m - p * T);
  const int64_t b = p / S;
  const int s = (int)(p - b * S);
  const int F = C + 1;
  const bool obs = w[(b * T + t) * S + s] != 0;
  f32x4 acc = *reinterpret_cast<const f32x4*>(pe + t * E + 4 * q);
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] += web[E * F + 4 * q + j];
  for (int c = 0; c < C; ++c) {
    const float xs = obs ? (x[((b * T + t) * C + c) * S + s] - mean[c]) * inv_sd[c] : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] += web[(4 * q + j) * F + c] * xs;
    if (q == 0) feats[m * F + c] = xs;
  }
  const float wf = obs ? 1.f : 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] += web[(4 * q + j) * F + C] * wf;
  if (q == 0) feats[m * F + C] = wf;
  *reinterpret_cast<f32x4*>(h + m * E + 4 * q) = acc;
}

__global__ void k_cast(const float* __restrict__ w, int N, int K, uint16_t* __restrict__ out,
                       uint16_t* __restrict__ out_t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * K) return;
  const int n = i / K, k = i % K;
  const uint16_t b = f2bf(w[i]);
  out[i] = b;
  if (out_t) out_t[k * N + n] = b;
}

// out[i] = sum_w part[w][i]: 64 outputs per workgroup, 16 lanes per output each
// summing every 16th partial, then the 16 sums added in a fixed order
__global__ __launch_bounds__(1024) void k_reduce(const float* __restrict__ part, int nparts, int len,
                                                 float* __restrict__ out) {
  __shared__ float red[16][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63), sl = threadIdx.x >> 6;
  float s = 0.f;
  if (col < len)
    for (int w = sl; w < nparts; w += 16) s += part[(int64_t)w * len + col];
  red[sl][threadIdx.x & 63] = s;
  __syncthreads();
  if (sl == 0 && col < len) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += red[k][threadIdx.x];
    out[col] = t;
  }
}

// dWe[e][f] = sum_m gh[m][e] feats[m][f], dbe[e] = sum_m gh[m][e]; lane = channel,
// four token slots per workgroup, partial sums per workgroup
__global__ __launch_bounds__(256) void k_embed_bwd(const float* __restrict__ gh, const float* __restrict__ feats,
                                                   int64_t M, int F, float* __restrict__ part) {
  __shared__ float red[4][E * 17];
  const int e = threadIdx.x & 63, slot = threadIdx.x >> 6;
  float acc[16], db = 0.f;
#pragma unroll
  for (int f = 0; f < 16; ++f) acc[f] = 0.f;
  // four tokens per iteration, their loads issued together
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t m0 = (int64_t)blockIdx.x * 4 + slot; m0 < M; m0 += 4 * stride) {
    float g[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) g[u] = m0 + u * stride < M ? gh[(m0 + u * stride) * E + e] : 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t m = m0 + u * stride;
      if (m >= M) break;
      db += g[u];
#pragma unroll
      for (int f = 0; f < 16; ++f)
        if (f < F) acc[f] += g[u] * feats[m * F + f];
    }
  }
#pragma unroll
  for (int f = 0; f < 16; ++f)
    if (f < F) red[slot][e * F + f] = acc[f];
  red[slot][E * F + e] = db;
  __syncthreads();
  const int len = E * F + E;
  for (int i = threadIdx.x; i < len; i += blockDim.x)
    part[(int64_t)blockIdx.x * len + i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
}

// ---------------------------------------------------------------------------
// layer norm: 16 lanes per row, 4 channels per lane
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ln_fwd(const float* __restrict__ h, int64_t M, const float* __restrict__ gb,
                                                uint16_t* __restrict__ out, float* __restrict__ mean,
                                                float* __restrict__ rstd) {
  const int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int q = threadIdx.x & 15;
  const bool ok = m < M;
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (ok) v = *reinterpret_cast<const f32x4*>(h + m * E + 4 * q);
  const float mu = sum16(v[0] + v[1] + v[2] + v[3]) * (1.f / E);
  float sq = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) sq += (v[j] - mu) * (v[j] - mu);
  const float rs = 1.f / sqrtf(sum16(sq) * (1.f / E) + LN_EPS);
  if (!ok) return;
  float y[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) y[j] = (v[j] - mu) * rs * gb[4 * q + j] + gb[E + 4 * q + j];
  u32x2 o = {pack2(y[0], y[1]), pack2(y[2], y[3])};
  *reinterpret_cast<u32x2*>(out + m * E + 4 * q) = o;
  if (q == 0) {
    mean[m] = mu;
    rstd[m] = rs;
  }
}

// gh += rstd (gx - mean(gx) - xhat mean(gx xhat)), gx = ga * gamma; partial
// sums of ga * xhat and ga per workgroup
__global__ __launch_bounds__(256) void k_ln_bwd(const float* __restrict__ ga, const float* __restrict__ h,
                                                const float* __restrict__ mean, const float* __restrict__ rstd,
                                                const float* __restrict__ gb, int64_t M, float* __restrict__ gh,
                                                float* __restrict__ part) {
  __shared__ float red[16][2 * E];
  const int slot = threadIdx.x >> 4, q = threadIdx.x & 15;
  float dg[4] = {0.f, 0.f, 0.f, 0.f}, db[4] = {0.f, 0.f, 0.f, 0.f};
  float gam[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) gam[j] = gb[4 * q + j];
  for (int64_t base = (int64_t)blockIdx.x * 16; base < M; base += (int64_t)gridDim.x * 16) {
    const int64_t m = base + slot;
    const bool ok = m < M;
    f32x4 a = {0.f, 0.f, 0.f, 0.f}, hv = {0.f, 0.f, 0.f, 0.f};
    float mu = 0.f, rs = 0.f;
    if (ok) {
      a = *reinterpret_cast<const f32x4*>(ga + m * E + 4 * q);
      hv = *reinterpret_cast<const f32x4*>(h + m * E + 4 * q);
      mu = mean[m];
      rs = rstd[m];
    }
    float xh[4], gx[4], s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      xh[j] = (hv[j] - mu) * rs;
      gx[j] = a[j] * gam[j];
      s1 += gx[j];
      s2 += gx[j] * xh[j];
      dg[j] += a[j] * xh[j];
      db[j] += a[j];
    }
    s1 = sum16(s1) * (1.f / E);
    s2 = sum16(s2) * (1.f / E);
    if (ok) {
      f32x4 g = *reinterpret_cast<const f32x4*>(gh + m * E + 4 * q);
#pragma unroll
      for (int j = 0; j < 4; ++j) g[j] += rs * (gx[j] - s1 - xh[j] * s2);
      *reinterpret_cast<f32x4*>(gh + m * E + 4 * q) = g;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    red[slot][4 * q + j] = dg[j];
    red[slot][E + 4 * q + j] = db[j];
  }
  __syncthreads();
  if (threadIdx.x < 2 * E) {
    float s = 0.f;
    for (int k = 0; k < 16; ++k) s += red[k][threadIdx.x];
    part[(int64_t)blockIdx.x * 2 * E + threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// token-wise product out[m][n] = sum_k x[m][k] w[n][k] (+ epilogue)
// Workgroup: 4 waves, one 64-column block of N (blockIdx.y); wave w owns
// columns 16w .. 16w+15 and keeps their weights in registers while the
// workgroup walks 64-row tiles staged in LDS.
// ---------------------------------------------------------------------------
template <int K, int MODE, bool AF32>
__global__ __launch_bounds__(256) void k_lin(const void* __restrict__ xin, const uint16_t* __restrict__ w,
                                             const float* __restrict__ bias, int N, const uint16_t* __restrict__ mask,
                                             const float* res, void* out, int64_t M) {
  constexpr int NS = K / 32;
  constexpr int RS = K + 8;  // LDS row stride in bf16 (16-byte pad)
  constexpr int CH = K / 8;
  __shared__ __attribute__((aligned(16))) uint16_t xs[64 * RS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int n = blockIdx.y * 64 + wave * 16 + r16;
  bf16x8 wb[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s)
    wb[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(w + (int64_t)n * K + 32 * s + 8 * g));
  const float bv = bias ? bias[n] : 0.f;
  const int64_t tiles = (M + 63) / 64;

  for (int64_t tix = blockIdx.x; tix < tiles; tix += gridDim.x) {
    const int64_t r0 = tix * 64;
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * CH; i += 256) {
      const int r = i / CH, c8 = i % CH;
      const int64_t row = r0 + r;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (row < M) {
        if constexpr (AF32) {
          const float* xf = static_cast<const float*>(xin) + row * K + 8 * c8;
          const f32x4 a = *reinterpret_cast<const f32x4*>(xf);
          const f32x4 b = *reinterpret_cast<const f32x4*>(xf + 4);
          v = u32x4{pack2(a[0], a[1]), pack2(a[2], a[3]), pack2(b[0], b[1]), pack2(b[2], b[3])};
        } else {
          v = *reinterpret_cast<const u32x4*>(static_cast<const uint16_t*>(xin) + row * K + 8 * c8);
        }
      }
      *reinterpret_cast<u32x4*>(xs + r * RS + 8 * c8) = v;
    }
    __syncthreads();
    f32x4 acc[4];
#pragma unroll
    for (int mm = 0; mm < 4; ++mm) acc[mm] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) {
        const u32x4 a = *reinterpret_cast<const u32x4*>(xs + (16 * mm + r16) * RS + 32 * s + 8 * g);
        acc[mm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), wb[s], acc[mm], 0, 0, 0);
      }
    if constexpr (MODE == 2 || MODE == 3) {
      // FP32 out: 16 lanes write 64 contiguous bytes of a row
#pragma unroll
      for (int mm = 0; mm < 4; ++mm)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t row = r0 + 16 * mm + 4 * g + j;
          if (row >= M) continue;
          const int64_t o = row * N + n;
          if constexpr (MODE == 2) static_cast<float*>(out)[o] = res[o] + acc[mm][j] + bv;
          else static_cast<float*>(out)[o] = acc[mm][j];
        }
    } else {
      // bfloat16 out: the 64 x 64 tile goes through LDS (reusing the input
      // tile) and leaves as 16-byte row pieces; the ReLU mask is applied there
      constexpr int OS = 64 + 8;
      static_assert(64 * OS <= 64 * RS, "output tile fits in the input tile");
      __syncthreads();
#pragma unroll
      for (int mm = 0; mm < 4; ++mm)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float v = MODE == 4 ? acc[mm][j] : acc[mm][j] + bv;
          xs[(16 * mm + 4 * g + j) * OS + wave * 16 + r16] = f2bf(MODE == 1 && v < 0.f ? 0.f : v);
        }
      __syncthreads();
      uint16_t* ob = static_cast<uint16_t*>(out);
      const int n0 = blockIdx.y * 64;
      for (int i = threadIdx.x; i < 64 * 8; i += 256) {
        const int r = i >> 3, c8 = i & 7;
        const int64_t row = r0 + r;
        if (row >= M) continue;
        u32x4 v = *reinterpret_cast<const u32x4*>(xs + r * OS + 8 * c8);
        if constexpr (MODE == 4) {
          const u32x4 mv = *reinterpret_cast<const u32x4*>(mask + row * N + n0 + 8 * c8);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t lo = (mv[q] & 0x7fffu) != 0u && !(mv[q] & 0x8000u) ? 0x0000ffffu : 0u;
            const uint32_t hi = ((mv[q] >> 16) & 0x7fffu) != 0u && !(mv[q] & 0x80000000u) ? 0xffff0000u : 0u;
            v[q] &= (lo | hi);
          }
        }
        *reinterpret_cast<u32x4*>(ob + row * N + n0 + 8 * c8) = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient dW[n][k] = sum_m bf16(dy[m][n]) x[m][k], db[n] = sum_m dy[m][n]
// Workgroup: one 64-row block of N (blockIdx.y), all K columns; walks chunks
// of 32 tokens staged transposed in LDS (pairs of token rows per 4-byte
// store, row stride 44) so each fragment is two 8-byte reads.  Wave w owns
// output rows 16w .. 16w+15.  Threads 0..127 stage dy (and add its column
// sums), threads 128..255 stage x.
// ---------------------------------------------------------------------------
template <int K, bool AF32>
__global__ __launch_bounds__(256) void k_wgrad(const void* __restrict__ dy, int N, const uint16_t* __restrict__ x,
                                               int64_t M, float* __restrict__ part) {
  constexpr int TK = 32;
  constexpr int XS = TK + 12;
  constexpr int CT = K / 16;
  __shared__ __attribute__((aligned(16))) uint16_t aT[64 * XS];
  __shared__ __attribute__((aligned(16))) uint16_t bT[K * XS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, r16 = lane & 15;
  const int nb = blockIdx.y * 64;
  f32x4 acc[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const int64_t chunks = (M + TK - 1) / TK;

  for (int64_t it = blockIdx.x; it < chunks; it += gridDim.x) {
    const int64_t m0 = it * TK;
    __syncthreads();
    if (threadIdx.x < 128) {
      const int up = threadIdx.x & 15, c0 = 8 * (threadIdx.x >> 4);
      const int64_t ma = m0 + 2 * up;
      u32x4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
      if constexpr (AF32) {
        const float* src = static_cast<const float*>(dy);
        f32x4 a0 = {0.f, 0.f, 0.f, 0.f}, b0 = a0, a1 = a0, b1 = a0;
        if (ma < M) {
          a0 = *reinterpret_cast<const f32x4*>(src + ma * N + nb + c0);
          b0 = *reinterpret_cast<const f32x4*>(src + ma * N + nb + c0 + 4);
        }
        if (ma + 1 < M) {
          a1 = *reinterpret_cast<const f32x4*>(src + (ma + 1) * N + nb + c0);
          b1 = *reinterpret_cast<const f32x4*>(src + (ma + 1) * N + nb + c0 + 4);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bsum[j] += a0[j] + a1[j];
          bsum[4 + j] += b0[j] + b1[j];
        }
        v0 = u32x4{pack2(a0[0], a0[1]), pack2(a0[2], a0[3]), pack2(b0[0], b0[1]), pack2(b0[2], b0[3])};
        v1 = u32x4{pack2(a1[0], a1[1]), pack2(a1[2], a1[3]), pack2(b1[0], b1[1]), pack2(b1[2], b1[3])};
      } else {
        const uint16_t* src = static_cast<const uint16_t*>(dy);
        if (ma < M) v0 = *reinterpret_cast<const u32x4*>(src + ma * N + nb + c0);
        if (ma + 1 < M) v1 = *reinterpret_cast<const u32x4*>(src + (ma + 1) * N + nb + c0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bsum[2 * q] += lo_bf(v0[q]) + lo_bf(v1[q]);
          bsum[2 * q + 1] += hi_bf(v0[q]) + hi_bf(v1[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<uint32_t*>(aT + (c0 + 2 * q) * XS + 2 * up) = (v0[q] & 0xffffu) | (v1[q] << 16);
        *reinterpret_cast<uint32_t*>(aT + (c0 + 2 * q + 1) * XS + 2 * up) = (v0[q] >> 16) | (v1[q] & 0xffff0000u);
      }
    } else {
      for (int i = threadIdx.x - 128; i < 16 * (K / 8); i += 128) {
        const int up = i & 15, c0 = 8 * (i >> 4);
        const int64_t ma = m0 + 2 * up;
        u32x4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
        if (ma < M) v0 = *reinterpret_cast<const u32x4*>(x + ma * K + c0);
        if (ma + 1 < M) v1 = *reinterpret_cast<const u32x4*>(x + (ma + 1) * K + c0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          *reinterpret_cast<uint32_t*>(bT + (c0 + 2 * q) * XS + 2 * up) = (v0[q] & 0xffffu) | (v1[q] << 16);
          *reinterpret_cast<uint32_t*>(bT + (c0 + 2 * q + 1) * XS + 2 * up) = (v0[q] >> 16) | (v1[q] & 0xffff0000u);
        }
      }
    }
    __syncthreads();
    const uint16_t* ar = aT + (16 * wave + r16) * XS + 8 * g;
    const u32x2 alo = *reinterpret_cast<const u32x2*>(ar), ahi = *reinterpret_cast<const u32x2*>(ar + 4);
    const bf16x8 a = __builtin_bit_cast(bf16x8, u32x4{alo[0], alo[1], ahi[0], ahi[1]});
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const uint16_t* br = bT + (16 * c + r16) * XS + 8 * g;
      const u32x2 blo = *reinterpret_cast<const u32x2*>(br), bhi = *reinterpret_cast<const u32x2*>(br + 4);
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          a, __builtin_bit_cast(bf16x8, u32x4{blo[0], blo[1], bhi[0], bhi[1]}), acc[c], 0, 0, 0);
    }
  }
  const int64_t len = (int64_t)N * K + N;
  float* pw = part + (int64_t)blockIdx.x * len;
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) pw[(int64_t)(nb + 16 * wave + 4 * g + j) * K + 16 * c + r16] = acc[c][j];
  if (threadIdx.x < 128) {
    // the 16 lanes of a channel group hold partial sums of its 8 columns
#pragma unroll
    for (int q = 0; q < 8; ++q) bsum[q] = sum16(bsum[q]);
    if ((threadIdx.x & 15) == 0) {
      const int c0 = 8 * (threadIdx.x >> 4);
#pragma unroll
      for (int q = 0; q < 8; ++q) pw[(int64_t)N * K + nb + c0 + q] = bsum[q];
    }
  }
}

// ---------------------------------------------------------------------------
// attention on the matrix cores
//
// Per (series, head) the scores of 16 keys x 16 queries are one MFMA with the
// key rows as A and the query rows as B (K = the 32 head channels), so a lane
// ends up holding 4 keys of one query.  Two such blocks (32 keys) give each
// lane 8 keys, {4g..4g+3} and {16+4g..16+4g+3} with g = lane/16, which is
// exactly the K slice a lane supplies as the B operand of the next MFMA: the
// probabilities (or score gradients) go from accumulator to operand without
// leaving the lane, and the other operand reads the same keys from a
// transposed copy in LDS.  Probabilities and score gradients are split into a
// bfloat16 high part and a bfloat16 remainder (two MFMAs), which keeps about 16
// significant bits; scores and value products are exact bfloat16 products
// summed in FP32.
// ---------------------------------------------------------------------------
constexpr float kScale = 0.17677669529663688f;  // 1/sqrt(32)
constexpr int ACH = 128;        // rows staged per chunk
constexpr int AWG = 8;          // wavefronts per attention workgroup (16 rows each)
constexpr int RSD = DH + 8;     // row-major LDS stride (bf16): 80 bytes
constexpr int TSD = ACH + 8;    // transposed LDS stride (bf16): 272 bytes

__device__ __forceinline__ u32x4 ld16(const uint16_t* p) { return *reinterpret_cast<const u32x4*>(p); }

// rows r0 .. r0+ACH-1 (zero from nr on) of one head's 32 columns, row-major, stride RSD
__device__ __forceinline__ void stage_r(uint16_t* dst, const uint16_t* base, int64_t stride, int col, int r0, int nr) {
  for (int i = threadIdx.x; i < ACH * 4; i += blockDim.x) {
    const int r = i >> 2, c = i & 3;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (r < nr) v = ld16(base + (int64_t)(r0 + r) * stride + col + 8 * c);
    *reinterpret_cast<u32x4*>(dst + r * RSD + 8 * c) = v;
  }
}
// the same rows transposed, dst[channel][row], stride TSD; pairs of rows per 4-byte store
__device__ __forceinline__ void stage_t(uint16_t* dst, const uint16_t* base, int64_t stride, int col, int r0, int nr) {
  for (int i = threadIdx.x; i < (ACH / 2) * 4; i += blockDim.x) {
    const int j = i >> 2, c = i & 3;
    u32x4 v0 = {0u, 0u, 0u, 0u}, v1 = {0u, 0u, 0u, 0u};
    if (2 * j < nr) v0 = ld16(base + (int64_t)(r0 + 2 * j) * stride + col + 8 * c);
    if (2 * j + 1 < nr) v1 = ld16(base + (int64_t)(r0 + 2 * j + 1) * stride + col + 8 * c);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<uint32_t*>(dst + (8 * c + 2 * q) * TSD + 2 * j) = (v0[q] & 0xffffu) | (v1[q] << 16);
      *reinterpret_cast<uint32_t*>(dst + (8 * c + 2 * q + 1) * TSD + 2 * j) = (v0[q] >> 16) | (v1[q] & 0xffff0000u);
    }
  }
}
// transposed copy of an LDS row-major copy (rows past the end are already zero)
__device__ __forceinline__ void transpose_lds(uint16_t* dst, const uint16_t* src) {
  for (int i = threadIdx.x; i < (ACH / 2) * 4; i += blockDim.x) {
    const int j = i >> 2, c = i & 3;
    const u32x4 v0 = *reinterpret_cast<const u32x4*>(src + (2 * j) * RSD + 8 * c);
    const u32x4 v1 = *reinterpret_cast<const u32x4*>(src + (2 * j + 1) * RSD + 8 * c);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<uint32_t*>(dst + (8 * c + 2 * q) * TSD + 2 * j) = (v0[q] & 0xffffu) | (v1[q] << 16);
      *reinterpret_cast<uint32_t*>(dst + (8 * c + 2 * q + 1) * TSD + 2 * j) = (v0[q] >> 16) | (v1[q] & 0xffff0000u);
    }
  }
}
// A operand from a transposed copy: channel row ch, the 8 rows {b+4g..b+4g+3, b+16+4g..+3}
__device__ __forceinline__ bf16x8 ld_t(const uint16_t* t, int ch, int b, int g) {
  const u32x2 x = *reinterpret_cast<const u32x2*>(t + ch * TSD + b + 4 * g);
  const u32x2 y = *reinterpret_cast<const u32x2*>(t + ch * TSD + b + 16 + 4 * g);
  return __builtin_bit_cast(bf16x8, u32x4{x[0], x[1], y[0], y[1]});
}
__device__ __forceinline__ bf16x8 ld_r(const uint16_t* r, int row, int g) {
  return __builtin_bit_cast(bf16x8, ld16(r + row * RSD + 8 * g));
}
// 8 FP32 values -> bfloat16 high parts and bfloat16 remainders
__device__ __forceinline__ void split8(const float* v, bf16x8& hi, bf16x8& lo) {
  u32x4 h, l;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint16_t a = f2bf(v[2 * q]), b = f2bf(v[2 * q + 1]);
    h[q] = (uint32_t)a | ((uint32_t)b << 16);
    l[q] = pack2(v[2 * q] - lo_bf(a), v[2 * q + 1] - lo_bf(b));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float max_g(float v) {
  v = fmaxf(v, __shfl_xor(v, 16));
  return fmaxf(v, __shfl_xor(v, 32));
}
__device__ __forceinline__ float sum_g(float v) {
  v += __shfl_xor(v, 16);
  return v + __shfl_xor(v, 32);
}
// lane's 4 accumulator rows 4g+r, r = 0..3, as 4 bfloat16 (8 bytes) at dst
__device__ __forceinline__ void st4(uint16_t* dst, f32x4 v, float s) {
  *reinterpret_cast<u32x2*>(dst) = u32x2{pack2(v[0] * s, v[1] * s), pack2(v[2] * s, v[3] * s)};
}

// Forward.  Workgroup: AWG waves x 16 queries (blockIdx.y selects 16 AWG queries);
// keys and transposed values staged ACH rows at a time; online softmax per
// 32-key block.  Lane (g, c) owns query c of its wave; row sums stay per lane
// until the end.
__global__ __launch_bounds__(64 * AWG) void k_attn_fwd(const uint16_t* __restrict__ qkv, int T, uint16_t* __restrict__ o,
                                                  float* __restrict__ lse) {
  __shared__ __attribute__((aligned(16))) uint16_t ks[ACH * RSD];
  __shared__ __attribute__((aligned(16))) uint16_t vt[DH * TSD];
  const int64_t p = blockIdx.x / NH;
  const int hd = blockIdx.x % NH;
  const uint16_t* base = qkv + p * (int64_t)T * QKV;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int qi = blockIdx.y * (16 * AWG) + wave * 16 + c;
  bf16x8 qb = __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
  if (qi < T) qb = __builtin_bit_cast(bf16x8, ld16(base + (int64_t)qi * QKV + DH * hd + 8 * g));
  float mx = -INFINITY, l = 0.f;
  f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < T; c0 += ACH) {
    const int nk = T - c0 < ACH ? T - c0 : ACH;
    __syncthreads();
    stage_r(ks, base, QKV, E + DH * hd, c0, nk);
    stage_t(vt, base, QKV, 2 * E + DH * hd, c0, nk);
    __syncthreads();
    for (int kb = 0; kb < nk; kb += 32) {
      const f32x4 sa = mfma(ld_r(ks, kb + c, g), qb, z4);
      const f32x4 sb = mfma(ld_r(ks, kb + 16 + c, g), qb, z4);
      float sv[8];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sv[r] = kb + 4 * g + r < nk ? sa[r] * kScale : -INFINITY;
        sv[4 + r] = kb + 16 + 4 * g + r < nk ? sb[r] * kScale : -INFINITY;
      }
      float bm = sv[0];
#pragma unroll
      for (int i = 1; i < 8; ++i) bm = fmaxf(bm, sv[i]);
      bm = max_g(bm);
      const float mn = fmaxf(mx, bm);
      const float cf = __expf(mx - mn);
      mx = mn;
      float pv[8], ps = 0.f;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        pv[i] = __expf(sv[i] - mx);
        ps += pv[i];
      }
      l = l * cf + ps;
      bf16x8 ph, pl;
      split8(pv, ph, pl);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bf16x8 a = ld_t(vt, 16 * t + c, kb, g);
        acc[t] = mfma(a, pl, acc[t] * cf);
        acc[t] = mfma(a, ph, acc[t]);
      }
    }
  }
  l = sum_g(l);
  if (qi >= T) return;
  uint16_t* dst = o + (p * T + qi) * (int64_t)E + DH * hd;
  st4(dst + 4 * g, acc[0], 1.f / l);
  st4(dst + 16 + 4 * g, acc[1], 1.f / l);
  if (g == 0) lse[(p * NH + hd) * (int64_t)T + qi] = mx + logf(l);
}

// Query gradient: dq = scale sum_k p (dp - delta) k.  Lane (g, c) owns query c
// of its wave; keys, values (row-major) and keys (transposed) staged per chunk.
__global__ __launch_bounds__(64 * AWG) void k_attn_bwd_q(const uint16_t* __restrict__ qkv, const uint16_t* __restrict__ o,
                                                    const uint16_t* __restrict__ go, const float* __restrict__ lse,
                                                    int T, uint16_t* __restrict__ dqkv) {
  __shared__ __attribute__((aligned(16))) uint16_t ks[ACH * RSD];
  __shared__ __attribute__((aligned(16))) uint16_t vs[ACH * RSD];
  __shared__ __attribute__((aligned(16))) uint16_t kt[DH * TSD];
  const int64_t p = blockIdx.x / NH;
  const int hd = blockIdx.x % NH;
  const uint16_t* base = qkv + p * (int64_t)T * QKV;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int qi = blockIdx.y * (16 * AWG) + wave * 16 + c;
  const bool act = qi < T;
  u32x4 qv = {0u, 0u, 0u, 0u}, dv = {0u, 0u, 0u, 0u}, ov = {0u, 0u, 0u, 0u};
  float L = 0.f;
  if (act) {
    qv = ld16(base + (int64_t)qi * QKV + DH * hd + 8 * g);
    dv = ld16(go + (p * T + qi) * (int64_t)E + DH * hd + 8 * g);
    ov = ld16(o + (p * T + qi) * (int64_t)E + DH * hd + 8 * g);
    L = lse[(p * NH + hd) * (int64_t)T + qi];
  }
  float dl = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q) dl += lo_bf(dv[q]) * lo_bf(ov[q]) + hi_bf(dv[q]) * hi_bf(ov[q]);
  dl = sum_g(dl);
  const bf16x8 qb = __builtin_bit_cast(bf16x8, qv), db = __builtin_bit_cast(bf16x8, dv);
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc[2] = {z4, z4};
  for (int c0 = 0; c0 < T; c0 += ACH) {
    const int nk = T - c0 < ACH ? T - c0 : ACH;
    __syncthreads();
    stage_r(ks, base, QKV, E + DH * hd, c0, nk);
    stage_r(vs, base, QKV, 2 * E + DH * hd, c0, nk);
    __syncthreads();
    transpose_lds(kt, ks);
    __syncthreads();
    for (int kb = 0; kb < nk; kb += 32) {
      const f32x4 sa = mfma(ld_r(ks, kb + c, g), qb, z4);
      const f32x4 sb = mfma(ld_r(ks, kb + 16 + c, g), qb, z4);
      const f32x4 pa = mfma(ld_r(vs, kb + c, g), db, z4);
      const f32x4 pb = mfma(ld_r(vs, kb + 16 + c, g), db, z4);
      float ds[8];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float ea = kb + 4 * g + r < nk ? __expf(sa[r] * kScale - L) : 0.f;
        const float eb = kb + 16 + 4 * g + r < nk ? __expf(sb[r] * kScale - L) : 0.f;
        ds[r] = ea * (pa[r] - dl);
        ds[4 + r] = eb * (pb[r] - dl);
      }
      bf16x8 hh, ll;
      split8(ds, hh, ll);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bf16x8 a = ld_t(kt, 16 * t + c, kb, g);
        acc[t] = mfma(a, ll, acc[t]);
        acc[t] = mfma(a, hh, acc[t]);
      }
    }
  }
  if (!act) return;
  uint16_t* dst = dqkv + (p * T + qi) * (int64_t)QKV + DH * hd;
  st4(dst + 4 * g, acc[0], kScale);
  st4(dst + 16 + 4 * g, acc[1], kScale);
}

// Key and value gradients: dv = sum_q p do, dk = scale sum_q p (dp - delta) q.
// Lane (g, c) owns key c of its wave; queries (row-major and transposed), output
// gradients (both), log-sum-exps and deltas staged per chunk.
__global__ __launch_bounds__(64 * AWG) void k_attn_bwd_kv(const uint16_t* __restrict__ qkv, const uint16_t* __restrict__ o,
                                                     const uint16_t* __restrict__ go, const float* __restrict__ lse,
                                                     int T, uint16_t* __restrict__ dqkv) {
  __shared__ __attribute__((aligned(16))) uint16_t qs[ACH * RSD];
  __shared__ __attribute__((aligned(16))) uint16_t dos[ACH * RSD];
  __shared__ __attribute__((aligned(16))) uint16_t qt[DH * TSD];
  __shared__ __attribute__((aligned(16))) uint16_t dt[DH * TSD];
  __shared__ __attribute__((aligned(16))) float ls[ACH];
  __shared__ __attribute__((aligned(16))) float dl[ACH];
  const int64_t p = blockIdx.x / NH;
  const int hd = blockIdx.x % NH;
  const uint16_t* base = qkv + p * (int64_t)T * QKV;
  const uint16_t* gob = go + p * (int64_t)T * E;
  const uint16_t* ob = o + p * (int64_t)T * E;
  const float* lb = lse + (p * NH + hd) * (int64_t)T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int kj = blockIdx.y * (16 * AWG) + wave * 16 + c;
  u32x4 kv = {0u, 0u, 0u, 0u}, vv = {0u, 0u, 0u, 0u};
  if (kj < T) {
    kv = ld16(base + (int64_t)kj * QKV + E + DH * hd + 8 * g);
    vv = ld16(base + (int64_t)kj * QKV + 2 * E + DH * hd + 8 * g);
  }
  const bf16x8 kb8 = __builtin_bit_cast(bf16x8, kv), vb8 = __builtin_bit_cast(bf16x8, vv);
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  f32x4 adv[2] = {z4, z4}, adk[2] = {z4, z4};
  for (int c0 = 0; c0 < T; c0 += ACH) {
    const int nq = T - c0 < ACH ? T - c0 : ACH;
    __syncthreads();
    stage_r(qs, base, QKV, DH * hd, c0, nq);
    stage_r(dos, gob, E, DH * hd, c0, nq);
    __syncthreads();
    transpose_lds(qt, qs);
    transpose_lds(dt, dos);
    for (int r = threadIdx.x; r < ACH; r += blockDim.x) {
      float d = 0.f, L = INFINITY;   // rows past the end: p = 0
      if (r < nq) {
        const uint16_t* b = ob + (int64_t)(c0 + r) * E + DH * hd;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          const u32x4 x = *reinterpret_cast<const u32x4*>(dos + r * RSD + 8 * cc), y = ld16(b + 8 * cc);
#pragma unroll
          for (int q = 0; q < 4; ++q) d += lo_bf(x[q]) * lo_bf(y[q]) + hi_bf(x[q]) * hi_bf(y[q]);
        }
        L = lb[c0 + r];
      }
      dl[r] = d;
      ls[r] = L;
    }
    __syncthreads();
    for (int qb = 0; qb < nq; qb += 32) {
      // scores and output-gradient products, queries as rows: lane holds queries 4g+r of each half
      const f32x4 sa = mfma(ld_r(qs, qb + c, g), kb8, z4);
      const f32x4 sb = mfma(ld_r(qs, qb + 16 + c, g), kb8, z4);
      const f32x4 pa = mfma(ld_r(dos, qb + c, g), vb8, z4);
      const f32x4 pb = mfma(ld_r(dos, qb + 16 + c, g), vb8, z4);
      // statistics of queries qb+4g..+3 and qb+16+4g..+3: four 16-byte reads
      const f32x4 la = *reinterpret_cast<const f32x4*>(ls + qb + 4 * g);
      const f32x4 lb4 = *reinterpret_cast<const f32x4*>(ls + qb + 16 + 4 * g);
      const f32x4 da = *reinterpret_cast<const f32x4*>(dl + qb + 4 * g);
      const f32x4 db = *reinterpret_cast<const f32x4*>(dl + qb + 16 + 4 * g);
      float pr[8], ds[8];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pr[r] = __expf(sa[r] * kScale - la[r]);
        pr[4 + r] = __expf(sb[r] * kScale - lb4[r]);
        ds[r] = pr[r] * (pa[r] - da[r]);
        ds[4 + r] = pr[4 + r] * (pb[r] - db[r]);
      }
      bf16x8 ph, pl, hh, ll;
      split8(pr, ph, pl);
      split8(ds, hh, ll);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bf16x8 a = ld_t(dt, 16 * t + c, qb, g);
        adv[t] = mfma(a, pl, adv[t]);
        adv[t] = mfma(a, ph, adv[t]);
        const bf16x8 b = ld_t(qt, 16 * t + c, qb, g);
        adk[t] = mfma(b, ll, adk[t]);
        adk[t] = mfma(b, hh, adk[t]);
      }
    }
  }
  if (kj >= T) return;
  uint16_t* dst = dqkv + (p * T + kj) * (int64_t)QKV + DH * hd;
  st4(dst + E + 4 * g, adk[0], kScale);
  st4(dst + E + 16 + 4 * g, adk[1], kScale);
  st4(dst + 2 * E + 4 * g, adv[0], 1.f);
  st4(dst + 2 * E + 16 + 4 * g, adv[1], 1.f);
}

// ---------------------------------------------------------------------------
// head
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sigmoid_d(double v) { return 1.0 / (1.0 + exp(-v)); }

__global__ __launch_bounds__(256) void k_head_fwd(const float* __restrict__ h, int64_t P, int T,
                                                  const float* __restrict__ hp, int S, int d, float lo, float hi,
                                                  float* __restrict__ s_out, float* __restrict__ mean,
                                                  float* __restrict__ rstd, float* __restrict__ lam) {
  const int64_t m = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int q = threadIdx.x & 15;
  const int64_t M = P * T;
  const bool ok = m < M;
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (ok) v = *reinterpret_cast<const f32x4*>(h + m * E + 4 * q);
  const float mu = sum16(v[0] + v[1] + v[2] + v[3]) * (1.f / E);
  float sq = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) sq += (v[j] - mu) * (v[j] - mu);
  const float rs = 1.f / sqrtf(sum16(sq) * (1.f / E) + LN_EPS);
  float dsum = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = 4 * q + j;
    dsum += ((v[j] - mu) * rs * hp[c] + hp[E + c]) * hp[2 * E + c];
  }
  const float sv = sum16(dsum) + hp[3 * E];
  if (!ok || q != 0) return;
  s_out[m] = sv;
  mean[m] = mu;
  rstd[m] = rs;
  const int64_t p = m / T;
  const int t = (int)(m - p * T);
  const int k = t - d / 2;
  if (k >= 0 && k < T - d) {
    const int64_t b = p / S;
    const int si = (int)(p - b * S);
    lam[(b * (T - d) + k) * S + si] = (float)exp10((double)lo + ((double)hi - (double)lo) * sigmoid_d(sv));
  }
}

__global__ __launch_bounds__(256) void k_head_bwd(const float* __restrict__ h, const float* __restrict__ s_in,
                                                  const float* __restrict__ mean, const float* __restrict__ rstd,
                                                  const float* __restrict__ hp, const float* __restrict__ glam,
                                                  int64_t P, int T, int S, int d, float lo, float hi,
                                                  float* __restrict__ gh, float* __restrict__ part) {
  __shared__ float red[16][3 * E + 1];
  const int slot = threadIdx.x >> 4, q = threadIdx.x & 15;
  const int64_t M = P * T;
  float dgf[4] = {0.f, 0.f, 0.f, 0.f}, dbf[4] = {0.f, 0.f, 0.f, 0.f}, dwh[4] = {0.f, 0.f, 0.f, 0.f};
  float dbh = 0.f;
  for (int64_t base = (int64_t)blockIdx.x * 16; base < M; base += (int64_t)gridDim.x * 16) {
    const int64_t m = base + slot;
    const bool ok = m < M;
    float gs = 0.f, mu = 0.f, rs = 0.f;
    f32x4 hv = {0.f, 0.f, 0.f, 0.f};
    if (ok) {
      const int64_t p = m / T;
      const int t = (int)(m - p * T);
      const int k = t - d / 2;
      if (k >= 0 && k < T - d) {
        const int64_t b = p / S;
        const int si = (int)(p - b * S);
        const double sg = sigmoid_d((double)s_in[m]);
        const double lv = exp10((double)lo + ((double)hi - (double)lo) * sg);
        gs = (float)((double)glam[(b * (T - d) + k) * S + si] * lv * 2.302585092994046 * ((double)hi - (double)lo) *
                     sg * (1.0 - sg));
      }
      hv = *reinterpret_cast<const f32x4*>(h + m * E + 4 * q);
      mu = mean[m];
      rs = rstd[m];
    }
    float xh[4], gx[4], s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 4 * q + j;
      xh[j] = (hv[j] - mu) * rs;
      const float gy = gs * hp[2 * E + c];
      dwh[j] += gs * (xh[j] * hp[c] + hp[E + c]);
      dgf[j] += gy * xh[j];
      dbf[j] += gy;
      gx[j] = gy * hp[c];
      s1 += gx[j];
      s2 += gx[j] * xh[j];
    }
    if (q == 0) dbh += gs;
    s1 = sum16(s1) * (1.f / E);
    s2 = sum16(s2) * (1.f / E);
    if (ok) {
      f32x4 o;
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = rs * (gx[j] - s1 - xh[j] * s2);
      *reinterpret_cast<f32x4*>(gh + m * E + 4 * q) = o;
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    red[slot][4 * q + j] = dgf[j];
    red[slot][E + 4 * q + j] = dbf[j];
    red[slot][2 * E + 4 * q + j] = dwh[j];
  }
  if (q == 0) red[slot][3 * E] = dbh;
  __syncthreads();
  if (threadIdx.x < 3 * E + 1) {
    float s = 0.f;
    for (int k = 0; k < 16; ++k) s += red[k][threadIdx.x];
    part[(int64_t)blockIdx.x * (3 * E + 1) + threadIdx.x] = s;
  }
}

}  // namespace whstf

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace whstf;

namespace {
int st(hipError_t e) { return e == hipSuccess ? 0 : -3; }
inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
constexpr int64_t kLinBlocks = 2048;
hipStream_t hs(void* s) { return static_cast<hipStream_t>(s); }
bool okn(int n) { return n == 64 || n == 128 || n == 192; }
}  // namespace

extern "C" {

int whs_tf_pe(const double* times, int T, float* pe, void* stream) {
  if (!times || !pe || T < 1) return -1;
  hipLaunchKernelGGL(k_pe, dim3(nblk((int64_t)T * (E / 2), 256)), dim3(256), 0, hs(stream), times, T, pe);
  return st(hipGetLastError());
}

int whs_tf_embed(const float* x, const uint8_t* w, int64_t P, int T, int C, int S, const float* mean,
                 const float* inv_sd, const float* pe, const float* web, float* feats, float* h, void* stream) {
  if (!x || !w || !mean || !inv_sd || !pe || !web || !feats || !h || P < 0 || T < 1 || C < 1 || C > 15 || S < 1)
    return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_embed, dim3(nblk(P * T * 16, 256)), dim3(256), 0, hs(stream), x, w, P, T, C, S, mean, inv_sd,
                     pe, web, feats, h);
  return st(hipGetLastError());
}

int whs_tf_ln_fwd(const float* h, int64_t M, const float* gb, uint16_t* out, float* mean, float* rstd,
                  void* stream) {
  if (!h || !gb || !out || !mean || !rstd || M < 0) return -1;
  if (M == 0) return 0;
  hipLaunchKernelGGL(k_ln_fwd, dim3(nblk(M * 16, 256)), dim3(256), 0, hs(stream), h, M, gb, out, mean, rstd);
  return st(hipGetLastError());
}

size_t whs_tf_ln_bwd_workspace_bytes(int parts) { return (size_t)(parts > 0 ? parts : 0) * 2 * E * sizeof(float); }

int whs_tf_ln_bwd(const float* ga, const float* h, const float* mean, const float* rstd, const float* gb,
                  int64_t M, float* gh, float* dgb, float* ws, size_t ws_bytes, int parts, void* stream) {
  if (!ga || !h || !mean || !rstd || !gb || !gh || !dgb || !ws || M < 1 || parts < 1) return -1;
  if (ws_bytes < whs_tf_ln_bwd_workspace_bytes(parts)) return -4;
  hipLaunchKernelGGL(k_ln_bwd, dim3(parts), dim3(256), 0, hs(stream), ga, h, mean, rstd, gb, M, gh, ws);
  hipLaunchKernelGGL(k_reduce, dim3(nblk(2 * E, 64)), dim3(1024), 0, hs(stream), ws, parts, 2 * E, dgb);
  return st(hipGetLastError());
}

int whs_tf_linear(const void* x, int x_f32, int K, const uint16_t* w, const float* bias, int N, int mode,
                  const uint16_t* mask, const float* res, void* out, int64_t M, void* stream) {
  if (!x || !w || !out || M < 0 || !okn(K) || !okn(N) || mode < 0 || mode > 4) return -1;
  if ((mode == 4 && !mask) || (mode == 2 && !res)) return -1;
  if (M == 0) return 0;
  const int64_t tiles = (M + 63) / 64;
  dim3 grid((unsigned)(tiles < kLinBlocks ? tiles : kLinBlocks), (unsigned)(N / 64));
#define WHS_LIN(KK, MO, AF)                                                                                   \
  hipLaunchKernelGGL((k_lin<KK, MO, AF>), grid, dim3(256), 0, hs(stream), x, w, bias, N, mask, res, out, M)
  if (K == 64 && !x_f32 && mode == 0) WHS_LIN(64, 0, false);
  else if (K == 64 && !x_f32 && mode == 1) WHS_LIN(64, 1, false);
  else if (K == 64 && !x_f32 && mode == 2) WHS_LIN(64, 2, false);
  else if (K == 64 && !x_f32 && mode == 3) WHS_LIN(64, 3, false);
  else if (K == 128 && !x_f32 && mode == 2) WHS_LIN(128, 2, false);
  else if (K == 128 && !x_f32 && mode == 3) WHS_LIN(128, 3, false);
  else if (K == 192 && !x_f32 && mode == 3) WHS_LIN(192, 3, false);
  else if (K == 64 && x_f32 && mode == 4) WHS_LIN(64, 4, true);
  else if (K == 64 && x_f32 && mode == 0) WHS_LIN(64, 0, true);
  else return -2;
#undef WHS_LIN
  return st(hipGetLastError());
}

size_t whs_tf_wgrad_workspace_bytes(int N, int K, int parts) {
  return (size_t)(parts > 0 ? parts : 0) * ((size_t)N * K + N) * sizeof(float);
}

int whs_tf_wgrad(const void* dy, int dy_f32, int N, const uint16_t* x, int K, int64_t M, float* dwb, float* ws,
                 size_t ws_bytes, int parts, void* stream) {
  if (!dy || !x || !dwb || !ws || M < 1 || parts < 1 || !okn(N) || (K != 64 && K != 128)) return -1;
  if (ws_bytes < whs_tf_wgrad_workspace_bytes(N, K, parts)) return -4;
  dim3 grid((unsigned)parts, (unsigned)(N / 64));
  if (K == 64 && dy_f32) hipLaunchKernelGGL((k_wgrad<64, true>), grid, dim3(256), 0, hs(stream), dy, N, x, M, ws);
  else if (K == 64) hipLaunchKernelGGL((k_wgrad<64, false>), grid, dim3(256), 0, hs(stream), dy, N, x, M, ws);
  else if (dy_f32) hipLaunchKernelGGL((k_wgrad<128, true>), grid, dim3(256), 0, hs(stream), dy, N, x, M, ws);
  else hipLaunchKernelGGL((k_wgrad<128, false>), grid, dim3(256), 0, hs(stream), dy, N, x, M, ws);
  const int len = N * K + N;
  hipLaunchKernelGGL(k_reduce, dim3(nblk(len, 64)), dim3(1024), 0, hs(stream), ws, parts, len, dwb);
  return st(hipGetLastError());
}

int whs_tf_attn_fwd(const uint16_t* qkv, int64_t P, int T, uint16_t* o, float* lse, void* stream) {
  if (!qkv || !o || !lse || P < 0 || T < 1 || T > MAXT) return -1;
  if (P == 0) return 0;
  const dim3 grid((unsigned)(P * NH), (unsigned)((T + 16 * AWG - 1) / (16 * AWG)));
  hipLaunchKernelGGL(k_attn_fwd, grid, dim3(64 * AWG), 0, hs(stream), qkv, T, o, lse);
  return st(hipGetLastError());
}

int whs_tf_attn_bwd(const uint16_t* qkv, const uint16_t* o, const uint16_t* go, const float* lse, int64_t P,
                    int T, uint16_t* dqkv, void* stream) {
  if (!qkv || !o || !go || !lse || !dqkv || P < 0 || T < 1 || T > MAXT) return -1;
  if (P == 0) return 0;
  const dim3 grid((unsigned)(P * NH), (unsigned)((T + 16 * AWG - 1) / (16 * AWG)));
  hipLaunchKernelGGL(k_attn_bwd_kv, grid, dim3(64 * AWG), 0, hs(stream), qkv, o, go, lse, T, dqkv);
  hipLaunchKernelGGL(k_attn_bwd_q, grid, dim3(64 * AWG), 0, hs(stream), qkv, o, go, lse, T, dqkv);
  return st(hipGetLastError());
}

int whs_tf_head_fwd(const float* h, int64_t P, int T, const float* hp, int S, int d, float lo, float hi, float* s,
                    float* mean, float* rstd, float* lam, void* stream) {
  if (!h || !hp || !s || !mean || !rstd || !lam || P < 0 || d < 1 || d > 4 || T <= d || S < 1 || !(hi > lo))
    return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_head_fwd, dim3(nblk(P * T * 16, 256)), dim3(256), 0, hs(stream), h, P, T, hp, S, d, lo, hi, s,
                     mean, rstd, lam);
  return st(hipGetLastError());
}

size_t whs_tf_head_bwd_workspace_bytes(int parts) {
  return (size_t)(parts > 0 ? parts : 0) * (3 * E + 1) * sizeof(float);
}

int whs_tf_head_bwd(const float* h, const float* s, const float* mean, const float* rstd, const float* hp,
                    const float* glam, int64_t P, int T, int S, int d, float lo, float hi, float* gh, float* dhp,
                    float* ws, size_t ws_bytes, int parts, void* stream) {
  if (!h || !s || !mean || !rstd || !hp || !glam || !gh || !dhp || !ws || P < 1 || d < 1 || d > 4 || T <= d ||
      S < 1 || parts < 1 || !(hi > lo))
    return -1;
  if (ws_bytes < whs_tf_head_bwd_workspace_bytes(parts)) return -4;
  hipLaunchKernelGGL(k_head_bwd, dim3(parts), dim3(256), 0, hs(stream), h, s, mean, rstd, hp, glam, P, T, S, d, lo,
                     hi, gh, ws);
  hipLaunchKernelGGL(k_reduce, dim3(nblk(3 * E + 1, 64)), dim3(1024), 0, hs(stream), ws, parts, 3 * E + 1, dhp);
  return st(hipGetLastError());
}

size_t whs_tf_embed_bwd_workspace_bytes(int F, int parts) {
  return (size_t)(parts > 0 ? parts : 0) * ((size_t)E * F + E) * sizeof(float);
}

int whs_tf_embed_bwd(const float* gh, const float* feats, int64_t M, int F, float* dweb, float* ws,
                     size_t ws_bytes, int parts, void* stream) {
  if (!gh || !feats || !dweb || !ws || M < 1 || F < 2 || F > 16 || parts < 1) return -1;
  if (ws_bytes < whs_tf_embed_bwd_workspace_bytes(F, parts)) return -4;
  hipLaunchKernelGGL(k_embed_bwd, dim3(parts), dim3(256), 0, hs(stream), gh, feats, M, F, ws);
  const int len = E * F + E;
  hipLaunchKernelGGL(k_reduce, dim3(nblk(len, 64)), dim3(1024), 0, hs(stream), ws, parts, len, dweb);
  return st(hipGetLastError());
}

int whs_tf_cast(const float* w, int N, int K, uint16_t* out, uint16_t* out_t, void* stream) {
  if (!w || !out || N < 1 || K < 1) return -1;
  hipLaunchKernelGGL(k_cast, dim3(nblk((int64_t)N * K, 256)), dim3(256), 0, hs(stream), w, N, K, out, out_t);
  return st(hipGetLastError());
}

}  // extern "C"

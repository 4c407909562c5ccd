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
// Attention is FP32 vector arithmetic: one lane per query (forward, query
// gradient) or per key (key and value gradients), the other side staged in
// LDS 256 rows at a time and read as wave-wide broadcasts, so any T fits in a
// fixed 32 KB and the results match an exact softmax to FP32 rounding.
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
constexpr int KC = 256;      // attention rows staged per chunk
constexpr int MAXT = 4096;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
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

// 32 bfloat16 (one head row, 64 bytes) -> FP32
__device__ __forceinline__ void load_row32(const uint16_t* src, float* dst) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const u32x4 v = *reinterpret_cast<const u32x4*>(src + 8 * c);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dst[8 * c + 2 * q] = lo_bf(v[q]);
      dst[8 * c + 2 * q + 1] = hi_bf(v[q]);
    }
  }
}
__device__ __forceinline__ void store_row32(uint16_t* dst, const float* v, float scale) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    u32x4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = pack2(v[8 * c + 2 * q] * scale, v[8 * c + 2 * q + 1] * scale);
    *reinterpret_cast<u32x4*>(dst + 8 * c) = o;
  }
}
__device__ __forceinline__ float dot32(const float* a, const float* b) {
  float s = 0.f;
#pragma unroll
  for (int d = 0; d < DH; ++d) s += a[d] * b[d];
  return s;
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

// one lane per (token, channel)
__global__ void k_embed(const float* __restrict__ x, const uint8_t* __restrict__ w, int64_t P, int T, int C, int S,
                        const float* __restrict__ mean, const float* __restrict__ inv_sd,
                        const float* __restrict__ pe, const float* __restrict__ web, float* __restrict__ feats,
                        float* __restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * T * E) return;
  const int64_t m = i / E;
  const int e = (int)(i - m * E);
  const int64_t p = m / T;
  const int t = (int)(m - p * T);
  const int64_t b = p / S;
  const int s = (int)(p - b * S);
  const int F = C + 1;
  const bool obs = w[(b * T + t) * S + s] != 0;
  float acc = web[E * F + e] + pe[t * E + e];
  for (int c = 0; c < C; ++c) {
    const float xs = obs ? (x[((b * T + t) * C + c) * S + s] - mean[c]) * inv_sd[c] : 0.f;
    acc += web[e * F + c] * xs;
    if (e == 0) feats[m * F + c] = xs;
  }
  const float wf = obs ? 1.f : 0.f;
  acc += web[e * F + C] * wf;
  if (e == 0) feats[m * F + C] = wf;
  h[m * E + e] = acc;
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

__global__ void k_reduce(const float* __restrict__ part, int nparts, int len, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
  for (int w = 0; w < nparts; ++w) s += part[(int64_t)w * len + i];
  out[i] = s;
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
  for (int64_t m = (int64_t)blockIdx.x * 4 + slot; m < M; m += (int64_t)gridDim.x * 4) {
    const float g = gh[m * E + e];
    db += g;
#pragma unroll
    for (int f = 0; f < 16; ++f)
      if (f < F) acc[f] += g * feats[m * F + f];
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
#pragma unroll
    for (int mm = 0; mm < 4; ++mm)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t row = r0 + 16 * mm + 4 * g + j;
        if (row >= M) continue;
        const int64_t o = row * N + n;
        const float v = acc[mm][j] + bv;
        if constexpr (MODE == 0) static_cast<uint16_t*>(out)[o] = f2bf(v);
        if constexpr (MODE == 1) static_cast<uint16_t*>(out)[o] = f2bf(v > 0.f ? v : 0.f);
        if constexpr (MODE == 2) static_cast<float*>(out)[o] = res[o] + v;
        if constexpr (MODE == 3) static_cast<float*>(out)[o] = acc[mm][j];
        if constexpr (MODE == 4) {
          const uint16_t mk = mask[o];
          static_cast<uint16_t*>(out)[o] = ((mk & 0x8000u) == 0u && (mk & 0x7fffu) != 0u) ? f2bf(acc[mm][j]) : 0;
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
// attention
// ---------------------------------------------------------------------------
constexpr float kScale = 0.17677669529663688f;  // 1/sqrt(32)

// stage rows r0 .. r0+nr-1 of one head's 32 columns (column offset col) into LDS
__device__ __forceinline__ void stage_rows(uint16_t* dst, const uint16_t* base, int64_t stride, int col, int r0,
                                           int nr) {
  for (int i = threadIdx.x; i < nr * 4; i += blockDim.x) {
    const int r = i >> 2, c = i & 3;
    *reinterpret_cast<u32x4*>(dst + r * DH + 8 * c) =
        *reinterpret_cast<const u32x4*>(base + (int64_t)(r0 + r) * stride + col + 8 * c);
  }
}

// grid (P*NH, query blocks); lane = query; online softmax over 16-key groups
__global__ __launch_bounds__(512) void k_attn_fwd(const uint16_t* __restrict__ qkv, int T, uint16_t* __restrict__ o,
                                                  float* __restrict__ lse) {
  __shared__ __attribute__((aligned(16))) uint16_t ks[KC * DH];
  __shared__ __attribute__((aligned(16))) uint16_t vs[KC * DH];
  const int64_t p = blockIdx.x / NH;
  const int hd = blockIdx.x % NH;
  const uint16_t* base = qkv + p * (int64_t)T * QKV;
  const int qi = blockIdx.y * blockDim.x + threadIdx.x;
  const bool act = qi < T;
  float qf[DH], acc[DH];
  float mx = -INFINITY, l = 0.f;
#pragma unroll
  for (int d = 0; d < DH; ++d) acc[d] = 0.f;
  if (act) {
    load_row32(base + (int64_t)qi * QKV + DH * hd, qf);
#pragma unroll
    for (int d = 0; d < DH; ++d) qf[d] *= kScale;
  }
  for (int c0 = 0; c0 < T; c0 += KC) {
    const int nk = T - c0 < KC ? T - c0 : KC;
    __syncthreads();
    stage_rows(ks, base, QKV, E + DH * hd, c0, nk);
    stage_rows(vs, base, QKV, 2 * E + DH * hd, c0, nk);
    __syncthreads();
    if (!act) continue;
    for (int j0 = 0; j0 < nk; j0 += 16) {
      float sc[16];
      float bm = -INFINITY;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        sc[jj] = -INFINITY;
        if (j0 + jj < nk) {
          float kf[DH];
          load_row32(ks + (j0 + jj) * DH, kf);
          sc[jj] = dot32(qf, kf);
        }
        bm = fmaxf(bm, sc[jj]);
      }
      if (bm > mx) {
        const float cf = __expf(mx - bm);
        l *= cf;
#pragma unroll
        for (int d = 0; d < DH; ++d) acc[d] *= cf;
        mx = bm;
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        if (j0 + jj < nk) {
          const float pj = __expf(sc[jj] - mx);
          l += pj;
          float vf[DH];
          load_row32(vs + (j0 + jj) * DH, vf);
#pragma unroll
          for (int d = 0; d < DH; ++d) acc[d] += pj * vf[d];
        }
      }
    }
  }
  if (!act) return;
  store_row32(o + (p * T + qi) * (int64_t)E + DH * hd, acc, 1.f / l);
  lse[(p * NH + hd) * (int64_t)T + qi] = mx + logf(l);
}

// key and value gradients: lane = key; queries (q, do, lse, delta) staged per chunk
__global__ __launch_bounds__(512) void k_attn_bwd_kv(const uint16_t* __restrict__ qkv, const uint16_t* __restrict__ o,
                                                     const uint16_t* __restrict__ go, const float* __restrict__ lse,
                                                     int T, uint16_t* __restrict__ dqkv) {
  __shared__ __attribute__((aligned(16))) uint16_t qs[KC * DH];
  __shared__ __attribute__((aligned(16))) uint16_t dos[KC * DH];
  __shared__ float ls[KC], dl[KC];
  const int64_t p = blockIdx.x / NH;
  const int hd = blockIdx.x % NH;
  const uint16_t* base = qkv + p * (int64_t)T * QKV;
  const uint16_t* gob = go + p * (int64_t)T * E;
  const uint16_t* ob = o + p * (int64_t)T * E;
  const float* lb = lse + (p * NH + hd) * (int64_t)T;
  const int kj = blockIdx.y * blockDim.x + threadIdx.x;
  const bool act = kj < T;
  float kf[DH], vf[DH], dk[DH], dv[DH];
#pragma unroll
  for (int d = 0; d < DH; ++d) {
    dk[d] = 0.f;
    dv[d] = 0.f;
  }
  if (act) {
    load_row32(base + (int64_t)kj * QKV + E + DH * hd, kf);
    load_row32(base + (int64_t)kj * QKV + 2 * E + DH * hd, vf);
  }
  for (int c0 = 0; c0 < T; c0 += KC) {
    const int nq = T - c0 < KC ? T - c0 : KC;
    __syncthreads();
    stage_rows(qs, base, QKV, DH * hd, c0, nq);
    stage_rows(dos, gob, E, DH * hd, c0, nq);
    for (int r = threadIdx.x; r < nq; r += blockDim.x) {
      float a[DH], b[DH];
      load_row32(gob + (int64_t)(c0 + r) * E + DH * hd, a);
      load_row32(ob + (int64_t)(c0 + r) * E + DH * hd, b);
      dl[r] = dot32(a, b);
      ls[r] = lb[c0 + r];
    }
    __syncthreads();
    if (!act) continue;
    for (int r = 0; r < nq; ++r) {
      float qf[DH], df[DH];
      load_row32(qs + r * DH, qf);
      load_row32(dos + r * DH, df);
      const float pr = __expf(dot32(qf, kf) * kScale - ls[r]);
      const float ds = pr * (dot32(df, vf) - dl[r]);
#pragma unroll
      for (int d = 0; d < DH; ++d) {
        dv[d] += pr * df[d];
        dk[d] += ds * qf[d];
      }
    }
  }
  if (!act) return;
  uint16_t* dst = dqkv + (p * T + kj) * (int64_t)QKV;
  store_row32(dst + E + DH * hd, dk, kScale);
  store_row32(dst + 2 * E + DH * hd, dv, 1.f);
}

// query gradients: lane = query; keys and values staged per chunk
__global__ __launch_bounds__(512) void k_attn_bwd_q(const uint16_t* __restrict__ qkv, const uint16_t* __restrict__ o,
                                                    const uint16_t* __restrict__ go, const float* __restrict__ lse,
                                                    int T, uint16_t* __restrict__ dqkv) {
  __shared__ __attribute__((aligned(16))) uint16_t ks[KC * DH];
  __shared__ __attribute__((aligned(16))) uint16_t vs[KC * DH];
  const int64_t p = blockIdx.x / NH;
  const int hd = blockIdx.x % NH;
  const uint16_t* base = qkv + p * (int64_t)T * QKV;
  const int qi = blockIdx.y * blockDim.x + threadIdx.x;
  const bool act = qi < T;
  float qf[DH], df[DH], dq[DH];
  float L = 0.f, delta = 0.f;
#pragma unroll
  for (int d = 0; d < DH; ++d) dq[d] = 0.f;
  if (act) {
    load_row32(base + (int64_t)qi * QKV + DH * hd, qf);
    load_row32(go + (p * T + qi) * (int64_t)E + DH * hd, df);
    float of[DH];
    load_row32(o + (p * T + qi) * (int64_t)E + DH * hd, of);
    delta = dot32(df, of);
    L = lse[(p * NH + hd) * (int64_t)T + qi];
  }
  for (int c0 = 0; c0 < T; c0 += KC) {
    const int nk = T - c0 < KC ? T - c0 : KC;
    __syncthreads();
    stage_rows(ks, base, QKV, E + DH * hd, c0, nk);
    stage_rows(vs, base, QKV, 2 * E + DH * hd, c0, nk);
    __syncthreads();
    if (!act) continue;
    for (int j = 0; j < nk; ++j) {
      float kf[DH], vf[DH];
      load_row32(ks + j * DH, kf);
      load_row32(vs + j * DH, vf);
      const float pr = __expf(dot32(qf, kf) * kScale - L);
      const float ds = pr * (dot32(df, vf) - delta);
#pragma unroll
      for (int d = 0; d < DH; ++d) dq[d] += ds * kf[d];
    }
  }
  if (!act) return;
  store_row32(dqkv + (p * T + qi) * (int64_t)QKV + DH * hd, dq, kScale);
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
// query (or key) blocks of an attention launch: at most 512 lanes each
void attn_shape(int T, unsigned& nb, unsigned& threads) {
  nb = (unsigned)((T + 511) / 512);
  const int per = (T + (int)nb - 1) / (int)nb;
  threads = (unsigned)(64 * ((per + 63) / 64));
}
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
  hipLaunchKernelGGL(k_embed, dim3(nblk(P * T * E, 256)), dim3(256), 0, hs(stream), x, w, P, T, C, S, mean, inv_sd,
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
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(2 * E), 0, hs(stream), ws, parts, 2 * E, dgb);
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
  hipLaunchKernelGGL(k_reduce, dim3(nblk(len, 256)), dim3(256), 0, hs(stream), ws, parts, len, dwb);
  return st(hipGetLastError());
}

int whs_tf_attn_fwd(const uint16_t* qkv, int64_t P, int T, uint16_t* o, float* lse, void* stream) {
  if (!qkv || !o || !lse || P < 0 || T < 1 || T > MAXT) return -1;
  if (P == 0) return 0;
  unsigned nb, th;
  attn_shape(T, nb, th);
  hipLaunchKernelGGL(k_attn_fwd, dim3((unsigned)(P * NH), nb), dim3(th), 0, hs(stream), qkv, T, o, lse);
  return st(hipGetLastError());
}

int whs_tf_attn_bwd(const uint16_t* qkv, const uint16_t* o, const uint16_t* go, const float* lse, int64_t P,
                    int T, uint16_t* dqkv, void* stream) {
  if (!qkv || !o || !go || !lse || !dqkv || P < 0 || T < 1 || T > MAXT) return -1;
  if (P == 0) return 0;
  unsigned nb, th;
  attn_shape(T, nb, th);
  hipLaunchKernelGGL(k_attn_bwd_kv, dim3((unsigned)(P * NH), nb), dim3(th), 0, hs(stream), qkv, o, go, lse, T, dqkv);
  hipLaunchKernelGGL(k_attn_bwd_q, dim3((unsigned)(P * NH), nb), dim3(th), 0, hs(stream), qkv, o, go, lse, T, dqkv);
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
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, hs(stream), ws, parts, 3 * E + 1, dhp);
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
  hipLaunchKernelGGL(k_reduce, dim3(nblk(len, 256)), dim3(256), 0, hs(stream), ws, parts, len, dweb);
  return st(hipGetLastError());
}

int whs_tf_cast(const float* w, int N, int K, uint16_t* out, uint16_t* out_t, void* stream) {
  if (!w || !out || N < 1 || K < 1) return -1;
  hipLaunchKernelGGL(k_cast, dim3(nblk((int64_t)N * K, 256)), dim3(256), 0, hs(stream), w, N, K, out, out_t);
  return st(hipGetLastError());
}

}  // extern "C"

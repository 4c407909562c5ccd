// Kernels of the weight network g_theta (Sec. II-C, Sec. IV-B): a stack of
// "same" 1-D convolutions with kernel 9 over time, bfloat16 operands on the
// matrix cores (v_mfma_f32_16x16x32_bf16) with FP32 accumulation, plus the
// bounded weight head, the masked MSE gradient and the Adam update.
//
// Activations are (P, T, C) bfloat16, channels contiguous, so the im2col row
// of output time t is the contiguous window x[t-4 .. t+4][0..C).  Weights are
// (Cout, 9, Cin) bfloat16.  Channel counts are 8, 16 or 64.
//
// MFMA 16x16x32 operand layout (checked on the device): lane l holds row
// l%16 of A and column l%16 of B, with K entries 8*(l/16) .. 8*(l/16)+7; the
// accumulator lane l holds rows 4*(l/16) .. +3 of column l%16.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "whs_net.h"

namespace whsnet {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

constexpr int KT = 9;    // taps
constexpr int HALO = 4;  // zero padding on each side
constexpr int TM = 64;   // output time rows per tile

// float -> bfloat16 bits, round to nearest even (gfx950 converts in one instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// one bit per bfloat16 value of a 16-byte chunk (8 channels) of a ReLU output:
// set where the value is > 0, which for these values (never negative) is where
// its bits are not zero
__device__ __forceinline__ uint8_t relu_bits(u32x4 v) {
  uint32_t b = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b |= min(v[q] & 0xffffu, 1u) << (2 * q);
    b |= min(v[q] >> 16, 1u) << (2 * q + 1);
  }
  return (uint8_t)b;
}
// keep the bfloat16 values of a 16-byte chunk whose bit is set, zero the rest
__device__ __forceinline__ u32x4 apply_bits(u32x4 v, uint32_t m) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    v[q] &= ((m >> (2 * q)) & 1u ? 0x0000ffffu : 0u) | ((m >> (2 * q + 1)) & 1u ? 0xffff0000u : 0u);
  return v;
}

// ---------------------------------------------------------------------------
// Convolution as implicit GEMM: out[t][n] = sum_{tap,c} Wt[n][tap][c] in[t+tap-4][c]
// MODE 0: + bias, ReLU, bfloat16 out (P,T,NOUT)
// MODE 1: + bias, FP32 out of channel 0 only (P,T)            (last layer; the
//         launcher runs k_conv_last instead, which computes only that channel)
// MODE 2: no bias, out *= (mask > 0), bfloat16 out (P,T,NOUT) (input gradient)
// MODE 3: as MODE 2 with the mask as bits (byte (p T + t) NOUT/8 + o/8, bit o%8)
// MODE 0 with `bits` set also writes the ReLU bits of its output in that layout
// (bit set where the stored bfloat16 value is > 0: the MODE 2 predicate), so
// the input gradient reads 1 bit per channel instead of the activation.
// A tile is 64 time rows of one series; wave w computes output channels
// 16w..16w+15 for all 64 rows (4 accumulator tiles).  Each workgroup loads
// its weights into registers once and then walks tiles blockIdx.x,
// blockIdx.x + gridDim.x, ... (the grid is bounded by the launcher).
// ---------------------------------------------------------------------------
template <int CIN, int NOUT, int MODE>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wt,
                                              const float* __restrict__ bias, const void* __restrict__ maskv,
                                              uint8_t* __restrict__ bits, void* __restrict__ out, int T, int ntiles,
                                              int64_t total) {
  constexpr int KTOT = KT * CIN;
  constexpr int NS = (KTOT + 31) / 32;      // K steps of 32
  constexpr int ROWS = TM + 2 * HALO;       // input window rows
  constexpr int RS = CIN + 8;               // LDS row stride in bf16 (16-byte pad)
  __shared__ __attribute__((aligned(16))) uint16_t win[ROWS * RS];
  __shared__ __attribute__((aligned(16))) uint16_t otile[TM * (NOUT + 8)];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;   // K group of this lane
  const int r16 = lane & 15;

  // weights of this wave's 16 output channels, all K steps, in registers
  bf16x8 wb[NS];
  const int n = wave * 16 + r16;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = 32 * s + 8 * g;
    const int tap = k / CIN, c = k % CIN;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (tap < KT) v = *reinterpret_cast<const u32x4*>(wt + ((int64_t)n * KT + tap) * CIN + c);
    wb[s] = __builtin_bit_cast(bf16x8, v);
  }
  const float bv = (MODE != 2 && bias) ? bias[n] : 0.f;

  // input window of a tile: rows t0-4 .. t0+67 (zero outside 0..T-1) in 16-byte
  // chunks, PRE per lane (the launcher uses NTH lanes per group); with PF the
  // next tile's window is fetched into registers while the current one is
  // computed. Only the 64-in, 64-out layers gain from it: the 64-lane groups
  // would need 36 more registers, and the thin-input layers lose occupancy
  // for a window too small to matter.
  constexpr int NTH = NOUT == 64 ? 256 : 64;
  constexpr bool PF = CIN == 64 && NOUT == 64;
  constexpr int CH = CIN / 8;
  constexpr int PRE = (ROWS * CH + NTH - 1) / NTH;
  u32x4 pre[PF ? PRE : 1];
  auto fetch = [&](int64_t tx) {
    if constexpr (!PF) return;
    const int64_t pp = tx / ntiles;
    const int tt0 = (int)(tx - pp * ntiles) * TM;
    const uint16_t* ip = in + pp * (int64_t)T * CIN;
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int i = (int)threadIdx.x + q * NTH;
      pre[q] = u32x4{0u, 0u, 0u, 0u};
      if (i < ROWS * CH) {
        const int t = tt0 - HALO + i / CH;
        if (t >= 0 && t < T) pre[q] = *reinterpret_cast<const u32x4*>(ip + (int64_t)t * CIN + 8 * (i % CH));
      }
    }
  };
  if (PF && (int64_t)blockIdx.x < total) fetch(blockIdx.x);

  for (int64_t tix = blockIdx.x; tix < total; tix += gridDim.x) {
  const int64_t p = tix / ntiles;
  const int t0 = (int)(tix - p * ntiles) * TM;
  __syncthreads();  // the previous tile's window and output tile are no longer read
  if constexpr (PF) {
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
      const int i = (int)threadIdx.x + q * NTH;
      if (i < ROWS * CH) *reinterpret_cast<u32x4*>(win + (i / CH) * RS + 8 * (i % CH)) = pre[q];
    }
  } else {
    const uint16_t* inp = in + p * (int64_t)T * CIN;
    for (int i = threadIdx.x; i < ROWS * CH; i += blockDim.x) {
      const int t = t0 - HALO + i / CH;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (t >= 0 && t < T) v = *reinterpret_cast<const u32x4*>(inp + (int64_t)t * CIN + 8 * (i % CH));
      *reinterpret_cast<u32x4*>(win + (i / CH) * RS + 8 * (i % CH)) = v;
    }
  }
  __syncthreads();
  if (PF && tix + gridDim.x < total) fetch(tix + gridDim.x);

  f32x4 acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = 32 * s + 8 * g;
    const int tap = k / CIN, c = k % CIN;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (tap < KT) v = *reinterpret_cast<const u32x4*>(win + (16 * m + r16 + tap) * RS + c);
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, v), wb[s], acc[m], 0, 0, 0);
    }
  }

  // epilogue: lane holds rows 16m + 4g + j, column n
  if constexpr (MODE == 1) {
    if (n == 0) {
      float* o = static_cast<float*>(out) + p * (int64_t)T;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int t = t0 + 16 * m + 4 * g + j;
          if (t < T) o[t] = acc[m][j] + bv;
        }
    }
  } else {
    constexpr int OS = NOUT + 8;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = 16 * m + 4 * g + j;
        float v = acc[m][j] + bv;
        if (MODE == 0) v = v > 0.f ? v : 0.f;
        otile[row * OS + n] = f2bf(v);
      }
    __syncthreads();
    uint16_t* o = static_cast<uint16_t*>(out) + p * (int64_t)T * NOUT;
    const uint16_t* mk = MODE == 2 ? static_cast<const uint16_t*>(maskv) + p * (int64_t)T * NOUT : nullptr;
    constexpr int OCH = NOUT / 8;
    const uint8_t* mb = MODE == 3 ? static_cast<const uint8_t*>(maskv) + p * (int64_t)T * OCH : nullptr;
    uint8_t* ob = MODE == 0 && bits ? bits + p * (int64_t)T * OCH : nullptr;
    for (int i = threadIdx.x; i < TM * OCH; i += blockDim.x) {
      const int r = i / OCH, c8 = i % OCH;
      const int t = t0 + r;
      if (t >= T) continue;
      u32x4 v = *reinterpret_cast<const u32x4*>(otile + r * OS + 8 * c8);
      if (MODE == 2) {
        const u32x4 mv = *reinterpret_cast<const u32x4*>(mk + (int64_t)t * NOUT + 8 * c8);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t lo = (mv[q] & 0x7fffu) != 0u && !(mv[q] & 0x8000u) ? 0x0000ffffu : 0u;
          const uint32_t hi = ((mv[q] >> 16) & 0x7fffu) != 0u && !(mv[q] & 0x80000000u) ? 0xffff0000u : 0u;
          v[q] &= (lo | hi);
        }
      }
      if (MODE == 3) v = apply_bits(v, mb[(int64_t)t * OCH + c8]);
      *reinterpret_cast<u32x4*>(o + (int64_t)t * NOUT + 8 * c8) = v;
      if (MODE == 0 && ob) ob[(int64_t)t * OCH + c8] = relu_bits(v);
    }
  }
  }  // tiles
}

// ---------------------------------------------------------------------------
// The 64-in, 64-out layers (MODE 0: + bias, ReLU; MODE 3: input gradient,
// out kept where its ReLU bit is set) as out^T = W . window on
// v_mfma_f32_32x32x16_bf16.  The
// weights are the A operand, in registers (lane l: output channel l % 32 of a
// 32-channel half, K entries 8 (l / 32) .. +7 of each 16-wide K step); the
// input window is the B operand, read from LDS (lane l: time row l % 32, 8
// channels).  A wavefront computes 64 time rows x all 64 channels, so each
// 1 KB LDS read feeds two 32x32x16 products (both channel halves) and four
// independent accumulators are in flight per K step.  The accumulators of a
// lane hold 4 consecutive channels of one time row (accumulator j: channel
// 8 (j / 4) + 4 (l / 32) + j % 4 of its half, time l % 32), which leave as
// 8-byte stores.  Tile: 256 time rows of one series, 64 per wavefront.
//
// Pipelined over the tiles a workgroup walks (blockIdx.x, + gridDim.x, ...):
// the next tile's input window goes straight from HBM into the other of two
// LDS buffers (buffer-to-LDS loads; rows outside the series read as zero
// through the buffer range) while this tile is computed, and a tile's output
// (staged in LDS) is stored during the first K steps of the next tile, so its
// LDS reads and stores overlap the products, and the one wait per tile is for
// memory operations issued a whole tile earlier.  MODE 3 loads a tile's
// ReLU bits (8 B per row) with its window and applies them to the sums, as
// integer masks on the packed bfloat16 values (lane-wise selects of the
// floats made the compiler spill); MODE 0 with `bits` writes its output's
// ReLU bits as the tile is stored.
// LDS rows are 128 B with the 16-byte chunks of row r permuted by XOR with
// (r >> 1) & 7, so the 16 rows read by a quarter wavefront hit distinct banks.
// ---------------------------------------------------------------------------
constexpr int TR64 = 256;  // time rows per tile of the 64-to-64 layers

template <int MODE>
__global__ __launch_bounds__(256, 1) void k_conv64(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wt,
                                                   const float* __restrict__ bias, const void* __restrict__ maskv,
                                                   uint8_t* __restrict__ bits, uint16_t* __restrict__ out, int T,
                                                   int ntiles, int64_t total) {
  static_assert(MODE == 0 || MODE == 3, "forward layer or input gradient with ReLU bits");
  constexpr int C = 64;
  constexpr int ROWS = TR64 + 2 * HALO;   // input window rows (264)
  constexpr int WB = ROWS * 128;          // bytes of one window buffer
  constexpr int OS = C + 8;               // output tile row stride in bf16 (144 B)
  constexpr int NS = KT * C / 16;         // K steps of 16
  typedef __attribute__((ext_vector_type(16))) float f32x16;
  typedef __attribute__((ext_vector_type(2))) uint32_t u32x2;
  typedef __attribute__((address_space(3))) void* lptr;
  // two window buffers as separate objects, so the compiler can tell the reads
  // of one from the loads in flight into the other and waits for neither
  __shared__ __attribute__((aligned(1024))) unsigned char win0[WB];
  __shared__ __attribute__((aligned(1024))) unsigned char win1[WB];
  // MODE 3: the ReLU bits of a tile, 8 bytes per row, loaded with its window
  __shared__ __attribute__((aligned(256))) unsigned char bits0[MODE == 3 ? TR64 * 8 : 4];
  __shared__ __attribute__((aligned(256))) unsigned char bits1[MODE == 3 ? TR64 * 8 : 4];
  __shared__ __attribute__((aligned(16))) uint16_t otile[TR64 * OS];
  __shared__ float sbias[C];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int hi = lane >> 5, l32 = lane & 31;

  bf16x8 wa[2][NS];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int n = 32 * h + l32;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int k = 16 * s + 8 * hi;
      const int tap = k / C, c = k % C;
      wa[h][s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(wt + ((int64_t)n * KT + tap) * C + c));
    }
  }
  if (threadIdx.x < C) sbias[threadIdx.x] = (MODE == 0 && bias) ? bias[threadIdx.x] : 0.f;

  auto tile_of = [&](int64_t tix, int64_t& p, int& t0) {
    p = tix / ntiles;
    t0 = (int)(tix - p * ntiles) * TR64;
  };
  // rows [r0, r0 + nrows) of a series (row r0 + r -> LDS row r) into an LDS
  // buffer: load i covers LDS rows 8i .. 8i+7; lane L fills slot L & 7 of row
  // 8i + (L >> 3) with chunk (L & 7) ^ ((row >> 1) & 7)
  auto dma_rows = [&](const uint16_t* series, int r0, int nrows, unsigned char* dst) {
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(series), (short)0, T * 128, 0x00020000);
    for (int i = wave; i < nrows / 8; i += 4) {
      const int r = 8 * i + (lane >> 3);
      const int chunk = (lane & 7) ^ ((r >> 1) & 7);
      const uint32_t off = (uint32_t)((r0 + r) * 128 + chunk * 16);  // rows before 0 wrap out of range
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lptr)(dst + 1024 * i), 16, off, 0, 0, 0);
    }
  };
  auto fetch = [&](int64_t tix, unsigned char* dst, unsigned char* bdst) {
    int64_t p;
    int t0;
    tile_of(tix, p, t0);
    dma_rows(in + p * (int64_t)T * C, t0 - HALO, ROWS, dst);
    if constexpr (MODE == 3) {
      // 8 bytes per row, loaded as dwords (T * 8 is a whole number of them, so
      // the buffer range zeroes exactly the rows past the series)
      const auto rs = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<uint8_t*>(static_cast<const uint8_t*>(maskv) + p * (int64_t)T * 8), (short)0, T * 8, 0x00020000);
      for (int i = wave; i < TR64 * 8 / 256; i += 4)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lptr)(bdst + 256 * i), 4,
                                                 (uint32_t)(t0 * 8 + 256 * i + 4 * lane), 0, 0, 0);
    }
  };
  // chunk q (of TR64 * 8 / 256) of the output tile of tile tix -> HBM
  auto store_chunk = [&](int64_t tix, int q) {
    int64_t p;
    int t0;
    tile_of(tix, p, t0);
    const int i = (int)threadIdx.x + 256 * q;
    const int r = i >> 3, c8 = i & 7;
    const int t = t0 + r;
    if (t >= T) return;
    u32x4 v = *reinterpret_cast<const u32x4*>(otile + r * OS + 8 * c8);
    *reinterpret_cast<u32x4*>(out + (p * (int64_t)T + t) * C + 8 * c8) = v;
    if (MODE == 0 && bits) bits[(p * (int64_t)T + t) * 8 + c8] = relu_bits(v);
  };
  constexpr int NSTORE = TR64 * 8 / 256;  // output chunks per thread
  static_assert(NSTORE <= KT * C / 16, "the stores ride on the first K steps");
  // one tile from window buffer cur while the next tile's window loads into nxt
  int64_t prev = -1;
  auto step = [&](int64_t tix, const unsigned char* cur, unsigned char* nxt, const unsigned char* bcur,
                  unsigned char* bnxt) {
    int64_t p;
    int t0;
    tile_of(tix, p, t0);
    // this tile's window and the previous tile's stores have landed
    __builtin_amdgcn_s_waitcnt(0x0070);  // vmcnt(0) lgkmcnt(0)
    __syncthreads();
    if (tix + gridDim.x < total) fetch(tix + gridDim.x, nxt, bnxt);

    // MODE 0: the sums start from the bias of the accumulator's channel
    f32x16 acc[2][2];  // [row block][channel half]
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x16 a0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 b4 = MODE == 0 ? *reinterpret_cast<const f32x4*>(sbias + 32 * h + 8 * q + 4 * hi)
                                   : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; ++e) a0[4 * q + e] = b4[e];
      }
      acc[0][h] = a0;
      acc[1][h] = a0;
    }
    // B fragments of K step s (rows 32 apart share the chunk permutation: the
    // second block reads 4 KB further)
    auto read_b = [&](int s, u32x4 (&v)[2]) {
      const int k = 16 * s + 8 * hi;
      const int tap = k / C, c8 = (k % C) >> 3;
      const int row = 64 * wave + l32 + tap;
      const unsigned char* src = cur + row * 128 + ((c8 ^ ((row >> 1) & 7)) << 4);
      v[0] = *reinterpret_cast<const u32x4*>(src);
      v[1] = *reinterpret_cast<const u32x4*>(src + 4096);
    };
    // fragments two K steps ahead: the reads of step s+2 are issued before the
    // products of step s (three register sets, so no read overwrites operands
    // still in use)
    u32x4 vb[3][2];
    read_b(0, vb[0]);
    read_b(1, vb[1]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (s + 2 < NS) read_b(s + 2, vb[(s + 2) % 3]);
      // the previous tile's output leaves while the products run
      if (s < NSTORE && prev >= 0) store_chunk(prev, s);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc[m][h] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wa[h][s], __builtin_bit_cast(bf16x8, vb[s % 3][m]),
                                                             acc[m][h], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // every wave has read the previous output tile out of LDS (only LDS
    // operations are waited for: the stores and the next window stay in flight)
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int row = 64 * wave + 32 * m + l32;
      // MODE 3: this row's 64 bits (bit c: channel c kept)
      uint64_t rb = 0;
      if constexpr (MODE == 3) rb = *reinterpret_cast<const uint64_t*>(bcur + 8 * row);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c0 = 32 * h + 8 * q + 4 * hi;  // first of the 4 channels
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            v[e] = acc[m][h][4 * q + e];
            if (MODE == 0) v[e] = v[e] > 0.f ? v[e] : 0.f;
          }
          u32x2 pk = {(uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                      (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16)};
          if constexpr (MODE == 3) {
            // the 4 bits of channels c0 .. c0 + 3, each widened to 16
            const uint32_t nib = (uint32_t)(h ? (rb >> 32) : rb) >> (8 * q + 4 * hi);
            pk[0] &= (0u - (nib & 1u)) & 0xffffu | (0u - ((nib >> 1) & 1u)) << 16;
            pk[1] &= (0u - ((nib >> 2) & 1u)) & 0xffffu | (0u - ((nib >> 3) & 1u)) << 16;
          }
          *reinterpret_cast<u32x2*>(otile + row * OS + c0) = pk;
        }
    }
    prev = tix;
  };

  if ((int64_t)blockIdx.x < total) fetch(blockIdx.x, win0, bits0);
  for (int64_t tix = blockIdx.x; tix < total; tix += 2 * (int64_t)gridDim.x) {
    step(tix, win0, win1, bits0, bits1);
    if (tix + gridDim.x < total) step(tix + gridDim.x, win1, win0, bits1, bits0);
  }
  if (prev >= 0) {
    __builtin_amdgcn_s_waitcnt(0x0070);  // every wave has written the last output tile
    __syncthreads();
    for (int q = 0; q < NSTORE; ++q) store_chunk(prev, q);
  }
}

// ---------------------------------------------------------------------------
// Inference through the whole network in one kernel: h (P, T) FP32 from the
// (P, T, 8) input, the activations of the three hidden layers kept in LDS.
// A tile is TRI = 224 output days of one series; each hidden layer computes
// 256 rows (its halo of 4 days per later layer included; rows outside the
// series are set to zero, the next layer's padding):
//   input rows  i <-> day t0 - 16 + i   (DMA, 16 B per row, next tile's in flight)
//   layer 0 out i <-> day t0 - 12 + i   (buffer A)
//   layer 1 out i <-> day t0 -  8 + i   (buffer B)
//   layer 2 out i <-> day t0 -  4 + i   (buffer A again)
//   h           i <-> day t0 + i
// so output row i of every layer reads input rows i .. i + 8.  Layers 0-2 run
// on v_mfma_f32_32x32x16_bf16 as out^T = W . window (weights the A operand in
// registers: wavefront w holds 32 output channels, 32 (w >> 1) .. +31, of all
// three layers, 316 registers; it computes rows 128 (w & 1) .. +127, four
// 32-row products per K step).  The last layer is u = A2 . W3 with W3 the
// (64 channels x 9 taps) matrix of its one real output channel, one
// v_mfma_f32_16x16x32_bf16 per 16 rows and 32 channels, then
// h[i] = bias + sum_tap u[i + tap][tap].  Sums start from the bias; each
// layer's outputs are rounded to bfloat16 after the ReLU, as in the layer
// kernels.  Hidden-layer rows are 128 B with 16-byte chunks permuted by XOR
// with (row >> 1) & 7 (conflict-free fragment reads).
// ---------------------------------------------------------------------------
constexpr int TRI = 224;        // output days per tile of the fused inference kernel
constexpr int NRI = 256;        // rows each hidden layer computes per tile
constexpr int NINR = 512;       // input rows staged (two loads of 64 rows per wavefront; 264 are read)
constexpr int ARS = NRI + 8;    // rows of a hidden-layer buffer (the last 8 stay zero)

__global__ __launch_bounds__(256, 1) void k_net_infer(const uint16_t* __restrict__ in8,
                                                      const uint16_t* __restrict__ w0,
                                                      const uint16_t* __restrict__ w1,
                                                      const uint16_t* __restrict__ w2,
                                                      const uint16_t* __restrict__ w3,
                                                      const float* __restrict__ b0, const float* __restrict__ b1,
                                                      const float* __restrict__ b2, const float* __restrict__ b3,
                                                      float* __restrict__ hout, int T, int ntiles, int64_t total) {
  constexpr int C = 64;
  constexpr int NS = KT * C / 16;  // K steps of the 64-channel layers
  constexpr int NS0 = 5;           // K steps of layer 0 (9 taps x 8 channels, the tenth tap zero)
  typedef __attribute__((ext_vector_type(16))) float f32x16;
  typedef __attribute__((ext_vector_type(2))) uint32_t u32x2;
  typedef __attribute__((address_space(3))) void* lptr;
  __shared__ __attribute__((aligned(1024))) unsigned char inb0[NINR * 16];
  __shared__ __attribute__((aligned(1024))) unsigned char inb1[NINR * 16];
  __shared__ __attribute__((aligned(1024))) unsigned char bufA[ARS * 128];
  __shared__ __attribute__((aligned(1024))) unsigned char bufB[ARS * 128];
  __shared__ float sbias[3 * C];
  // layer 0's weights (64 x 9 x 8) and the last layer's channel-0 weights (9 x 64),
  // read from LDS when used (28 registers would not fit beside the others)
  __shared__ __attribute__((aligned(16))) uint16_t sw0[C * KT * 8];
  __shared__ __attribute__((aligned(16))) uint16_t sw3[KT * C];
  float* const ubuf = reinterpret_cast<float*>(bufB);  // u[row][16], after layer 2 has read B

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rg = wave & 1, chh = wave >> 1;
  const int hi = lane >> 5, l32 = lane & 31;
  const int n = 32 * chh + l32;  // output channel of this lane's A rows

  // the two 64-channel layers' weights stay in registers
  bf16x8 wz1[NS], wz2[NS];
  for (int i = threadIdx.x; i < C * KT * 8 / 8; i += blockDim.x)
    reinterpret_cast<u32x4*>(sw0)[i] = reinterpret_cast<const u32x4*>(w0)[i];
  for (int i = threadIdx.x; i < KT * C / 8; i += blockDim.x)
    reinterpret_cast<u32x4*>(sw3)[i] = reinterpret_cast<const u32x4*>(w3)[i];  // output channel 0's rows
  auto load_w0 = [&](bf16x8 (&wz0)[NS0]) {
#pragma unroll
    for (int s = 0; s < NS0; ++s) {
      const int tap = 2 * s + hi;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (tap < KT) v = *reinterpret_cast<const u32x4*>(sw0 + (n * KT + tap) * 8);
      wz0[s] = __builtin_bit_cast(bf16x8, v);
    }
  };
  auto load_w3 = [&](bf16x8 (&wz3)[2]) {
    // 16x16x32 B operand: column (tap) lane % 16, channels 32 ks + 8 (lane / 16) .. +7
    const int tap = lane & 15, cg = lane >> 4;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      u32x4 v = {0u, 0u, 0u, 0u};
      if (tap < KT) v = *reinterpret_cast<const u32x4*>(sw3 + tap * C + 32 * ks + 8 * cg);
      wz3[ks] = __builtin_bit_cast(bf16x8, v);
    }
  };
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int k = 16 * s + 8 * hi;
    const int tap = k / C, c = k % C;
    wz1[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(w1 + ((int64_t)n * KT + tap) * C + c));
    wz2[s] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(w2 + ((int64_t)n * KT + tap) * C + c));
  }
  if (threadIdx.x < C) {
    sbias[threadIdx.x] = b0[threadIdx.x];
    sbias[C + threadIdx.x] = b1[threadIdx.x];
    sbias[2 * C + threadIdx.x] = b2[threadIdx.x];
  }
  const float bias3 = b3[0];
  // rows NRI .. ARS-1 of both hidden-layer buffers are read (by rows no later
  // layer uses) but never written: zero them once
  for (int i = threadIdx.x; i < 8 * 128 / 4; i += blockDim.x) {
    reinterpret_cast<uint32_t*>(bufA + NRI * 128)[i] = 0u;
    reinterpret_cast<uint32_t*>(bufB + NRI * 128)[i] = 0u;
  }

  auto tile_of = [&](int64_t tix, int64_t& p, int& t0) {
    p = tix / ntiles;
    t0 = (int)(tix - p * ntiles) * TRI;
  };
  // input rows day t0-16 .. into an input buffer (zero outside the series);
  // issued by every wavefront whether or not there is a tile (tix >= total
  // loads zeros through an empty range), so the wait counts are the same on
  // every path and waiting for other loads never waits for these
  auto fetch = [&](int64_t tix, unsigned char* dst) {
    int64_t p;
    int t0;
    const bool any = tix < total;
    tile_of(any ? tix : 0, p, t0);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(in8 + p * (int64_t)T * 8), (short)0,
                                                      any ? T * 16 : 0, 0x00020000);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = 2 * wave + j;
      const uint32_t off = (uint32_t)((t0 - 16 + 64 * i + lane) * 16);  // days before 0 wrap out of range
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lptr)(dst + 1024 * i), 16, off, 0, 0, 0);
    }
  };
  auto lds_barrier = [&]() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS only, the loads in flight stay in flight
    __builtin_amdgcn_s_barrier();
  };
  // accumulators of a layer start from its bias (lane channels 32 chh + 8 q + 4 hi + e)
  auto init_acc = [&](int layer, f32x16 (&acc)[2]) {
    f32x16 a0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 b4 = *reinterpret_cast<const f32x4*>(sbias + layer * C + 32 * chh + 8 * q + 4 * hi);
#pragma unroll
      for (int e = 0; e < 4; ++e) a0[4 * q + e] = b4[e];
    }
    acc[0] = a0;
    acc[1] = a0;
  };
  // ReLU, zero rows outside the series, bfloat16, into a hidden-layer buffer;
  // row i of the layer is day t0 - off + i; acc holds rows r0 + 32 b + l32
  auto epilogue = [&](f32x16 (&acc)[2], int r0, unsigned char* dst, int t0, int off) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int row = r0 + 32 * b + l32;
      const int t = t0 - off + row;
      const bool in = t >= 0 && t < T;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float a = acc[b][4 * q + e];
          v[e] = (in && a > 0.f) ? a : 0.f;
        }
        const u32x2 pk = {(uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16),
                          (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16)};
        const int c8 = 4 * chh + q;
        *reinterpret_cast<u32x2*>(dst + row * 128 + ((c8 ^ ((row >> 1) & 7)) << 4) + 8 * hi) = pk;
      }
    }
  };
  // a 64-channel layer: src rows i + tap -> acc rows i, i = r0 + 32 b + l32 (two blocks)
  auto layer64 = [&](const bf16x8 (&wz)[NS], const unsigned char* src, int r0, f32x16 (&acc)[2]) {
    auto read_b = [&](int s, u32x4 (&v)[2]) {
      const int k = 16 * s + 8 * hi;
      const int tap = k / C, c8 = (k % C) >> 3;
      const int row = r0 + l32 + tap;
      // rows 32 apart share the chunk permutation
      const unsigned char* a = src + row * 128 + ((c8 ^ ((row >> 1) & 7)) << 4);
      v[0] = *reinterpret_cast<const u32x4*>(a);
      v[1] = *reinterpret_cast<const u32x4*>(a + 4096);
    };
    // fragments three K steps ahead (four register sets)
    u32x4 vb[4][2];
    read_b(0, vb[0]);
    read_b(1, vb[1]);
    read_b(2, vb[2]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (s + 3 < NS) read_b(s + 3, vb[(s + 3) & 3]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wz[s], __builtin_bit_cast(bf16x8, vb[s & 3][b]), acc[b], 0,
                                                         0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  float hprev = 0.f;
  int64_t prev = -1;
  // h of the previous tile; a buffer store on every path (dropped through the
  // range where there is no row to write), like the loads above
  auto store_h = [&]() {
    int64_t p;
    int t0;
    tile_of(prev >= 0 ? prev : 0, p, t0);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(hout + p * (int64_t)T, (short)0, prev >= 0 ? T * 4 : 0,
                                                      0x00020000);
    const int t = t0 + (int)threadIdx.x;
    const uint32_t off = ((int)threadIdx.x < TRI && t < T) ? (uint32_t)t * 4u : 0x80000000u;
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, hprev), rs, off, 0, 0);
  };
  auto step = [&](int64_t tix, const unsigned char* cur, unsigned char* nxt) {
    int64_t p;
    int t0;
    tile_of(tix, p, t0);
    __builtin_amdgcn_s_waitcnt(0x0070);  // this tile's input and the previous tile's h stores have landed
    __syncthreads();
    fetch(tix + gridDim.x, nxt);
    store_h();

    f32x16 acc[2];
    // layer 0: input rows i + tap (16 B rows, 8 channels; the tenth tap reads nothing)
    bf16x8 wz0[NS0];
    load_w0(wz0);
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const int r0 = 128 * rg + 64 * pass;
      init_acc(0, acc);
#pragma unroll
      for (int s = 0; s < NS0; ++s) {
        const int tap = 2 * s + hi;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int row = r0 + 32 * b + l32 + tap;
          u32x4 v = *reinterpret_cast<const u32x4*>(cur + 16 * (tap < KT ? row : 0));
          if (tap >= KT) v = u32x4{0u, 0u, 0u, 0u};
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wz0[s], __builtin_bit_cast(bf16x8, v), acc[b], 0, 0, 0);
        }
      }
      epilogue(acc, r0, bufA, t0, 12);
    }
    lds_barrier();
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const int r0 = 128 * rg + 64 * pass;
      init_acc(1, acc);
      layer64(wz1, bufA, r0, acc);
      epilogue(acc, r0, bufB, t0, 8);
    }
    lds_barrier();
    // layer 2 reads B and writes A (layer 0's output, which every wave has read)
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const int r0 = 128 * rg + 64 * pass;
      init_acc(2, acc);
      layer64(wz2, bufB, r0, acc);
      epilogue(acc, r0, bufA, t0, 4);
    }
    lds_barrier();  // every wave has written its rows of A and read B, which u overwrites
    // last layer: u[row][tap] = sum_c A2[row][c] W3[tap][c]; wave w: rows 64 w .. +63
    {
      const int r16 = lane & 15, cg = lane >> 4;
      bf16x8 wz3[2];
      load_w3(wz3);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = 64 * wave + 16 * b + r16;
        f32x4 u = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const int c8 = 4 * ks + cg;
          const u32x4 v = *reinterpret_cast<const u32x4*>(bufA + row * 128 + ((c8 ^ ((row >> 1) & 7)) << 4));
          u = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, v), wz3[ks], u, 0, 0, 0);
        }
        // accumulator: rows 4 cg .. +3 of the block, column (tap) r16
#pragma unroll
        for (int j = 0; j < 4; ++j) ubuf[(64 * wave + 16 * b + 4 * cg + j) * 16 + r16] = u[j];
      }
    }
    lds_barrier();
    if (threadIdx.x < TRI) {
      float h = bias3;
#pragma unroll
      for (int tap = 0; tap < KT; ++tap) h += ubuf[((int)threadIdx.x + tap) * 16 + tap];
      hprev = h;
    }
    prev = tix;
  };

  fetch(blockIdx.x, inb0);
  for (int64_t tix = blockIdx.x; tix < total; tix += 2 * (int64_t)gridDim.x) {
    step(tix, inb0, inb1);
    if (tix + gridDim.x < total) step(tix + gridDim.x, inb1, inb0);
  }
  __builtin_amdgcn_s_waitcnt(0x0070);  // the last (empty) input load before the kernel ends
  store_h();
}

// ---------------------------------------------------------------------------
// Last layer, one real output channel: h[t] = bias + sum_{tap,c} W[tap][c]
// in[t+tap-4][c] (64 input channels), FP32 out (P, T).  Vector arithmetic: a
// 64-row tile's input window sits in LDS, four lanes share an output row (16
// channels each, all nine taps) and add their sums with two lane swaps; the
// weights of channel 0 are read from LDS as wave-wide broadcasts.  Channels
// 1..15 of the padded weights are not read.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_conv_last(const uint16_t* __restrict__ in, const uint16_t* __restrict__ wt,
                                                   const float* __restrict__ bias, float* __restrict__ out, int T,
                                                   int ntiles, int64_t total) {
  constexpr int CIN = 64;
  constexpr int ROWS = TM + 2 * HALO;
  constexpr int RS = CIN + 8;  // LDS row stride in bf16 (16-byte pad)
  __shared__ __attribute__((aligned(16))) uint16_t win[ROWS * RS];
  __shared__ __attribute__((aligned(16))) uint16_t wl[KT * CIN];
  for (int i = threadIdx.x; i < KT * CIN; i += blockDim.x) wl[i] = wt[i];  // output channel 0: (9, 64)
  const float bv = bias ? bias[0] : 0.f;
  const int r = threadIdx.x >> 2, q = threadIdx.x & 3;  // output row of the tile, channel quarter
  for (int64_t tix = blockIdx.x; tix < total; tix += gridDim.x) {
    const int64_t p = tix / ntiles;
    const int t0 = (int)(tix - p * ntiles) * TM;
    const uint16_t* inp = in + p * (int64_t)T * CIN;
    __syncthreads();  // the weights are staged; the previous window is no longer read
    for (int i = threadIdx.x; i < ROWS * (CIN / 8); i += blockDim.x) {
      const int rr = i / (CIN / 8), c8 = i % (CIN / 8);
      const int t = t0 - HALO + rr;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (t >= 0 && t < T) v = *reinterpret_cast<const u32x4*>(inp + (int64_t)t * CIN + 8 * c8);
      *reinterpret_cast<u32x4*>(win + rr * RS + 8 * c8) = v;
    }
    __syncthreads();
    float acc = 0.f;
#pragma unroll
    for (int tap = 0; tap < KT; ++tap) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const u32x4 a = *reinterpret_cast<const u32x4*>(win + (r + tap) * RS + 16 * q + 8 * h);
        const u32x4 b = *reinterpret_cast<const u32x4*>(wl + tap * CIN + 16 * q + 8 * h);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          acc += bf2f((uint16_t)(a[k] & 0xffffu)) * bf2f((uint16_t)(b[k] & 0xffffu));
          acc += bf2f((uint16_t)(a[k] >> 16)) * bf2f((uint16_t)(b[k] >> 16));
        }
      }
    }
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    const int t = t0 + r;
    if (q == 0 && t < T) out[p * (int64_t)T + t] = acc + bv;
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: gW[n][tap][c] = sum_{p,t} gy[p,t,n] in[p,t+tap-4,c],
// gb[n] = sum gy[p,t,n].  GEMM with K = time, done as
//   gW[n][tap][c] = sum_u gy[u-tap+4][n] in[u][c]
// so the input operand (columns c, 32 consecutive u) is the same for all
// nine taps and the tap only shifts the gradient operand.  Each work item is
// 32 time rows of one series, staged in LDS transposed (channel-major, pairs
// of time rows per 4-byte store) so every operand fragment is a contiguous
// read: the input fragments directly, and each tap's gradient fragment is cut
// from a 16-element window with funnel shifts.  Workgroup w writes partial
// sums to part[w]; k_wgrad_reduce adds them in a fixed order (deterministic).
// ---------------------------------------------------------------------------
template <int CIN, int NOUT>
__global__ __launch_bounds__(256) void k_wgrad(const uint16_t* __restrict__ in, const uint16_t* __restrict__ gy,
                                               float* __restrict__ part, int64_t P, int T) {
  constexpr int NN = KT * CIN;               // GEMM N (tap, c)
  constexpr int CT = (CIN + 15) / 16;        // column tiles of 16 channels
  constexpr int NT = KT * CT;                // accumulator tiles per wave
  constexpr int TK = 32;                     // time rows per item
  constexpr int GR = TK + 2 * HALO;          // gradient rows per item
  // LDS row strides in bf16: 4 mod 8, so channel rows 8 apart fall 16 banks apart
  // (the staging stores of one instruction spread over all banks); fragments are
  // then read as 8-byte pieces
  constexpr int XS = TK + 12;
  constexpr int GS = GR + 4;
  constexpr int XROWS = CT * 16;             // channel rows of xT (zero rows pad CIN = 8)
  __shared__ __attribute__((aligned(16))) uint16_t xT[XROWS * XS];
  __shared__ __attribute__((aligned(16))) uint16_t gT[NOUT * GS];
  typedef __attribute__((ext_vector_type(2))) uint32_t u32x2;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int r16 = lane & 15;
  const int m = wave * 16 + r16;  // output channel of this lane's A row
  const int64_t chunks = (T + TK - 1) / TK;
  const int64_t items = P * chunks;

  f32x4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  if (CIN < XROWS) {
    for (int i = threadIdx.x; i < (XROWS - CIN) * XS; i += blockDim.x) xT[CIN * XS + i] = 0;
  }

  // A unit of the staging is a pair of rows x 8 channels (two 16-byte loads).
  // The next item's units are loaded into registers while this item's
  // products run, and stored to LDS (transposed) after the barrier.
  constexpr int NTH = NOUT == 64 ? 256 : 64;  // threads per workgroup (as launched)
  constexpr int XU = (TK / 2) * (CIN / 8), GU = (GR / 2) * (NOUT / 8);
  constexpr int UX = (XU + NTH - 1) / NTH, UG = (GU + NTH - 1) / NTH;  // units per thread
  u32x4 px0[UX], px1[UX], pg0[UG], pg1[UG];
  auto fetch_item = [&](int64_t it) {
#pragma unroll
    for (int k = 0; k < UX; ++k) px0[k] = px1[k] = u32x4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < UG; ++k) pg0[k] = pg1[k] = u32x4{0u, 0u, 0u, 0u};
    if (it >= items) return;
    const int64_t p = it / chunks;
    const int t0 = (int)(it - p * chunks) * TK;
    const uint16_t* ip = in + p * (int64_t)T * CIN;
    const uint16_t* gp = gy + p * (int64_t)T * NOUT;
#pragma unroll
    for (int k = 0; k < UX; ++k) {
      const int i = (int)threadIdx.x + NTH * k;
      if (i >= XU) break;
      const int up = i % (TK / 2), c0 = 8 * (i / (TK / 2));
      const int t = t0 + 2 * up;
      if (t < T) px0[k] = *reinterpret_cast<const u32x4*>(ip + (int64_t)t * CIN + c0);
      if (t + 1 < T) px1[k] = *reinterpret_cast<const u32x4*>(ip + (int64_t)(t + 1) * CIN + c0);
    }
#pragma unroll
    for (int k = 0; k < UG; ++k) {
      const int i = (int)threadIdx.x + NTH * k;
      if (i >= GU) break;
      const int rp = i % (GR / 2), n0 = 8 * (i / (GR / 2));
      const int t = t0 - HALO + 2 * rp;
      if (t >= 0 && t < T) pg0[k] = *reinterpret_cast<const u32x4*>(gp + (int64_t)t * NOUT + n0);
      if (t + 1 >= 0 && t + 1 < T) pg1[k] = *reinterpret_cast<const u32x4*>(gp + (int64_t)(t + 1) * NOUT + n0);
    }
  };
  fetch_item(blockIdx.x);

  for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
    __syncthreads();
    // the item's units into LDS: each stores 8 dwords, the (t, t+1) pair of one channel
#pragma unroll
    for (int k = 0; k < UX; ++k) {
      const int i = (int)threadIdx.x + NTH * k;
      if (i >= XU) break;
      const int up = i % (TK / 2), c0 = 8 * (i / (TK / 2));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<uint32_t*>(xT + (c0 + 2 * q) * XS + 2 * up) = (px0[k][q] & 0xffffu) | (px1[k][q] << 16);
        *reinterpret_cast<uint32_t*>(xT + (c0 + 2 * q + 1) * XS + 2 * up) =
            (px0[k][q] >> 16) | (px1[k][q] & 0xffff0000u);
      }
    }
#pragma unroll
    for (int k = 0; k < UG; ++k) {
      const int i = (int)threadIdx.x + NTH * k;
      if (i >= GU) break;
      const int rp = i % (GR / 2), n0 = 8 * (i / (GR / 2));
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<uint32_t*>(gT + (n0 + 2 * q) * GS + 2 * rp) = (pg0[k][q] & 0xffffu) | (pg1[k][q] << 16);
        *reinterpret_cast<uint32_t*>(gT + (n0 + 2 * q + 1) * GS + 2 * rp) =
            (pg0[k][q] >> 16) | (pg1[k][q] & 0xffff0000u);
      }
    }
    __syncthreads();
    fetch_item(it + gridDim.x);
    // gradient window of this lane: rows 8g .. 8g+15 of channel m (taps cut 8 of them)
    uint32_t W[8];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const u32x2 v = *reinterpret_cast<const u32x2*>(gT + m * GS + 8 * g + 4 * h);
      W[2 * h] = v[0];
      W[2 * h + 1] = v[1];
    }
    // input fragments: column c = 16 ct + r16, rows 8g .. 8g+7
    bf16x8 bx[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const uint16_t* src = xT + (16 * ct + r16) * XS + 8 * g;
      const u32x2 lo = *reinterpret_cast<const u32x2*>(src);
      const u32x2 hi = *reinterpret_cast<const u32x2*>(src + 4);
      const u32x4 v = {lo[0], lo[1], hi[0], hi[1]};
      bx[ct] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
    for (int tap = 0; tap < KT; ++tap) {
      // rows 8g + j - tap + 8 of the window, j = 0..7: elements e .. e+7 with e = 8 - tap
      const int e = 8 - tap;
      u32x4 av;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int lo = (e >> 1) + q;
        av[q] = (e & 1) ? __builtin_amdgcn_alignbit(W[lo + 1 < 8 ? lo + 1 : 7], W[lo], 16) : W[lo];
      }
      const bf16x8 a = __builtin_bit_cast(bf16x8, av);
      if (tap == HALO) {
#pragma unroll
        for (int q = 0; q < 4; ++q) bsum += bf2f((uint16_t)(av[q] & 0xffffu)) + bf2f((uint16_t)(av[q] >> 16));
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
        acc[tap * CT + ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bx[ct], acc[tap * CT + ct], 0, 0, 0);
    }
  }
  // partial sums: part[w][n][tap * CIN + c] (NOUT x NN), then the bias after them
  float* pw = part + (int64_t)blockIdx.x * (NOUT * NN + NOUT);
#pragma unroll
  for (int tap = 0; tap < KT; ++tap)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = wave * 16 + 4 * g + j;  // output channel
        const int c = 16 * ct + r16;
        if (c < CIN) pw[row * NN + tap * CIN + c] = acc[tap * CT + ct][j];
      }
  // bias: the four K groups of a channel hold partial sums
  bsum += __shfl_xor(bsum, 16);
  bsum += __shfl_xor(bsum, 32);
  if (g == 0) pw[NOUT * NN + m] = bsum;
}

// out[i] = sum_w part[w][i]: 64 outputs per workgroup, 16 lanes per output each
// summing every 16th partial, then the 16 sums added in a fixed order
__global__ __launch_bounds__(1024) void k_wgrad_reduce(const float* __restrict__ part, int nparts, int len,
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

// ---------------------------------------------------------------------------
// Backward of the last layer on its one real output channel (h = channel 0;
// the padded channels 1..15 carry zero gradient), vector arithmetic:
//   dx[t][c] = mask(t, c) * sum_tap W[0][tap][c] gh[t + 4 - tap]   (bf16 out)
//   grad[tap][c] = sum_t gh[t] x[t + tap - 4][c],  grad_bias = sum_t gh[t]
// with gh the stored bfloat16 dL/dh, FP32 sums, the mask the input's ReLU bits:
// the rounding points of the 16-channel calls, without their 15 zero channels.
// ---------------------------------------------------------------------------
constexpr int LASTW = KT * 64;        // weights of output channel 0
constexpr int LASTP = LASTW + 1;      // one partial: the weights' gradient, then the bias's
constexpr int LASTR = 256;            // days per tile

// gh of days t0 - 4 .. t0 + LASTR + 3 of series p into LDS (zero outside 0..T-1)
__device__ __forceinline__ void last_stage_gh(const uint16_t* __restrict__ gh, int64_t p, int T, int t0, float* sg) {
  for (int i = threadIdx.x; i < LASTR + 2 * HALO; i += blockDim.x) {
    const int s = t0 - HALO + i;
    sg[i] = (s >= 0 && s < T) ? bf2f(gh[p * (int64_t)T + s]) : 0.f;
  }
}

// workgroups walk tiles of 256 days of one series (blockIdx.x, + gridDim.x,
// ...) with the weights of their 8 channels in registers; thread (r, c8) takes
// days t0 + r + 32 k and channels 8 c8 .. +7: 16 bytes of dx per day
__global__ __launch_bounds__(256) void k_last_dgrad(const uint16_t* __restrict__ gh, const uint16_t* __restrict__ w,
                                                    const uint8_t* __restrict__ bits, uint16_t* __restrict__ dx,
                                                    int T, int ntiles, int64_t total) {
  __shared__ float sw[LASTW];
  __shared__ float sg[LASTR + 2 * HALO];
  for (int i = threadIdx.x; i < LASTW; i += blockDim.x) sw[i] = bf2f(w[i]);
  __syncthreads();
  const int c8 = threadIdx.x & 7, r = threadIdx.x >> 3;
  float wr[KT][8];
#pragma unroll
  for (int tap = 0; tap < KT; ++tap)
#pragma unroll
    for (int e = 0; e < 8; ++e) wr[tap][e] = sw[tap * 64 + 8 * c8 + e];
  for (int64_t tix = blockIdx.x; tix < total; tix += gridDim.x) {
  const int64_t p = tix / ntiles;
  const int t0 = (int)(tix - p * ntiles) * LASTR;
  __syncthreads();  // the previous tile's gh is no longer read
  last_stage_gh(gh, p, T, t0, sg);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < LASTR / 32; ++k) {
    const int i = r + 32 * k;  // day t0 + i
    const bool in = t0 + i < T;
    float acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = 0.f;
    // dx day t takes gh day t + 4 - tap, LDS entry i + 8 - tap
#pragma unroll
    for (int tap = 0; tap < KT; ++tap) {
      const float g = sg[i + 2 * HALO - tap];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] = __builtin_fmaf(wr[tap][e], g, acc[e]);
    }
    u32x4 v;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (uint32_t)f2bf(acc[2 * q]) | ((uint32_t)f2bf(acc[2 * q + 1]) << 16);
    const int64_t row = p * (int64_t)T + (in ? t0 + i : T - 1);
    v = apply_bits(v, bits[row * 8 + c8]);
    if (in) *reinterpret_cast<u32x4*>(dx + row * 64 + 8 * c8) = v;
  }
  }  // tiles
}

// workgroup b walks tiles b, b + parts, ...; thread (r, c8) adds days t0 + r +
// 32 k, channels 8 c8 .. +7; the sums are added over the wavefront by lane
// swaps and over the four wavefronts in LDS, in a fixed order
__global__ __launch_bounds__(256) void k_last_wgrad(const uint16_t* __restrict__ x, const uint16_t* __restrict__ gh,
                                                    float* __restrict__ part, int T, int ntiles, int64_t total) {
  __shared__ float red[4][LASTP];
  __shared__ float sg[LASTR + 2 * HALO];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c8 = threadIdx.x & 7, r = threadIdx.x >> 3;
  float acc[KT][8];
#pragma unroll
  for (int tap = 0; tap < KT; ++tap)
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[tap][e] = 0.f;
  float gb = 0.f;
  for (int64_t tix = blockIdx.x; tix < total; tix += gridDim.x) {
    const int64_t p = tix / ntiles;
    const int t0 = (int)(tix - p * ntiles) * LASTR;
    __syncthreads();  // the previous tile's gh is no longer read
    last_stage_gh(gh, p, T, t0, sg);
    __syncthreads();
    // all eight days' rows loaded first (days past the series read the last
    // day and count as zero)
    u32x4 xv[LASTR / 32];
#pragma unroll
    for (int k = 0; k < LASTR / 32; ++k) {
      const int t = t0 + r + 32 * k;
      xv[k] = *reinterpret_cast<const u32x4*>(x + (p * (int64_t)T + (t < T ? t : T - 1)) * 64 + 8 * c8);
    }
#pragma unroll
    for (int k = 0; k < LASTR / 32; ++k) {
      const int i = r + 32 * k;  // x day t0 + i
      const bool in = t0 + i < T;
      float xf[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        xf[2 * q] = in ? bf2f((uint16_t)(xv[k][q] & 0xffffu)) : 0.f;
        xf[2 * q + 1] = in ? bf2f((uint16_t)(xv[k][q] >> 16)) : 0.f;
      }
      // x day t enters grad[tap] with gh day t + 4 - tap, LDS entry i + 8 - tap
#pragma unroll
      for (int tap = 0; tap < KT; ++tap) {
        const float g = sg[i + 2 * HALO - tap];
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[tap][e] = __builtin_fmaf(g, xf[e], acc[tap][e]);
      }
      if (c8 == 0 && in) gb += sg[i + HALO];
    }
  }
  // over the eight days of the wavefront (lanes 8 apart share c8)
#pragma unroll
  for (int off = 8; off < 64; off <<= 1) {
#pragma unroll
    for (int tap = 0; tap < KT; ++tap)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[tap][e] += __shfl_xor(acc[tap][e], off);
    gb += __shfl_xor(gb, off);
  }
  if (lane < 8) {
#pragma unroll
    for (int tap = 0; tap < KT; ++tap)
#pragma unroll
      for (int e = 0; e < 8; ++e) red[wave][tap * 64 + 8 * c8 + e] = acc[tap][e];
    if (lane == 0) red[wave][LASTW] = gb;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < LASTP; j += blockDim.x)
    part[(int64_t)blockIdx.x * LASTP + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
}

// grad (16, 9, 64) + 16 of the padded layer: channel 0's rows and bias from the
// partials, 64 of them per workgroup, 16 lanes per output each adding every
// 16th partial, then the 16 sums in a fixed order (as k_wgrad_reduce); the
// workgroups past those zero every other entry
constexpr int LASTRB = (LASTP + 63) / 64;  // reducing workgroups

__global__ __launch_bounds__(1024) void k_last_reduce(const float* __restrict__ part, int nparts,
                                                      float* __restrict__ grad) {
  constexpr int NW = 16 * LASTW;  // padded weights, then 16 biases
  if ((int)blockIdx.x >= LASTRB) {
    const int j = ((int)blockIdx.x - LASTRB) * 1024 + (int)threadIdx.x;
    if (j < NW + 16 && j >= LASTW && j != NW) grad[j] = 0.f;
    return;
  }
  __shared__ float red[16][64];
  const int col = blockIdx.x * 64 + (threadIdx.x & 63), sl = threadIdx.x >> 6;
  float s = 0.f;
  if (col < LASTP)
    for (int w = sl; w < nparts; w += 16) s += part[(int64_t)w * LASTP + col];
  red[sl][threadIdx.x & 63] = s;
  __syncthreads();
  if (sl == 0 && col < LASTP) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += red[k][threadIdx.x];
    grad[col < LASTW ? col : NW] = t;
  }
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------

// Network input (P, T, 8): x standardised where observed (0 elsewhere), w,
// then four time features per day (feat: (T, 4)), then two zero channels.
__global__ void k_net_input(const float* __restrict__ x, const uint8_t* __restrict__ w, int64_t P, int T, int S,
                            float mean, float inv_sd, const float* __restrict__ feat, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * T) return;
  const int64_t p = i / T;
  const int t = (int)(i - p * T);
  const int64_t b = p / S;
  const int s = (int)(p - b * S);
  const int64_t off = (b * T + t) * S + s;
  const bool obs = w[off] != 0;
  const float xs = obs ? (x[off] - mean) * inv_sd : 0.f;
  u32x4 v;
  v[0] = (uint32_t)f2bf(xs) | ((uint32_t)f2bf(obs ? 1.f : 0.f) << 16);
  v[1] = (uint32_t)f2bf(feat[t * 4 + 0]) | ((uint32_t)f2bf(feat[t * 4 + 1]) << 16);
  v[2] = (uint32_t)f2bf(feat[t * 4 + 2]) | ((uint32_t)f2bf(feat[t * 4 + 3]) << 16);
  v[3] = 0u;
  *reinterpret_cast<u32x4*>(out + i * 8) = v;
}

__device__ __forceinline__ float sigm(float h) { return 1.f / (1.f + __expf(-h)); }

// Bounded head: log10 lambda = lo + (hi-lo) sigmoid(h) per day; difference row
// k takes day k + d/2; written in the interleaved per-difference layout.
__global__ void k_head_fwd(const float* __restrict__ h, int64_t P, int T, int S, int d, float lo, float hi,
                           float* __restrict__ lam) {
  const int Td = T - d;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * Td) return;
  const int64_t p = i / Td;
  const int k = (int)(i - p * Td);
  const float hv = h[p * (int64_t)T + k + d / 2];
  const float e = lo + (hi - lo) * sigm(hv);
  const int64_t b = p / S;
  const int s = (int)(p - b * S);
  lam[(b * Td + k) * S + s] = exp10f(e);
}

// dL/dh from dL/dlambda (interleaved) into channel 0 of a (P, T, 16) bfloat16
// gradient (channels 1..15 zero), the padded output of the last layer.
template <int CH>
__global__ void k_head_bwd(const float* __restrict__ h, const float* __restrict__ glam, int64_t P, int T, int S,
                           int d, float lo, float hi, uint16_t* __restrict__ gh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * T) return;
  const int64_t p = i / T;
  const int t = (int)(i - p * T);
  const int k = t - d / 2;
  float g = 0.f;
  if (k >= 0 && k < T - d) {
    const int64_t b = p / S;
    const int s = (int)(p - b * S);
    const float hv = h[i];
    const float sg = sigm(hv);
    const float lamv = exp10f(lo + (hi - lo) * sg);
    g = glam[(b * (T - d) + k) * S + s] * lamv * 2.302585093f * (hi - lo) * sg * (1.f - sg);
  }
  if constexpr (CH == 1) {
    gh[i] = f2bf(g);
  } else {
    u32x4 z = {0u, 0u, 0u, 0u};
    u32x4 v = z;
    v[0] = (uint32_t)f2bf(g);
    *reinterpret_cast<u32x4*>(gh + i * 16) = v;
    *reinterpret_cast<u32x4*>(gh + i * 16 + 8) = z;
  }
}

// g = 2 (z - x) / n at held-out points (0 elsewhere), and sum of squares into *loss.
// Grid-stride over the elements; the squares are summed in FP64 per lane, then
// per workgroup, with one atomic per workgroup (a bounded grid keeps them few).
constexpr int kMseBlocks = 1024;
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ z, const float* __restrict__ x,
                                             const uint8_t* __restrict__ hold, int64_t n_elem, float inv_n,
                                             float* __restrict__ g, double* __restrict__ loss) {
  __shared__ double red[4];
  double sq = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_elem; i += stride) {
    const bool h = hold[i] != 0;
    const float r = h ? z[i] - x[i] : 0.f;
    g[i] = 2.f * r * inv_n;
    sq += (double)r * (double)r;
  }
  for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
  __syncthreads();
  if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] + red[1] + red[2] + red[3]);
}

// Homoscedastic head: every series gets lambda = 10^(lo + (hi - lo) sigmoid(theta)).
__global__ void k_scalar_head_fwd(const float* __restrict__ theta, int64_t P, float lo, float hi,
                                  float* __restrict__ lam) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const double s = 1.0 / (1.0 + exp(-(double)theta[0]));
  lam[i] = (float)exp10((double)lo + ((double)hi - (double)lo) * s);
}

// dL/dtheta = (sum_p glam[p]) dlambda/dtheta; one workgroup, FP64, fixed order.
__global__ __launch_bounds__(1024) void k_scalar_head_bwd(const float* __restrict__ theta,
                                                          const float* __restrict__ glam, int64_t P, float lo,
                                                          float hi, float* __restrict__ grad) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < P; i += blockDim.x) s += (double)glam[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) tot += red[wv];
    const double sg = 1.0 / (1.0 + exp(-(double)theta[0]));
    const double lam = exp10((double)lo + ((double)hi - (double)lo) * sg);
    grad[0] = (float)(tot * lam * 2.302585092994046 * ((double)hi - (double)lo) * sg * (1.0 - sg));
  }
}

// Adam with bias correction on FP32 master weights (n_out, 9, n_in) of which
// the first n_real output rows are trained; writes the bfloat16 forward copy
// (n_out_pad, 9, n_in) and the transposed, tap-flipped copy used by the
// input gradient (n_in, 9, n_out_pad).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_pack_weights(const float* __restrict__ w, int n_real, int n_out_pad, int n_in,
                               uint16_t* __restrict__ wf, uint16_t* __restrict__ wd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = n_out_pad * KT * n_in;
  if (i >= total) return;
  const int o = i / (KT * n_in);
  const int rem = i - o * KT * n_in;
  const int tap = rem / n_in, c = rem % n_in;
  const uint16_t b = o < n_real ? f2bf(w[(o * KT + tap) * n_in + c]) : (uint16_t)0;
  wf[i] = b;
  if (wd) wd[(c * KT + (KT - 1 - tap)) * n_out_pad + o] = b;
}

}  // namespace whsnet

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

using namespace whsnet;

namespace {
int st(hipError_t e) { return e == hipSuccess ? 0 : -3; }
inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
constexpr int64_t kConvBlocks = 4096;
// one resident workgroup of the 64-to-64 kernel per compute unit
int64_t conv64_blocks() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || n < 1)
    n = 256;
  return n;
}
bool okc(int c) { return c == 8 || c == 16 || c == 64; }
}  // namespace

extern "C" {

int whs_net_conv_fwd(const uint16_t* in, int cin, const uint16_t* w, const float* bias, int cout, int mode,
                     const void* mask, void* out, uint8_t* bits, int64_t P, int T, void* stream) {
  if (!in || !w || !out || P < 0 || T < 1 || !okc(cin) || (cout != 16 && cout != 64)) return -1;
  if (mode < 0 || mode > 3 || (mode >= 2 && !mask) || (bits && mode != 0)) return -1;
  // one series' 64-channel rows within a 32-bit buffer range (pipelined kernels)
  if ((int64_t)T * 128 >= ((int64_t)1 << 31)) return -2;
  if (P == 0) return 0;
  const int ntiles = (int)nblk(T, TM);
  const int64_t total = P * ntiles;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // enough workgroups to fill the chip several times over; each walks tiles
  dim3 grid((unsigned)(total < kConvBlocks ? total : kConvBlocks));
  dim3 block(cout == 64 ? 256 : 64);
#define WHS_CONV(CI, CO, MO) \
  hipLaunchKernelGGL((k_conv<CI, CO, MO>), grid, block, 0, s, in, w, bias, mask, bits, out, T, ntiles, total)
  // the 64-to-64 layers: 256-row tiles, one persistent workgroup per CU
  const int nt64 = (int)nblk(T, TR64);
  const int64_t tot64 = P * nt64;
  const int64_t nb64 = conv64_blocks();
  const dim3 grid64((unsigned)(tot64 < nb64 ? tot64 : nb64));
  if (cin == 8 && cout == 64 && mode == 0) WHS_CONV(8, 64, 0);
  else if (cin == 64 && cout == 64 && mode == 0)
    hipLaunchKernelGGL((k_conv64<0>), grid64, dim3(256), 0, s, in, w, bias, nullptr, bits,
                       static_cast<uint16_t*>(out), T, nt64, tot64);
  else if (cin == 64 && cout == 16 && mode == 1) {
    // one real output channel: the vector kernel, 256 lanes per workgroup
    hipLaunchKernelGGL(k_conv_last, grid, dim3(256), 0, s, in, w, bias, static_cast<float*>(out), T, ntiles, total);
  }
  else if (cin == 64 && cout == 64 && mode == 2) WHS_CONV(64, 64, 2);
  else if (cin == 16 && cout == 64 && mode == 2) WHS_CONV(16, 64, 2);
  else if (cin == 64 && cout == 64 && mode == 3)
    hipLaunchKernelGGL((k_conv64<3>), grid64, dim3(256), 0, s, in, w, bias, mask, nullptr,
                       static_cast<uint16_t*>(out), T, nt64, tot64);
  else if (cin == 16 && cout == 64 && mode == 3) WHS_CONV(16, 64, 3);
  else return -2;
#undef WHS_CONV
  return st(hipGetLastError());
}

int whs_net_infer(const uint16_t* in8, const uint16_t* w0, const uint16_t* w1, const uint16_t* w2,
                  const uint16_t* w3, const float* b0, const float* b1, const float* b2, const float* b3, float* h,
                  int64_t P, int T, void* stream) {
  if (!in8 || !w0 || !w1 || !w2 || !w3 || !b0 || !b1 || !b2 || !b3 || !h || P < 0 || T < 1) return -1;
  if ((int64_t)T * 16 >= ((int64_t)1 << 31)) return -2;  // one series' input within a 32-bit buffer range
  if (P == 0) return 0;
  const int nt = (int)nblk(T, TRI);
  const int64_t total = P * nt;
  const int64_t nb = conv64_blocks();
  hipLaunchKernelGGL(k_net_infer, dim3((unsigned)(total < nb ? total : nb)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), in8, w0, w1, w2, w3, b0, b1, b2, b3, h, T, nt, total);
  return st(hipGetLastError());
}

size_t whs_net_wgrad_workspace_bytes(int cin, int cout, int parts) {
  return (size_t)parts * ((size_t)cout * KT * cin + cout) * sizeof(float);
}

int whs_net_conv_wgrad(const uint16_t* in, int cin, const uint16_t* gy, int cout, float* grad, float* ws,
                       size_t ws_bytes, int parts, int64_t P, int T, void* stream) {
  if (!in || !gy || !grad || !ws || P < 1 || T < 1 || parts < 1 || !okc(cin) ||
      (cout != 16 && cout != 64))
    return -1;
  if (ws_bytes < whs_net_wgrad_workspace_bytes(cin, cout, parts)) return -4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  dim3 block(cout == 64 ? 256 : 64);
  if (cin == 8 && cout == 64) hipLaunchKernelGGL((k_wgrad<8, 64>), dim3(parts), block, 0, s, in, gy, ws, P, T);
  else if (cin == 64 && cout == 64) hipLaunchKernelGGL((k_wgrad<64, 64>), dim3(parts), block, 0, s, in, gy, ws, P, T);
  else if (cin == 64 && cout == 16) hipLaunchKernelGGL((k_wgrad<64, 16>), dim3(parts), block, 0, s, in, gy, ws, P, T);
  else return -2;
  const int len = cout * KT * cin + cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk(len, 64)), dim3(1024), 0, s, ws, parts, len, grad);
  return st(hipGetLastError());
}

int whs_net_input(const float* x, const uint8_t* w, int64_t P, int T, int S, float mean, float inv_sd,
                  const float* feat, uint16_t* out, void* stream) {
  if (!x || !w || !feat || !out || P < 0 || T < 1 || S < 1) return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_net_input, dim3(nblk(P * T, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), x, w, P,
                     T, S, mean, inv_sd, feat, out);
  return st(hipGetLastError());
}

int whs_net_head_fwd(const float* h, int64_t P, int T, int S, int d, float lo, float hi, float* lam, void* stream) {
  if (!h || !lam || P < 0 || T <= d || d < 1 || S < 1) return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_head_fwd, dim3(nblk(P * (T - d), 256)), dim3(256), 0, static_cast<hipStream_t>(stream), h,
                     P, T, S, d, lo, hi, lam);
  return st(hipGetLastError());
}

int whs_net_head_bwd(const float* h, const float* glam, int64_t P, int T, int S, int d, float lo, float hi,
                     uint16_t* gh16, void* stream) {
  if (!h || !glam || !gh16 || P < 0 || T <= d || d < 1 || S < 1) return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_head_bwd<16>, dim3(nblk(P * T, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), h, glam,
                     P, T, S, d, lo, hi, gh16);
  return st(hipGetLastError());
}

int whs_net_head_bwd1(const float* h, const float* glam, int64_t P, int T, int S, int d, float lo, float hi,
                      uint16_t* gh, void* stream) {
  if (!h || !glam || !gh || P < 0 || T <= d || d < 1 || S < 1) return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_head_bwd<1>, dim3(nblk(P * T, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), h, glam,
                     P, T, S, d, lo, hi, gh);
  return st(hipGetLastError());
}

size_t whs_net_last_bwd_workspace_bytes(int parts) { return parts > 0 ? (size_t)parts * LASTP * sizeof(float) : 0; }

int whs_net_last_bwd(const uint16_t* x, const uint16_t* gh, const uint16_t* w, const uint8_t* bits, uint16_t* dx,
                     float* grad, float* ws, size_t ws_bytes, int parts, int64_t P, int T, void* stream) {
  if (!x || !gh || !w || !bits || !dx || !grad || !ws || P < 1 || T < 1 || parts < 1) return -1;
  if (ws_bytes < whs_net_last_bwd_workspace_bytes(parts)) return -4;
  const int nt = (int)nblk(T, LASTR);
  const int64_t total = P * nt;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_last_wgrad, dim3((unsigned)parts), dim3(256), 0, s, x, gh, ws, T, nt, total);
  hipLaunchKernelGGL(k_last_reduce, dim3(LASTRB + nblk(16 * LASTW + 16, 1024)), dim3(1024), 0, s, ws, parts, grad);
  hipLaunchKernelGGL(k_last_dgrad, dim3((unsigned)(total < kConvBlocks ? total : kConvBlocks)), dim3(256), 0, s, gh, w,
                     bits, dx, T, nt, total);
  return st(hipGetLastError());
}

int whs_net_scalar_head_fwd(const float* theta, int64_t P, float lo, float hi, float* lam, void* stream) {
  if (!theta || !lam || P < 0 || !(hi > lo)) return -1;
  if (P == 0) return 0;
  hipLaunchKernelGGL(k_scalar_head_fwd, dim3(nblk(P, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), theta,
                     P, lo, hi, lam);
  return st(hipGetLastError());
}

int whs_net_scalar_head_bwd(const float* theta, const float* glam, int64_t P, float lo, float hi,
                            float* grad_theta, void* stream) {
  if (!theta || !glam || !grad_theta || P < 1 || !(hi > lo)) return -1;
  hipLaunchKernelGGL(k_scalar_head_bwd, dim3(1), dim3(1024), 0, static_cast<hipStream_t>(stream), theta, glam, P,
                     lo, hi, grad_theta);
  return st(hipGetLastError());
}

int whs_net_mse(const float* z, const float* x, const uint8_t* hold, int64_t n_elem, float inv_n, float* g,
                double* loss, void* stream) {
  if (!z || !x || !hold || !g || n_elem < 0) return -1;
  if (n_elem == 0) return 0;
  const int64_t blocks = nblk(n_elem, 256) < kMseBlocks ? nblk(n_elem, 256) : kMseBlocks;
  hipLaunchKernelGGL(k_mse, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream), z, x, hold,
                     n_elem, inv_n, g, loss);
  return st(hipGetLastError());
}

int whs_net_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 int step, void* stream) {
  if (!p || !g || !m || !v || n < 0 || step < 1) return -1;
  if (n == 0) return 0;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), p, g, m, v, n, lr,
                     b1, b2, eps, c1, c2);
  return st(hipGetLastError());
}

int whs_net_pack_weights(const float* w, int n_real, int n_out_pad, int n_in, uint16_t* wf, uint16_t* wd,
                         void* stream) {
  if (!w || !wf || n_real < 1 || n_out_pad < n_real || n_in < 1) return -1;
  const int total = n_out_pad * KT * n_in;
  hipLaunchKernelGGL(k_pack_weights, dim3(nblk(total, 256)), dim3(256), 0, static_cast<hipStream_t>(stream), w,
                     n_real, n_out_pad, n_in, wf, wd);
  return st(hipGetLastError());
}

}  // extern "C"

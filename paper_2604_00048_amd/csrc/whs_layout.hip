// Layout changes between series-contiguous arrays (P, L) and the interleaved
// time-major layout (ceil(P/64), L, 64) the throughput kernels read: element
// (p, j) sits at p*L + j in one and at ((p/64)*L + j)*64 + p%64 in the other.
// A workgroup moves one tile through LDS so both sides are read and written in
// whole rows.  Interleaving zero-fills the slots of the last block that hold no
// series.  Elements of 1, 4 and 8 bytes take wide accesses where the pointers
// and row lengths allow them; one element per access otherwise (an interleaved
// copy not 16-byte aligned, byte rows whose start or length is not a multiple
// of 4).
#include <hip/hip_runtime.h>

#include "whs_kernels.h"

namespace whs {
namespace {

template <typename E>
__global__ __launch_bounds__(256) void k_interleave(const E* __restrict__ src, E* __restrict__ dst, int64_t P,
                                                    int64_t L, int to_interleaved) {
  __shared__ E tile[64][65];
  const int64_t b = blockIdx.x;
  const int64_t j0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  if (to_interleaved) {
    for (int r = ty; r < 64; r += 4) {
      const int64_t p = b * 64 + r, j = j0 + tx;
      tile[r][tx] = (p < P && j < L) ? src[p * L + j] : E(0);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
      const int64_t j = j0 + r;
      if (j < L) dst[(b * L + j) * 64 + tx] = tile[tx][r];
    }
  } else {
    for (int r = ty; r < 64; r += 4) {
      const int64_t j = j0 + r;
      tile[tx][r] = j < L ? src[(b * L + j) * 64 + tx] : E(0);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
      const int64_t p = b * 64 + r, j = j0 + tx;
      if (p < P && j < L) dst[p * L + j] = tile[r][tx];
    }
  }
}

// Workgroups go out round-robin over the 8 XCDs.  The k-th workgroup of XCD x
// takes tile x * (grid / 8) + k of a numbering with the step tile fastest, so
// the tiles that share a series block's rows run at about the same time on one
// XCD, whose L2 then joins the halves of the cache lines they split.  The grid
// is a multiple of 8; a workgroup past the last tile returns at once.
__device__ inline bool xcd_tile(int64_t n_step_tiles, int64_t n_tiles, int64_t& b, int64_t& by) {
  const int64_t id = blockIdx.x, per = gridDim.x / 8;
  const int64_t u = (id % 8) * per + id / 8;
  if (u >= n_tiles) return false;
  b = u / n_step_tiles;
  by = u % n_step_tiles;
  return true;
}

// 4- and 8-byte elements, a tile of 64 series x TJ steps (a 256-byte piece of
// each series row).  The series-contiguous side is read or written V elements per
// access (its rows start V-aligned: L % V == 0), the interleaved side 16 bytes per
// access.
template <typename E, int V>
__global__ __launch_bounds__(256) void k_interleave_wide(const E* __restrict__ src, E* __restrict__ dst, int64_t P,
                                                         int64_t L, int to_interleaved, int64_t ny) {
  constexpr int TJ = 256 / (int)sizeof(E);  // steps per tile
  constexpr int IV = 16 / (int)sizeof(E);   // elements per access on the interleaved side
  constexpr int kLanes = TJ / V;            // lanes per series row on the contiguous side
  constexpr int kRows = 256 / kLanes;       // series rows per pass there
  constexpr int kILanes = 64 / IV;          // lanes per step row on the interleaved side
  constexpr int kIRows = 256 / kILanes;     // step rows per pass there
  constexpr int kPitch = TJ + 1;
  using vec = E __attribute__((ext_vector_type(V)));
  using ivec = E __attribute__((ext_vector_type(IV)));
  __shared__ E tile[64 * kPitch];  // [series][step]
  int64_t b, by;
  if (!xcd_tile(ny, ny * ((P + 63) / 64), b, by)) return;
  const int64_t j0 = by * TJ;
  const int t = threadIdx.x;
  const int c = t % kLanes, r0 = t / kLanes;   // contiguous side: V-element column, first series
  const int q = t % kILanes, jr = t / kILanes;  // interleaved side: series group, first step
  if (to_interleaved) {
#pragma unroll
    for (int i = 0; i < 64 / kRows; ++i) {
      const int r = r0 + kRows * i;
      const int64_t p = b * 64 + r, j = j0 + V * c;
      vec v = vec(E(0));
      if (p < P && j < L) v = *reinterpret_cast<const vec*>(src + p * L + j);
#pragma unroll
      for (int e = 0; e < V; ++e) tile[r * kPitch + V * c + e] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TJ / kIRows; ++i) {
      const int jj = jr + kIRows * i;
      const int64_t j = j0 + jj;
      if (j < L) {
        ivec o;
#pragma unroll
        for (int m = 0; m < IV; ++m) o[m] = tile[(IV * q + m) * kPitch + jj];
        *reinterpret_cast<ivec*>(dst + (b * L + j) * 64 + IV * q) = o;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < TJ / kIRows; ++i) {
      const int jj = jr + kIRows * i;
      const int64_t j = j0 + jj;
      ivec v = ivec(E(0));
      if (j < L) v = *reinterpret_cast<const ivec*>(src + (b * L + j) * 64 + IV * q);
#pragma unroll
      for (int m = 0; m < IV; ++m) tile[(IV * q + m) * kPitch + jj] = v[m];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 64 / kRows; ++i) {
      const int r = r0 + kRows * i;
      const int64_t p = b * 64 + r, j = j0 + V * c;
      if (p < P && j < L) {
        vec v;
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = tile[r * kPitch + V * c + e];
        *reinterpret_cast<vec*>(dst + p * L + j) = v;
      }
    }
  }
}

// Byte k of word m of a becomes byte m of word k of the result: a 4 x 4 byte
// transpose (four series by four steps).
__device__ inline void transpose_bytes(const uint32_t a[4], uint32_t o[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
    o[k] = ((a[0] >> (8 * k)) & 0xffu) | (((a[1] >> (8 * k)) & 0xffu) << 8) | (((a[2] >> (8 * k)) & 0xffu) << 16) |
           (((a[3] >> (8 * k)) & 0xffu) << 24);
}

// 1-byte elements, a tile of 64 series x 256 steps held in LDS as 4-step words
// of each series.  The series-contiguous side is read or written W words per
// lane (64 / W lanes cover a series' 256 steps; L % (4 W) == 0), the
// interleaved side 16 bytes per lane (16 series of one step); each lane turns
// four 4-series x 4-step byte squares around in registers between the two.
template <int W>
__global__ __launch_bounds__(256) void k_interleave1(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst,
                                                     int64_t P, int64_t L, int to_interleaved, int64_t ny) {
  using vec = uint32_t __attribute__((ext_vector_type(W)));
  constexpr int kLanes = 64 / W;        // lanes per series row on the contiguous side (W words each)
  constexpr int kRows = 256 / kLanes;   // series rows per pass there
  __shared__ uint32_t tile[64 * 65];    // [series][4-step word], pitch 65 words
  int64_t b, by;
  if (!xcd_tile(ny, ny * ((P + 63) / 64), b, by)) return;
  const int64_t j0 = by * 256;
  const int t = threadIdx.x;
  const int c = t % kLanes, r0 = t / kLanes;  // contiguous side: W-word column, first series
  const int h = t & 3, cw = t >> 2;           // interleaved side: 16-series group, 4-step word of the tile
  const int64_t Lw = L / 4, jw = j0 / 4 + W * c;
  if (to_interleaved) {
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
#pragma unroll
    for (int i = 0; i < 64 / kRows; ++i) {
      const int r = r0 + kRows * i;
      const int64_t p = b * 64 + r;
      vec v = vec(0u);
      if (p < P && jw < Lw) v = *reinterpret_cast<const vec*>(s + p * Lw + jw);
#pragma unroll
      for (int e = 0; e < W; ++e) tile[r * 65 + W * c + e] = v[e];
    }
    __syncthreads();
    uint32_t o[4][4];  // [step k][series quad e]
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t a[4], r[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = tile[(16 * h + 4 * e + m) * 65 + cw];
      transpose_bytes(a, r);
#pragma unroll
      for (int k = 0; k < 4; ++k) o[k][e] = r[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t j = j0 + 4 * cw + k;
      if (j < L)
        *reinterpret_cast<uint4*>(dst + (b * L + j) * 64 + 16 * h) = make_uint4(o[k][0], o[k][1], o[k][2], o[k][3]);
    }
  } else {
    uint32_t in[4][4];  // [step k][series quad e]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t j = j0 + 4 * cw + k;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (j < L) v = *reinterpret_cast<const uint4*>(src + (b * L + j) * 64 + 16 * h);
      in[k][0] = v.x;
      in[k][1] = v.y;
      in[k][2] = v.z;
      in[k][3] = v.w;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t a[4], r[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = in[k][e];
      transpose_bytes(a, r);
#pragma unroll
      for (int m = 0; m < 4; ++m) tile[(16 * h + 4 * e + m) * 65 + cw] = r[m];
    }
    __syncthreads();
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
    for (int i = 0; i < 64 / kRows; ++i) {
      const int r = r0 + kRows * i;
      const int64_t p = b * 64 + r;
      if (p < P && jw < Lw) {
        vec v;
#pragma unroll
        for (int e = 0; e < W; ++e) v[e] = tile[r * 65 + W * c + e];
        *reinterpret_cast<vec*>(d + p * Lw + jw) = v;
      }
    }
  }
}

}  // namespace

// A launch counts at most 2^32 - 1 work-items.
constexpr int64_t kMaxGroups = (int64_t)0xffffffff / 256;

bool interleave_fits(int64_t P, int64_t L, int elem_bytes) {
  const int64_t nb = (P + 63) / 64;
  if (P <= 0 || L <= 0) return true;
  // the wide kernels' 1-D grid (tiles of 256 bytes of a series row), and the
  // one-element kernel's 2-D grid
  const int64_t steps = elem_bytes == 8 ? 32 : 64;
  return (nb * ((L + steps - 1) / steps) + 7) / 8 * 8 <= kMaxGroups && nb <= kMaxGroups && (L + 63) / 64 <= 65535;
}

hipError_t launch_interleave(const void* src, void* dst, int64_t P, int64_t L, int elem_bytes, bool to_interleaved,
                             hipStream_t stream) {
  if (P <= 0 || L <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P + 63) / 64), (unsigned)((L + 63) / 64));
  const int dir = to_interleaved ? 1 : 0;
  // alignment of the series-contiguous and the interleaved pointer
  const uintptr_t ac = reinterpret_cast<uintptr_t>(to_interleaved ? src : dst);
  const uintptr_t ai = reinterpret_cast<uintptr_t>(to_interleaved ? dst : src);
  // the wide kernels take a 1-D grid of a multiple of 8 workgroups
  const int64_t nb = (P + 63) / 64;
  auto grid1 = [&](int64_t steps_per_tile, int64_t& ny) {
    ny = (L + steps_per_tile - 1) / steps_per_tile;
    return (nb * ny + 7) / 8 * 8;
  };
  const bool narrow_fits = nb <= kMaxGroups && (L + 63) / 64 <= 65535;
  int64_t ny = 0, n = 0;
  switch (elem_bytes) {
    case 1:
      n = grid1(256, ny);
      if (n <= kMaxGroups && L % 8 == 0 && ac % 8 == 0 && ai % 16 == 0) {
        hipLaunchKernelGGL(k_interleave1<2>, dim3((unsigned)n), dim3(256), 0, stream,
                           static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst), P, L, dir, ny);
      } else if (n <= kMaxGroups && L % 4 == 0 && ac % 4 == 0 && ai % 16 == 0) {
        hipLaunchKernelGGL(k_interleave1<1>, dim3((unsigned)n), dim3(256), 0, stream,
                           static_cast<const uint8_t*>(src), static_cast<uint8_t*>(dst), P, L, dir, ny);
      } else if (narrow_fits) {
        hipLaunchKernelGGL(k_interleave<uint8_t>, grid, dim3(256), 0, stream, static_cast<const uint8_t*>(src),
                           static_cast<uint8_t*>(dst), P, L, dir);
      } else {
        return hipErrorInvalidValue;
      }
      break;
    case 4: {
      const float* s4 = static_cast<const float*>(src);
      float* d4 = static_cast<float*>(dst);
      n = grid1(64, ny);
      const dim3 g((unsigned)n);
      if (n > kMaxGroups || ai % 16 != 0) {
        if (!narrow_fits) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_interleave<float>, grid, dim3(256), 0, stream, s4, d4, P, L, dir);
      } else if (L % 4 == 0 && ac % 16 == 0)
        hipLaunchKernelGGL((k_interleave_wide<float, 4>), g, dim3(256), 0, stream, s4, d4, P, L, dir, ny);
      else if (L % 2 == 0 && ac % 8 == 0)
        hipLaunchKernelGGL((k_interleave_wide<float, 2>), g, dim3(256), 0, stream, s4, d4, P, L, dir, ny);
      else
        hipLaunchKernelGGL((k_interleave_wide<float, 1>), g, dim3(256), 0, stream, s4, d4, P, L, dir, ny);
      break;
    }
    case 8: {
      const double* s8 = static_cast<const double*>(src);
      double* d8 = static_cast<double*>(dst);
      n = grid1(32, ny);
      const dim3 g((unsigned)n);
      if (n > kMaxGroups || ai % 16 != 0) {
        if (!narrow_fits) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_interleave<double>, grid, dim3(256), 0, stream, s8, d8, P, L, dir);
      } else if (L % 2 == 0 && ac % 16 == 0)
        hipLaunchKernelGGL((k_interleave_wide<double, 2>), g, dim3(256), 0, stream, s8, d8, P, L, dir, ny);
      else
        hipLaunchKernelGGL((k_interleave_wide<double, 1>), g, dim3(256), 0, stream, s8, d8, P, L, dir, ny);
      break;
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace whs

// Layout changes between series-contiguous arrays (P, L) and the interleaved
// time-major layout (ceil(P/64), L, 64) the throughput kernels read: element
// (p, j) sits at p*L + j in one and at ((p/64)*L + j)*64 + p%64 in the other.
// A workgroup moves one 64 x 64 tile through LDS so both sides are read and
// written in 64-element rows.  Interleaving zero-fills the slots of the last
// block that hold no series.
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

}  // namespace

hipError_t launch_interleave(const void* src, void* dst, int64_t P, int64_t L, int elem_bytes, bool to_interleaved,
                             hipStream_t stream) {
  if (P <= 0 || L <= 0) return hipSuccess;
  const dim3 grid((unsigned)((P + 63) / 64), (unsigned)((L + 63) / 64));
  const int dir = to_interleaved ? 1 : 0;
  switch (elem_bytes) {
    case 1:
      hipLaunchKernelGGL(k_interleave<uint8_t>, grid, dim3(256), 0, stream, static_cast<const uint8_t*>(src),
                         static_cast<uint8_t*>(dst), P, L, dir);
      break;
    case 4:
      hipLaunchKernelGGL(k_interleave<float>, grid, dim3(256), 0, stream, static_cast<const float*>(src),
                         static_cast<float*>(dst), P, L, dir);
      break;
    case 8:
      hipLaunchKernelGGL(k_interleave<double>, grid, dim3(256), 0, stream, static_cast<const double*>(src),
                         static_cast<double*>(dst), P, L, dir);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace whs

// GCV weight selection: launches of the grid-search kernel.
#include <hip/hip_runtime.h>

#include "whs_fast.h"
#include "whs_kernels.h"

namespace whs {

// tile depth of the GCV kernel (its reverse sweep also keeps 1/Dp per step)
constexpr int gcv_tile(int D) { return D <= 2 ? 16 : 8; }

size_t gcv_checkpoint_bytes(int64_t P, int S, int T, int D) {
  const int64_t nb = (P + S - 1) / S;
  const int64_t nt = (T + gcv_tile(D) - 1) / gcv_tile(D);
  int nf = 0;
  switch (D) {
    case 1: nf = ck_fields<1, 1>(); break;
    case 2: nf = ck_fields<2, 1>(); break;
    case 3: nf = ck_fields<3, 1>(); break;
    case 4: nf = ck_fields<4, 1>(); break;
    default: return 0;
  }
  return (size_t)nb * nt * nf * S * sizeof(double);
}

template <int D, typename TS>
static hipError_t gcv_t(const GcvLaunch& L, hipStream_t stream) {
  GcvArgs a;
  a.P = L.P;
  a.T = L.T;
  a.S = L.S;
  constexpr int B = gcv_tile(D);
  a.nt = (L.T + B - 1) / B;
  a.n_grid = L.n_grid;
  a.w = L.w;
  a.x = L.x;
  a.grid = L.grid;
  a.lam_best = L.lam_best;
  a.scores = L.scores;
  a.info = L.info;
  a.ck = L.ws;
  const int threads = 256;
  const int64_t blocks = (L.P + threads - 1) / threads;
  hipLaunchKernelGGL((k_gcv<D, B, TS>), dim3((unsigned)blocks), dim3(threads), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_gcv(const GcvLaunch& L, hipStream_t stream) {
  switch (L.D) {
    case 1: return L.f64 ? gcv_t<1, double>(L, stream) : gcv_t<1, float>(L, stream);
    case 2: return L.f64 ? gcv_t<2, double>(L, stream) : gcv_t<2, float>(L, stream);
    case 3: return L.f64 ? gcv_t<3, double>(L, stream) : gcv_t<3, float>(L, stream);
    case 4: return L.f64 ? gcv_t<4, double>(L, stream) : gcv_t<4, float>(L, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace whs

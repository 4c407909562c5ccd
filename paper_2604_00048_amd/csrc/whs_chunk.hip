// Several lanes per series: the partition form of the banded solve.
//
// One workgroup of 256 lanes owns one series (interleave 1: the series'
// samples are contiguous).  The series is cut into K <= 256 chunks of at
// most MMAX samples.  Chunk k keeps its last d rows as an interface J_k
// (except the last chunk); the rest is its interior I_k.  Ordering the
// unknowns as (all interiors, then all interfaces) and eliminating the
// interiors first is a Cholesky factorisation of a symmetric permutation of
// Omega, so it keeps the stability of the sequential sweep:
//
//  pass 1  each lane factors its interior (LDL^T from a zero state) and keeps
//          L, 1/Dp and y = L^{-1} b in registers; alongside it propagates
//          W_T = L^{-1} (coupling of I_k to J_{k-1}) and W_B = L^{-1}
//          (coupling of I_k to J_k) and accumulates the Schur complement
//          terms as sums of squares  G = sum_t W_t^T Dp_t^{-1} W_t,
//          g = sum_t W_t^T Dp_t^{-1} y_t.
//  join    the interface system S xi = r is block tridiagonal with d x d
//          blocks: S_kk = Omega_JJ - G_BB(k) - G_TT(k+1),
//          S_k,k+1 = -G_TB(k+1),  r_k = b_J - g_B(k) - g_T(k+1).
//          It is solved by block cyclic reduction in LDS (odd-even
//          elimination: again Cholesky of a permuted SPD matrix).
//  pass 3  each interior is re-solved with the interface values moved to
//          the right-hand side, from the factor kept in registers.
//
// The series' inputs are read from HBM once (staged in LDS with coalesced
// loads) and every output is written once: no re-reads, no checkpoints.
// The adjoint runs the same solve on g, then forms grad_x = W u and
// grad_lambda_k = -(D u)_k (D z)_k from u in LDS and z in HBM.
//
// Orders d = 1, 2 and one band; everything else uses the two-sweep kernels.
#include <hip/hip_runtime.h>

#include "whs_fast.h"
#include "whs_kernels.h"
#include "whs_step.h"

namespace whs {

namespace {

constexpr int kThreads = 256;  // lanes per series (four wavefronts)
constexpr int kMmax = 13;      // samples per chunk at most

struct ChunkArgs {
  int64_t P;
  int T;
  const uint8_t* w;
  const void* lam;
  const void* rhs;  // x (solve) or g (adjoint)
  const void* zin;  // z (adjoint)
  void* out;        // z (solve) or grad_x (adjoint)
  void* glam;       // grad_lambda (adjoint)
  int32_t* info;
};

template <typename T>
__device__ __forceinline__ size_t align8(T v) {
  return ((size_t)v + 7) & ~(size_t)7;
}

// inverse of a small SPD matrix by LDL^T; returns false if a pivot is not
// positive and finite
template <int D>
__device__ __forceinline__ bool spd_inverse(const double (&B)[D][D], double (&Bi)[D][D]) {
  if constexpr (D == 1) {
    Bi[0][0] = 1.0 / B[0][0];
    return pivot_good(B[0][0]);
  } else {
    // D = 2: B = [a b; b c] = L diag(d1, d2) L^T with l = b / a
    const double a = B[0][0], b = B[1][0], c = B[1][1];
    const double d1 = a;
    const double l = b / a;
    const double d2 = c - l * b;
    const double i2 = 1.0 / d2;
    Bi[1][1] = i2;
    Bi[0][1] = Bi[1][0] = -l * i2;
    Bi[0][0] = 1.0 / d1 + l * l * i2;
    return pivot_good(d1) && pivot_good(d2);
  }
}

template <int D>
__device__ __forceinline__ void mm(const double (&X)[D][D], const double (&Y)[D][D], double (&Z)[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s = __builtin_fma(X[i][k], Y[k][j], s);
      Z[i][j] = s;
    }
}

// LDS view of one interface row of the block-tridiagonal system
//   A_i x_{i-s} + B_i x_i + C_i x_{i+s} = r_i,  plus its solution X_i.
template <int D>
struct Iface {
  double* base;
  static constexpr int kRow = 3 * D * D + 2 * D;
  __device__ double* row(int i) const { return base + (size_t)i * kRow; }
  __device__ void load(int i, double (&A)[D][D], double (&B)[D][D], double (&C)[D][D], double (&r)[D]) const {
    const double* p = row(i);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        A[a][b] = p[a * D + b];
        B[a][b] = p[D * D + a * D + b];
        C[a][b] = p[2 * D * D + a * D + b];
      }
#pragma unroll
    for (int a = 0; a < D; ++a) r[a] = p[3 * D * D + a];
  }
  __device__ void store(int i, const double (&A)[D][D], const double (&B)[D][D], const double (&C)[D][D],
                        const double (&r)[D]) const {
    double* p = row(i);
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        p[a * D + b] = A[a][b];
        p[D * D + a * D + b] = B[a][b];
        p[2 * D * D + a * D + b] = C[a][b];
      }
#pragma unroll
    for (int a = 0; a < D; ++a) p[3 * D * D + a] = r[a];
  }
  __device__ double* X(int i) const { return row(i) + 3 * D * D + D; }
};

template <int D, typename TS, bool BWD, bool PERDIFF>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_chunk(ChunkArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int T = a.T;
  const int64_t p = blockIdx.x;
  const int tid = threadIdx.x;
  constexpr uint32_t ES = sizeof(TS);

  // ---- LDS layout -------------------------------------------------------
  const size_t bx = align8((size_t)T * ES);
  const size_t bl = PERDIFF ? align8((size_t)(T - D) * ES) : 0;
  const size_t nG = (size_t)kThreads * (2 * D * D + D) * 8;
  const size_t nI = (size_t)kThreads * Iface<D>::kRow * 8;
  size_t region = bx + bl;
  if (nG > region) region = nG;
  if (nI > region) region = nI;
  TS* xs = reinterpret_cast<TS*>(lds);                // x or g; later z or u
  TS* ls = reinterpret_cast<TS*>(lds + bx);           // per-difference weights
  double* gx = reinterpret_cast<double*>(lds);        // exchange of the Schur terms
  Iface<D> ifc{reinterpret_cast<double*>(lds)};       // interface system
  uint8_t* ws = lds + region;                         // w
  const size_t tail = align8(T) > 32 ? align8(T) : 32;
  int* flags = reinterpret_cast<int*>(lds + region + tail);  // [0] failed, [1] observed count

  // ---- stage the series in LDS (coalesced) ------------------------------
  const auto rx = make_rsrc(static_cast<const TS*>(a.rhs) + p * T, (uint32_t)T * ES);
  const auto rw = make_rsrc(a.w + p * T, (uint32_t)T);
  if (tid == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
  int nobs = 0;
  for (int t = tid; t < T; t += kThreads) {
    xs[t] = bload<TS>(rx, (uint32_t)t * ES);
    const uint8_t wv = (uint8_t)__builtin_amdgcn_raw_buffer_load_b8(rw, (uint32_t)t, 0, 0);
    ws[t] = wv;
    nobs += wv != 0;
  }
  double lam_scalar = 0.0;
  if constexpr (PERDIFF) {
    const auto rl = make_rsrc(static_cast<const TS*>(a.lam) + p * (T - D), (uint32_t)(T - D) * ES);
    for (int t = tid; t < T - D; t += kThreads) ls[t] = bload<TS>(rl, (uint32_t)t * ES);
  } else {
    lam_scalar = to_f64(static_cast<const TS*>(a.lam)[p]);
  }
  __syncthreads();
  if (nobs) atomicAdd(&flags[1], nobs);

  auto lam_at = [&](int k) -> double {
    if (k < 0 || k >= T - D) return 0.0;
    if constexpr (PERDIFF) return to_f64(ls[k]);
    else return lam_scalar;
  };
  auto rhs_at = [&](int t) -> double {
    const double v = to_f64(xs[t]);
    if constexpr (BWD) return v;
    else return ws[t] != 0 ? v : 0.0;
  };
  auto omega_at = [&](int t, double (&om)[D + 1]) {
    double lwv[D + 1];
#pragma unroll
    for (int m = 0; m <= D; ++m) lwv[m] = lam_at(t - m);
    omega_row<D>(lwv, ws[t] != 0 ? 1.0 : 0.0, om);
  };

  // ---- chunk of this lane -----------------------------------------------
  const int K = (T + kMmax - 1) / kMmax;  // <= kThreads (checked on the host)
  const int k = tid;
  const bool act = k < K;
  const int s0 = act ? (int)(((int64_t)k * T) / K) : 0;
  const int e = act ? (int)(((int64_t)(k + 1) * T) / K) : 0;
  const bool hasJ = act && k < K - 1;
  const bool hasL = act && k > 0;
  const int ie = hasJ ? e - D : e;
  const int n = act ? ie - s0 : 0;  // interior rows, 1..kMmax

  // Omega rows of the interface J_k (rows ie .. ie+D-1)
  double omJ[D][D + 1];
  double bJ[D];
#pragma unroll
  for (int r = 0; r < D; ++r) {
    if (hasJ) {
      omega_at(ie + r, omJ[r]);
      bJ[r] = rhs_at(ie + r);
    } else {
#pragma unroll
      for (int i = 0; i <= D; ++i) omJ[r][i] = 0.0;
      bJ[r] = 0.0;
    }
  }

  // ---- pass 1: factor the interior, keep it, accumulate Schur terms ------
  double Ls[kMmax][D + 1], IDs[kMmax], Ys[kMmax];
#pragma unroll
  for (int i = 0; i < kMmax; ++i) {
#pragma unroll
    for (int j = 0; j <= D; ++j) Ls[i][j] = 0.0;
    IDs[i] = 0.0;
    Ys[i] = 0.0;
  }
  double rt0[D][D];  // Omega[s0 + r, s0 - D + c]: coupling of the first rows to J_{k-1}
  double WT[D + 1][D], WB[D + 1][D];
  double GTT[D][D], GTb[D], GBB[D][D], GBb[D], GTB[D][D];
#pragma unroll
  for (int r = 0; r <= D; ++r)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      WT[r][c] = 0.0;
      WB[r][c] = 0.0;
    }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    GTb[r] = 0.0;
    GBb[r] = 0.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      rt0[r][c] = 0.0;
      GTT[r][c] = 0.0;
      GBB[r][c] = 0.0;
      GTB[r][c] = 0.0;
    }
  }
  bool ok = true;
  State<D, 1> st;
  st.zero();
#pragma unroll
  for (int i = 0; i < kMmax; ++i) {
    if (i < n) {
      const int t = s0 + i;
      double om[D + 1], l[D + 1], dt, invdt, yt[1];
      omega_at(t, om);
      ldl_step<D, 1>(st, om, l, dt, invdt);
      ok = ok && pivot_good(dt);
      const double b[1] = {rhs_at(t)};
      fwd_step<D, 1>(st, l, b, yt);
#pragma unroll
      for (int j = 1; j <= D; ++j) Ls[i][j] = l[j];
      IDs[i] = invdt;
      Ys[i] = yt[0];
      // right-hand sides of W_T (first D rows) and W_B (last D rows)
      double rt[D], rb[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        rt[c] = (hasL && i < D && c >= i) ? om[(i + D - c) <= D ? (i + D - c) : 0] : 0.0;
        if (i < D) rt0[i < D ? i : 0][c] = rt[c];
        rb[c] = 0.0;
      }
      const int rr = i - (n - D);  // index among the last D interior rows
#pragma unroll
      for (int q = 0; q < D; ++q) {
        if (hasJ && rr == q) {
#pragma unroll
          for (int c = 0; c <= q; ++c) rb[c] = omJ[c][D + c - q];
        }
      }
      double wt[D], wb[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        double s1 = rt[c], s2 = rb[c];
#pragma unroll
        for (int j = 1; j <= D; ++j) {
          s1 = __builtin_fma(-l[j], WT[j][c], s1);
          s2 = __builtin_fma(-l[j], WB[j][c], s2);
        }
        wt[c] = s1;
        wb[c] = s2;
      }
#pragma unroll
      for (int j = D; j >= 2; --j)
#pragma unroll
        for (int c = 0; c < D; ++c) {
          WT[j][c] = WT[j - 1][c];
          WB[j][c] = WB[j - 1][c];
        }
#pragma unroll
      for (int c = 0; c < D; ++c) {
        WT[1][c] = wt[c];
        WB[1][c] = wb[c];
      }
      double vt[D], vb[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        vt[c] = wt[c] * invdt;
        vb[c] = wb[c] * invdt;
      }
#pragma unroll
      for (int r = 0; r < D; ++r) {
        GTb[r] = __builtin_fma(vt[r], yt[0], GTb[r]);
        GBb[r] = __builtin_fma(vb[r], yt[0], GBb[r]);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          GTT[r][c] = __builtin_fma(vt[r], wt[c], GTT[r][c]);
          GBB[r][c] = __builtin_fma(vb[r], wb[c], GBB[r][c]);
          GTB[r][c] = __builtin_fma(vt[r], wb[c], GTB[r][c]);
        }
      }
    }
  }
  if (!ok) flags[0] = 1;
  __syncthreads();  // staging of x and lambda is no longer read

  // ---- join: exchange the top terms with the left neighbour -------------
  constexpr int GW = 2 * D * D + D;
  if (hasL) {
    double* g = gx + (size_t)k * GW;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      g[2 * D * D + r] = GTb[r];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        g[r * D + c] = GTT[r][c];
        g[D * D + r * D + c] = GTB[r][c];
      }
    }
  }
  __syncthreads();
  double Am[D][D], Bm[D][D], Cm[D][D], rv[D];
  if (hasJ) {
    const double* g = gx + (size_t)(k + 1) * GW;
    const bool next_has_j = k + 1 < K - 1;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      rv[r] = bJ[r] - GBb[r] - g[2 * D * D + r];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        // Omega_JJ[r][c] = Omega[ie + r, ie + c]
        const double ojj = r >= c ? omJ[r][r - c >= 0 ? r - c : 0] : omJ[c][c - r >= 0 ? c - r : 0];
        Bm[r][c] = ojj - GBB[r][c] - g[r * D + c];
        Cm[r][c] = next_has_j ? -g[D * D + r * D + c] : 0.0;
        Am[r][c] = hasL ? -GTB[c][r] : 0.0;
      }
    }
  }
  __syncthreads();  // every neighbour term has been read
  const int nJ = K - 1;
  if (hasJ) ifc.store(k, Am, Bm, Cm, rv);
  __syncthreads();

  // ---- block cyclic reduction on the nJ interface rows -------------------
  bool cr_ok = true;
  int s = 1;
  while (nJ / s > 1) {
    // kept rows i = 2 s (m + 1) - 1 absorb their neighbours i - s and i + s
    const int i = 2 * s * (tid + 1) - 1;
    if (i < nJ) {
      double A[D][D], B[D][D], C[D][D], r[D];
      double A1[D][D], B1[D][D], C1[D][D], r1[D], B1i[D][D], al[D][D], t1[D][D];
      ifc.load(i, A, B, C, r);
      ifc.load(i - s, A1, B1, C1, r1);
      cr_ok = spd_inverse<D>(B1, B1i) && cr_ok;
      mm<D>(A, B1i, al);  // alpha = A_i B_{i-s}^{-1}
      double An[D][D], Cn[D][D];
      mm<D>(al, C1, t1);
#pragma unroll
      for (int x = 0; x < D; ++x)
#pragma unroll
        for (int y = 0; y < D; ++y) B[x][y] -= t1[x][y];
      mm<D>(al, A1, t1);
#pragma unroll
      for (int x = 0; x < D; ++x) {
#pragma unroll
        for (int y = 0; y < D; ++y) {
          An[x][y] = -t1[x][y];
          r[x] = __builtin_fma(-al[x][y], r1[y], r[x]);
        }
      }
#pragma unroll
      for (int x = 0; x < D; ++x)
#pragma unroll
        for (int y = 0; y < D; ++y) Cn[x][y] = 0.0;
      if (i + s < nJ) {
        double A2[D][D], B2[D][D], C2[D][D], r2[D], B2i[D][D], ga[D][D];
        ifc.load(i + s, A2, B2, C2, r2);
        cr_ok = spd_inverse<D>(B2, B2i) && cr_ok;
        mm<D>(C, B2i, ga);  // gamma = C_i B_{i+s}^{-1}
        mm<D>(ga, A2, t1);
#pragma unroll
        for (int x = 0; x < D; ++x)
#pragma unroll
          for (int y = 0; y < D; ++y) B[x][y] -= t1[x][y];
        mm<D>(ga, C2, t1);
#pragma unroll
        for (int x = 0; x < D; ++x) {
#pragma unroll
          for (int y = 0; y < D; ++y) {
            Cn[x][y] = -t1[x][y];
            r[x] = __builtin_fma(-ga[x][y], r2[y], r[x]);
          }
        }
      }
      // symmetrise the pivot block (it is symmetric in exact arithmetic)
#pragma unroll
      for (int x = 0; x < D; ++x)
#pragma unroll
        for (int y = 0; y < x; ++y) {
          const double m = 0.5 * (B[x][y] + B[y][x]);
          B[x][y] = m;
          B[y][x] = m;
        }
      ifc.store(i, An, B, Cn, r);
    }
    __syncthreads();
    s *= 2;
  }
  if (nJ > 0 && tid == 0) {
    // the one row left at this level: i = s - 1, no neighbours
    double A[D][D], B[D][D], C[D][D], r[D], Bi[D][D];
    ifc.load(s - 1, A, B, C, r);
    cr_ok = spd_inverse<D>(B, Bi) && cr_ok;
    double* X = ifc.X(s - 1);
#pragma unroll
    for (int x = 0; x < D; ++x) {
      double v = 0.0;
#pragma unroll
      for (int y = 0; y < D; ++y) v = __builtin_fma(Bi[x][y], r[y], v);
      X[x] = v;
    }
  }
  __syncthreads();
  while (s > 1) {
    s /= 2;
    // rows active at stride s but eliminated there: i = s (2m + 1) - 1
    const int i = s * (2 * tid + 1) - 1;
    if (i < nJ) {
      double A[D][D], B[D][D], C[D][D], r[D], Bi[D][D];
      ifc.load(i, A, B, C, r);
      cr_ok = spd_inverse<D>(B, Bi) && cr_ok;
      if (i - s >= 0) {
        const double* Xl = ifc.X(i - s);
#pragma unroll
        for (int x = 0; x < D; ++x)
#pragma unroll
          for (int y = 0; y < D; ++y) r[x] = __builtin_fma(-A[x][y], Xl[y], r[x]);
      }
      if (i + s < nJ) {
        const double* Xr = ifc.X(i + s);
#pragma unroll
        for (int x = 0; x < D; ++x)
#pragma unroll
          for (int y = 0; y < D; ++y) r[x] = __builtin_fma(-C[x][y], Xr[y], r[x]);
      }
      double* X = ifc.X(i);
#pragma unroll
      for (int x = 0; x < D; ++x) {
        double v = 0.0;
#pragma unroll
        for (int y = 0; y < D; ++y) v = __builtin_fma(Bi[x][y], r[y], v);
        X[x] = v;
      }
    }
    __syncthreads();
  }
  if (!cr_ok) flags[0] = 1;
  double xiL[D], xiR[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    xiL[c] = hasL ? ifc.X(k - 1)[c] : 0.0;
    xiR[c] = hasJ ? ifc.X(k)[c] : 0.0;
  }
  __syncthreads();  // the interface area is reused for the outputs below

  const bool failed = flags[0] != 0 || flags[1] < D;
  const double qnan = __builtin_nan("");
  if (failed) {
    // rare path: the exact first failing pivot by a plain rescan on one lane
    if (tid == 0) {
      int info = 0;
      State<D, 1> sq;
      sq.zero();
      const auto rl = make_rsrc(PERDIFF ? static_cast<const TS*>(a.lam) + p * (T - D) : static_cast<const TS*>(a.lam),
                                PERDIFF ? (uint32_t)(T - D) * ES : 0u);
      for (int t = 0; t < T && info == 0; ++t) {
        double lwv[D + 1];
        lwv[0] = (t < T - D) ? (PERDIFF ? to_f64(bload<TS>(rl, (uint32_t)t * ES)) : lam_scalar) : 0.0;
#pragma unroll
        for (int m = 1; m <= D; ++m) lwv[m] = sq.lw[m];
        double om[D + 1], l[D + 1], dt, invdt;
        omega_row<D>(lwv, ws[t] != 0 ? 1.0 : 0.0, om);
        ldl_step<D, 1>(sq, om, l, dt, invdt);
#pragma unroll
        for (int m = D; m >= 2; --m) sq.lw[m] = sq.lw[m - 1];
        sq.lw[1] = lwv[0];
        if (!pivot_good(dt)) info = t + 1;
      }
      if (info == 0) info = T;  // fewer than d observations, or a failure the rescan does not see
      if (a.info) a.info[p] = info;
    }
    for (int t = tid; t < T; t += kThreads) {
      if (a.out) static_cast<TS*>(a.out)[p * T + t] = from_f64<TS>(qnan);
    }
    if constexpr (BWD) {
      if (a.glam) {
        if constexpr (PERDIFF) {
          for (int t = tid; t < T - D; t += kThreads) static_cast<TS*>(a.glam)[p * (T - D) + t] = from_f64<TS>(qnan);
        } else if (tid == 0) {
          static_cast<TS*>(a.glam)[p] = from_f64<TS>(qnan);
        }
      }
    }
    return;
  }

  // ---- pass 3: interiors with the interface values moved to the right ----
  if (act) {
    double yc[D + 1];
#pragma unroll
    for (int j = 0; j <= D; ++j) yc[j] = 0.0;
#pragma unroll
    for (int i = 0; i < kMmax; ++i) {
      if (i < n) {
        double cv = 0.0;
        if (i < D) {
#pragma unroll
          for (int c = 0; c < D; ++c) cv = __builtin_fma(rt0[i < D ? i : 0][c], xiL[c], cv);
        }
        const int rr = i - (n - D);
#pragma unroll
        for (int q = 0; q < D; ++q) {
          if (hasJ && rr == q) {
#pragma unroll
            for (int c = 0; c <= q; ++c) cv = __builtin_fma(omJ[c][D + c - q], xiR[c], cv);
          }
        }
#pragma unroll
        for (int j = 1; j <= D; ++j) cv = __builtin_fma(-Ls[i][j], yc[j], cv);
#pragma unroll
        for (int j = D; j >= 2; --j) yc[j] = yc[j - 1];
        yc[1] = cv;
        Ys[i] -= cv;
      }
    }
    double zn[D + 1];
#pragma unroll
    for (int j = 0; j <= D; ++j) zn[j] = 0.0;
#pragma unroll
    for (int i = kMmax - 1; i >= 0; --i) {
      if (i < n) {
        double zt = Ys[i] * IDs[i];
#pragma unroll
        for (int j = 1; j <= D; ++j) {
          if (i + j < kMmax) zt = __builtin_fma(-Ls[i + j < kMmax ? i + j : 0][j], zn[j], zt);
        }
#pragma unroll
        for (int j = D; j >= 2; --j) zn[j] = zn[j - 1];
        zn[1] = zt;
        xs[s0 + i] = from_f64<TS>(zt);
      }
    }
    if (hasJ) {
#pragma unroll
      for (int r = 0; r < D; ++r) xs[ie + r] = from_f64<TS>(xiR[r]);
    }
  }
  __syncthreads();

  // ---- outputs ----------------------------------------------------------
  if (tid == 0 && a.info) a.info[p] = 0;
  if constexpr (!BWD) {
    const auto ro = make_rsrc(static_cast<TS*>(a.out) + p * T, (uint32_t)T * ES);
    for (int t = tid; t < T; t += kThreads) bstore<TS>(ro, (uint32_t)t * ES, xs[t]);
  } else {
    if (a.out) {
      const auto ro = make_rsrc(static_cast<TS*>(a.out) + p * T, (uint32_t)T * ES);
      for (int t = tid; t < T; t += kThreads) bstore<TS>(ro, (uint32_t)t * ES, ws[t] != 0 ? xs[t] : TS(0));
    }
    if (a.glam) {
      const auto rz = make_rsrc(static_cast<const TS*>(a.zin) + p * T, (uint32_t)T * ES);
      double gsum = 0.0;
      const auto rg = make_rsrc(static_cast<TS*>(a.glam) + (PERDIFF ? p * (T - D) : 0),
                                PERDIFF ? (uint32_t)(T - D) * ES : 0u);
      for (int kk = tid; kk < T - D; kk += kThreads) {
        double du = 0.0, dz = 0.0;
#pragma unroll
        for (int j = 0; j <= D; ++j) {
          du = __builtin_fma(cdiff<D>(j), to_f64(xs[kk + j]), du);
          dz = __builtin_fma(cdiff<D>(j), to_f64(bload<TS>(rz, (uint32_t)(kk + j) * ES)), dz);
        }
        const double gk = -du * dz;
        if constexpr (PERDIFF) bstore<TS>(rg, (uint32_t)kk * ES, from_f64<TS>(gk));
        else gsum += gk;
      }
      if constexpr (!PERDIFF) {
        // block sum: wavefront butterfly, then one value per wavefront in LDS
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) gsum += __shfl_xor(gsum, off);
        __syncthreads();
        double* red = reinterpret_cast<double*>(lds + region);  // w is no longer needed
        if ((tid & 63) == 0) red[tid >> 6] = gsum;
        __syncthreads();
        if (tid == 0) {
          double tot = 0.0;
          for (int wv = 0; wv < kThreads / 64; ++wv) tot += red[wv];
          static_cast<TS*>(a.glam)[p] = from_f64<TS>(tot);
        }
      }
    }
  }
}

template <int D>
size_t chunk_lds_bytes(int T, size_t es, bool perdiff) {
  const size_t bx = ((size_t)T * es + 7) & ~(size_t)7;
  const size_t bl = perdiff ? (((size_t)(T - D) * es + 7) & ~(size_t)7) : 0;
  const size_t nG = (size_t)kThreads * (2 * D * D + D) * 8;
  const size_t nI = (size_t)kThreads * Iface<D>::kRow * 8;
  size_t region = bx + bl;
  if (nG > region) region = nG;
  if (nI > region) region = nI;
  const size_t tail = (((size_t)T + 7) & ~(size_t)7) > 32 ? (((size_t)T + 7) & ~(size_t)7) : 32;
  return region + tail + 16;  // w (or the 4-value reduction), then two flags
}

template <int D, typename TS, bool BWD, bool PERDIFF>
hipError_t chunk_t(const LaunchDesc& L, hipStream_t stream) {
  ChunkArgs a;
  a.P = L.P;
  a.T = L.T;
  a.w = L.w;
  a.lam = L.lam;
  a.rhs = L.rhs;
  a.zin = L.zin;
  a.out = L.out;
  a.glam = L.glam;
  a.info = L.info;
  const size_t lds = chunk_lds_bytes<D>(L.T, sizeof(TS), PERDIFF);
  hipLaunchKernelGGL((k_chunk<D, TS, BWD, PERDIFF>), dim3((unsigned)L.P), dim3(kThreads), lds, stream, a);
  return hipGetLastError();
}

template <int D, bool BWD>
hipError_t chunk_d(const LaunchDesc& L, hipStream_t stream) {
  if (L.f64) return L.perdiff ? chunk_t<D, double, BWD, true>(L, stream) : chunk_t<D, double, BWD, false>(L, stream);
  return L.perdiff ? chunk_t<D, float, BWD, true>(L, stream) : chunk_t<D, float, BWD, false>(L, stream);
}

}  // namespace

// The partition kernel takes a call when the series are contiguous (interleave
// 1), one band, order 1 or 2, the factor is recomputed (no whs_factor input),
// D is the daily-grid operator, and a series fits 256 chunks of 13 samples.
bool chunk_path(const LaunchDesc& L) {
  if (L.S != 1 || L.C != 1 || L.D < 1 || L.D > 2 || L.fac || L.coef) return false;
  // one workgroup per series; a grid counts at most 2^32 - 1 work-items, so larger
  // batches take the one-lane kernel
  if (L.T > kThreads * kMmax || L.P < 1 || L.P > (int64_t)0xffffffff / kThreads) return false;
  const size_t lds = L.D == 1 ? chunk_lds_bytes<1>(L.T, L.f64 ? 8 : 4, L.perdiff)
                              : chunk_lds_bytes<2>(L.T, L.f64 ? 8 : 4, L.perdiff);
  return lds <= 64 * 1024;
}

hipError_t launch_chunk(const LaunchDesc& L, bool bwd, hipStream_t stream) {
  if (L.D == 1) return bwd ? chunk_d<1, true>(L, stream) : chunk_d<1, false>(L, stream);
  return bwd ? chunk_d<2, true>(L, stream) : chunk_d<2, false>(L, stream);
}

}  // namespace whs

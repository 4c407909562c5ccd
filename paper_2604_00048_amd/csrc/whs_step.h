// Per-lane banded LDL^T recurrence of the Whittaker-Henderson system.
//
// One lane owns one series.  At time t the lane assembles row t of
// Omega = W + D^T Lambda D (eq. (3)) from the 0/1 flag w_t and the last d+1
// smoothing weights, performs one step of the banded factorisation
// Omega = L diag(Dp) L^T (Sec. III-A), and one step of the forward
// substitution L y = W x for C right-hand sides.  Everything is FP64 in
// registers; arrays are indexed with compile-time constants only, so the
// state lives in VGPRs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace whs {

constexpr long long binom(int n, int k) {
  long long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// c_j of the order-D difference on unit spacing: (-1)^(D-j) C(D, j).
template <int D>
__host__ __device__ constexpr double cdiff(int j) {
  return (((D - j) & 1) ? -1.0 : 1.0) * static_cast<double>(binom(D, j));
}

// 1/x to full FP64 accuracy for positive normal x: hardware estimate plus two
// Newton-Raphson corrections r <- r + r (1 - x r).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double to_f64(float v) { return static_cast<double>(v); }
__device__ __forceinline__ double to_f64(double v) { return v; }
template <typename TS> __device__ __forceinline__ TS from_f64(double v);
template <> __device__ __forceinline__ float from_f64<float>(double v) { return static_cast<float>(v); }
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }

// Recurrence state carried from step t-1 to step t.
//   invD[j]  = 1 / Dp[t-j]                 (j = 1..D)
//   R[j][k]  = L[t-j, t-j-k]               (j = 1..D-1, k = 1..D-j)
//   y[j][c]  = y[t-j][c]                   (j = 1..D)
//   lw[m]    = lambda_{t-m}                (m = 1..D; per-difference weights)
//   cw[m][j] = c_{t-m, j}                  (m = 1..D; rows of D on uneven times)
// Index 0 entries are unused.  A zero state is the state before t = 0: rows
// with negative index contribute nothing because Omega has no entries there.
template <int D, int C>
struct State {
  double invD[D + 1];
  double R[D + 1][D + 1];
  double y[D + 1][C];
  double lw[D + 1];
  double cw[D + 1][D + 1];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j <= D; ++j) {
      invD[j] = 0.0;
      lw[j] = 0.0;
#pragma unroll
      for (int k = 0; k <= D; ++k) cw[j][k] = 0.0;
#pragma unroll
      for (int k = 0; k <= D; ++k) R[j][k] = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) y[j][c] = 0.0;
    }
  }
};

// Number of FP64 checkpoint fields: invD (D), R triangle (D(D-1)/2), y (D*C).
// The per-difference weight window is re-read from lambda instead.
template <int D, int C>
__host__ __device__ constexpr int ck_fields() {
  return D + D * (D - 1) / 2 + D * C;
}

template <int D, int C>
__device__ __forceinline__ void ck_store(const State<D, C>& st, double* ck, int S) {
  int f = 0;
#pragma unroll
  for (int j = 1; j <= D; ++j) ck[(f++) * S] = st.invD[j];
#pragma unroll
  for (int j = 1; j < D; ++j)
#pragma unroll
    for (int k = 1; k <= D - j; ++k) ck[(f++) * S] = st.R[j][k];
#pragma unroll
  for (int j = 1; j <= D; ++j)
#pragma unroll
    for (int c = 0; c < C; ++c) ck[(f++) * S] = st.y[j][c];
}

template <int D, int C>
__device__ __forceinline__ void ck_load(State<D, C>& st, const double* ck, int S) {
  int f = 0;
#pragma unroll
  for (int j = 1; j <= D; ++j) st.invD[j] = ck[(f++) * S];
#pragma unroll
  for (int j = 1; j < D; ++j)
#pragma unroll
    for (int k = 1; k <= D - j; ++k) st.R[j][k] = ck[(f++) * S];
#pragma unroll
  for (int j = 1; j <= D; ++j)
#pragma unroll
    for (int c = 0; c < C; ++c) st.y[j][c] = ck[(f++) * S];
}

// Row t of Omega below and on the diagonal: om[i] = Omega[t, t-i], i = 0..D,
// from Omega[r, s] = w_r [r = s] + sum_k lambda_k c_{r-k} c_{s-k}.  With
// lw[m] = lambda_{t-m}: om[i] = [i = 0] w_t + sum_{m=i..D} lw[m] c_m c_{m-i}.
// Weights outside 0..T-D-1 must already be zero in lw.
template <int D>
__device__ __forceinline__ void omega_row(const double (&lw)[D + 1], double wt, double (&om)[D + 1]) {
#pragma unroll
  for (int i = 0; i <= D; ++i) {
    double a = 0.0;
#pragma unroll
    for (int m = i; m <= D; ++m) a = __builtin_fma(lw[m], cdiff<D>(m) * cdiff<D>(m - i), a);
    om[i] = a;
  }
  om[0] += wt;
}

// The same row when D has its own coefficients per row (uneven sample times,
// Sec. II): with cw[m][j] = c_{t-m, j} (row t-m of D),
// om[i] = [i = 0] w_t + sum_{m=i..D} lw[m] c_{t-m, m} c_{t-m, m-i}.
template <int D>
__device__ __forceinline__ void omega_row_tab(const double (&lw)[D + 1], const double (&cw)[D + 1][D + 1], double wt,
                                              double (&om)[D + 1]) {
#pragma unroll
  for (int i = 0; i <= D; ++i) {
    double a = 0.0;
#pragma unroll
    for (int m = i; m <= D; ++m) a = __builtin_fma(lw[m] * cw[m][m], cw[m][m - i], a);
    om[i] = a;
  }
  om[0] += wt;
}

// One LDL^T step for row t given om[] (Omega[t, t-i]).
// Outputs l[j] = L[t, t-j] (j = 1..D), Dp[t] and its reciprocal, and shifts
// the factor part of the state.  a_j = L[t,t-j] Dp[t-j] satisfies
// a_j = Omega[t,t-j] - sum_{m>j} a_m L[t-j, t-m], and
// Dp[t] = Omega[t,t] - sum_j a_j L[t,t-j].
template <int D, int C>
__device__ __forceinline__ void ldl_step(State<D, C>& st, const double (&om)[D + 1], double (&l)[D + 1],
                                         double& dt, double& invdt) {
  double a[D + 1];
#pragma unroll
  for (int j = D; j >= 1; --j) {
    double acc = om[j];
#pragma unroll
    for (int m = j + 1; m <= D; ++m) acc = __builtin_fma(-a[m], st.R[j][m - j], acc);
    a[j] = acc;
    l[j] = acc * st.invD[j];
  }
  double dd = om[0];
#pragma unroll
  for (int j = 1; j <= D; ++j) dd = __builtin_fma(-a[j], l[j], dd);
  dt = dd;
  invdt = rcp64(dd);
  // shift: row t becomes row (t+1)-1
#pragma unroll
  for (int j = D - 1; j >= 2; --j)
#pragma unroll
    for (int k = 1; k <= D - j; ++k) st.R[j][k] = st.R[j - 1][k];
  if (D >= 2) {
#pragma unroll
    for (int k = 1; k <= D - 1; ++k) st.R[1][k] = l[k];
  }
#pragma unroll
  for (int j = D; j >= 2; --j) st.invD[j] = st.invD[j - 1];
  st.invD[1] = invdt;
}

// One forward-substitution step y_t = b_t - sum_j L[t,t-j] y_{t-j}; shifts y.
template <int D, int C>
__device__ __forceinline__ void fwd_step(State<D, C>& st, const double (&l)[D + 1], const double (&b)[C],
                                         double (&yt)[C]) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    double acc = b[c];
#pragma unroll
    for (int j = 1; j <= D; ++j) acc = __builtin_fma(-l[j], st.y[j][c], acc);
    yt[c] = acc;
  }
#pragma unroll
  for (int j = D; j >= 2; --j)
#pragma unroll
    for (int c = 0; c < C; ++c) st.y[j][c] = st.y[j - 1][c];
#pragma unroll
  for (int c = 0; c < C; ++c) st.y[1][c] = yt[c];
}

__device__ __forceinline__ bool pivot_ok(double dt) {
  return dt > 0.0 && dt < __builtin_huge_val();
}

}  // namespace whs

// Generalised cross-validation of a scalar weight over a grid, in one forward
// sweep per grid value.
//
// For a grid value lambda, Omega = W + lambda D^T D and b = W x.  The score is
// GCV = m RSS / (m - ED)^2 with m = sum_t w_t, RSS = sum_t w_t (x_t - z_t)^2
// and ED = sum_t w_t (Omega^{-1})_tt.  Both sums are derivatives along the
// perturbation Omega + eps W (weights 0/1, so W^2 = W):
//
//   ED  = tr(Omega^{-1} W) = d/deps log det(Omega + eps W)        (Jacobi)
//       = sum_t Dp'_t / Dp_t,
//   RSS = d/deps min_z [(1 + eps) |x - z|_W^2 + lambda |D z|^2]   (envelope)
//       = sum_t w_t x_t^2 - d/deps [b_eps^T Omega_eps^{-1} b_eps],  b_eps = (1 + eps) W x,
//       = sum_t w_t x_t^2 - sum_t d/deps (y_t^2 / Dp_t),
//
// where Omega = L diag(Dp) L^T and y = L^{-1} b.  The kernel runs the LDL^T
// recurrence and forward substitution of the solve kernels together with
// their derivatives (forward-mode, om'[0] = w_t, om'[i > 0] = 0, b' = b), so
// it needs no reverse sweep, no checkpoints and no workspace.  x is taken
// relative to the first observed value of its series (the smoother keeps
// constants, so RSS does not change), which keeps sum w x^2 and the explained
// part from cancelling for series far from zero.
//
// G grid values share one pass: each tile of x and w is loaded once for G
// recurrences, interleaved step by step.
#pragma once

#include <hip/hip_runtime.h>

#include "whs_fast.h"

namespace whs {

struct GcvArgs {
  int64_t P;
  int T, S, nt, n_grid;
  const uint8_t* w;
  const void* x;
  const double* grid;
  void* lam_best;
  double* scores;
  int32_t* info;
};

// the factor window, the forward-substitution window and their derivatives
template <int D>
struct DualState {
  double invD[D + 1], R[D + 1][D + 1], y[D + 1];
  double dinvD[D + 1], dR[D + 1][D + 1], dy[D + 1];
  double ds, ed;  // half the derivative of sum y^2 / Dp, and sum Dp' / Dp

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j <= D; ++j) {
      invD[j] = dinvD[j] = y[j] = dy[j] = 0.0;
#pragma unroll
      for (int k = 0; k <= D; ++k) R[j][k] = dR[j][k] = 0.0;
    }
    ds = ed = 0.0;
  }
};

// One step of LDL^T and forward substitution (the same operations as
// ldl_step and fwd_step) with the derivatives along W; row t of Omega is
// om[i] = Omega[t, t-i].  v: row t lies inside the series (its terms count).
template <int D>
__device__ __forceinline__ void dual_step(DualState<D>& st, const double (&om)[D + 1], double wt, double b, bool v,
                                          double& dt) {
  // a_j = L[t,t-j] Dp[t-j]; its derivative is zero for j = D (om'[D] = 0 and
  // no earlier term), which the loops below skip
  double a[D + 1], da[D + 1], l[D + 1], dl[D + 1];
#pragma unroll
  for (int j = D; j >= 1; --j) {
    double acc = om[j], dacc = 0.0;
#pragma unroll
    for (int m = j + 1; m <= D; ++m) {
      acc = __builtin_fma(-a[m], st.R[j][m - j], acc);
      const double t1 = -a[m] * st.dR[j][m - j];
      dacc = (m == j + 1) ? t1 : dacc + t1;
      if (m < D) dacc = __builtin_fma(-da[m], st.R[j][m - j], dacc);
    }
    a[j] = acc;
    da[j] = dacc;
    l[j] = acc * st.invD[j];
    dl[j] = (j == D) ? acc * st.dinvD[j] : __builtin_fma(dacc, st.invD[j], acc * st.dinvD[j]);
  }
  double dd = om[0], ddd = wt;
#pragma unroll
  for (int j = 1; j <= D; ++j) {
    dd = __builtin_fma(-a[j], l[j], dd);
    ddd = __builtin_fma(-a[j], dl[j], ddd);
    if (j < D) ddd = __builtin_fma(-da[j], l[j], ddd);
  }
  dt = dd;
  const double invdt = rcp64(dd);
  const double e = ddd * invdt;  // Dp'/Dp
  const double dinvdt = -e * invdt;
#pragma unroll
  for (int j = D - 1; j >= 2; --j)
#pragma unroll
    for (int k = 1; k <= D - j; ++k) {
      st.R[j][k] = st.R[j - 1][k];
      st.dR[j][k] = st.dR[j - 1][k];
    }
  if (D >= 2) {
#pragma unroll
    for (int k = 1; k <= D - 1; ++k) {
      st.R[1][k] = l[k];
      st.dR[1][k] = dl[k];
    }
  }
#pragma unroll
  for (int j = D; j >= 2; --j) {
    st.invD[j] = st.invD[j - 1];
    st.dinvD[j] = st.dinvD[j - 1];
  }
  st.invD[1] = invdt;
  st.dinvD[1] = dinvdt;
  double yt = b, dyt = b;
#pragma unroll
  for (int j = 1; j <= D; ++j) {
    yt = __builtin_fma(-l[j], st.y[j], yt);
    dyt = __builtin_fma(-l[j], st.dy[j], __builtin_fma(-dl[j], st.y[j], dyt));
  }
#pragma unroll
  for (int j = D; j >= 2; --j) {
    st.y[j] = st.y[j - 1];
    st.dy[j] = st.dy[j - 1];
  }
  st.y[1] = yt;
  st.dy[1] = dyt;
  // half of d/deps (y^2 / Dp) = q (y' - q Dp' / 2) with q = y / Dp
  const double q = yt * invdt;
  const double half = __builtin_fma(-0.5 * q, ddd, dyt);
  st.ds = v ? __builtin_fma(q, half, st.ds) : st.ds;
  st.ed = v ? st.ed + e : st.ed;
}

template <int D, int B, typename TS, int G>
struct Gcv : Fast<D, 1, B, TS, false, false> {
  using Base = Fast<D, 1, B, TS, false, false>;
  using typename Base::Tile;

  // A tile is interior when every row it touches has the full weight window
  // (t0 >= D and t0 + B <= T - D): there row t of Omega is the constant row
  // omi (computed once per grid value) plus w_t on the diagonal, which is
  // what omega_row gives for a window of equal weights.
  __device__ __forceinline__ bool interior(int t0) const { return t0 >= D && t0 + B <= this->T - D; }

  __device__ __forceinline__ void interior_row(double lam, double (&omi)[D + 1]) const {
    double lwv[D + 1];
#pragma unroll
    for (int m = 0; m <= D; ++m) lwv[m] = lam;
    omega_row<D>(lwv, 0.0, omi);
  }

  // one tile for the G recurrences, step by step
  template <bool INT>
  __device__ __forceinline__ void tile_g(DualState<D> (&st)[G], const Tile& tl, int t0, const double (&lam)[G],
                                         const double (&omi)[G][D + 1], bool (&ok)[G], TS& shift, bool& have,
                                         double& sx, int& nobs) const {
    const int T = this->T;
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int t = t0 + s;
      const bool obs = tl.w[s] != 0u;
      const bool v = INT || t < T;
      // relative to the first observed value (rows before it have b = 0)
      shift = (obs && !have) ? tl.x[s][0] : shift;
      have = have || obs;
      const double xs = obs ? to_f64(tl.x[s][0]) - to_f64(shift) : 0.0;
      const double wt = obs ? 1.0 : 0.0;
      sx = __builtin_fma(xs, xs, sx);
      nobs += obs;
#pragma unroll
      for (int c = 0; c < G; ++c) {
        double om[D + 1];
        if constexpr (INT) {
#pragma unroll
          for (int i = 0; i <= D; ++i) om[i] = omi[c][i];
          om[0] += wt;
        } else {
          // lw[m] = lambda_{t-m}, zero outside the rows 0..T-D-1 of D
          double lwv[D + 1];
#pragma unroll
          for (int m = 0; m <= D; ++m) lwv[m] = (t - m >= 0 && t - m < T - D) ? lam[c] : 0.0;
          omega_row<D>(lwv, wt, om);
        }
        double dt;
        dual_step<D>(st[c], om, wt, xs, v, dt);
        ok[c] = ok[c] & (pivot_good(dt) | !v);
      }
    }
  }

  __device__ void run(const GcvArgs& g) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wave_off = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x + wave_off;
    if (p0 >= g.P) return;
    const int64_t bidx = p0 / g.S;
    const int s_in = (int)(p - bidx * g.S);
    this->T = g.T;
    this->S = g.S;
    this->Ctot = 1;
    this->c0 = 0;
    this->nt = g.nt;
    this->Rx = (uint32_t)g.S * sizeof(TS);
    this->xb = static_cast<const TS*>(g.x) + bidx * g.T * g.S;
    this->wb = g.w + bidx * g.T * g.S;
    this->lb = nullptr;
    this->zb = nullptr;
    this->ob = nullptr;
    this->gb = nullptr;
    this->ckb = nullptr;
    this->accum = false;
    const bool live = p < g.P;
    constexpr uint32_t kDead = 0x80000000u;
    this->lx = live ? (uint32_t)s_in * (uint32_t)sizeof(TS) : kDead;
    this->lw = live ? (uint32_t)s_in : kDead;
    this->lc = kDead;
    const int T = g.T, nt = g.nt;

    double best = __builtin_huge_val();
    int best_i = -1;
    int first_info = 0;
    for (int g0 = 0; g0 < g.n_grid; g0 += G) {
      // a last group past the end of the grid repeats its last value (scores unused)
      double lam[G], omi[G][D + 1];
      DualState<D> st[G];
      int bad_tile[G];
#pragma unroll
      for (int c = 0; c < G; ++c) {
        lam[c] = g.grid[g0 + c < g.n_grid ? g0 + c : g.n_grid - 1];
        interior_row(lam[c], omi[c]);
        st[c].zero();
        bad_tile[c] = -1;
      }
      TS shift = TS(0);
      bool have = false;
      double sx = 0.0;
      int nobs = 0;
      Tile A, Bt;
      this->template load_tile<false>(A, 0);
      for (int j = 0; j < nt; ++j) {
        this->template load_tile<false>(Bt, (j + 1) * B);
        bool ok[G];
#pragma unroll
        for (int c = 0; c < G; ++c) ok[c] = true;
        if (interior(j * B)) tile_g<true>(st, A, j * B, lam, omi, ok, shift, have, sx, nobs);
        else tile_g<false>(st, A, j * B, lam, omi, ok, shift, have, sx, nobs);
#pragma unroll
        for (int c = 0; c < G; ++c)
          if (!ok[c] && bad_tile[c] < 0) bad_tile[c] = j;
        A = Bt;
      }
      const double m = (double)nobs;
#pragma unroll
      for (int c = 0; c < G; ++c) {
        int info = 0;
        if (live && bad_tile[c] >= 0) {
          this->lam_scalar = lam[c];
          info = this->first_bad_pivot((bad_tile[c] + 1) * B);
        }
        if (info == 0 && nobs < D) info = T;
        const int gi = g0 + c;
        if (gi == 0) first_info = info;
        const double rss = sx - 2.0 * st[c].ds;
        const double den = m - st[c].ed;
        const double score = (info == 0) ? m * rss / (den * den) : __builtin_nan("");
        if (gi < g.n_grid) {
          if (live && g.scores) g.scores[p * g.n_grid + gi] = score;
          if (score < best) {  // NaN never wins; the first minimum is kept
            best = score;
            best_i = gi;
          }
        }
      }
    }
    if (live) {
      static_cast<TS*>(g.lam_best)[p] = from_f64<TS>(best_i >= 0 ? g.grid[best_i] : __builtin_nan(""));
      if (g.info) g.info[p] = best_i >= 0 ? 0 : first_info;
    }
  }
};

template <int D, int B, typename TS, int G>
__global__ __launch_bounds__(256) void k_gcv(GcvArgs a) {
  Gcv<D, B, TS, G> k;
  k.run(a);
}

}  // namespace whs

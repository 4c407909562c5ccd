// Two lanes per series (uneven-batch plan): a series' rows are split at a
// separator S = [m, m+d) of d rows.  The top part [0, m+d) is factored in time
// order; the bottom part [m, T) is factored on the time-reversed series:
// reversing time maps Omega to the smoother matrix of the reversed weights,
// J Omega J = J W J + (D J)^T Lambda (D J) with D J = (-1)^d J' D on the daily
// grid, so the same recurrence (Sec. III-A) applies to the reversed rows and
// reversed weights.  Both parts continue through S, so each ends holding the
// last d rows of its factor, which give its Schur contribution on S:
//   Lp Dp Lp^T = Omega_SS - E^T A^{-1} E,    Lp yp = b_S - E^T A^{-1} b,
// (A the part's interior block, E its coupling to S).  Summing both and
// removing the Omega_SS counted twice gives the separator system
//   (Yt + Yb - Omega_SS) z_S = ct + cb - b_S,
// which both lanes solve with the same operations (the same z_S), and each
// part back-substitutes its interior from z_S.  This is Cholesky of a
// symmetric permutation of Omega (interiors first, S last), so it keeps the
// accuracy of the sequential sweep, and it halves the dependent chain of a
// long series.  Forward solve, one band, daily grid.
//
// Each part runs on its own virtual rows v in [-pad, Tv): Tv = m+d (top) or
// T-m (bottom), physical row v (top) or T-1-v (bottom).  The pad rows in front
// align the last tile with the end of S, so S sits at fixed positions of the
// last tile; they are identity rows (w = 1, x = 0, no weight), which leave the
// factor of the real rows unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include "whs_fast.h"
#include "whs_step.h"

namespace whs {

// Per-lane separator data of one part, physical order of S: the lower
// triangle of its Schur term (d(d+1)/2 values) and its right-hand side (d).
template <int D>
struct SepPart {
  double Y[D * (D + 1) / 2];
  double c[D];
};

template <int D>
__device__ __forceinline__ int tri(int r, int q) { return r * (r + 1) / 2 + q; }  // r >= q

template <int D, int B, typename TS, bool PERDIFF>
struct Twist {
  static constexpr int NF = ck_fields<D, 1>();
  static constexpr uint32_t ES = sizeof(TS);

  struct Tile {
    TS x[B];
    uint32_t w[B];
    TS lam[B];
  };

  // wave-uniform
  const TS* xb;      // first row of the block, x
  const uint8_t* wb;
  const TS* lb;      // per-difference weights of the block
  TS* zb;
  double* ckb;
  int T, m, Tv, pad, ntv, S;
  bool rev;
  uint32_t Rx;       // bytes per row of x / z
  // per lane
  uint32_t lx, lw, lc;
  double lam_scalar;

  // physical row of virtual row v, and the row of D whose weight enters at v
  __device__ __forceinline__ int prow(int v) const { return rev ? T - 1 - v : v; }
  __device__ __forceinline__ int krow(int v) const { return rev ? T - D - 1 - v : v; }

  // Rows of the tile at virtual v0 that lie inside the part, [0, Tv): the first
  // physical row of that span (`base`, 0 when empty), their count, and K0 such
  // that element s of the tile is row K0 + s (time order) or K0 - s (reversed)
  // of the span; elements outside it fall outside the buffer range and read as
  // zero.  Tiles past either end of the part (prefetches, pad rows) never
  // address rows outside it.
  __device__ __forceinline__ void span(int v0, int& base, int& nrows, int& K0) const {
    const int vs = v0 > 0 ? v0 : 0;
    const int ve = (v0 + B < Tv) ? v0 + B : Tv;
    nrows = ve > vs ? ve - vs : 0;
    if (nrows == 0) {
      base = 0;
      K0 = -B;  // every element off the (empty) span
    } else if (!rev) {
      base = vs;
      K0 = v0 - vs;
    } else {
      base = T - ve;
      K0 = ve - 1 - v0;
    }
  }

  // tile of virtual rows [v0, v0+B); rows outside the part read as zero
  __device__ __forceinline__ void load_tile(Tile& tl, int v0) const {
    int base, nrows, K0;
    span(v0, base, nrows, K0);
    const auto rx = make_rsrc(xb + (int64_t)base * S, (uint32_t)nrows * Rx);
    const auto rw = make_rsrc(wb + (int64_t)base * S, (uint32_t)nrows * S);
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int r = rev ? K0 - s : K0 + s;  // row within the span; negative wraps past the range
      tl.x[s] = bload<TS>(rx, lx + (uint32_t)r * Rx);
      tl.w[s] = __builtin_amdgcn_raw_buffer_load_b8(rw, lw + (uint32_t)r * (uint32_t)S, 0, 0);
    }
    if constexpr (PERDIFF) {
      // rows of D entering at the tile's rows inside the part: k = v (time
      // order) or T-D-1-v (reversed), kept within 0..T-D-1
      const int Td = T - D;
      const int vs = v0 > 0 ? v0 : 0;
      const int ve = (v0 + B < Tv) ? v0 + B : Tv;
      int kb = 0, kn = 0, k0 = -B;
      if (ve > vs) {
        if (!rev) {
          kb = vs;
          const int ke = ve < Td ? ve : Td;
          kn = ke > kb ? ke - kb : 0;
          k0 = v0 - kb;
        } else {
          const int hi = Td - 1 - vs, lo = Td - ve;  // rows of D at v = vs and v = ve-1
          kb = lo > 0 ? lo : 0;
          kn = hi >= kb ? hi - kb + 1 : 0;
          k0 = Td - 1 - v0 - kb;
        }
        if (kn == 0) {
          kb = 0;
          k0 = -B;
        }
      }
      const auto rl = make_rsrc(lb + (int64_t)(kn > 0 ? kb : 0) * S, (uint32_t)kn * S * ES);
#pragma unroll
      for (int s = 0; s < B; ++s) {
        const int r = rev ? k0 - s : k0 + s;
        tl.lam[s] = bload<TS>(rl, lx + (uint32_t)r * (uint32_t)S * ES);
      }
    }
  }

  __device__ __forceinline__ double lam_at(const Tile& tl, int s, int v) const {
    if constexpr (PERDIFF) {
      return to_f64(tl.lam[s]);
    } else {
      const int k = krow(v);
      return (v >= 0 && k >= 0 && k < T - D) ? lam_scalar : 0.0;
    }
  }

  __device__ __forceinline__ void step(State<D, 1>& st, const Tile& tl, int s, int v, double (&l)[D + 1],
                                       double& dt, double& invdt, double& yt) const {
    const bool obs = tl.w[s] != 0u || v < 0;  // pad rows are identity rows
    const double lt = lam_at(tl, s, v);
    double lwv[D + 1];
    lwv[0] = lt;
#pragma unroll
    for (int q = 1; q <= D; ++q) lwv[q] = st.lw[q];
    double om[D + 1];
    omega_row<D>(lwv, obs ? 1.0 : 0.0, om);
    ldl_step<D, 1>(st, om, l, dt, invdt);
#pragma unroll
    for (int q = D; q >= 2; --q) st.lw[q] = st.lw[q - 1];
    st.lw[1] = lt;
    double b[1] = {to_f64(obs ? tl.x[s] : TS(0))};
    double y1[1];
    fwd_step<D, 1>(st, l, b, y1);
    yt = y1[0];
  }

  __device__ __forceinline__ void store_ck(const State<D, 1>& st, int j) const {
    const auto r = make_rsrc(ckb, (uint32_t)ntv * NF * 64 * 8u);
    const uint32_t base = lc + (uint32_t)(j * NF) * 64u * 8u;
    int f = 0;
#pragma unroll
    for (int jj = 1; jj <= D; ++jj) bstore<double, kStream>(r, base + (uint32_t)(f++ * 64 * 8), st.invD[jj]);
#pragma unroll
    for (int jj = 1; jj < D; ++jj)
#pragma unroll
      for (int k = 1; k <= D - jj; ++k) bstore<double, kStream>(r, base + (uint32_t)(f++ * 64 * 8), st.R[jj][k]);
#pragma unroll
    for (int jj = 1; jj <= D; ++jj) bstore<double, kStream>(r, base + (uint32_t)(f++ * 64 * 8), st.y[jj][0]);
  }

  // state at the start of tile j: checkpoint plus the weights of the D rows before it
  __device__ __forceinline__ void restore(State<D, 1>& st, int j) const {
    const auto r = make_rsrc(ckb, (uint32_t)ntv * NF * 64 * 8u);
    const uint32_t base = lc + (uint32_t)(j * NF) * 64u * 8u;
    int f = 0;
#pragma unroll
    for (int jj = 1; jj <= D; ++jj) st.invD[jj] = bload<double, kStream>(r, base + (uint32_t)(f++ * 64 * 8));
#pragma unroll
    for (int jj = 1; jj < D; ++jj)
#pragma unroll
      for (int k = 1; k <= D - jj; ++k) st.R[jj][k] = bload<double, kStream>(r, base + (uint32_t)(f++ * 64 * 8));
#pragma unroll
    for (int jj = 1; jj <= D; ++jj) st.y[jj][0] = bload<double, kStream>(r, base + (uint32_t)(f++ * 64 * 8));
    const int v0 = -pad + j * B;
    st.lw[0] = 0.0;
    const auto rl = make_rsrc(lb ? (const void*)lb : (const void*)wb, PERDIFF ? (uint32_t)(T - D) * S * ES : 0u);
#pragma unroll
    for (int q = 1; q <= D; ++q) {
      const int v = v0 - q;
      const int k = krow(v);
      const bool ok = v >= 0 && k >= 0 && k < T - D;
      if constexpr (PERDIFF) {
        st.lw[q] = to_f64(bload<TS>(rl, ok ? lx + (uint32_t)k * (uint32_t)S * ES : 0x80000000u));
      } else {
        st.lw[q] = ok ? lam_scalar : 0.0;
      }
    }
  }

  // Sweep 1 over every tile; returns false if a pivot failed.  On return `st`
  // holds the last D rows of the part's factor (the rows of S).
  __device__ bool sweep1(State<D, 1>& st, int& nobs, int nobs_to) const {
    st.zero();
    bool ok = true;
    Tile A, Bt;
    load_tile(A, -pad);
    for (int j = 0; j < ntv; j += 2) {
      load_tile(Bt, -pad + (j + 1) * B);
      store_ck(st, j);
      ok = ok & fwd_tile(st, A, -pad + j * B, nobs, nobs_to);
      load_tile(A, -pad + (j + 2) * B);
      if (j + 1 < ntv) {
        store_ck(st, j + 1);
        ok = ok & fwd_tile(st, Bt, -pad + (j + 1) * B, nobs, nobs_to);
      }
    }
    return ok;
  }

  __device__ __forceinline__ bool fwd_tile(State<D, 1>& st, const Tile& tl, int v0, int& nobs, int nobs_to) const {
    bool ok = true;
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int v = v0 + s;
      double l[D + 1], dt, invdt, yt;
      step(st, tl, s, v, l, dt, invdt, yt);
      nobs += (tl.w[s] != 0u && v >= 0 && v < nobs_to) ? 1 : 0;
      ok = ok & pivot_good(dt);
    }
    return ok;
  }

  // Schur term and right-hand side of this part on S, physical order of S.
  __device__ void separator_part(const State<D, 1>& st, SepPart<D>& out) const {
    // virtual order: S rows u = 0..D-1 are virtual rows Tv-D+u; the state
    // after the last of them holds invD[j] = 1/Dp at u = D-j and
    // R[j][k] = L[u, u-k] at u = D-j
    double L[D][D], Dp[D], y[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
#pragma unroll
      for (int q = 0; q < D; ++q) L[u][q] = (q == u) ? 1.0 : 0.0;
      Dp[u] = 1.0 / st.invD[D - u];
      y[u] = st.y[D - u][0];
    }
#pragma unroll
    for (int jj = 1; jj < D; ++jj)
#pragma unroll
      for (int k = 1; k <= D - jj; ++k) L[D - jj][D - jj - k] = st.R[jj][k];
    // Y = L Dp L^T, c = L y (virtual order), then to physical order of S
    // (reversed for the bottom part; indices stay compile-time constants)
    double Yv[D][D], cv[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
      double cu = 0.0;
#pragma unroll
      for (int q = 0; q <= u; ++q) cu = __builtin_fma(L[u][q], y[q], cu);
      cv[u] = cu;
#pragma unroll
      for (int u2 = 0; u2 <= u; ++u2) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q <= u2; ++q) a = __builtin_fma(L[u][q] * Dp[q], L[u2][q], a);
        Yv[u][u2] = a;
        Yv[u2][u] = a;
      }
    }
#pragma unroll
    for (int r = 0; r < D; ++r) {
      out.c[r] = rev ? cv[D - 1 - r] : cv[r];
#pragma unroll
      for (int r2 = 0; r2 <= r; ++r2) out.Y[tri<D>(r, r2)] = rev ? Yv[D - 1 - r][D - 1 - r2] : Yv[r][r2];
    }
  }

  // Omega_SS (lower triangle) and b_S of the physical rows m..m+D-1.
  __device__ void separator_omega(double (&Om)[D * (D + 1) / 2], double (&bS)[D]) const {
    const auto rw = make_rsrc(wb, (uint32_t)T * S);
    const auto rx = make_rsrc(xb, (uint32_t)T * Rx);
    const auto rl = make_rsrc(lb ? (const void*)lb : (const void*)wb, PERDIFF ? (uint32_t)(T - D) * S * ES : 0u);
#pragma unroll
    for (int i = 0; i < D * (D + 1) / 2; ++i) Om[i] = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      const int t = m + r;
      const bool obs = __builtin_amdgcn_raw_buffer_load_b8(rw, lw + (uint32_t)t * (uint32_t)S, 0, 0) != 0u;
      Om[tri<D>(r, r)] += obs ? 1.0 : 0.0;
      bS[r] = obs ? to_f64(bload<TS>(rx, lx + (uint32_t)t * Rx)) : 0.0;
    }
    // rows k of D touching S twice: lambda_k c_{t-k} c_{t'-k} for t, t' in S
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) {
      const int k = m - D + q;
      const bool ok = k >= 0 && k < T - D;
      double lk;
      if constexpr (PERDIFF) {
        lk = to_f64(bload<TS>(rl, ok ? lx + (uint32_t)k * (uint32_t)S * ES : 0x80000000u));
      } else {
        lk = ok ? lam_scalar : 0.0;
      }
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int r2 = 0; r2 <= r; ++r2) {
          const int a = m + r - k, b = m + r2 - k;  // positions in row k
          if (a >= 0 && a <= D && b >= 0 && b <= D) Om[tri<D>(r, r2)] = __builtin_fma(lk, cdiff<D>(a) * cdiff<D>(b), Om[tri<D>(r, r2)]);
        }
    }
  }

  // Sweep 2: reverse tiles over the part, z of S given in virtual order.
  __device__ void sweep2(const double (&zSv)[D], bool failed, bool store_S) const {
    double zn[D + 1], lcr[D + 1][D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      zn[i] = 0.0;
#pragma unroll
      for (int k = 0; k <= D; ++k) lcr[i][k] = 0.0;
    }
    Tile A, Bt;
    int j = ntv - 1;
    load_tile(A, -pad + j * B);
    rev_tile<true>(A, j, zSv, zn, lcr, failed, store_S);
    for (j = ntv - 2; j >= 0; j -= 2) {
      load_tile(Bt, -pad + j * B);
      if (j - 1 >= 0) load_tile(A, -pad + (j - 1) * B);
      rev_tile<false>(Bt, j, zSv, zn, lcr, failed, store_S);
      if (j - 1 >= 0) rev_tile<false>(A, j - 1, zSv, zn, lcr, failed, store_S);
    }
  }

  template <bool LAST>
  __device__ __forceinline__ void rev_tile(const Tile& tl, int j, const double (&zSv)[D], double (&zn)[D + 1],
                                           double (&lc_)[D + 1][D + 1], bool failed, bool store_S) const {
    State<D, 1> st;
    restore(st, j);
    const int v0 = -pad + j * B;
    double lt[B][D + 1];
    double yd[B];
#pragma unroll
    for (int s = 0; s < B; ++s) {
      double l[D + 1], dt, invdt, yt;
      step(st, tl, s, v0 + s, l, dt, invdt, yt);
#pragma unroll
      for (int i = 1; i <= D; ++i) lt[s][i] = l[i];
      yd[s] = yt * invdt;
    }
    int base, nrows, K0;
    span(v0, base, nrows, K0);
    // the S rows of the last tile are stored by one part only
    const int nst = (LAST && !store_S) ? (rev ? nrows - D : nrows) : nrows;
    const int sh = (LAST && !store_S && rev) ? D : 0;  // bottom: S rows are the lowest physical rows of its range
    const auto ro = make_rsrc(zb + (int64_t)(base + sh) * S, (uint32_t)(nst > 0 ? nst : 0) * Rx);
    const double qnan = __builtin_nan("");
#pragma unroll
    for (int s = B - 1; s >= 0; --s) {
      double zt;
      if (LAST && s >= B - D) {
        zt = zSv[s - (B - D)];
      } else {
        double acc = yd[s];
#pragma unroll
        for (int i = 1; i <= D; ++i) {
          const double li = (s + i < B) ? lt[s + i < B ? s + i : 0][i] : lc_[s + i - B < 0 ? 0 : s + i - B][i];
          acc = __builtin_fma(-li, zn[i], acc);
        }
        zt = acc;
      }
      const int r = (rev ? K0 - s : K0 + s) - sh;
      bstore<TS, kStream>(ro, lx + (uint32_t)r * Rx, from_f64<TS>(failed ? qnan : zt));
#pragma unroll
      for (int i = D; i >= 2; --i) zn[i] = zn[i - 1];
      zn[1] = zt;
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int i = 0; i <= D; ++i) lc_[r][i] = lt[r][i];
  }

  // exact index of the first failing pivot of the whole series, time order
  __device__ int first_bad_pivot() const {
    State<D, 1> st;
    st.zero();
    const auto rw = make_rsrc(wb, (uint32_t)T * S);
    const auto rl = make_rsrc(lb ? (const void*)lb : (const void*)wb, PERDIFF ? (uint32_t)(T - D) * S * ES : 0u);
    for (int t = 0; t < T; ++t) {
      const bool obs = __builtin_amdgcn_raw_buffer_load_b8(rw, lw + (uint32_t)(t * S), 0, 0) != 0;
      const double ltv = PERDIFF ? to_f64(bload<TS>(rl, lx + (uint32_t)(t * S) * ES)) : (t < T - D ? lam_scalar : 0.0);
      double lwv[D + 1];
      lwv[0] = ltv;
      for (int q = 1; q <= D; ++q) lwv[q] = st.lw[q];
      double om[D + 1], l[D + 1], dt, invdt;
      omega_row<D>(lwv, obs ? 1.0 : 0.0, om);
      ldl_step<D, 1>(st, om, l, dt, invdt);
      for (int q = D; q >= 2; --q) st.lw[q] = st.lw[q - 1];
      st.lw[1] = ltv;
      if (!pivot_good(dt)) return t + 1;
    }
    return 0;
  }
};

// LDL^T solve of the D x D separator system (lower triangle given); false if
// a pivot is not positive and finite.
template <int D>
__device__ __forceinline__ bool solve_separator(const double (&A)[D * (D + 1) / 2], const double (&rhs)[D],
                                                double (&z)[D]) {
  double L[D][D], Dp[D], y[D];
  bool ok = true;
#pragma unroll
  for (int r = 0; r < D; ++r) {
#pragma unroll
    for (int q = 0; q < r; ++q) {
      double a = A[tri<D>(r, q)];
#pragma unroll
      for (int p = 0; p < q; ++p) a = __builtin_fma(-L[r][p] * Dp[p], L[q][p], a);
      L[r][q] = a / Dp[q];
    }
    double dd = A[tri<D>(r, r)];
#pragma unroll
    for (int p = 0; p < r; ++p) dd = __builtin_fma(-L[r][p] * Dp[p], L[r][p], dd);
    Dp[r] = dd;
    ok = ok & pivot_good(dd);
  }
#pragma unroll
  for (int r = 0; r < D; ++r) {
    double a = rhs[r];
#pragma unroll
    for (int p = 0; p < r; ++p) a = __builtin_fma(-L[r][p], y[p], a);
    y[r] = a;
  }
#pragma unroll
  for (int r = D - 1; r >= 0; --r) {
    double a = y[r] / Dp[r];
#pragma unroll
    for (int p = r + 1; p < D; ++p) a = __builtin_fma(-L[p][r], z[p], a);
    z[r] = a;
  }
  return ok;
}

}  // namespace whs

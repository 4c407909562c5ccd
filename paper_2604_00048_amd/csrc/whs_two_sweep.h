#pragma once
// Fused banded Whittaker-Henderson solve and its adjoint for gfx950 (templates).
//
// One lane = one series; the interleaved time-major layout makes the time-t
// values of the S series of a block one contiguous row, so every load and
// store of a wavefront is a single coalesced transaction.  Each kernel runs
// two sweeps per series (Sec. III-A):
//
//   sweep 1 (t ascending)  assemble row t of Omega, one LDL^T step, one
//                          forward-substitution step; every B steps the
//                          recurrence state is checkpointed to the workspace.
//   sweep 2 (tiles in reverse) restore the tile's checkpoint, recompute the
//                          tile's factor rows and y into registers, then back
//                          substitute t descending and store the result.
//
// The factor is never stored: sweep 2 re-reads the tile inputs (a tile of B
// steps is B coalesced rows) instead of writing and reading (d+1+C) FP64
// values per step.  Tile inputs are prefetched one tile ahead into
// registers.
#include <hip/hip_runtime.h>

#include "whs_fast.h"
#include "whs_kernels.h"
#include "whs_step.h"

namespace whs {

enum class Src { Fused, Factor };
enum class Mode { Solve, Backward };

struct Args {
  int64_t P;
  int T;
  int S;
  int Ctot;   // RHS count of the arrays
  int c0;     // first RHS handled by this launch
  int nt;     // tiles per series
  const uint8_t* w;
  const void* lam;
  const double* fac;
  const void* rhs;   // x (solve) or g (backward)
  const void* zin;   // z (backward)
  void* out;         // z (solve) or grad_x (backward)
  void* glam;        // grad_lambda (backward)
  int32_t* info;
  double* ck;        // workspace: [b][tile][field][S]
  int write_info;    // only the first RHS group writes info
  int glam_accum;    // later RHS groups add their share of grad_lambda
};

template <int D, int C, int B, typename TS, Src SRC, Mode MODE, bool PERDIFF>
struct Kern {
  static constexpr int NF = ck_fields<D, C>();
  static constexpr bool FUSED = SRC == Src::Fused;
  static constexpr bool BWD = MODE == Mode::Backward;

  struct Tile {
    uint32_t w[B];
    TS lam[B];
    TS r[B][C];
    double f[B][D + 1];
    TS z[B][C];
  };

  // Per-series views.
  const uint8_t* ws;   // w[t] at ws[t*S]
  const TS* ls;        // lambda_t at ls[t*S] (per-difference) or *ls (scalar)
  const double* fs;    // factor[i][t] at fs[(i*T + t)*S]
  const TS* rs;        // rhs[t][c] at rs[(t*Ctot + c)*S]
  const TS* zs;        // z[t][c]
  TS* os;              // out[t][c]
  TS* gls;             // grad_lambda
  double* cks;         // checkpoint j field f at cks[(j*NF + f)*S]
  int T, S, Ctot;
  bool accum;
  double lam_scalar;

  // ---- loads -------------------------------------------------------------
  template <bool FULL, bool SWEEP2>
  __device__ __forceinline__ void load_tile(Tile& tl, int t0) const {
    const int Td = T - D;
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int t = t0 + s;
      const bool v = FULL || t < T;
      tl.w[s] = v ? static_cast<uint32_t>(ws[(int64_t)t * S]) : 0u;
      if constexpr (FUSED && PERDIFF) {
        const bool vl = FULL || t < Td;
        tl.lam[s] = vl ? ls[(int64_t)t * S] : TS(0);
      }
#pragma unroll
      for (int c = 0; c < C; ++c) tl.r[s][c] = v ? rs[((int64_t)t * Ctot + c) * S] : TS(0);
      if constexpr (!FUSED) {
#pragma unroll
        for (int i = 0; i <= D; ++i) {
          const int tt = t - i;
          const bool vi = (FULL || t < T) && tt >= 0;
          tl.f[s][i] = vi ? fs[((int64_t)i * T + tt) * S] : 0.0;
        }
      }
      if constexpr (BWD && SWEEP2) {
#pragma unroll
        for (int c = 0; c < C; ++c) tl.z[s][c] = v ? zs[((int64_t)t * Ctot + c) * S] : TS(0);
      }
    }
  }

  // ---- one step of sweep 1 / of the tile recompute -------------------------
  // Returns l[] = L[t, t-j], invdt = 1/Dp[t] and y_t; updates the state.
  template <bool FULL>
  __device__ __forceinline__ void step(State<D, C>& st, const Tile& tl, int s, int t, double (&l)[D + 1],
                                       double& dt, double& invdt, double (&yt)[C]) const {
    const bool obs = tl.w[s] != 0u;
    if constexpr (FUSED) {
      double lw[D + 1];
      double lt;
      if constexpr (PERDIFF) {
        lt = to_f64(tl.lam[s]);  // zero beyond T-D-1 (load predicate)
      } else {
        lt = (FULL || t < T - D) ? lam_scalar : 0.0;
      }
      lw[0] = lt;
#pragma unroll
      for (int m = 1; m <= D; ++m) lw[m] = st.lw[m];
      double om[D + 1];
      omega_row<D>(lw, obs ? 1.0 : 0.0, om);
      ldl_step<D, C>(st, om, l, dt, invdt);
#pragma unroll
      for (int m = D; m >= 2; --m) st.lw[m] = st.lw[m - 1];
      st.lw[1] = lt;
    } else {
      // Factor given in Cholesky form F[i][t] = Lc[t+i, t]:
      // L[t, t-j] = F[j][t-j] / F[0][t-j], Dp[t] = F[0][t]^2.
      const double f0 = tl.f[s][0];
      const double i0 = rcp64(f0);
#pragma unroll
      for (int j = 1; j <= D; ++j) l[j] = tl.f[s][j] * st.invD[j];
      dt = f0;
      invdt = i0 * i0;
#pragma unroll
      for (int j = D; j >= 2; --j) st.invD[j] = st.invD[j - 1];
      st.invD[1] = i0;
    }
    double b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double v = to_f64(tl.r[s][c]);
      b[c] = BWD ? v : (obs ? v : 0.0);
    }
    fwd_step<D, C>(st, l, b, yt);
  }

  // Restore the state at the start of tile j (j >= 1).
  __device__ __forceinline__ void restore(State<D, C>& st, int j, const double (&ckv)[NF],
                                          const double (&lwin)[D + 1]) const {
    int f = 0;
#pragma unroll
    for (int jj = 1; jj <= D; ++jj) st.invD[jj] = ckv[f++];
#pragma unroll
    for (int jj = 1; jj < D; ++jj)
#pragma unroll
      for (int k = 1; k <= D - jj; ++k) st.R[jj][k] = ckv[f++];
#pragma unroll
    for (int jj = 1; jj <= D; ++jj)
#pragma unroll
      for (int c = 0; c < C; ++c) st.y[jj][c] = ckv[f++];
#pragma unroll
    for (int m = 0; m <= D; ++m) st.lw[m] = lwin[m];
  }

  __device__ __forceinline__ void load_ck(int j, double (&ckv)[NF], double (&lwin)[D + 1]) const {
    const int t0 = j * B;
#pragma unroll
    for (int f = 0; f < NF; ++f) ckv[f] = cks[((int64_t)j * NF + f) * S];
    lwin[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= D; ++m) {
      const int k = t0 - m;  // >= 0 since B >= D and j >= 1
      if constexpr (FUSED && PERDIFF) {
        lwin[m] = (k < T - D) ? to_f64(ls[(int64_t)k * S]) : 0.0;
      } else {
        lwin[m] = (k < T - D) ? lam_scalar : 0.0;
      }
    }
  }

  __device__ __forceinline__ bool full_tile(int t0) const { return t0 + B <= T - D; }

  // ---- the kernel body -------------------------------------------------------
  __device__ void run(const Args& a, int64_t p) {
    const int64_t bidx = p / a.S;
    const int sl = static_cast<int>(p - bidx * a.S);
    T = a.T;
    S = a.S;
    Ctot = a.Ctot;
    const int nt = a.nt;
    ws = a.w + (int64_t)bidx * T * S + sl;
    if constexpr (FUSED) {
      if constexpr (PERDIFF) {
        ls = static_cast<const TS*>(a.lam) + (int64_t)bidx * (T - D) * S + sl;
        lam_scalar = 0.0;
      } else {
        ls = nullptr;
        lam_scalar = to_f64(static_cast<const TS*>(a.lam)[p]);
      }
      fs = nullptr;
    } else {
      ls = nullptr;
      lam_scalar = 0.0;
      fs = a.fac + (int64_t)bidx * (D + 1) * T * S + sl;
    }
    rs = static_cast<const TS*>(a.rhs) + ((int64_t)bidx * T * Ctot + a.c0) * S + sl;
    zs = BWD ? static_cast<const TS*>(a.zin) + ((int64_t)bidx * T * Ctot + a.c0) * S + sl : nullptr;
    os = a.out ? static_cast<TS*>(a.out) + ((int64_t)bidx * T * Ctot + a.c0) * S + sl : nullptr;
    gls = nullptr;
    accum = a.glam_accum != 0;
    if (BWD && a.glam) {
      gls = PERDIFF ? static_cast<TS*>(a.glam) + (int64_t)bidx * (T - D) * S + sl
                    : static_cast<TS*>(a.glam) + p;
    }
    cks = a.ck + (int64_t)bidx * nt * NF * S + sl;

    // ---------------- sweep 1 ----------------
    State<D, C> st;
    st.zero();
    int info = 0;
    int nobs = 0;
    Tile cur, nxt;
    if (full_tile(0)) load_tile<true, false>(cur, 0); else load_tile<false, false>(cur, 0);
    for (int j = 0; j < nt; ++j) {
      const int t0 = j * B;
      if (j + 1 < nt) {
        if (full_tile(t0 + B)) load_tile<true, false>(nxt, t0 + B); else load_tile<false, false>(nxt, t0 + B);
      }
      if (j > 0) ck_store<D, C>(st, cks + (int64_t)j * NF * S, S);
      if (full_tile(t0)) {
#pragma unroll
        for (int s = 0; s < B; ++s) {
          double l[D + 1], dt, invdt, yt[C];
          step<true>(st, cur, s, t0 + s, l, dt, invdt, yt);
          nobs += cur.w[s] != 0u;
          if (!pivot_ok(dt) && info == 0) info = t0 + s + 1;
        }
      } else {
#pragma unroll
        for (int s = 0; s < B; ++s) {
          const int t = t0 + s;
          if (t < T) {
            double l[D + 1], dt, invdt, yt[C];
            step<false>(st, cur, s, t, l, dt, invdt, yt);
            nobs += cur.w[s] != 0u;
            if (!pivot_ok(dt) && info == 0) info = t + 1;
          }
        }
      }
      cur = nxt;
    }
    if (info == 0 && FUSED && nobs < D) info = T;
    const bool failed = info != 0;
    if (a.info && a.write_info) a.info[p] = info;

    // ---------------- sweep 2 ----------------
    const double qnan = __builtin_nan("");
    double zn[D + 1][C];   // result at t+1..t+D
    double xn[D + 1][C];   // backward: z input at t+1..t+D
    double lc[D + 1][D + 1];  // l rows of the first D steps of the following tile
#pragma unroll
    for (int i = 0; i <= D; ++i) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        zn[i][c] = 0.0;
        xn[i][c] = 0.0;
      }
#pragma unroll
      for (int k = 0; k <= D; ++k) lc[i][k] = 0.0;
    }
    double gsum = 0.0;
    double ckc[NF], ckn[NF], lwc[D + 1], lwn[D + 1];
#pragma unroll
    for (int f = 0; f < NF; ++f) ckn[f] = 0.0;
#pragma unroll
    for (int m = 0; m <= D; ++m) lwn[m] = 0.0;
    {
      const int j = nt - 1;
      if (full_tile(j * B)) load_tile<true, true>(cur, j * B); else load_tile<false, true>(cur, j * B);
      if (j > 0) load_ck(j, ckc, lwc);
    }
    for (int j = nt - 1; j >= 0; --j) {
      const int t0 = j * B;
      if (j > 0) {
        const int tp = t0 - B;
        if (full_tile(tp)) load_tile<true, true>(nxt, tp); else load_tile<false, true>(nxt, tp);
        if (j > 1) load_ck(j - 1, ckn, lwn);
      }
      State<D, C> rs_;
      if (j > 0) restore(rs_, j, ckc, lwc); else rs_.zero();
      double lt[B][D + 1];
      double yd[B][C];
      const bool full = full_tile(t0);
#pragma unroll
      for (int s = 0; s < B; ++s) {
        const int t = t0 + s;
        double l[D + 1], dt, invdt, yt[C];
        if (full) {
          step<true>(rs_, cur, s, t, l, dt, invdt, yt);
        } else {
          step<false>(rs_, cur, s, t, l, dt, invdt, yt);
        }
        const bool v = full || t < T;
#pragma unroll
        for (int i = 1; i <= D; ++i) lt[s][i] = v ? l[i] : 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) yd[s][c] = v ? yt[c] * invdt : 0.0;
      }
      // back substitution, t descending
#pragma unroll
      for (int s = B - 1; s >= 0; --s) {
        const int t = t0 + s;
        double zt[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          double acc = yd[s][c];
#pragma unroll
          for (int i = 1; i <= D; ++i) {
            const double li = (s + i < B) ? lt[s + i < B ? s + i : 0][i] : lc[s + i - B < 0 ? 0 : s + i - B][i];
            acc = __builtin_fma(-li, zn[i][c], acc);
          }
          zt[c] = acc;
        }
        const bool v = full || t < T;
        if constexpr (!BWD) {
          if (v && os) {
#pragma unroll
            for (int c = 0; c < C; ++c) os[((int64_t)t * Ctot + c) * S] = from_f64<TS>(failed ? qnan : zt[c]);
          }
        } else {
          const bool obs = cur.w[s] != 0u;
          if (v && os) {
#pragma unroll
            for (int c = 0; c < C; ++c)
              os[((int64_t)t * Ctot + c) * S] = from_f64<TS>(failed ? qnan : (obs ? zt[c] : 0.0));
          }
          // grad_lambda_t = -sum_c (D u_c)_t (D z_c)_t  for t <= T-D-1
          double zin[C];
#pragma unroll
          for (int c = 0; c < C; ++c) zin[c] = to_f64(cur.z[s][c]);
          double gt = 0.0;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            double du = cdiff<D>(0) * zt[c];
            double dz = cdiff<D>(0) * zin[c];
#pragma unroll
            for (int i = 1; i <= D; ++i) {
              du = __builtin_fma(cdiff<D>(i), zn[i][c], du);
              dz = __builtin_fma(cdiff<D>(i), xn[i][c], dz);
            }
            gt = __builtin_fma(-du, dz, gt);
          }
          const bool vk = full || t < T - D;
          if constexpr (PERDIFF) {
            if (vk && gls) {
              const int64_t o = (int64_t)t * S;
              const double prev = accum ? to_f64(gls[o]) : 0.0;
              gls[o] = from_f64<TS>(failed ? qnan : prev + gt);
            }
          } else {
            gsum += vk ? gt : 0.0;
          }
          if (v) {
#pragma unroll
            for (int i = D; i >= 2; --i)
#pragma unroll
              for (int c = 0; c < C; ++c) xn[i][c] = xn[i - 1][c];
#pragma unroll
            for (int c = 0; c < C; ++c) xn[1][c] = zin[c];
          }
        }
        if (v) {
#pragma unroll
          for (int i = D; i >= 2; --i)
#pragma unroll
            for (int c = 0; c < C; ++c) zn[i][c] = zn[i - 1][c];
#pragma unroll
          for (int c = 0; c < C; ++c) zn[1][c] = zt[c];
        }
      }
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int i = 0; i <= D; ++i) lc[r][i] = (r < B) ? lt[r < B ? r : 0][i] : 0.0;
      cur = nxt;
#pragma unroll
      for (int f = 0; f < NF; ++f) ckc[f] = ckn[f];
#pragma unroll
      for (int m = 0; m <= D; ++m) lwc[m] = lwn[m];
    }
    if constexpr (BWD && !PERDIFF) {
      if (gls) {
        const double prev = accum ? to_f64(*gls) : 0.0;
        *gls = from_f64<TS>(failed ? qnan : prev + gsum);
      }
    }
  }
};

template <int D, int C, int B, typename TS, Src SRC, Mode MODE, bool PERDIFF>
__global__ __launch_bounds__(256) void k_two_sweep(Args a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  Kern<D, C, B, TS, SRC, MODE, PERDIFF> k;
  k.run(a, p);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

// Steps per tile: the deepest tile whose kernel compiles without register
// spills for this order, band group and storage type (ES bytes per value).
// The uneven-time kernels also carry a window of D's rows.
template <int D, int C, bool TAB = false, int ES = 4>
constexpr int tile_depth() {
  if (C != 1) return 8;
  if (TAB) return D == 1 ? 16 : D == 4 ? 8 : 12;  // as deep as the adjoint with a weight per difference row
  if (D <= 2) return ES == 4 ? 24 : 16;
  if (D == 3) return ES == 4 ? 16 : 12;
  return 12;
}

// The fast solve of 2 or 3 bands in FP32 storage (order <= 2, even times) has
// room for 16 steps: two bands with either weight kind, three with one weight
// per series.  With uneven times, one band takes 16 steps (order <= 2) or 12
// except in the adjoint with a weight per difference row, and the solve of a
// 4-band group in FP32 (order <= 2) 12.  Never shallower than tile_depth,
// which sizes the checkpoints.
template <int D, int C, bool TAB, int ES, bool BWD, bool PERDIFF>
constexpr int fast_tile_depth() {
  if (!TAB && !BWD && ES == 4 && D <= 2 && (C == 2 || (C == 3 && !PERDIFF))) return 16;
  if (TAB && C == 1 && !(BWD && PERDIFF)) return D <= 2 ? 16 : 12;
  if (TAB && C == 4 && !BWD && ES == 4 && D <= 2) return 12;
  return tile_depth<D, C, TAB, ES>();
}

template <int D, int C, typename TS, Src SRC, Mode MODE, bool PERDIFF, bool TAB = false, bool WB = false>
hipError_t launch_fast(const LaunchDesc& L, int c0, int write_info, hipStream_t stream) {
  constexpr int B = fast_tile_depth<D, C, TAB, (int)sizeof(TS), MODE == Mode::Backward, PERDIFF>();
  static_assert(B >= tile_depth<D, C, TAB, (int)sizeof(TS)>(), "checkpoints are sized for tile_depth");
  FastArgs f;
  f.P = L.P;
  f.T = L.T;
  f.S = L.S;
  f.Ctot = L.C;
  f.c0 = c0;
  f.nt = (L.T + B - 1) / B;
  f.w = L.w;
  f.lam = L.lam;
  f.rhs = L.rhs;
  f.zin = L.zin;
  f.out = L.out;
  f.glam = L.glam;
  f.info = L.info;
  f.ck = L.ws;
  f.coef = L.coef;
  f.write_info = write_info;
  f.glam_accum = c0 > 0;
  const int threads = 256;
  const int64_t blocks = (L.P + threads - 1) / threads;
  hipLaunchKernelGGL((k_fast<D, C, B, TS, MODE == Mode::Backward, PERDIFF, TAB, WB>), dim3((unsigned)blocks),
                     dim3(threads), 0, stream, f);
  return hipGetLastError();
}

// The generic kernels take tile_depth steps, except that reading a given factor
// (d+1 FP64 values per step) leaves room for only 16 steps at order 2 in FP32
// storage.  Never shallower than the FP64 tile, which sizes the checkpoints.
template <int D, int C, int ES, Src SRC>
constexpr int generic_tile_depth() {
  if (SRC == Src::Factor && D == 2 && ES == 4 && C == 1) return 16;
  return tile_depth<D, C, false, ES>();
}

template <int D, int C, typename TS, Src SRC, Mode MODE, bool PERDIFF>
hipError_t launch_generic(const LaunchDesc& L, int c0, int write_info, hipStream_t stream) {
  constexpr int B = generic_tile_depth<D, C, (int)sizeof(TS), SRC>();
  static_assert(B >= tile_depth<D, C, false, 8>() || B >= tile_depth<D, C, false, 4>(),
                "checkpoints are sized for the shallower of the two storage types' tiles");
  Args a;
  a.P = L.P;
  a.T = L.T;
  a.S = L.S;
  a.Ctot = L.C;
  a.c0 = c0;
  a.nt = (L.T + B - 1) / B;
  a.w = L.w;
  a.lam = L.lam;
  a.fac = L.fac;
  a.rhs = L.rhs;
  a.zin = L.zin;
  a.out = L.out;
  a.glam = L.glam;
  a.info = L.info;
  a.ck = L.ws;
  a.write_info = write_info;
  a.glam_accum = c0 > 0;
  const int threads = 256;
  const int64_t blocks = (L.P + threads - 1) / threads;
  hipLaunchKernelGGL((k_two_sweep<D, C, B, TS, SRC, MODE, PERDIFF>), dim3((unsigned)blocks), dim3(threads), 0,
                     stream, a);
  return hipGetLastError();
}

// checkpoint bytes of one band group, for either storage type (the shallower
// tile of the two decides)
template <int D, int C, bool TAB = false>
size_t ck_bytes_for(int64_t nb, int S, int T) {
  constexpr int B4 = tile_depth<D, C, TAB, 4>();
  constexpr int B8 = tile_depth<D, C, TAB, 8>();
  constexpr int B = B4 < B8 ? B4 : B8;
  const int64_t nt = (T + B - 1) / B;
  return (size_t)nb * nt * ck_fields<D, C>() * S * sizeof(double);
}

// RHS group sizes.  A call covers C bands by greedy groups, each one launch
// that recomputes the same factor.  On the fast path (interleave a multiple of
// 64, weights and mask given) the largest group is the largest one whose kernel
// compiles without register spills for its order, storage type and weight
// kind:
//   solve, order <= 2: 5 bands; 4 in FP64 with a weight per difference row at
//     order 2; 3 in FP32 with one weight per series (its 16-step tiles move
//     fewer checkpoint bytes per day than the 8-step tiles of 5 bands);
//   solve, order 3 and 4: 3 bands;
//   adjoint, order 1: 3; order 2: 3, but 2 in FP64 with one weight per series;
//     order 3: 3 in FP32 with a weight per difference row, else 2; order 4: 3
//     in FP32 with a weight per difference row, 2 in FP64 with one, else 1.
// The generic path (any interleave, or a given factor) uses 2 and 1.
inline bool fast_path(const LaunchDesc& L) { return !L.fac && L.S % 64 == 0 && L.P < ((int64_t)1 << 31); }

constexpr int max_group(int D, bool bwd, bool f64, bool perdiff) {
  if (!bwd) {
    if (D >= 3) return 3;
    if (!f64 && !perdiff) return 3;
    return (D == 2 && f64 && perdiff) ? 4 : 5;
  }
  switch (D) {
    case 1: return 3;
    case 2: return (f64 && !perdiff) ? 2 : 3;
    case 3: return (!f64 && perdiff) ? 3 : 2;
    default: return perdiff ? (f64 ? 2 : 3) : 1;
  }
}

inline int next_group(int remaining, bool fast, int D, bool bwd, bool f64, bool perdiff) {
  if (fast) {
    const int g = max_group(D, bwd, f64, perdiff);
    return remaining < g ? remaining : g;
  }
  return remaining >= 2 ? 2 : 1;
}

template <int D>
inline size_t ck_bytes_d(int64_t nb, int S, int T, int g) {
  switch (g) {
    case 5: return ck_bytes_for<D, 5>(nb, S, T);
    case 4: return ck_bytes_for<D, 4>(nb, S, T);
    case 3: return ck_bytes_for<D, 3>(nb, S, T);
    case 2: return ck_bytes_for<D, 2>(nb, S, T);
    default: return ck_bytes_for<D, 1>(nb, S, T);
  }
}

// Band groups of the uneven-time kernels: the solve takes 4 and 1.  The
// adjoint takes the widest group whose kernel compiles without register
// spills: 4 bands only for FP32 storage with a weight per difference row at
// order <= 2, else 2 bands (orders 1 and 2; order 3 except FP64 with one weight
// per series; order 4 with a weight per difference row), else 1.
inline int tab_max_group(bool bwd, int D, bool f64, bool perdiff) {
  if (!bwd) return 4;
  if (D <= 2 && !f64 && perdiff) return 4;
  if (D <= 2 || (D == 3 && !(f64 && !perdiff)) || (D == 4 && perdiff)) return 2;
  return 1;
}

inline int next_group_tab(int remaining, bool bwd = false, int D = 1, bool f64 = false, bool perdiff = true) {
  const int g = tab_max_group(bwd, D, f64, perdiff);
  if (remaining >= g) return g;
  return remaining >= 2 && g >= 2 && bwd ? 2 : 1;
}

template <int D>
inline size_t ck_bytes_tab_d(int64_t nb, int S, int T, int g) {
  if (g == 4) return ck_bytes_for<D, 4, true>(nb, S, T);
  if (g == 2) return ck_bytes_for<D, 2, true>(nb, S, T);
  return ck_bytes_for<D, 1, true>(nb, S, T);
}

template <int D, typename TS, Src SRC, Mode MODE, bool PERDIFF>
hipError_t run_groups(const LaunchDesc& L, hipStream_t stream) {
  const bool fast = SRC == Src::Fused && fast_path(L);
  constexpr bool kBwd = MODE == Mode::Backward;
  // groups wider than this are never chosen (and not compiled) for this variant
  constexpr int kMaxG = max_group(D, kBwd, sizeof(TS) == 8, PERDIFF);
  int c0 = 0;
  while (c0 < L.C) {
    const int g = next_group(L.C - c0, fast, D, kBwd, sizeof(TS) == 8, PERDIFF);
    const int wi = c0 == 0;  // the first group writes info; later groups add to grad_lambda
    hipError_t e = hipErrorInvalidValue;
    if constexpr (SRC == Src::Fused) {
      // weights as bits: one band, one launch (the ABI admits nothing else)
      if (fast && L.wbits) return L.C == 1 ? launch_fast<D, 1, TS, SRC, MODE, PERDIFF, false, true>(L, 0, 1, stream)
                                           : hipErrorInvalidValue;
      if (fast) {
        switch (g) {
          case 5:
            if constexpr (kMaxG >= 5) e = launch_fast<D, 5, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream);
            break;
          case 4:
            if constexpr (kMaxG >= 4) e = launch_fast<D, 4, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream);
            break;
          case 3:
            if constexpr (kMaxG >= 3) e = launch_fast<D, 3, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream);
            break;
          case 2:
            if constexpr (kMaxG >= 2) e = launch_fast<D, 2, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream);
            break;
          default: e = launch_fast<D, 1, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream); break;
        }
        if (e != hipSuccess) return e;
        c0 += g;
        continue;
      }
    }
    e = g == 2 ? launch_generic<D, 2, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream)
               : launch_generic<D, 1, TS, SRC, MODE, PERDIFF>(L, c0, wi, stream);
    if (e != hipSuccess) return e;
    c0 += g;
  }
  return hipSuccess;
}

// Uneven sample times (a coefficient table for D): fast path only, built for
// 4 and 1 bands per launch, and 2 for the adjoint.
template <int D, typename TS, Mode MODE, bool PERDIFF>
hipError_t run_groups_tab(const LaunchDesc& L, hipStream_t stream) {
  constexpr bool kBwd = MODE == Mode::Backward;
  int c0 = 0;
  while (c0 < L.C) {
    const int g = next_group_tab(L.C - c0, kBwd, D, sizeof(TS) == 8, PERDIFF);
    const int wi = c0 == 0;
    hipError_t e;
    if (g == 4) {
      // the adjoint takes 4 bands only where tab_max_group allows them
      if constexpr (!kBwd || (D <= 2 && sizeof(TS) == 4 && PERDIFF))
        e = launch_fast<D, 4, TS, Src::Fused, MODE, PERDIFF, true>(L, c0, wi, stream);
      else e = hipErrorInvalidValue;  // never chosen
    } else if (g == 2) {
      // 2 bands: the adjoint only, where tab_max_group allows at least 2
      constexpr bool kF64 = sizeof(TS) == 8;
      if constexpr (kBwd && (D <= 2 || (D == 3 && !(kF64 && !PERDIFF)) || (D == 4 && PERDIFF)))
        e = launch_fast<D, 2, TS, Src::Fused, MODE, PERDIFF, true>(L, c0, wi, stream);
      else e = hipErrorInvalidValue;  // never chosen
    } else {
      e = launch_fast<D, 1, TS, Src::Fused, MODE, PERDIFF, true>(L, c0, wi, stream);
    }
    if (e != hipSuccess) return e;
    c0 += g;
  }
  return hipSuccess;
}

template <int D, Mode MODE>
hipError_t run_mode_tab_d(const LaunchDesc& L, hipStream_t stream) {
  if (L.f64) return L.perdiff ? run_groups_tab<D, double, MODE, true>(L, stream)
                              : run_groups_tab<D, double, MODE, false>(L, stream);
  return L.perdiff ? run_groups_tab<D, float, MODE, true>(L, stream) : run_groups_tab<D, float, MODE, false>(L, stream);
}

// All storage types and weight kinds of one order and mode.
template <int D, Mode MODE>
hipError_t run_mode_d(const LaunchDesc& L, hipStream_t stream) {
  if (L.fac) {
    // a given factor needs no weights; only the gradient layout depends on their kind
    if constexpr (MODE == Mode::Backward) {
      if (L.f64) return L.perdiff ? run_groups<D, double, Src::Factor, MODE, true>(L, stream)
                                  : run_groups<D, double, Src::Factor, MODE, false>(L, stream);
      return L.perdiff ? run_groups<D, float, Src::Factor, MODE, true>(L, stream)
                       : run_groups<D, float, Src::Factor, MODE, false>(L, stream);
    } else {
      if (L.f64) return run_groups<D, double, Src::Factor, MODE, false>(L, stream);
      return run_groups<D, float, Src::Factor, MODE, false>(L, stream);
    }
  }
  if (L.f64) return L.perdiff ? run_groups<D, double, Src::Fused, MODE, true>(L, stream)
                              : run_groups<D, double, Src::Fused, MODE, false>(L, stream);
  return L.perdiff ? run_groups<D, float, Src::Fused, MODE, true>(L, stream)
                   : run_groups<D, float, Src::Fused, MODE, false>(L, stream);
}

}  // namespace whs

// Fast path of the two-sweep kernels: interleave S a multiple of 64, so one
// wavefront reads one block of series and every block pointer is uniform.
//
// Memory is accessed through per-wave buffer resources (SGPR descriptors with
// a byte range): no per-lane 64-bit address arithmetic, and rows beyond the
// end of a series read as zero and drop stores, so partial tiles need no
// branches around their loads.  Tile inputs are double-buffered in registers
// (two named buffers, no copies), so the loads of tile j+1 are in flight
// while tile j is computed.
#pragma once

#include <hip/hip_runtime.h>

#include "whs_kernels.h"
#include "whs_step.h"

namespace whs {

constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nbytes, kRsrcWord3);
}

// Cache policy of a buffer access.  kStream marks data touched once more at
// most, far in the future or never (the reverse sweep's inputs, results,
// checkpoints): non-temporal, so it does not displace lines still to be reused.
constexpr int kKeep = 0;
constexpr int kStream = 2;  // NT bit of the gfx950 cache-policy operand

template <typename TS, int POL = kKeep>
__device__ __forceinline__ TS bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(TS) == 4)
    return __builtin_bit_cast(TS, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, POL));
  else
    return __builtin_bit_cast(TS, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, POL));
}
template <typename TS, int POL = kKeep>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, TS v) {
  if constexpr (sizeof(TS) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, off, 0, POL);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) int, v), r, off, 0,
                                          POL);
}

// positive normal or subnormal: the only acceptable pivots
__device__ __forceinline__ bool pivot_good(double dt) { return __builtin_amdgcn_class(dt, (1 << 7) | (1 << 8)); }

struct FastArgs {
  int64_t P;
  int T, S, Ctot, c0, nt;
  const uint8_t* w;
  const void* lam;
  const void* rhs;
  const void* zin;
  void* out;
  void* glam;
  int32_t* info;
  double* ck;
  const double* coef;  // rows of D on uneven times, (T-D) x (D+1); null on the daily grid
  int write_info;
  int glam_accum;
};

template <int D, int C, int B, typename TS, bool BWD, bool PERDIFF, bool TAB = false, bool WB = false>
struct Fast {
  static constexpr int NF = ck_fields<D, C>();
  static constexpr uint32_t ES = sizeof(TS);

  struct Tile {
    TS x[B][C];
    uint32_t w[WB ? 1 : B];  // 0/1 weights (bytes)
    uint32_t wm;             // the same as bits s of one register (weights as bits)
    TS lam[B];
    TS z[B][C];
  };
  // the 0/1 weight of step s of a tile
  static __device__ __forceinline__ bool wt(const Tile& tl, int s) {
    if constexpr (WB) return (tl.wm >> s) & 1u;
    else return tl.w[s] != 0u;
  }

  // wave-uniform
  const TS* xb;
  const uint8_t* wb;
  const TS* lb;
  const TS* zb;
  TS* ob;
  TS* gb;
  double* ckb;
  const double* ctab;  // coefficient table (TAB only); the same for every series
  int T, S, Ctot, c0, nt;
  uint32_t Rx;  // bytes per row of x / z / g
  // per lane
  uint32_t lx, lw, lc;
  double lam_scalar;
  bool accum;
  // w as bits (WB): a row of w is S / 8 bytes and lane s reads bit s & 31 (its
  // lane index & 31) of the dword at byte lw (every lane of the dword reads the
  // same address)
  static constexpr bool wbits = WB;

  // the 0/1 weight of this lane at row `row` of the w range rw
  template <int POLICY>
  __device__ __forceinline__ uint32_t load_w(const __amdgpu_buffer_rsrc_t rw, int row) const {
    if constexpr (WB)
      return (__builtin_amdgcn_raw_buffer_load_b32(rw, lw + (uint32_t)(row * (S >> 3)), 0, POLICY) >>
              (__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)) & 31u)) & 1u;
    else
      return __builtin_amdgcn_raw_buffer_load_b8(rw, lw + (uint32_t)(row * S), 0, POLICY);
  }
  __device__ __forceinline__ uint32_t w_row_bytes() const { return WB ? (uint32_t)(S >> 3) : (uint32_t)S; }

  // row k of D's coefficient table (wave-uniform); zero outside 0..T-D-1
  __device__ __forceinline__ void crow(int k, double (&c)[D + 1]) const {
    const bool in = k >= 0 && k < T - D;
    const double* r = ctab + (int64_t)(in ? k : 0) * (D + 1);
#pragma unroll
    for (int j = 0; j <= D; ++j) c[j] = in ? r[j] : 0.0;
  }

  // rows of a tile starting at t0 that lie inside [0, lim); 0 for tiles outside
  __device__ __forceinline__ int rows_from(int t0, int lim) const {
    if (t0 < 0 || t0 >= lim) return 0;
    const int r = lim - t0;
    return r > B ? B : r;
  }

  template <bool SWEEP2>
  __device__ __forceinline__ void load_tile(Tile& tl, int t0) const {
    const int rows = rows_from(t0, T);
    const int tb = rows > 0 ? t0 : 0;
    const auto rx = make_rsrc(xb + (int64_t)tb * Ctot * S, rows * Rx);
    const auto rw = make_rsrc(wb + (int64_t)tb * w_row_bytes(), rows * w_row_bytes());
#pragma unroll
    for (int s = 0; s < B; ++s) {
#pragma unroll
      for (int c = 0; c < C; ++c)
        tl.x[s][c] = bload<TS, SWEEP2 ? kStream : kKeep>(rx, lx + (uint32_t)((s * Ctot + c0 + c) * S) * ES);
      if constexpr (WB) {
        if (s == 0) tl.wm = 0u;
        tl.wm |= load_w<SWEEP2 ? kStream : kKeep>(rw, s) << s;
      } else {
        tl.w[s] = load_w<SWEEP2 ? kStream : kKeep>(rw, s);
      }
    }
    if constexpr (PERDIFF) {
      const int rl = rows_from(t0, T - D);
      const int tl0 = rl > 0 ? t0 : 0;
      const auto rlm = make_rsrc(lb + (int64_t)tl0 * S, rl * S * ES);
#pragma unroll
      for (int s = 0; s < B; ++s) tl.lam[s] = bload<TS, SWEEP2 ? kStream : kKeep>(rlm, lx + (uint32_t)(s * S) * ES);
    }
    if constexpr (BWD && SWEEP2) {
      const auto rz = make_rsrc(zb + (int64_t)tb * Ctot * S, rows * Rx);
#pragma unroll
      for (int s = 0; s < B; ++s)
#pragma unroll
        for (int c = 0; c < C; ++c)
          tl.z[s][c] = bload<TS, kStream>(rz, lx + (uint32_t)((s * Ctot + c0 + c) * S) * ES);
    }
  }

  // one step of the recurrence (sweep 1 and the sweep-2 recompute)
  template <bool FULL>
  __device__ __forceinline__ void step(State<D, C>& st, const Tile& tl, int s, int t, double (&l)[D + 1],
                                       double& dt, double& invdt, double (&yt)[C]) const {
    const bool obs = wt(tl, s);
    double lt;
    if constexpr (PERDIFF) {
      lt = to_f64(tl.lam[s]);
    } else {
      lt = (FULL || t < T - D) ? lam_scalar : 0.0;
    }
    double lwv[D + 1];
    lwv[0] = lt;
#pragma unroll
    for (int m = 1; m <= D; ++m) lwv[m] = st.lw[m];
    double om[D + 1];
    if constexpr (TAB) {
      double cwv[D + 1][D + 1];
      crow(t, cwv[0]);
#pragma unroll
      for (int m = 1; m <= D; ++m)
#pragma unroll
        for (int j = 0; j <= D; ++j) cwv[m][j] = st.cw[m][j];
      omega_row_tab<D>(lwv, cwv, obs ? 1.0 : 0.0, om);
#pragma unroll
      for (int m = D; m >= 2; --m)
#pragma unroll
        for (int j = 0; j <= D; ++j) st.cw[m][j] = st.cw[m - 1][j];
#pragma unroll
      for (int j = 0; j <= D; ++j) st.cw[1][j] = cwv[0][j];
    } else {
      omega_row<D>(lwv, obs ? 1.0 : 0.0, om);
    }
    ldl_step<D, C>(st, om, l, dt, invdt);
#pragma unroll
    for (int m = D; m >= 2; --m) st.lw[m] = st.lw[m - 1];
    st.lw[1] = lt;
    double b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      if constexpr (BWD) {
        b[c] = to_f64(tl.x[s][c]);
      } else {
        b[c] = to_f64(obs ? tl.x[s][c] : TS(0));
      }
    }
    fwd_step<D, C>(st, l, b, yt);
  }

  __device__ __forceinline__ void store_ck(const State<D, C>& st, int j) const {
    const auto r = make_rsrc(ckb, (uint32_t)nt * NF * S * 8u);
    int f = 0;
    const uint32_t base = lc + (uint32_t)(j * NF) * S * 8u;
#pragma unroll
    for (int jj = 1; jj <= D; ++jj) bstore<double, kStream>(r, base + (uint32_t)(f++ * S * 8), st.invD[jj]);
#pragma unroll
    for (int jj = 1; jj < D; ++jj)
#pragma unroll
      for (int k = 1; k <= D - jj; ++k) bstore<double, kStream>(r, base + (uint32_t)(f++ * S * 8), st.R[jj][k]);
#pragma unroll
    for (int jj = 1; jj <= D; ++jj)
#pragma unroll
      for (int c = 0; c < C; ++c) bstore<double, kStream>(r, base + (uint32_t)(f++ * S * 8), st.y[jj][c]);
  }

  // checkpoint of tile j plus the weight window lambda_{t0-1..t0-D};
  // tiles outside 0..nt-1 read as zero (the state before t = 0)
  __device__ __forceinline__ void load_ck(int j, double (&ckv)[NF], double (&lwin)[D + 1]) const {
    const auto r = make_rsrc(ckb, (j >= 0 && j < nt) ? (uint32_t)nt * NF * S * 8u : 0u);
    const int jc = (j >= 0 && j < nt) ? j : 0;
    const uint32_t base = lc + (uint32_t)(jc * NF) * S * 8u;
#pragma unroll
    for (int f = 0; f < NF; ++f) ckv[f] = bload<double, kStream>(r, base + (uint32_t)(f * S * 8));
    const int t0 = j * B;
    lwin[0] = 0.0;
    if constexpr (PERDIFF) {
      const auto rl = make_rsrc(lb, (uint32_t)(T - D) * S * ES);
#pragma unroll
      for (int m = 1; m <= D; ++m) lwin[m] = to_f64(bload<TS>(rl, lx + (uint32_t)((t0 - m) * S) * ES));
    } else {
#pragma unroll
      for (int m = 1; m <= D; ++m) {
        const int k = t0 - m;
        lwin[m] = (k >= 0 && k < T - D) ? lam_scalar : 0.0;
      }
    }
  }

  __device__ __forceinline__ void restore(State<D, C>& st, const double (&ckv)[NF],
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

  __device__ __forceinline__ bool full_tile(int t0) const { return t0 + B <= T - D; }

  // sweep-1 pass over one tile; returns false if a pivot failed in it
  template <bool FULL>
  __device__ __forceinline__ bool fwd_tile(State<D, C>& st, const Tile& tl, int t0, int& nobs) const {
    bool ok = true;
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int t = t0 + s;
      double l[D + 1], dt, invdt, yt[C];
      step<FULL>(st, tl, s, t, l, dt, invdt, yt);
      nobs += wt(tl, s) ? 1 : 0;
      ok = ok & (pivot_good(dt) | (!FULL && t >= T));
    }
    return ok;
  }

  // sweep-2: recompute one tile from its checkpoint and back substitute it
  template <bool FULL>
  __device__ __forceinline__ void rev_tile(const Tile& tl, int t0, const double (&ckv)[NF],
                                           const double (&lwin)[D + 1], double (&zn)[D + 1][C],
                                           double (&xn)[D + 1][C], double (&lc_)[D + 1][D + 1], bool failed,
                                           double& gsum) const {
    State<D, C> st;
    restore(st, ckv, lwin);
    if constexpr (TAB) {
#pragma unroll
      for (int m = 1; m <= D; ++m) crow(t0 - m, st.cw[m]);
    }
    double lt[B][D + 1];
    double yd[B][C];
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int t = t0 + s;
      double l[D + 1], dt, invdt, yt[C];
      step<FULL>(st, tl, s, t, l, dt, invdt, yt);
      const bool v = FULL || t < T;
#pragma unroll
      for (int i = 1; i <= D; ++i) lt[s][i] = v ? l[i] : 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) yd[s][c] = v ? yt[c] * invdt : 0.0;
    }
    const double qnan = __builtin_nan("");
    const int rows = rows_from(t0, T);
    const int tb = rows > 0 ? t0 : 0;
    const auto ro = make_rsrc(ob ? (const void*)(ob + (int64_t)tb * Ctot * S) : (const void*)ckb,
                              ob ? rows * Rx : 0u);
    const int rlr = rows_from(t0, T - D);
    const auto rg = make_rsrc(gb ? (const void*)(gb + (int64_t)(rlr > 0 ? t0 : 0) * S) : (const void*)ckb,
                              (BWD && PERDIFF && gb) ? rlr * S * ES : 0u);
#pragma unroll
    for (int s = B - 1; s >= 0; --s) {
      const int t = t0 + s;
      double zt[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double acc = yd[s][c];
#pragma unroll
        for (int i = 1; i <= D; ++i) {
          const double li = (s + i < B) ? lt[s + i < B ? s + i : 0][i] : lc_[s + i - B < 0 ? 0 : s + i - B][i];
          acc = __builtin_fma(-li, zn[i][c], acc);
        }
        zt[c] = acc;
      }
      if constexpr (!BWD) {
#pragma unroll
        for (int c = 0; c < C; ++c)
          bstore<TS, kStream>(ro, lx + (uint32_t)((s * Ctot + c0 + c) * S) * ES, from_f64<TS>(failed ? qnan : zt[c]));
      } else {
        const bool obs = wt(tl, s);
        if (ob) {
#pragma unroll
          for (int c = 0; c < C; ++c)
            bstore<TS, kStream>(ro, lx + (uint32_t)((s * Ctot + c0 + c) * S) * ES,
                       from_f64<TS>(failed ? qnan : (obs ? zt[c] : 0.0)));
        }
        double zin[C];
#pragma unroll
        for (int c = 0; c < C; ++c) zin[c] = to_f64(tl.z[s][c]);
        double crw[D + 1];  // coefficients of row t of D
        if constexpr (TAB) {
          crow(t, crw);
        } else {
#pragma unroll
          for (int i = 0; i <= D; ++i) crw[i] = cdiff<D>(i);
        }
        double gt = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          double du = crw[0] * zt[c];
          double dz = crw[0] * zin[c];
#pragma unroll
          for (int i = 1; i <= D; ++i) {
            du = __builtin_fma(crw[i], zn[i][c], du);
            dz = __builtin_fma(crw[i], xn[i][c], dz);
          }
          gt = __builtin_fma(-du, dz, gt);
        }
        if constexpr (PERDIFF) {
          if (gb) {
            const uint32_t o = lx + (uint32_t)(s * S) * ES;
            const double prev = accum ? to_f64(bload<TS>(rg, o)) : 0.0;
            bstore<TS, kStream>(rg, o, from_f64<TS>(failed ? qnan : prev + gt));
          }
        } else {
          gsum += (FULL || t < T - D) ? gt : 0.0;
        }
        if (FULL || t < T) {
#pragma unroll
          for (int i = D; i >= 2; --i)
#pragma unroll
            for (int c = 0; c < C; ++c) xn[i][c] = xn[i - 1][c];
#pragma unroll
          for (int c = 0; c < C; ++c) xn[1][c] = zin[c];
        }
      }
      if (FULL || t < T) {
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
      for (int i = 0; i <= D; ++i) lc_[r][i] = lt[r][i];
  }

  // Rare path: exact index of the first failing pivot, by a plain rescan.
  __device__ int first_bad_pivot(int t_end) const {
    State<D, C> st;
    st.zero();
    const auto rw = make_rsrc(wb, (uint32_t)T * w_row_bytes());
    const auto rl = make_rsrc(lb ? (const void*)lb : (const void*)wb, PERDIFF ? (uint32_t)(T - D) * S * ES : 0u);
    for (int t = 0; t < t_end && t < T; ++t) {
      const bool obs = load_w<0>(rw, t) != 0;
      const double ltv = PERDIFF ? to_f64(bload<TS>(rl, lx + (uint32_t)(t * S) * ES)) : (t < T - D ? lam_scalar : 0.0);
      double lwv[D + 1];
      lwv[0] = ltv;
      for (int m = 1; m <= D; ++m) lwv[m] = st.lw[m];
      double om[D + 1], l[D + 1], dt, invdt;
      if constexpr (TAB) {
        double cwv[D + 1][D + 1];
        crow(t, cwv[0]);
        for (int m = 1; m <= D; ++m)
          for (int j = 0; j <= D; ++j) cwv[m][j] = st.cw[m][j];
        omega_row_tab<D>(lwv, cwv, obs ? 1.0 : 0.0, om);
        for (int m = D; m >= 2; --m)
          for (int j = 0; j <= D; ++j) st.cw[m][j] = st.cw[m - 1][j];
        for (int j = 0; j <= D; ++j) st.cw[1][j] = cwv[0][j];
      } else {
        omega_row<D>(lwv, obs ? 1.0 : 0.0, om);
      }
      ldl_step<D, C>(st, om, l, dt, invdt);
      for (int m = D; m >= 2; --m) st.lw[m] = st.lw[m - 1];
      st.lw[1] = ltv;
      if (!pivot_good(dt)) return t + 1;
    }
    return 0;
  }

  // Set the wave-uniform pointers for block `bidx` of the batch described by
  // `a` (whose array pointers are the batch's first block) and run both sweeps.
  // `s_in` is the lane's slot in the block, `p` its series index in `a`.
  __device__ void run_block(const FastArgs& a, int64_t bidx, int s_in, int64_t p) {
    T = a.T;
    S = a.S;
    Ctot = a.Ctot;
    c0 = a.c0;
    nt = a.nt;
    Rx = (uint32_t)Ctot * S * ES;
    xb = static_cast<const TS*>(a.rhs) + bidx * T * Ctot * S;
    wb = a.w + bidx * T * (int64_t)w_row_bytes();
    lb = PERDIFF ? static_cast<const TS*>(a.lam) + bidx * (T - D) * S : nullptr;
    zb = BWD ? static_cast<const TS*>(a.zin) + bidx * T * Ctot * S : nullptr;
    ob = a.out ? static_cast<TS*>(a.out) + bidx * T * Ctot * S : nullptr;
    gb = (BWD && a.glam && PERDIFF) ? static_cast<TS*>(a.glam) + bidx * (T - D) * S : nullptr;
    ctab = a.coef;
    accum = a.glam_accum != 0;
    const bool live = p < a.P;
    // padding slots of the last block: an offset beyond every buffer range
    // makes their loads read zero and drops their stores
    constexpr uint32_t kDead = 0x80000000u;
    lx = live ? (uint32_t)s_in * ES : kDead;
    lw = live ? (WB ? ((uint32_t)s_in >> 5) << 2 : (uint32_t)s_in) : kDead;
    lc = live ? (uint32_t)s_in * 8u : kDead;
    lam_scalar = (!PERDIFF && live) ? to_f64(static_cast<const TS*>(a.lam)[p]) : 0.0;

    // ---------------- sweep 1 ----------------
    State<D, C> st;
    st.zero();
    int nobs = 0;
    int bad_tile = -1;
    Tile A, Bt;
    load_tile<false>(A, 0);
    for (int j = 0; j < nt; j += 2) {
      load_tile<false>(Bt, (j + 1) * B);
      store_ck(st, j);
      bool ok = full_tile(j * B) ? fwd_tile<true>(st, A, j * B, nobs) : fwd_tile<false>(st, A, j * B, nobs);
      if (!ok && bad_tile < 0) bad_tile = j;
      load_tile<false>(A, (j + 2) * B);
      if (j + 1 < nt) {
        store_ck(st, j + 1);
        ok = full_tile((j + 1) * B) ? fwd_tile<true>(st, Bt, (j + 1) * B, nobs)
                                    : fwd_tile<false>(st, Bt, (j + 1) * B, nobs);
        if (!ok && bad_tile < 0) bad_tile = j + 1;
      }
    }
    int info = 0;
    if (live && bad_tile >= 0) info = first_bad_pivot((bad_tile + 1) * B);
    if (info == 0 && nobs < D) info = T;
    const bool failed = info != 0;
    if (live && a.info && a.write_info) a.info[p] = info;

    // ---------------- sweep 2 ----------------
    double zn[D + 1][C], xn[D + 1][C], lcr[D + 1][D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        zn[i][c] = 0.0;
        xn[i][c] = 0.0;
      }
#pragma unroll
      for (int k = 0; k <= D; ++k) lcr[i][k] = 0.0;
    }
    double gsum = 0.0;
    double ckA[NF], ckB[NF], lwA[D + 1], lwB[D + 1];
    int j = nt - 1;
    load_tile<true>(A, j * B);
    load_ck(j, ckA, lwA);
    for (; j >= 0; j -= 2) {
      load_tile<true>(Bt, (j - 1) * B);
      load_ck(j - 1, ckB, lwB);
      if (full_tile(j * B)) rev_tile<true>(A, j * B, ckA, lwA, zn, xn, lcr, failed, gsum);
      else rev_tile<false>(A, j * B, ckA, lwA, zn, xn, lcr, failed, gsum);
      load_tile<true>(A, (j - 2) * B);
      load_ck(j - 2, ckA, lwA);
      if (j - 1 >= 0) {
        if (full_tile((j - 1) * B)) rev_tile<true>(Bt, (j - 1) * B, ckB, lwB, zn, xn, lcr, failed, gsum);
        else rev_tile<false>(Bt, (j - 1) * B, ckB, lwB, zn, xn, lcr, failed, gsum);
      }
    }
    if constexpr (BWD && !PERDIFF) {
      if (a.glam && live) {
        TS* g = static_cast<TS*>(a.glam) + p;
        const double prev = accum ? to_f64(*g) : 0.0;
        *g = from_f64<TS>(failed ? __builtin_nan("") : prev + gsum);
      }
    }
  }

  __device__ void run(const FastArgs& a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wave_off = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x + wave_off;  // first series of this wavefront
    if (p0 >= a.P) return;  // whole wavefront past the batch: its block does not exist
    const int64_t bidx = p0 / a.S;
    ckb = a.ck + bidx * a.nt * NF * a.S;
    run_block(a, bidx, (int)(p - bidx * a.S), p);
  }
};

template <int D, int C, int B, typename TS, bool BWD, bool PERDIFF, bool TAB, bool WB = false>
__global__ __launch_bounds__(256) void k_fast(FastArgs a) {
  Fast<D, C, B, TS, BWD, PERDIFF, TAB, WB> k;
  k.run(a);
}

}  // namespace whs

namespace whs {

// ---------------------------------------------------------------------------
// Posterior variance: the diagonal of Omega^{-1}.
//
// Sweep 1 factors the series (no right-hand side: x reads as zero through an
// empty buffer range) and checkpoints the state as in the solve kernel; the
// reverse sweep recomputes each tile and runs the selected-inverse recurrence
// of Sigma = Omega^{-1} on the LDL^T factor,
//   Sigma[t, t+j] = -sum_i L[t+i, t] Sigma[t+i, t+j]      (j >= 1)
//   Sigma[t, t]   = 1/Dp[t] - sum_i L[t+i, t] Sigma[t+i, t],
// carrying the d x d block Sigma[t+1..t+d, t+1..t+d] and storing Sigma[t, t]
// for every t.
// ---------------------------------------------------------------------------

struct VarArgs {
  int64_t P;
  int T, S, nt;
  const uint8_t* w;
  const void* lam;
  void* var;
  int32_t* info;
  double* ck;
};

template <int D, int B, typename TS, bool PERDIFF>
struct Var : Fast<D, 1, B, TS, false, PERDIFF> {
  using Base = Fast<D, 1, B, TS, false, PERDIFF>;
  using typename Base::Tile;
  static constexpr int NF = Base::NF;

  template <bool FULL>
  __device__ __forceinline__ void rev_tile_var(const Tile& tl, int t0, const double (&ckv)[NF],
                                               const double (&lwin)[D + 1], double (&sg)[D + 1][D + 1],
                                               double (&lcr)[D + 1][D + 1], TS* vb, bool failed) const {
    State<D, 1> st;
    this->restore(st, ckv, lwin);
    double lt[B][D + 1];
    double id[B];
#pragma unroll
    for (int s = 0; s < B; ++s) {
      const int t = t0 + s;
      double l[D + 1], dt, invdt, yt[1];
      this->template step<FULL>(st, tl, s, t, l, dt, invdt, yt);
      const bool v = FULL || t < this->T;
#pragma unroll
      for (int i = 1; i <= D; ++i) lt[s][i] = v ? l[i] : 0.0;
      id[s] = v ? invdt : 0.0;
    }
    const int rows = this->rows_from(t0, this->T);
    const auto ro = make_rsrc(vb + (int64_t)(rows > 0 ? t0 : 0) * this->S, rows * this->S * Base::ES);
    const double qnan = __builtin_nan("");
#pragma unroll
    for (int s = B - 1; s >= 0; --s) {
      const int t = t0 + s;
      double L[D + 1];
#pragma unroll
      for (int i = 1; i <= D; ++i)
        L[i] = (s + i < B) ? lt[s + i < B ? s + i : 0][i] : lcr[s + i - B < 0 ? 0 : s + i - B][i];
      double sj[D + 1];
#pragma unroll
      for (int j = 1; j <= D; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 1; i <= D; ++i) acc = __builtin_fma(-L[i], sg[i - 1][j - 1], acc);
        sj[j] = acc;
      }
      double stt = id[s];
#pragma unroll
      for (int i = 1; i <= D; ++i) stt = __builtin_fma(-L[i], sj[i], stt);
      bstore<TS>(ro, this->lx + (uint32_t)(s * this->S) * Base::ES, from_f64<TS>(failed ? qnan : stt));
      if (FULL || t < this->T) {
#pragma unroll
        for (int a = D - 1; a >= 1; --a)
#pragma unroll
          for (int b = D - 1; b >= 1; --b) sg[a][b] = sg[a - 1][b - 1];
        sg[0][0] = stt;
#pragma unroll
        for (int b = 1; b < D; ++b) {
          sg[0][b] = sj[b];
          sg[b][0] = sj[b];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int i = 0; i <= D; ++i) lcr[r][i] = lt[r][i];
  }

  __device__ void run(const VarArgs& g) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wave_off = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~63u));
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x + wave_off;
    if (p0 >= g.P) return;
    const int64_t bidx = p0 / g.S;
    const int s_in = (int)(p - bidx * g.S);
    const int T = g.T, nt = g.nt;
    this->T = T;
    this->S = g.S;
    this->Ctot = 1;
    this->c0 = 0;
    this->nt = nt;
    this->Rx = 0;  // no right-hand side: every x load is out of range and reads zero
    this->wb = g.w + bidx * T * g.S;
    this->xb = reinterpret_cast<const TS*>(this->wb);
    this->lb = PERDIFF ? static_cast<const TS*>(g.lam) + bidx * (T - D) * g.S : nullptr;
    this->zb = nullptr;
    this->ob = nullptr;
    this->gb = nullptr;
    this->ckb = g.ck + bidx * nt * NF * g.S;
    this->accum = false;
    const bool live = p < g.P;
    constexpr uint32_t kDead = 0x80000000u;
    this->lx = live ? (uint32_t)s_in * Base::ES : kDead;
    this->lw = live ? (uint32_t)s_in : kDead;
    this->lc = live ? (uint32_t)s_in * 8u : kDead;
    this->lam_scalar = (!PERDIFF && live) ? to_f64(static_cast<const TS*>(g.lam)[p]) : 0.0;
    TS* vb = static_cast<TS*>(g.var) + bidx * T * g.S;

    State<D, 1> st;
    st.zero();
    int nobs = 0, bad_tile = -1;
    Tile A, Bt;
    this->template load_tile<false>(A, 0);
    for (int j = 0; j < nt; j += 2) {
      this->template load_tile<false>(Bt, (j + 1) * B);
      this->store_ck(st, j);
      bool ok = this->full_tile(j * B) ? this->template fwd_tile<true>(st, A, j * B, nobs)
                                       : this->template fwd_tile<false>(st, A, j * B, nobs);
      if (!ok && bad_tile < 0) bad_tile = j;
      this->template load_tile<false>(A, (j + 2) * B);
      if (j + 1 < nt) {
        this->store_ck(st, j + 1);
        ok = this->full_tile((j + 1) * B) ? this->template fwd_tile<true>(st, Bt, (j + 1) * B, nobs)
                                          : this->template fwd_tile<false>(st, Bt, (j + 1) * B, nobs);
        if (!ok && bad_tile < 0) bad_tile = j + 1;
      }
    }
    int info = 0;
    if (live && bad_tile >= 0) info = this->first_bad_pivot((bad_tile + 1) * B);
    if (info == 0 && nobs < D) info = T;
    if (live && g.info) g.info[p] = info;
    const bool failed = info != 0;

    double sg[D + 1][D + 1], lcr[D + 1][D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i)
#pragma unroll
      for (int k = 0; k <= D; ++k) {
        sg[i][k] = 0.0;
        lcr[i][k] = 0.0;
      }
    double ckA[NF], ckB[NF], lwA[D + 1], lwB[D + 1];
    int j = nt - 1;
    this->template load_tile<true>(A, j * B);
    this->load_ck(j, ckA, lwA);
    for (; j >= 0; j -= 2) {
      this->template load_tile<true>(Bt, (j - 1) * B);
      this->load_ck(j - 1, ckB, lwB);
      if (this->full_tile(j * B)) rev_tile_var<true>(A, j * B, ckA, lwA, sg, lcr, vb, failed);
      else rev_tile_var<false>(A, j * B, ckA, lwA, sg, lcr, vb, failed);
      this->template load_tile<true>(A, (j - 2) * B);
      this->load_ck(j - 2, ckA, lwA);
      if (j - 1 >= 0) {
        if (this->full_tile((j - 1) * B)) rev_tile_var<true>(Bt, (j - 1) * B, ckB, lwB, sg, lcr, vb, failed);
        else rev_tile_var<false>(Bt, (j - 1) * B, ckB, lwB, sg, lcr, vb, failed);
      }
    }
  }
};

template <int D, int B, typename TS, bool PERDIFF>
__global__ __launch_bounds__(256) void k_var(VarArgs a) {
  Var<D, B, TS, PERDIFF> k;
  k.run(a);
}

}  // namespace whs

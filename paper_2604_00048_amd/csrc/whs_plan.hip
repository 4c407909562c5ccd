// Uneven batches in one persistent launch.
//
// A plan covers groups of series that share a length T and an order d (the
// mask pads nothing: each group keeps its own T).  Work items are blocks of
// 64 series of one group, sorted longest-first on the host and served from
// a device queue: every resident wavefront takes the next item with one
// atomic, so long series start first and short ones fill the tail.  The
// kernel resets its own queue counters when the last wavefront leaves, so a
// launch can be replayed from a graph without a memset node.
//
// Long series can take two lanes (the autotuner decides per length): the two
// wavefronts of a workgroup solve the top and the bottom part of the same 64
// series and meet at a separator of d rows (whs_twist.h), which halves the
// dependent chain that otherwise sets the batch time.  That kernel serves
// units of work: one split block (both wavefronts) or two whole blocks (one
// each).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "whs.h"
#include "whs_fast.h"
#include "whs_kernels.h"
#include "whs_twist.h"

namespace whs {

struct GroupDev {
  int64_t x_off, w_off, lam_off, info_off, n_series;
  int32_t T, d;
};

struct PlanArgs {
  const GroupDev* groups;
  const int2* items;  // (group, block)
  int n_items;
  int n_waves;        // resident wavefronts of the persistent grid
  int* queue;         // [0] next item, [1] finished wavefronts
  const uint8_t* w;
  const void* lam;
  const void* x;
  void* z;
  int32_t* info;
  double* ck;         // one checkpoint slot per wavefront
  int64_t ck_stride;  // doubles per slot
  const int4* units;  // two-lane kernel: (kind, item, item, 0); kind 1 = one item split over both wavefronts
  int n_units;
};

// tile depth per order for each tuning profile: 0 = (8,8,8,8),
// 1 = (16,16,12,8), 2 = (24,16,16,8), order 3 at most 12 with a weight per
// difference row; deeper tiles store fewer checkpoints but hold more
// registers: these are the deepest that compile without spills
__host__ __device__ constexpr int plan_tile(int prof, int d, bool pd) {
  return d >= 4 ? 8
       : d == 3 ? (prof == 0 ? 8 : (prof == 1 || pd) ? 12 : 16)
                : (prof == 0 ? 8 : (prof == 1 ? 16 : (d == 1 ? 24 : 16)));
}

template <int D, int B, typename TS, bool PERDIFF>
__device__ __forceinline__ void plan_item(const PlanArgs& a, const GroupDev& G, int64_t bidx, double* slot) {
  constexpr int S = 64;
  FastArgs f;
  f.P = G.n_series;
  f.T = G.T;
  f.S = S;
  f.Ctot = 1;
  f.c0 = 0;
  f.nt = (G.T + B - 1) / B;
  f.w = a.w + G.w_off;
  f.lam = static_cast<const TS*>(a.lam) + G.lam_off;
  f.rhs = static_cast<const TS*>(a.x) + G.x_off;
  f.zin = nullptr;
  f.out = static_cast<TS*>(a.z) + G.x_off;
  f.glam = nullptr;
  f.info = a.info ? a.info + G.info_off : nullptr;
  f.ck = slot;
  f.write_info = 1;
  f.glam_accum = 0;
  Fast<D, 1, B, TS, false, PERDIFF> k;
  k.ckb = slot;
  const int lane = threadIdx.x & 63;
  k.run_block(f, bidx, lane, bidx * S + lane);
}

template <int PROF, typename TS, bool PERDIFF>
__global__ __launch_bounds__(256) void k_plan(PlanArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  double* slot = a.ck + (int64_t)wave * a.ck_stride;
  for (;;) {
    int item = 0;
    if (lane == 0) item = atomicAdd(&a.queue[0], 1);
    item = __builtin_amdgcn_readlane(item, 0);
    if (item >= a.n_items) break;
    const int2 it = a.items[item];
    const GroupDev G = a.groups[it.x];
    switch (G.d) {
      case 1: plan_item<1, plan_tile(PROF, 1, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
      case 2: plan_item<2, plan_tile(PROF, 2, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
      case 3: plan_item<3, plan_tile(PROF, 3, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
      default: plan_item<4, plan_tile(PROF, 4, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
    }
  }
  // the last wavefront to leave rewinds the queue for the next launch
  if (lane == 0) {
    __threadfence();
    const int done = atomicAdd(&a.queue[1], 1);
    if (done == a.n_waves - 1) {
      atomicExch(&a.queue[0], 0);
      atomicExch(&a.queue[1], 0);
    }
  }
}

// separator exchange between the two wavefronts of a workgroup: per part, the
// lower triangle of its Schur term and its right-hand side (order d <= 4)
constexpr int kSepFields = 4 * 5 / 2 + 4;

template <int D>
__host__ __device__ constexpr int split_point(int T) { return (T - D) / 2; }

template <int D, int B, typename TS, bool PERDIFF>
__device__ __forceinline__ void twist_item(const PlanArgs& a, const GroupDev& G, int64_t bidx, double* slot,
                                           int half, double (*sep)[kSepFields][64], int (*flag)[64]) {
  constexpr int NY = D * (D + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int T = G.T;
  Twist<D, B, TS, PERDIFF> k;
  k.T = T;
  k.S = 64;
  k.m = split_point<D>(T);
  k.rev = half == 1;
  k.Tv = k.rev ? T - k.m : k.m + D;
  k.ntv = (k.Tv + B - 1) / B;
  k.pad = k.ntv * B - k.Tv;
  k.Rx = 64u * (uint32_t)sizeof(TS);
  k.xb = static_cast<const TS*>(a.x) + G.x_off + bidx * T * 64;
  k.zb = static_cast<TS*>(a.z) + G.x_off + bidx * T * 64;
  k.wb = a.w + G.w_off + bidx * T * 64;
  k.lb = PERDIFF ? static_cast<const TS*>(a.lam) + G.lam_off + bidx * (T - D) * 64 : nullptr;
  k.ckb = slot;
  const int64_t p = bidx * 64 + lane;
  const bool live = p < G.n_series;
  constexpr uint32_t kDead = 0x80000000u;
  k.lx = live ? (uint32_t)lane * (uint32_t)sizeof(TS) : kDead;
  k.lw = live ? (uint32_t)lane : kDead;
  k.lc = live ? (uint32_t)lane * 8u : kDead;
  k.lam_scalar = (!PERDIFF && live) ? to_f64(static_cast<const TS*>(a.lam)[G.lam_off + p]) : 0.0;

  State<D, 1> st;
  int nobs = 0;
  const bool ok = k.sweep1(st, nobs, k.rev ? k.Tv - D : k.Tv);  // S counted once, by the top part
  SepPart<D> sp;
  k.separator_part(st, sp);
#pragma unroll
  for (int i = 0; i < NY; ++i) sep[half][i][lane] = sp.Y[i];
#pragma unroll
  for (int r = 0; r < D; ++r) sep[half][NY + r][lane] = sp.c[r];
  flag[half][lane] = (ok ? 1 : 0) | (nobs << 1);
  __syncthreads();
  const int o = 1 - half;
  double A[NY], rhs[D], Om[NY], bS[D];
  k.separator_omega(Om, bS);
#pragma unroll
  for (int i = 0; i < NY; ++i) A[i] = (sp.Y[i] + sep[o][i][lane]) - Om[i];
#pragma unroll
  for (int r = 0; r < D; ++r) rhs[r] = (sp.c[r] + sep[o][NY + r][lane]) - bS[r];
  const int fo = flag[o][lane];
  double zS[D];
  const bool sep_ok = solve_separator<D>(A, rhs, zS);
  const bool failed = !(ok && (fo & 1) && sep_ok) || nobs + (fo >> 1) < D;
  if (half == 0 && live && a.info) {
    int info = 0;
    if (failed) {
      info = k.first_bad_pivot();
      if (info == 0) info = T;  // too few observations, or a separator pivot lost to rounding
    }
    a.info[G.info_off + p] = info;
  }
  double zSv[D];
#pragma unroll
  for (int u = 0; u < D; ++u) zSv[u] = k.rev ? zS[D - 1 - u] : zS[u];
  k.sweep2(zSv, failed, !k.rev);
}

template <int PROF, typename TS, bool PERDIFF>
__device__ __forceinline__ void whole_item(const PlanArgs& a, int item, double* slot) {
  const int2 it = a.items[item];
  const GroupDev G = a.groups[it.x];
  switch (G.d) {
    case 1: plan_item<1, plan_tile(PROF, 1, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
    case 2: plan_item<2, plan_tile(PROF, 2, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
    case 3: plan_item<3, plan_tile(PROF, 3, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
    default: plan_item<4, plan_tile(PROF, 4, PERDIFF), TS, PERDIFF>(a, G, it.y, slot); break;
  }
}

// Two wavefronts per workgroup; a.n_waves counts workgroups here.
template <int PROF, typename TS, bool PERDIFF>
__global__ __launch_bounds__(128) void k_plan2(PlanArgs a) {
  __shared__ int s_unit[2];
  __shared__ double s_sep[2][kSepFields][64];
  __shared__ int s_flag[2][64];
  const int half = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double* slot = a.ck + ((int64_t)blockIdx.x * 2 + half) * a.ck_stride;
  for (int round = 0;; ++round) {
    // the unit slot alternates: a wavefront still reading last round's slot
    // cannot see it overwritten before the next barrier
    if (threadIdx.x == 0) s_unit[round & 1] = atomicAdd(&a.queue[0], 1);
    __syncthreads();
    const int u = s_unit[round & 1];
    if (u >= a.n_units) break;
    const int4 U = a.units[u];
    if (U.x == 0) {
      const int item = half == 0 ? U.y : U.z;
      if (item >= 0) whole_item<PROF, TS, PERDIFF>(a, item, slot);
    } else {
      const int2 it = a.items[U.y];
      const GroupDev G = a.groups[it.x];
      switch (G.d) {
        case 1: twist_item<1, plan_tile(PROF, 1, PERDIFF), TS, PERDIFF>(a, G, it.y, slot, half, s_sep, s_flag); break;
        case 2: twist_item<2, plan_tile(PROF, 2, PERDIFF), TS, PERDIFF>(a, G, it.y, slot, half, s_sep, s_flag); break;
        case 3: twist_item<3, plan_tile(PROF, 3, PERDIFF), TS, PERDIFF>(a, G, it.y, slot, half, s_sep, s_flag); break;
        default: twist_item<4, plan_tile(PROF, 4, PERDIFF), TS, PERDIFF>(a, G, it.y, slot, half, s_sep, s_flag); break;
      }
    }
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const int done = atomicAdd(&a.queue[1], 1);
    if (done == a.n_waves - 1) {
      atomicExch(&a.queue[0], 0);
      atomicExch(&a.queue[1], 0);
    }
  }
}

}  // namespace whs

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

using whs::GroupDev;
using whs::PlanArgs;

constexpr int kProfiles[] = {0, 1, 2};

struct Config {
  int tile = 1;            // tile profile (see plan_tile)
  int waves_per_block = 4;
  int waves_per_simd = 1;  // resident wavefronts per SIMD of the persistent grid
  int split_T = 0;         // series of at least this length take two lanes (0: none); two-wavefront blocks
};

template <int PROF, typename TS, bool PD>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&whs::k_plan<PROF, TS, PD>);
}

template <int PROF, typename TS, bool PD>
const void* kernel2_ptr() {
  return reinterpret_cast<const void*>(&whs::k_plan2<PROF, TS, PD>);
}

const void* pick_kernel2(int prof, bool f64, bool pd) {
  switch (prof) {
    case 0: return f64 ? (pd ? kernel2_ptr<0, double, true>() : kernel2_ptr<0, double, false>())
                       : (pd ? kernel2_ptr<0, float, true>() : kernel2_ptr<0, float, false>());
    case 2: return f64 ? (pd ? kernel2_ptr<2, double, true>() : kernel2_ptr<2, double, false>())
                       : (pd ? kernel2_ptr<2, float, true>() : kernel2_ptr<2, float, false>());
    default: return f64 ? (pd ? kernel2_ptr<1, double, true>() : kernel2_ptr<1, double, false>())
                        : (pd ? kernel2_ptr<1, float, true>() : kernel2_ptr<1, float, false>());
  }
}

const void* pick_kernel(int prof, bool f64, bool pd) {
  switch (prof) {
    case 0: return f64 ? (pd ? kernel_ptr<0, double, true>() : kernel_ptr<0, double, false>())
                       : (pd ? kernel_ptr<0, float, true>() : kernel_ptr<0, float, false>());
    case 2: return f64 ? (pd ? kernel_ptr<2, double, true>() : kernel_ptr<2, double, false>())
                       : (pd ? kernel_ptr<2, float, true>() : kernel_ptr<2, float, false>());
    default: return f64 ? (pd ? kernel_ptr<1, double, true>() : kernel_ptr<1, double, false>())
                        : (pd ? kernel_ptr<1, float, true>() : kernel_ptr<1, float, false>());
  }
}

int ck_fields_d(int d) {
  switch (d) {
    case 1: return whs::ck_fields<1, 1>();
    case 2: return whs::ck_fields<2, 1>();
    case 3: return whs::ck_fields<3, 1>();
    default: return whs::ck_fields<4, 1>();
  }
}

}  // namespace

struct whs_plan {
  int device = 0;
  int n_cu = 0;
  bool f64 = false;
  bool perdiff = false;
  std::vector<whs_group> host_groups;
  GroupDev* d_groups = nullptr;
  int2* d_items = nullptr;
  int n_items = 0;
  std::vector<int64_t> item_cost;  // per item, with its group
  std::vector<int> item_group;
  int4* d_units = nullptr;         // units of the two-lane kernel for cfg.split_T
  int n_units = 0;
  int units_split_T = -1;          // split_T the units were built for
  int* d_queue = nullptr;
  double* d_ck = nullptr;
  size_t ck_capacity = 0;  // doubles
  Config cfg;
  std::string key;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node = nullptr;
  PlanArgs graph_args{};
  std::mutex mu;
};

namespace {

int split_point_d(int d, int T) {
  switch (d) {
    case 1: return whs::split_point<1>(T);
    case 2: return whs::split_point<2>(T);
    case 3: return whs::split_point<3>(T);
    default: return whs::split_point<4>(T);
  }
}

// a group is split when the configuration asks for it and both parts keep a
// few tiles of interior
bool group_split(const whs_group& g, int split_T) { return split_T > 0 && g.T >= split_T && g.T >= 64; }

int64_t max_ck_doubles(const whs_plan* pl, int prof) {
  int64_t mx = 0;
  for (const auto& g : pl->host_groups) {
    const int B = whs::plan_tile(prof, g.d, pl->perdiff);
    int64_t nt = (g.T + B - 1) / B;
    const int m = split_point_d(g.d, g.T);
    nt = std::max<int64_t>(nt, std::max<int64_t>((m + g.d + B - 1) / B, (g.T - m + B - 1) / B));
    mx = std::max<int64_t>(mx, nt * ck_fields_d(g.d) * 64);
  }
  return mx;
}

bool two_lane(const Config& c) { return c.split_T > 0; }

// resident wavefronts of the persistent grid (both kernels), a multiple of the
// wavefronts per workgroup
int grid_waves(const whs_plan* pl, const Config& c) {
  const int waves = pl->n_cu * 4 * c.waves_per_simd;
  const int per_block = two_lane(c) ? 2 : c.waves_per_block;
  const int work = two_lane(c) ? 2 * pl->n_units : pl->n_items;
  return std::max(per_block, std::min(waves / per_block * per_block, ((work + per_block - 1) / per_block) * per_block));
}

// Units of the two-lane kernel: split blocks alone, whole blocks in pairs,
// in order of decreasing cost per wavefront (longest processing time first).
int build_units(whs_plan* pl, int split_T) {
  if (pl->units_split_T == split_T) return WHS_OK;
  std::vector<std::pair<int64_t, int>> pieces;  // (cost per wavefront, item; negative = split)
  for (int i = 0; i < pl->n_items; ++i) {
    const whs_group& g = pl->host_groups[pl->item_group[i]];
    if (group_split(g, split_T))
      pieces.push_back({pl->item_cost[i] / 2 + 1, -(i + 1)});
    else
      pieces.push_back({pl->item_cost[i], i});
  }
  std::stable_sort(pieces.begin(), pieces.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<int4> units;
  int pending = -1;
  for (const auto& pc : pieces) {
    if (pc.second < 0) {
      units.push_back(int4{1, -pc.second - 1, -1, 0});
    } else if (pending < 0) {
      pending = pc.second;
    } else {
      units.push_back(int4{0, pending, pc.second, 0});
      pending = -1;
    }
  }
  if (pending >= 0) units.push_back(int4{0, pending, -1, 0});
  if (pl->d_units) hipFree(pl->d_units);
  pl->d_units = nullptr;
  pl->n_units = (int)units.size();
  if (hipMalloc(&pl->d_units, sizeof(int4) * std::max<size_t>(units.size(), 1)) != hipSuccess) return WHS_ERR_HIP;
  if (!units.empty() &&
      hipMemcpy(pl->d_units, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice) != hipSuccess)
    return WHS_ERR_HIP;
  pl->units_split_T = split_T;
  return WHS_OK;
}

int ensure_ck(whs_plan* pl, const Config& c) {
  if (two_lane(c) && build_units(pl, c.split_T) != WHS_OK) return WHS_ERR_HIP;
  const size_t need = (size_t)grid_waves(pl, c) * (size_t)max_ck_doubles(pl, c.tile);
  if (need <= pl->ck_capacity) return WHS_OK;
  if (pl->d_ck) hipFree(pl->d_ck);
  pl->d_ck = nullptr;
  pl->ck_capacity = 0;
  if (hipMalloc(&pl->d_ck, std::max<size_t>(need, 1) * sizeof(double)) != hipSuccess) return WHS_ERR_HIP;
  pl->ck_capacity = need;
  return WHS_OK;
}

PlanArgs make_args(whs_plan* pl, const Config& c, const uint8_t* w, const void* lam, const void* x, void* z,
                   int32_t* info) {
  PlanArgs a{};
  a.groups = pl->d_groups;
  a.items = pl->d_items;
  a.n_items = pl->n_items;
  a.n_waves = grid_waves(pl, c);
  a.queue = pl->d_queue;
  a.w = w;
  a.lam = lam;
  a.x = x;
  a.z = z;
  a.info = info;
  a.ck = pl->d_ck;
  a.ck_stride = max_ck_doubles(pl, c.tile);
  a.units = pl->d_units;
  a.n_units = pl->n_units;
  if (two_lane(c)) a.n_waves /= 2;  // the two-lane kernel counts workgroups
  return a;
}

const void* kernel_for(const whs_plan* pl, const Config& c) {
  return two_lane(c) ? pick_kernel2(c.tile, pl->f64, pl->perdiff) : pick_kernel(c.tile, pl->f64, pl->perdiff);
}

dim3 grid_for(const Config& c, const PlanArgs& a) { return dim3(two_lane(c) ? a.n_waves : a.n_waves / c.waves_per_block); }
dim3 block_for(const Config& c) { return dim3(two_lane(c) ? 128 : 64 * c.waves_per_block); }

int launch(whs_plan* pl, const Config& c, const PlanArgs& a, hipStream_t stream) {
  void* args[] = {const_cast<PlanArgs*>(&a)};
  hipError_t e = hipLaunchKernel(kernel_for(pl, c), grid_for(c, a), block_for(c), args, 0, stream);
  return e == hipSuccess ? WHS_OK : WHS_ERR_HIP;
}

std::string cache_path() {
  if (const char* p = std::getenv("WHS_TUNE_CACHE")) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/whs_tune.txt";
}

bool cache_lookup(const std::string& key, Config& c) {
  FILE* f = std::fopen(cache_path().c_str(), "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[3900];
    int b, wpb, m, sp = 0;
    const int n = std::sscanf(line, "%3899s %d %d %d %d", k, &b, &wpb, &m, &sp);
    if (n >= 4 && key == k) {
      c.tile = b;
      c.waves_per_block = wpb;
      c.waves_per_simd = m;
      c.split_T = n == 5 ? sp : 0;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const std::string& key, const Config& c) {
  const std::string path = cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) mkdir(path.substr(0, slash).c_str(), 0755);  // best effort
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), c.tile, c.waves_per_block, c.waves_per_simd, c.split_T);
  std::fclose(f);
}

}  // namespace

extern "C" {

int whs_plan_create(whs_plan** out, const whs_group* groups, int32_t n_groups, int32_t n_rhs, int32_t dtype,
                    int32_t lambda_kind, int32_t interleave) {
  if (!out) return WHS_ERR_ARG;
  *out = nullptr;
  if (!groups || n_groups < 1) return WHS_ERR_ARG;
  if (dtype != WHS_F32 && dtype != WHS_F64) return WHS_ERR_ARG;
  if (lambda_kind != WHS_LAMBDA_SCALAR && lambda_kind != WHS_LAMBDA_PER_DIFF) return WHS_ERR_ARG;
  if (n_rhs != 1 || interleave != 64) return WHS_ERR_UNSUPPORTED;
  std::vector<GroupDev> gd;
  std::vector<std::pair<int64_t, int2>> items;
  for (int g = 0; g < n_groups; ++g) {
    const whs_group& G = groups[g];
    if (G.n_series < 0 || G.T < 1 || G.d < 1 || G.T <= G.d) return WHS_ERR_ARG;
    if (G.d > 4) return WHS_ERR_UNSUPPORTED;
    if (G.x_off < 0 || G.w_off < 0 || G.lam_off < 0 || G.info_off < 0) return WHS_ERR_ARG;
    // blocks of 64 series are addressed through 32-bit buffer ranges (x, z at
    // 8 bytes per value, and the per-wavefront checkpoint slot at up to 14
    // FP64 fields per 8-step tile): both stay below 2^31 bytes
    if ((int64_t)G.T * 64 * 8 * 2 >= ((int64_t)1 << 31)) return WHS_ERR_UNSUPPORTED;
    gd.push_back(GroupDev{G.x_off, G.w_off, G.lam_off, G.info_off, G.n_series, G.T, G.d});
    const int64_t nb = (G.n_series + 63) / 64;
    if (nb > 0x7fffffff) return WHS_ERR_UNSUPPORTED;
    const int64_t cost = (int64_t)G.T * (G.d + 2);
    for (int64_t b = 0; b < nb; ++b) items.push_back({cost, int2{g, (int)b}});
  }
  if (items.size() > 0x7fffffff) return WHS_ERR_UNSUPPORTED;
  // longest processing time first
  std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  auto* pl = new whs_plan();
  pl->f64 = dtype == WHS_F64;
  pl->perdiff = lambda_kind == WHS_LAMBDA_PER_DIFF;
  pl->host_groups.assign(groups, groups + n_groups);
  pl->n_items = (int)items.size();
  for (const auto& it : items) {
    pl->item_cost.push_back(it.first);
    pl->item_group.push_back(it.second.x);
  }
  hipGetDevice(&pl->device);
  hipDeviceGetAttribute(&pl->n_cu, hipDeviceAttributeMultiprocessorCount, pl->device);
  if (pl->n_cu <= 0) pl->n_cu = 256;
  std::vector<int2> it(items.size());
  for (size_t i = 0; i < items.size(); ++i) it[i] = items[i].second;
  bool ok = hipMalloc(&pl->d_groups, sizeof(GroupDev) * gd.size()) == hipSuccess &&
            hipMalloc(&pl->d_items, sizeof(int2) * std::max<size_t>(it.size(), 1)) == hipSuccess &&
            hipMalloc(&pl->d_queue, 2 * sizeof(int)) == hipSuccess;
  ok = ok && hipMemcpy(pl->d_groups, gd.data(), sizeof(GroupDev) * gd.size(), hipMemcpyHostToDevice) == hipSuccess;
  if (ok && !it.empty())
    ok = hipMemcpy(pl->d_items, it.data(), sizeof(int2) * it.size(), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemset(pl->d_queue, 0, 2 * sizeof(int)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  // tuning key: device, types and the (T, d, blocks) multiset
  char buf[128];
  std::snprintf(buf, sizeof buf, "cu%d|%s|%s", pl->n_cu, pl->f64 ? "f64" : "f32", pl->perdiff ? "pd" : "sc");
  pl->key = buf;
  for (const auto& g : pl->host_groups) {
    std::snprintf(buf, sizeof buf, "|%dx%dx%lld", g.T, g.d, (long long)((g.n_series + 63) / 64));
    pl->key += buf;
  }
  Config c;
  if (cache_lookup(pl->key, c)) pl->cfg = c;
  ok = ok && ensure_ck(pl, pl->cfg) == WHS_OK;
  if (!ok) {
    whs_plan_destroy(pl);
    return WHS_ERR_HIP;
  }
  *out = pl;
  return WHS_OK;
}

void whs_plan_destroy(whs_plan* pl) {
  if (!pl) return;
  if (pl->exec) hipGraphExecDestroy(pl->exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  if (pl->d_groups) hipFree(pl->d_groups);
  if (pl->d_items) hipFree(pl->d_items);
  if (pl->d_queue) hipFree(pl->d_queue);
  if (pl->d_ck) hipFree(pl->d_ck);
  if (pl->d_units) hipFree(pl->d_units);
  delete pl;
}

int whs_plan_solve(whs_plan* pl, const uint8_t* w, const void* lambda, const void* x, void* z, int32_t* info,
                   void* stream) {
  if (!pl || !w || !lambda || !x || !z) return WHS_ERR_ARG;
  std::lock_guard<std::mutex> lk(pl->mu);
  if (pl->n_items == 0) return WHS_OK;
  const PlanArgs a = make_args(pl, pl->cfg, w, lambda, x, z, info);
  return launch(pl, pl->cfg, a, static_cast<hipStream_t>(stream));
}

int whs_plan_graph_launch(whs_plan* pl, const uint8_t* w, const void* lambda, const void* x, void* z,
                          int32_t* info, void* stream) {
  if (!pl || !w || !lambda || !x || !z) return WHS_ERR_ARG;
  std::lock_guard<std::mutex> lk(pl->mu);
  if (pl->n_items == 0) return WHS_OK;
  const PlanArgs a = make_args(pl, pl->cfg, w, lambda, x, z, info);
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(kernel_for(pl, pl->cfg));
  kp.gridDim = grid_for(pl->cfg, a);
  kp.blockDim = block_for(pl->cfg);
  kp.sharedMemBytes = 0;
  pl->graph_args = a;
  void* args[] = {&pl->graph_args};
  kp.kernelParams = args;
  kp.extra = nullptr;
  if (!pl->exec) {
    if (hipGraphCreate(&pl->graph, 0) != hipSuccess) return WHS_ERR_HIP;
    if (hipGraphAddKernelNode(&pl->node, pl->graph, nullptr, 0, &kp) != hipSuccess) return WHS_ERR_HIP;
    if (hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess) return WHS_ERR_HIP;
  } else if (hipGraphExecKernelNodeSetParams(pl->exec, pl->node, &kp) != hipSuccess) {
    return WHS_ERR_HIP;
  }
  return hipGraphLaunch(pl->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? WHS_OK : WHS_ERR_HIP;
}

int whs_plan_autotune(whs_plan* pl, const uint8_t* w, const void* lambda, const void* x, void* z, int32_t force,
                      void* stream) {
  if (!pl || !w || !lambda || !x || !z) return WHS_ERR_ARG;
  std::lock_guard<std::mutex> lk(pl->mu);
  if (pl->n_items == 0) return WHS_OK;
  Config cached;
  if (!force && cache_lookup(pl->key, cached)) {
    pl->cfg = cached;
    return ensure_ck(pl, cached);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return WHS_ERR_HIP;
  float best = 1e30f;
  Config best_c = pl->cfg;
  // lanes per series: none split, or every group of at least T split for
  // each length T within a factor four of the longest
  std::vector<int> splits{0};
  int tmax = 0;
  for (const auto& g : pl->host_groups) tmax = std::max(tmax, g.T);
  for (const auto& g : pl->host_groups)
    if (4 * g.T >= tmax && g.T >= 64 && std::find(splits.begin(), splits.end(), g.T) == splits.end())
      splits.push_back(g.T);
  std::vector<Config> cands;
  for (int prof : kProfiles)
    for (int sp : splits)
      for (int wpb : sp ? std::vector<int>{2} : std::vector<int>{1, 2, 4})
        for (int m : {1, 2}) cands.push_back(Config{prof, wpb, m, sp});
  for (const Config& c : cands) {
    if (ensure_ck(pl, c) != WHS_OK) continue;
    const PlanArgs a = make_args(pl, c, w, lambda, x, z, nullptr);
    if (launch(pl, c, a, s) != WHS_OK) continue;  // warm-up
    hipEventRecord(e0, s);
    for (int r = 0; r < 3; ++r) launch(pl, c, a, s);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_c = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  pl->cfg = best_c;
  if (pl->exec) {  // the graph node must be rebuilt for the new kernel
    hipGraphExecDestroy(pl->exec);
    hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
  }
  cache_store(pl->key, best_c);
  return ensure_ck(pl, best_c);
}

int whs_plan_set_config(whs_plan* pl, int32_t tile, int32_t waves_per_block, int32_t waves_per_simd,
                        int32_t split_T) {
  if (!pl || tile < 0 || tile > 2 || (waves_per_simd != 1 && waves_per_simd != 2) || split_T < 0) return WHS_ERR_ARG;
  if (split_T > 0 ? waves_per_block != 2 : (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4))
    return WHS_ERR_ARG;
  std::lock_guard<std::mutex> lk(pl->mu);
  const Config c{tile, waves_per_block, waves_per_simd, split_T};
  const int st = ensure_ck(pl, c);
  if (st != WHS_OK) return st;
  pl->cfg = c;
  if (pl->exec) {  // the graph node must be rebuilt for the new kernel
    hipGraphExecDestroy(pl->exec);
    hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
  }
  return WHS_OK;
}

int whs_plan_lanes(const whs_plan* pl, int32_t group, int32_t* lanes_per_series) {
  if (!pl || !lanes_per_series || group < 0 || group >= (int32_t)pl->host_groups.size()) return WHS_ERR_ARG;
  *lanes_per_series = group_split(pl->host_groups[group], pl->cfg.split_T) ? 2 : 1;
  return WHS_OK;
}

int whs_plan_config(const whs_plan* pl, int32_t* tile, int32_t* waves_per_block, int32_t* waves_per_simd,
                    int32_t* n_items) {
  if (!pl) return WHS_ERR_ARG;
  if (tile) *tile = pl->cfg.tile;
  if (waves_per_block) *waves_per_block = pl->cfg.waves_per_block;
  if (waves_per_simd) *waves_per_simd = pl->cfg.waves_per_simd;
  if (n_items) *n_items = pl->n_items;
  return WHS_OK;
}

}  // extern "C"

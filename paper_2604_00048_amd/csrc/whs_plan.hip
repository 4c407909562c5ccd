// Uneven batches in one persistent launch.
//
// A plan covers groups of series that share a length T and an order d (the
// mask pads nothing: each group keeps its own T).  Work items are blocks of
// 64 series of one group, sorted longest-first on the host and served from
// a device queue: every resident wavefront takes the next item with one
// atomic, so long series start first and short ones fill the tail.  The
// kernel resets its own queue counters when the last wavefront leaves, so a
// launch can be replayed from a graph without a memset node.
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
};

// tile depth per order for each tuning profile: 0 = (8,8,8,8),
// 1 = (16,16,8,8), 2 = (24,16,8,8); deeper tiles store fewer checkpoints
// but hold more registers, which the higher orders cannot afford
__host__ __device__ constexpr int plan_tile(int prof, int d) {
  return d >= 3 ? 8 : (prof == 0 ? 8 : (prof == 1 ? 16 : (d == 1 ? 24 : 16)));
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
      case 1: plan_item<1, plan_tile(PROF, 1), TS, PERDIFF>(a, G, it.y, slot); break;
      case 2: plan_item<2, plan_tile(PROF, 2), TS, PERDIFF>(a, G, it.y, slot); break;
      case 3: plan_item<3, plan_tile(PROF, 3), TS, PERDIFF>(a, G, it.y, slot); break;
      default: plan_item<4, plan_tile(PROF, 4), TS, PERDIFF>(a, G, it.y, slot); break;
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
};

template <int PROF, typename TS, bool PD>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&whs::k_plan<PROF, TS, PD>);
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

int64_t max_ck_doubles(const whs_plan* pl, int prof) {
  int64_t mx = 0;
  for (const auto& g : pl->host_groups) {
    const int B = whs::plan_tile(prof, g.d);
    const int64_t nt = (g.T + B - 1) / B;
    mx = std::max<int64_t>(mx, nt * ck_fields_d(g.d) * 64);
  }
  return mx;
}

int grid_waves(const whs_plan* pl, const Config& c) {
  const int waves = pl->n_cu * 4 * c.waves_per_simd;
  const int per_block = c.waves_per_block;
  return std::max(per_block, std::min(waves, ((pl->n_items + per_block - 1) / per_block) * per_block));
}

int ensure_ck(whs_plan* pl, const Config& c) {
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
  return a;
}

int launch(whs_plan* pl, const Config& c, const PlanArgs& a, hipStream_t stream) {
  const int threads = 64 * c.waves_per_block;
  const int blocks = a.n_waves / c.waves_per_block;
  void* args[] = {const_cast<PlanArgs*>(&a)};
  hipError_t e = hipLaunchKernel(pick_kernel(c.tile, pl->f64, pl->perdiff), dim3(blocks), dim3(threads), args, 0,
                                 stream);
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
    int b, wpb, m;
    if (std::sscanf(line, "%3899s %d %d %d", k, &b, &wpb, &m) == 4 && key == k) {
      c.tile = b;
      c.waves_per_block = wpb;
      c.waves_per_simd = m;
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
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), c.tile, c.waves_per_block, c.waves_per_simd);
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
  kp.func = const_cast<void*>(pick_kernel(pl->cfg.tile, pl->f64, pl->perdiff));
  kp.gridDim = dim3(a.n_waves / pl->cfg.waves_per_block);
  kp.blockDim = dim3(64 * pl->cfg.waves_per_block);
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
  for (int prof : kProfiles) {
    for (int wpb : {1, 2, 4}) {
      for (int m : {1, 2}) {
        Config c{prof, wpb, m};
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

// C-ABI entry points of libwhs: argument validation and dispatch.
#include <hip/hip_runtime.h>

#include <mutex>

#include "whs.h"
#include "whs_kernels.h"

namespace {

constexpr int kMaxD = 4;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t elem(const whs_desc* d) { return d->dtype == WHS_F64 ? 8 : 4; }

// Interleaves that are a multiple of 64 run the kernels that address one block
// of S series through 32-bit buffer ranges, with byte offset 2^31 marking the
// padding lanes of a partial block: every per-block array (x, z, g, grad_x,
// w, lambda, and each kernel's checkpoint area) must stay below 2^31 bytes.
// Other interleaves use 64-bit addressing and have no such limit.
bool block_ranges_fit(const whs_desc* d) {
  if (d->interleave % 64 != 0) return true;
  constexpr uint64_t kLim = (uint64_t)1 << 31;
  const uint64_t rows = (uint64_t)d->T * (uint64_t)d->interleave;  // < 2^62
  if (rows >= kLim) return false;                                  // w; also bounds the products below
  if (rows * (uint64_t)d->n_rhs * elem(d) >= kLim) return false;   // x, z, g, grad_x (lambda is smaller)
  const int64_t S = d->interleave;
  if (whs::checkpoint_bytes(S, (int)S, d->T, d->d, d->n_rhs) >= kLim) return false;
  if (whs::var_checkpoint_bytes(S, (int)S, d->T, d->d) >= kLim) return false;
  return true;
}

int check_desc(const whs_desc* d) {
  if (!d) return WHS_ERR_ARG;
  if (d->n_series < 0 || d->T < 1 || d->d < 1 || d->n_rhs < 1 || d->interleave < 1) return WHS_ERR_ARG;
  if (d->dtype != WHS_F32 && d->dtype != WHS_F64) return WHS_ERR_ARG;
  if (d->lambda_kind != WHS_LAMBDA_SCALAR && d->lambda_kind != WHS_LAMBDA_PER_DIFF) return WHS_ERR_ARG;
  if (d->w_format != WHS_W_BYTES && d->w_format != WHS_W_BITS) return WHS_ERR_ARG;
  if (d->d > kMaxD) return WHS_ERR_UNSUPPORTED;
  if (d->T <= d->d) return WHS_ERR_ARG;
  // grid of ceil(P/256) blocks must fit one launch dimension
  if (d->n_series > (int64_t)0x7fffffff * 256) return WHS_ERR_UNSUPPORTED;
  if (!block_ranges_fit(d)) return WHS_ERR_UNSUPPORTED;
  return WHS_OK;
}

whs::LaunchDesc make_launch(const whs_desc* d) {
  whs::LaunchDesc L{};
  L.P = d->n_series;
  L.T = d->T;
  L.D = d->d;
  L.C = d->n_rhs;
  L.S = d->interleave;
  L.f64 = d->dtype == WHS_F64;
  L.perdiff = d->lambda_kind == WHS_LAMBDA_PER_DIFF;
  L.wbits = d->w_format == WHS_W_BITS;
  return L;
}

// Weights as bits are read by the fused one-band two-sweep kernels on the
// daily grid only: interleave a multiple of 64 (a block's row of w is then
// whole dwords), no given factor, P < 2^31 (the same conditions select those
// kernels), one band
bool bits_ok(const whs_desc* d, const double* factor) {
  if (d->w_format != WHS_W_BITS) return true;
  return d->interleave % 64 == 0 && !factor && d->n_series < ((int64_t)1 << 31) && d->n_rhs == 1;
}

int hip_status(hipError_t e) { return e == hipSuccess ? WHS_OK : WHS_ERR_HIP; }

// Series-contiguous calls (interleave 1) with a large enough workspace run the
// interleaved kernels on copies: slots for x (or g), z, grad_x, w, lambda and
// grad_lambda, then the interleaved kernels' checkpoints.
size_t up256(size_t n) { return (n + 255) / 256 * 256; }

struct Staged {
  size_t x, w, lam, ck;
  size_t total() const { return 3 * x + w + 2 * lam + ck; }
};

Staged staged_sizes(const whs_desc* d) {
  const size_t nb = (size_t)((d->n_series + 63) / 64);
  const size_t e = elem(d);
  Staged s{};
  s.x = up256(nb * 64 * (size_t)d->T * (size_t)d->n_rhs * e);
  s.w = up256(nb * 64 * (size_t)d->T);
  s.lam = d->lambda_kind == WHS_LAMBDA_PER_DIFF ? up256(nb * 64 * (size_t)(d->T - d->d) * e) : 0;
  s.ck = whs::checkpoint_bytes(d->n_series, 64, d->T, d->d, d->n_rhs);
  return s;
}

// Whether a series-contiguous call can run the interleaved kernels on copies:
// the copies' grids fit a launch, and one block of 64 series stays within the
// interleaved kernels' 32-bit ranges.
bool staged_fits(const whs_desc* d) {
  if (d->interleave != 1 || d->n_series <= 0 || d->n_series >= ((int64_t)1 << 31)) return false;
  if (!whs::interleave_fits(d->n_series, (int64_t)d->T * d->n_rhs, (int)elem(d))) return false;
  whs_desc d64 = *d;
  d64.interleave = 64;
  return block_ranges_fit(&d64);
}

bool use_staged(const whs_desc* d, const double* factor, size_t ws_bytes) {
  return !factor && staged_fits(d) && ws_bytes >= staged_sizes(d).total();
}

// GCV on copies: slots for x and w
size_t gcv_staged_bytes(const whs_desc* d) {
  const size_t nb = (size_t)((d->n_series + 63) / 64);
  return up256(nb * 64 * (size_t)d->T * elem(d)) + up256(nb * 64 * (size_t)d->T);
}

// The variance on copies: slots for w, lambda (per difference row), var, then
// the interleaved kernel's checkpoints
size_t var_staged_bytes(const whs_desc* d) {
  const size_t nb = (size_t)((d->n_series + 63) / 64);
  const size_t e = elem(d);
  const size_t lam = d->lambda_kind == WHS_LAMBDA_PER_DIFF ? up256(nb * 64 * (size_t)(d->T - d->d) * e) : 0;
  return up256(nb * 64 * (size_t)d->T) + lam + up256(nb * 64 * (size_t)d->T * e) +
         whs::var_checkpoint_bytes(d->n_series, 64, d->T, d->d);
}

struct Slots {
  char *x, *z, *gx, *lam, *glam;
  uint8_t* w;
  double* ck;
};

Slots carve(const Staged& s, void* ws) {
  char* p = static_cast<char*>(ws);
  Slots o{};
  o.x = p;
  o.z = (p += s.x);
  o.gx = (p += s.x);
  o.w = reinterpret_cast<uint8_t*>(p += s.x);
  o.lam = (p += s.w);
  o.glam = (p += s.lam);
  o.ck = reinterpret_cast<double*>(p += s.lam);
  return o;
}

hipError_t solve_staged(const whs_desc* d, const double* coef, const uint8_t* w, const void* lambda, const void* x,
                        void* z, int32_t* info, void* ws, hipStream_t s) {
  const Slots o = carve(staged_sizes(d), ws);
  const int64_t P = d->n_series, LX = (int64_t)d->T * d->n_rhs;
  const int e = (int)elem(d);
  const bool pd = d->lambda_kind == WHS_LAMBDA_PER_DIFF;
  hipError_t err = whs::launch_interleave(x, o.x, P, LX, e, true, s);
  if (err == hipSuccess) err = whs::launch_interleave(w, o.w, P, d->T, 1, true, s);
  if (err == hipSuccess && pd) err = whs::launch_interleave(lambda, o.lam, P, d->T - d->d, e, true, s);
  if (err != hipSuccess) return err;
  whs::LaunchDesc L = make_launch(d);
  L.S = 64;
  L.coef = coef;
  L.w = o.w;
  L.lam = pd ? static_cast<const void*>(o.lam) : lambda;
  L.rhs = o.x;
  L.out = o.z;
  L.info = info;
  L.ws = o.ck;
  err = whs::launch_solve(L, s);
  if (err != hipSuccess) return err;
  return whs::launch_interleave(o.z, z, P, LX, e, false, s);
}

hipError_t backward_staged(const whs_desc* d, const double* coef, const uint8_t* w, const void* lambda, const void* z,
                           const void* g, void* grad_x, void* grad_lambda, int32_t* info, void* ws, hipStream_t s) {
  const Slots o = carve(staged_sizes(d), ws);
  const int64_t P = d->n_series, LX = (int64_t)d->T * d->n_rhs;
  const int e = (int)elem(d);
  const bool pd = d->lambda_kind == WHS_LAMBDA_PER_DIFF;
  hipError_t err = whs::launch_interleave(g, o.x, P, LX, e, true, s);
  if (err == hipSuccess) err = whs::launch_interleave(z, o.z, P, LX, e, true, s);
  if (err == hipSuccess) err = whs::launch_interleave(w, o.w, P, d->T, 1, true, s);
  if (err == hipSuccess && pd) err = whs::launch_interleave(lambda, o.lam, P, d->T - d->d, e, true, s);
  if (err != hipSuccess) return err;
  whs::LaunchDesc L = make_launch(d);
  L.S = 64;
  L.coef = coef;
  L.w = o.w;
  L.lam = pd ? static_cast<const void*>(o.lam) : lambda;
  L.rhs = o.x;
  L.zin = o.z;
  L.out = grad_x ? o.gx : nullptr;
  L.glam = grad_lambda ? (pd ? static_cast<void*>(o.glam) : grad_lambda) : nullptr;
  L.info = info;
  L.ws = o.ck;
  err = whs::launch_backward(L, s);
  if (err == hipSuccess && grad_x) err = whs::launch_interleave(o.gx, grad_x, P, LX, e, false, s);
  if (err == hipSuccess && grad_lambda && pd)
    err = whs::launch_interleave(o.glam, grad_lambda, P, d->T - d->d, e, false, s);
  return err;
}

// Workspace of whs_solve_noalloc: a library-owned device array, one copy per
// GPU, held until the process ends.  Host code never passes its name to a
// kernel or a copy: the address of each device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of `scratch` (nullptr on failure).
void* scratch_for_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char* whs_status_str(int status) {
  switch (status) {
    case WHS_OK: return "ok";
    case WHS_ERR_ARG: return "invalid argument (descriptor, null or misaligned pointer)";
    case WHS_ERR_UNSUPPORTED:
      return "unsupported configuration (order d > 4, too many series, or a block of interleaved series of 2 GiB or more)";
    case WHS_ERR_HIP: return "HIP runtime or launch error";
    case WHS_ERR_WORKSPACE: return "workspace missing or smaller than whs_workspace_bytes()";
    default: return "unknown status";
  }
}

int whs_version(void) { return 100; }

#ifndef WHS_BUILD_ID
#define WHS_BUILD_ID "unknown"
#endif
const char* whs_build_id(void) { return WHS_BUILD_ID; }

size_t whs_workspace_bytes(const whs_desc* desc) {
  if (check_desc(desc) != WHS_OK || desc->n_series == 0) return 0;
  return whs::checkpoint_bytes(desc->n_series, desc->interleave, desc->T, desc->d, desc->n_rhs);
}

size_t whs_interleave_workspace_bytes(const whs_desc* desc) {
  if (check_desc(desc) != WHS_OK || desc->n_series == 0 || desc->interleave != 1) return 0;
  if (!staged_fits(desc)) return 0;
  return staged_sizes(desc).total();
}

size_t whs_factor_bytes(const whs_desc* desc) {
  if (check_desc(desc) != WHS_OK) return 0;
  const int64_t nb = (desc->n_series + desc->interleave - 1) / desc->interleave;
  return (size_t)nb * desc->interleave * (desc->d + 1) * (size_t)desc->T * sizeof(double);
}

int whs_factor(const whs_desc* desc, const uint8_t* w, const void* lambda, double* factor, int32_t* info,
               void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->w_format == WHS_W_BITS) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !lambda || !factor) return WHS_ERR_ARG;
  if (!aligned(lambda, elem(desc)) || !aligned(factor, 8) || !aligned(info, 4)) return WHS_ERR_ARG;
  whs::LaunchDesc L = make_launch(desc);
  L.w = w;
  L.lam = lambda;
  L.fac = factor;
  L.info = info;
  return hip_status(whs::launch_factor(L, static_cast<hipStream_t>(stream)));
}

int whs_solve(const whs_desc* desc, const uint8_t* w, const void* lambda, const double* factor, const void* x,
              void* z, int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (!bits_ok(desc, factor)) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !x || !z) return WHS_ERR_ARG;
  if (!factor && !lambda) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(x, e) || !aligned(z, e) || (lambda && !aligned(lambda, e)) || !aligned(factor, 8) ||
      !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  if (use_staged(desc, factor, workspace_bytes))
    return hip_status(solve_staged(desc, nullptr, w, lambda, x, z, info, workspace, static_cast<hipStream_t>(stream)));
  whs::LaunchDesc L = make_launch(desc);
  L.w = w;
  L.lam = lambda;
  L.fac = factor;
  L.rhs = x;
  L.out = z;
  L.info = info;
  L.ws = static_cast<double*>(workspace);
  return hip_status(whs::launch_solve(L, static_cast<hipStream_t>(stream)));
}

size_t whs_solve_noalloc_max_bytes(void) { return kNoallocScratchBytes; }

int whs_solve_noalloc(const whs_desc* desc, const uint8_t* w, const void* lambda, const void* x, void* z,
                      int32_t* info, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->n_series == 0) return WHS_OK;
  if (whs_workspace_bytes(desc) > kNoallocScratchBytes) return WHS_ERR_UNSUPPORTED;
  if (!w || !lambda || !x || !z) return WHS_ERR_ARG;
  void* ws = scratch_for_current_device();
  if (!ws) return WHS_ERR_HIP;
  // the scratch array is passed as an ordinary workspace: whs_solve picks the
  // interleaved copies for interleave 1 when they fit, and allocates nothing
  return whs_solve(desc, w, lambda, nullptr, x, z, info, ws, kNoallocScratchBytes, stream);
}

int whs_backward(const whs_desc* desc, const uint8_t* w, const void* lambda, const double* factor, const void* z,
                 const void* g, void* grad_x, void* grad_lambda, int32_t* info, void* workspace,
                 size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (!bits_ok(desc, factor)) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !z || !g) return WHS_ERR_ARG;
  if (!factor && !lambda) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(z, e) || !aligned(g, e) || !aligned(grad_x, e) || !aligned(grad_lambda, e) ||
      (lambda && !aligned(lambda, e)) || !aligned(factor, 8) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  if (!grad_x && !grad_lambda && !info) return WHS_OK;
  if (use_staged(desc, factor, workspace_bytes))
    return hip_status(backward_staged(desc, nullptr, w, lambda, z, g, grad_x, grad_lambda, info, workspace,
                                      static_cast<hipStream_t>(stream)));
  whs::LaunchDesc L = make_launch(desc);
  L.w = w;
  L.lam = lambda;
  L.fac = factor;
  L.rhs = g;
  L.zin = z;
  L.out = grad_x;
  L.glam = grad_lambda;
  L.info = info;
  L.ws = static_cast<double*>(workspace);
  return hip_status(whs::launch_backward(L, static_cast<hipStream_t>(stream)));
}

int whs_diff_coef(const double* times, int32_t T, int32_t d, double* coef, void* stream) {
  if (d < 1 || T <= d) return d > kMaxD ? WHS_ERR_UNSUPPORTED : WHS_ERR_ARG;
  if (d > kMaxD) return WHS_ERR_UNSUPPORTED;
  if (!times || !coef || !aligned(times, 8) || !aligned(coef, 8)) return WHS_ERR_ARG;
  return hip_status(whs::launch_diff_coef(times, T, d, coef, static_cast<hipStream_t>(stream)));
}

int whs_solve_coef(const whs_desc* desc, const double* coef, const uint8_t* w, const void* lambda, const void* x,
                   void* z, int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->w_format == WHS_W_BITS) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return desc->interleave % 64 == 0 || desc->interleave == 1 ? WHS_OK : WHS_ERR_UNSUPPORTED;
  const bool stg = use_staged(desc, nullptr, workspace_bytes);
  if (!stg && (desc->interleave % 64 != 0 || desc->n_series >= ((int64_t)1 << 31))) return WHS_ERR_UNSUPPORTED;
  if (!coef || !w || !lambda || !x || !z) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(coef, 8) || !aligned(x, e) || !aligned(z, e) || !aligned(lambda, e) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  if (stg) return hip_status(solve_staged(desc, coef, w, lambda, x, z, info, workspace, static_cast<hipStream_t>(stream)));
  whs::LaunchDesc L = make_launch(desc);
  L.coef = coef;
  L.w = w;
  L.lam = lambda;
  L.rhs = x;
  L.out = z;
  L.info = info;
  L.ws = static_cast<double*>(workspace);
  return hip_status(whs::launch_solve(L, static_cast<hipStream_t>(stream)));
}

int whs_backward_coef(const whs_desc* desc, const double* coef, const uint8_t* w, const void* lambda, const void* z,
                      const void* g, void* grad_x, void* grad_lambda, int32_t* info, void* workspace,
                      size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->w_format == WHS_W_BITS) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return desc->interleave % 64 == 0 || desc->interleave == 1 ? WHS_OK : WHS_ERR_UNSUPPORTED;
  const bool stg = use_staged(desc, nullptr, workspace_bytes);
  if (!stg && (desc->interleave % 64 != 0 || desc->n_series >= ((int64_t)1 << 31))) return WHS_ERR_UNSUPPORTED;
  if (!coef || !w || !lambda || !z || !g) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(coef, 8) || !aligned(z, e) || !aligned(g, e) || !aligned(grad_x, e) || !aligned(grad_lambda, e) ||
      !aligned(lambda, e) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  if (!grad_x && !grad_lambda && !info) return WHS_OK;
  if (stg)
    return hip_status(backward_staged(desc, coef, w, lambda, z, g, grad_x, grad_lambda, info, workspace,
                                      static_cast<hipStream_t>(stream)));
  whs::LaunchDesc L = make_launch(desc);
  L.coef = coef;
  L.w = w;
  L.lam = lambda;
  L.rhs = g;
  L.zin = z;
  L.out = grad_x;
  L.glam = grad_lambda;
  L.info = info;
  L.ws = static_cast<double*>(workspace);
  return hip_status(whs::launch_backward(L, static_cast<hipStream_t>(stream)));
}

size_t whs_gcv_workspace_bytes(const whs_desc* desc) {
  // one forward sweep, nothing kept; series-contiguous calls copy x and w
  if (check_desc(desc) != WHS_OK || !staged_fits(desc)) return 0;
  return gcv_staged_bytes(desc);
}

int whs_gcv(const whs_desc* desc, const uint8_t* w, const void* x, const double* grid, int32_t n_grid,
            void* lambda_best, double* scores, int32_t* info, void* workspace, size_t workspace_bytes,
            void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->w_format == WHS_W_BITS) return WHS_ERR_UNSUPPORTED;
  if (desc->n_rhs != 1 || desc->lambda_kind != WHS_LAMBDA_SCALAR) return WHS_ERR_UNSUPPORTED;
  if ((desc->interleave % 64 != 0 && desc->interleave != 1) || desc->n_series >= ((int64_t)1 << 31))
    return WHS_ERR_UNSUPPORTED;
  if (n_grid < 1) return WHS_ERR_ARG;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !x || !grid || !lambda_best) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(x, e) || !aligned(lambda_best, e) || !aligned(grid, 8) || !aligned(scores, 8) || !aligned(info, 4))
    return WHS_ERR_ARG;
  const bool staged = desc->interleave == 1;
  if (staged) {
    if (!staged_fits(desc)) return WHS_ERR_UNSUPPORTED;
    if (!workspace || workspace_bytes < gcv_staged_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  whs::GcvLaunch L{};
  L.P = desc->n_series;
  L.T = desc->T;
  L.D = desc->d;
  L.S = desc->interleave;
  L.n_grid = n_grid;
  L.f64 = desc->dtype == WHS_F64;
  L.w = w;
  L.x = x;
  L.grid = grid;
  L.lam_best = lambda_best;
  L.scores = scores;
  L.info = info;
  if (staged) {
    // lambda_best, scores and info are per series in either layout
    char* xs = static_cast<char*>(workspace);
    uint8_t* ws8 = reinterpret_cast<uint8_t*>(xs + up256((size_t)((L.P + 63) / 64) * 64 * (size_t)L.T * e));
    hipError_t err = whs::launch_interleave(x, xs, L.P, L.T, (int)e, true, s);
    if (err == hipSuccess) err = whs::launch_interleave(w, ws8, L.P, L.T, 1, true, s);
    if (err != hipSuccess) return hip_status(err);
    L.S = 64;
    L.x = xs;
    L.w = ws8;
  }
  return hip_status(whs::launch_gcv(L, s));
}

size_t whs_variance_workspace_bytes(const whs_desc* desc) {
  if (check_desc(desc) != WHS_OK || desc->n_series == 0) return 0;
  if (desc->interleave == 1) return staged_fits(desc) ? var_staged_bytes(desc) : 0;
  return whs::var_checkpoint_bytes(desc->n_series, desc->interleave, desc->T, desc->d);
}

int whs_variance(const whs_desc* desc, const uint8_t* w, const void* lambda, void* var, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->w_format == WHS_W_BITS) return WHS_ERR_UNSUPPORTED;
  if (desc->n_rhs != 1) return WHS_ERR_ARG;
  if ((desc->interleave % 64 != 0 && desc->interleave != 1) || desc->n_series >= ((int64_t)1 << 31))
    return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !lambda || !var) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(lambda, e) || !aligned(var, e) || !aligned(info, 4)) return WHS_ERR_ARG;
  const bool staged = desc->interleave == 1;
  if (staged && !staged_fits(desc)) return WHS_ERR_UNSUPPORTED;
  if (!workspace || workspace_bytes < whs_variance_workspace_bytes(desc) || !aligned(workspace, 8))
    return WHS_ERR_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  whs::LaunchDesc L = make_launch(desc);
  L.w = w;
  L.lam = lambda;
  L.out = var;
  L.info = info;
  L.ws = static_cast<double*>(workspace);
  if (!staged) return hip_status(whs::launch_var(L, s));
  // copies of w and lambda (per difference row) in, var out; a scalar lambda
  // and info are per series in either layout
  const size_t nb = (size_t)((L.P + 63) / 64);
  const bool pd = desc->lambda_kind == WHS_LAMBDA_PER_DIFF;
  char* p = static_cast<char*>(workspace);
  uint8_t* wc = reinterpret_cast<uint8_t*>(p);
  char* lc = (p += up256(nb * 64 * (size_t)L.T));
  char* vc = (p += pd ? up256(nb * 64 * (size_t)(L.T - L.D) * e) : 0);
  double* ck = reinterpret_cast<double*>(p += up256(nb * 64 * (size_t)L.T * e));
  hipError_t err = whs::launch_interleave(w, wc, L.P, L.T, 1, true, s);
  if (err == hipSuccess && pd) err = whs::launch_interleave(lambda, lc, L.P, L.T - L.D, (int)e, true, s);
  if (err != hipSuccess) return hip_status(err);
  L.S = 64;
  L.w = wc;
  L.lam = pd ? static_cast<const void*>(lc) : lambda;
  L.out = vc;
  L.ws = ck;
  err = whs::launch_var(L, s);
  if (err == hipSuccess) err = whs::launch_interleave(vc, var, L.P, L.T, (int)e, false, s);
  return hip_status(err);
}

}  // extern "C"

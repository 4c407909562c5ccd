// C-ABI entry points of libwhs: argument validation and dispatch.
#include <hip/hip_runtime.h>

#include "whs.h"
#include "whs_kernels.h"

namespace {

constexpr int kMaxD = 4;

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int check_desc(const whs_desc* d) {
  if (!d) return WHS_ERR_ARG;
  if (d->n_series < 0 || d->T < 1 || d->d < 1 || d->n_rhs < 1 || d->interleave < 1) return WHS_ERR_ARG;
  if (d->dtype != WHS_F32 && d->dtype != WHS_F64) return WHS_ERR_ARG;
  if (d->lambda_kind != WHS_LAMBDA_SCALAR && d->lambda_kind != WHS_LAMBDA_PER_DIFF) return WHS_ERR_ARG;
  if (d->d > kMaxD) return WHS_ERR_UNSUPPORTED;
  if (d->T <= d->d) return WHS_ERR_ARG;
  // grid of ceil(P/256) blocks must fit one launch dimension
  if (d->n_series > (int64_t)0x7fffffff * 256) return WHS_ERR_UNSUPPORTED;
  return WHS_OK;
}

size_t elem(const whs_desc* d) { return d->dtype == WHS_F64 ? 8 : 4; }

whs::LaunchDesc make_launch(const whs_desc* d) {
  whs::LaunchDesc L{};
  L.P = d->n_series;
  L.T = d->T;
  L.D = d->d;
  L.C = d->n_rhs;
  L.S = d->interleave;
  L.f64 = d->dtype == WHS_F64;
  L.perdiff = d->lambda_kind == WHS_LAMBDA_PER_DIFF;
  return L;
}

int hip_status(hipError_t e) { return e == hipSuccess ? WHS_OK : WHS_ERR_HIP; }

}  // namespace

extern "C" {

const char* whs_status_str(int status) {
  switch (status) {
    case WHS_OK: return "ok";
    case WHS_ERR_ARG: return "invalid argument (descriptor, null or misaligned pointer)";
    case WHS_ERR_UNSUPPORTED: return "unsupported configuration (order d > 4 or too many series)";
    case WHS_ERR_HIP: return "HIP runtime or launch error";
    case WHS_ERR_WORKSPACE: return "workspace missing or smaller than whs_workspace_bytes()";
    default: return "unknown status";
  }
}

int whs_version(void) { return 100; }

size_t whs_workspace_bytes(const whs_desc* desc) {
  if (check_desc(desc) != WHS_OK || desc->n_series == 0) return 0;
  return whs::checkpoint_bytes(desc->n_series, desc->interleave, desc->T, desc->d, desc->n_rhs);
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
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !x || !z) return WHS_ERR_ARG;
  if (!factor && !lambda) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(x, e) || !aligned(z, e) || (lambda && !aligned(lambda, e)) || !aligned(factor, 8) ||
      !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
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

int whs_backward(const whs_desc* desc, const uint8_t* w, const void* lambda, const double* factor, const void* z,
                 const void* g, void* grad_x, void* grad_lambda, int32_t* info, void* workspace,
                 size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !z || !g) return WHS_ERR_ARG;
  if (!factor && !lambda) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(z, e) || !aligned(g, e) || !aligned(grad_x, e) || !aligned(grad_lambda, e) ||
      (lambda && !aligned(lambda, e)) || !aligned(factor, 8) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  if (!grad_x && !grad_lambda && !info) return WHS_OK;
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
  if (desc->interleave % 64 != 0 || desc->n_series >= ((int64_t)1 << 31)) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!coef || !w || !lambda || !x || !z) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(coef, 8) || !aligned(x, e) || !aligned(z, e) || !aligned(lambda, e) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
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
  if (desc->interleave % 64 != 0 || desc->n_series >= ((int64_t)1 << 31)) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!coef || !w || !lambda || !z || !g) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(coef, 8) || !aligned(z, e) || !aligned(g, e) || !aligned(grad_x, e) || !aligned(grad_lambda, e) ||
      !aligned(lambda, e) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_workspace_bytes(desc) || !aligned(workspace, 8)) return WHS_ERR_WORKSPACE;
  if (!grad_x && !grad_lambda && !info) return WHS_OK;
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
  if (check_desc(desc) != WHS_OK || desc->n_series == 0) return 0;
  return whs::gcv_checkpoint_bytes(desc->n_series, desc->interleave, desc->T, desc->d);
}

int whs_gcv(const whs_desc* desc, const uint8_t* w, const void* x, const double* grid, int32_t n_grid,
            void* lambda_best, double* scores, int32_t* info, void* workspace, size_t workspace_bytes,
            void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->n_rhs != 1 || desc->lambda_kind != WHS_LAMBDA_SCALAR) return WHS_ERR_UNSUPPORTED;
  if (desc->interleave % 64 != 0 || desc->n_series >= ((int64_t)1 << 31)) return WHS_ERR_UNSUPPORTED;
  if (n_grid < 1) return WHS_ERR_ARG;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !x || !grid || !lambda_best) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(x, e) || !aligned(lambda_best, e) || !aligned(grid, 8) || !aligned(scores, 8) || !aligned(info, 4))
    return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_gcv_workspace_bytes(desc) || !aligned(workspace, 8))
    return WHS_ERR_WORKSPACE;
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
  L.ws = static_cast<double*>(workspace);
  return hip_status(whs::launch_gcv(L, static_cast<hipStream_t>(stream)));
}

size_t whs_variance_workspace_bytes(const whs_desc* desc) {
  if (check_desc(desc) != WHS_OK || desc->n_series == 0) return 0;
  return whs::var_checkpoint_bytes(desc->n_series, desc->interleave, desc->T, desc->d);
}

int whs_variance(const whs_desc* desc, const uint8_t* w, const void* lambda, void* var, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream) {
  int st = check_desc(desc);
  if (st != WHS_OK) return st;
  if (desc->n_rhs != 1) return WHS_ERR_ARG;
  if (desc->interleave % 64 != 0 || desc->n_series >= ((int64_t)1 << 31)) return WHS_ERR_UNSUPPORTED;
  if (desc->n_series == 0) return WHS_OK;
  if (!w || !lambda || !var) return WHS_ERR_ARG;
  const size_t e = elem(desc);
  if (!aligned(lambda, e) || !aligned(var, e) || !aligned(info, 4)) return WHS_ERR_ARG;
  if (!workspace || workspace_bytes < whs_variance_workspace_bytes(desc) || !aligned(workspace, 8))
    return WHS_ERR_WORKSPACE;
  whs::LaunchDesc L = make_launch(desc);
  L.w = w;
  L.lam = lambda;
  L.out = var;
  L.info = info;
  L.ws = static_cast<double*>(workspace);
  return hip_status(whs::launch_var(L, static_cast<hipStream_t>(stream)));
}

}  // extern "C"

// SpMV shape autotuning: every level of a hierarchy is multiplied with each
// row-group shape in FP64 and (when built) FP32, and the fastest shape is
// kept per level and precision; on the fine level the FP64 residual product
// of the refinement loop is timed and chosen on its own.  The timed launches
// are the ones the solver issues, on the library stream, bracketed by HIP
// events.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "spmv.h"

namespace rt {
namespace {

// One untimed launch, then reps timed ones of the product in `mode`: the
// Krylov loop's y = A x with x.y partials (SP_DOT), or the refinement's FP64
// residual r = b - A x with its FP32 copy, partials and componentwise maxima
// (SP_RESID, FP64 only).
template <typename T, int MODE>
int time_shape(rt_ctx* ctx, const Level& L, const T* val, const T* diag, T* y, float* y32,
               double* part, double* pmax, int shape, int reps, double* us) {
  hipStream_t st = ctx->stream;
  auto launch = [&]() {
    return launch_spmv_level<T, MODE>(st, L, val, diag, diag, diag, nullptr, y, y32, part, nullptr,
                                      shape, nullptr, nullptr, pmax, nullptr);
  };
  RT_CHECK(launch());
  RT_CHECK_HIP(hipEventRecord(ctx->ev0, st));
  for (int r = 0; r < reps; ++r) RT_CHECK(launch());
  RT_CHECK_HIP(hipEventRecord(ctx->ev1, st));
  RT_CHECK_HIP(hipEventSynchronize(ctx->ev1));
  float ms = 0.f;
  RT_CHECK_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  *us = 1e3 * (double)ms / reps;
  return RT_OK;
}

}  // namespace
}  // namespace rt

extern "C" {

int rt_spmv_shapes(int* g, int* ent, int* tiled, int max) {
  using namespace rt;
  for (int s = 0; s < kNumSpmvShapes && s < max; ++s) {
    if (g) g[s] = kSpmvShapes[s].g;
    if (ent) ent[s] = kSpmvShapes[s].ent;
    if (tiled) tiled[s] = kSpmvShapes[s].tiled ? 1 : 0;
  }
  return kNumSpmvShapes;
}

int rt_matrix_set_spmv_shape(rt_matrix* A, int level, int precision, int shape) {
  using namespace rt;
  clear_error();
  if (!A || level < 0 || level >= (int)A->levels.size() ||
      (precision != RT_PREC_FP64 && precision != RT_PREC_MIXED &&
       precision != RT_PRODUCT_RESIDUAL) || shape < -1 || shape >= kNumSpmvShapes) {
    set_error("rt_matrix_set_spmv_shape: bad matrix, level, precision or shape");
    return RT_E_ARG;
  }
  Level& L = A->levels[level];
  (precision == RT_PREC_FP64 ? L.shape64 : precision == RT_PREC_MIXED ? L.shape32 : L.shape_res) =
      shape;
  return RT_OK;
}

int rt_matrix_tune(rt_ctx* ctx, rt_matrix* A, int reps, rt_tune_report* rep) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || reps < 1) {
    set_error("rt_matrix_tune: NULL argument or reps < 1");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  rt_tune_report local{};
  rt_tune_report* r = rep ? rep : &local;
  std::memset(r, 0, sizeof(*r));
  const int nl = std::min<int>((int)A->levels.size(), RT_MAX_LEVELS);
  r->levels = nl;
  r->shapes = std::min(kNumSpmvShapes, RT_MAX_SHAPES);
  int64_t nmax = 0;
  for (int l = 0; l < nl; ++l) nmax = std::max(nmax, A->levels[l].n);
  DevBuf<double> y, part, pmax;
  DevBuf<float> y32;
  RT_CHECK(y.reserve(std::max<int64_t>(nmax, 1)));
  RT_CHECK(y32.reserve(std::max<int64_t>(nmax, 1)));
  RT_CHECK(part.reserve(max_partials(nmax)));
  RT_CHECK(pmax.reserve(max_partials(nmax)));
  for (int l = 0; l < nl; ++l) {
    Level& L = A->levels[l];
    r->chosen[l][0] = r->chosen[l][1] = r->chosen[l][2] = -1;
    if (L.n == 0) continue;
    for (int p = 0; p < 3; ++p) {
      if (p == 1 && !A->has_fp32) continue;
      if (p == 2 && (l > 0 || !A->has_fp32)) continue;   // refinement residuals: fine level
      double best = 0.0;
      int arg = -1;
      for (int s = 0; s < r->shapes; ++s) {
        if (kSpmvShapes[s].tiled && !L.tiled) continue;
        double us = 0.0;
        if (p == 0)
          RT_CHECK((time_shape<double, SP_DOT>(ctx, L, L.val64.p, L.diag64.p, y.p, nullptr, part.p,
                                               nullptr, s, reps, &us)));
        else if (p == 1)
          RT_CHECK((time_shape<float, SP_DOT>(ctx, L, L.val32.p, L.diag32.p, (float*)y.p, nullptr,
                                              part.p, nullptr, s, reps, &us)));
        else
          RT_CHECK((time_shape<double, SP_RESID>(ctx, L, L.val64.p, L.diag64.p, y.p, y32.p, part.p,
                                                 pmax.p, s, reps, &us)));
        r->us[l][p][s] = us;
        if (arg < 0 || us < best) {
          best = us;
          arg = s;
        }
      }
      r->chosen[l][p] = arg;
      (p == 0 ? L.shape64 : p == 1 ? L.shape32 : L.shape_res) = arg;
    }
  }
  return RT_OK;
}

int rt_matrix_set_cycle_depth(rt_matrix* A, int depth) {
  using namespace rt;
  clear_error();
  if (!A || depth < 0) {
    set_error("rt_matrix_set_cycle_depth: NULL matrix or negative depth");
    return RT_E_ARG;
  }
  A->cycle_levels = depth;
  return RT_OK;
}

int rt_matrix_tune_depth(rt_ctx* ctx, rt_matrix* A, const double* b, const double* x0,
                         const rt_solve_opts* opts, int reps, rt_depth_report* rep) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || !opts || reps < 1 || (A->n > 0 && (!b || !x0))) {
    set_error("rt_matrix_tune_depth: NULL argument or reps < 1");
    return RT_E_ARG;
  }
  if (opts->precond != 1) {
    set_error("rt_matrix_tune_depth: the solve options must use the V-cycle (precond 1)");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt_depth_report local{};
  rt_depth_report* r = rep ? rep : &local;
  *r = rt_depth_report{};
  const int nl = std::min<int>((int)A->levels.size(), RT_MAX_LEVELS);
  r->depths = nl;
  r->chosen = nl;
  if (A->n == 0 || nl == 0) return RT_OK;
  DevBuf<double> x;
  {
    rt::StreamScope scope(ctx->stream);
    RT_CHECK(x.reserve(A->n));
  }
  const int keep = A->cycle_levels;
  double best = 0.0;
  int arg = -1;
  for (int d = 1; d <= nl; ++d) {
    A->cycle_levels = d;
    double total = 0.0;
    int status = RT_OK;
    rt_solve_stats st{};
    for (int k = 0; k < reps; ++k) {
      RT_CHECK_HIP(hipMemcpyAsync(x.p, x0, sizeof(double) * A->n, hipMemcpyDeviceToDevice,
                                  ctx->stream));
      const int s = rt_solve(ctx, A, b, x.p, opts, &st);
      if (s < 0) {
        A->cycle_levels = keep;
        return s;
      }
      if (s == RT_NOT_CONVERGED) status = RT_NOT_CONVERGED;
      total += st.seconds;
    }
    r->seconds[d - 1] = total / reps;
    r->iterations[d - 1] = st.iterations;
    r->status[d - 1] = status;
    if (status == RT_OK && (arg < 0 || r->seconds[d - 1] < best)) {
      best = r->seconds[d - 1];
      arg = d;
    }
  }
  clear_error();   // a depth that did not converge is only left out
  r->chosen = arg > 0 ? arg : nl;
  A->cycle_levels = r->chosen == nl ? 0 : r->chosen;
  return RT_OK;
}

}  // extern "C"

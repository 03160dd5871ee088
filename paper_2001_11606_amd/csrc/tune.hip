// SpMV shape autotuning: every level of a hierarchy is multiplied with each
// row-group shape in FP64 and (when built) FP32, and the fastest shape is
// kept per level and precision.  The timed launch is the one the Krylov loop
// issues (y = A x with the per-block x.y partials), on the library stream,
// bracketed by HIP events.
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "spmv.h"

namespace rt {
namespace {

template <typename T>
int time_shape(rt_ctx* ctx, const Level& L, const T* val, const T* diag, T* y, double* part,
               int shape, int reps, double* us) {
  hipStream_t st = ctx->stream;
  // one untimed launch, then reps timed ones
  RT_CHECK((launch_spmv_level<T, SP_DOT>(st, L, val, diag, diag, nullptr, nullptr, y, nullptr, part,
                                         nullptr, shape)));
  RT_CHECK_HIP(hipEventRecord(ctx->ev0, st));
  for (int r = 0; r < reps; ++r)
    RT_CHECK((launch_spmv_level<T, SP_DOT>(st, L, val, diag, diag, nullptr, nullptr, y, nullptr,
                                           part, nullptr, shape)));
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
      (precision != RT_PREC_FP64 && precision != RT_PREC_MIXED) || shape < -1 ||
      shape >= kNumSpmvShapes) {
    set_error("rt_matrix_set_spmv_shape: bad matrix, level, precision or shape");
    return RT_E_ARG;
  }
  Level& L = A->levels[level];
  (precision == RT_PREC_FP64 ? L.shape64 : L.shape32) = shape;
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
  DevBuf<double> y, part;
  RT_CHECK(y.reserve(std::max<int64_t>(nmax, 1)));
  RT_CHECK(part.reserve(max_partials(nmax)));
  for (int l = 0; l < nl; ++l) {
    Level& L = A->levels[l];
    r->chosen[l][0] = r->chosen[l][1] = -1;
    if (L.n == 0) continue;
    for (int p = 0; p < 2; ++p) {
      if (p == 1 && !A->has_fp32) continue;
      double best = 0.0;
      int arg = -1;
      for (int s = 0; s < r->shapes; ++s) {
        if (kSpmvShapes[s].tiled && !L.tiled) continue;
        double us = 0.0;
        if (p == 0)
          RT_CHECK(time_shape<double>(ctx, L, L.val64.p, L.diag64.p, y.p, part.p, s, reps, &us));
        else
          RT_CHECK(time_shape<float>(ctx, L, L.val32.p, L.diag32.p, (float*)y.p, part.p, s, reps,
                                     &us));
        r->us[l][p][s] = us;
        if (arg < 0 || us < best) {
          best = us;
          arg = s;
        }
      }
      r->chosen[l][p] = arg;
      (p == 0 ? L.shape64 : L.shape32) = arg;
    }
  }
  return RT_OK;
}

}  // extern "C"

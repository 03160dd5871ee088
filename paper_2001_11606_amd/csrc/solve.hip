// Preconditioned conjugate gradients for the V-scaled radiation system
// (the D^-1 operator of Sec. 3.2), FP64 and mixed precision.
//
// The paper solves the diffusion equation with AMG-preconditioned GMRES; the
// V-scaled matrix here is symmetric positive definite, so CG applies.  The
// paper warm-starts with E^l; the caller passes the initial guess in x.
//
// FP64:  PCG on A x = b, stop when ||r||_2 <= tol ||b||_2 (recursive residual).
// MIXED: r = b - A x in FP64; repeat { FP32 PCG on A d = r (FP32 matrix, FP32
//        vectors and arithmetic) to a relative reduction inner_tol (or just
//        enough to reach tol); x += d in FP64; r = b - A x in FP64 } until
//        ||r||_2 <= tol ||b||_2 -- the classical iterative refinement.
//
// Scalars (alpha, beta, r.z, ...) stay on the device; block partials of the
// dot products are combined in FP64 by a one-block kernel in a fixed order.
// The stopping test runs on the device too: the kernel that forms ||r||^2
// sets a stop flag once it meets the threshold (or on breakdown), and every
// kernel of the iteration does nothing once the flag is set.  The host queues
// several iterations between reads of the state -- as many as the observed
// convergence rate says are still needed, scaled down so that it rarely
// queues past the end -- so an iteration costs no host round trip, and the
// arithmetic is the same as stopping after each iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "reduce.h"
#include "spmv.h"

namespace rt {
namespace {

enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_RR0, S_BB, S_BAD, S_ITS, S_STOP, S_COUNT };
enum { FIN_ALPHA = 0, FIN_BETA, FIN_RZ, FIN_RR, FIN_BB };
enum { PROF_SPMV64 = 0, PROF_SPMV32 = 1, PROF_RESID64 = 2, PROF_KINDS = 3 };

// One block: combine the partials and update the scalars.  In the loop
// (FIN_ALPHA, FIN_BETA) nothing happens once *stop is set; FIN_BETA counts the
// iteration and sets *stop when ||r||^2 <= thr2 (or is not a number);
// FIN_ALPHA sets it on breakdown (p.Ap not positive).  FIN_RZ starts a loop.
__global__ void __launch_bounds__(kBlock)
k_finalize(int op, int np, const double* __restrict__ pa, const double* __restrict__ pb,
           double* __restrict__ s, int32_t* __restrict__ stop, double thr2) {
  __shared__ double red[kBlock / kWave];
  if ((op == FIN_ALPHA || op == FIN_BETA) && *stop) return;
  // four independent running sums per thread keep four loads in flight; they
  // are combined in a fixed order, so the result is the same on every run
  double a4[4] = {0.0, 0.0, 0.0, 0.0}, b4[4] = {0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 3 * kBlock < np; i += 4 * kBlock) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a4[u] += pa[i + u * kBlock];
    if (pb) {
#pragma unroll
      for (int u = 0; u < 4; ++u) b4[u] += pb[i + u * kBlock];
    }
  }
  for (int u = 0; i < np; i += kBlock, ++u) {
    a4[u] += pa[i];
    if (pb) b4[u] += pb[i];
  }
  double a = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  double b = (b4[0] + b4[1]) + (b4[2] + b4[3]);
  a = block_sum(a, red);
  if (pb) b = block_sum(b, red);
  if (threadIdx.x != 0) return;
  switch (op) {
    case FIN_ALPHA:
      s[S_PQ] = a;
      if (a > 0.0 && isfinite(a)) {
        s[S_ALPHA] = s[S_RZ] / a;
      } else {
        s[S_ALPHA] = 0.0;
        s[S_BAD] = 1.0;
        s[S_STOP] = 1.0;
        *stop = 1;
      }
      break;
    case FIN_BETA:   // a = ||r||^2, b = r.z (new)
      s[S_RR] = a;
      s[S_BETA] = b / s[S_RZ];
      s[S_RZ] = b;
      s[S_ITS] += 1.0;
      if (!(a > thr2)) {
        s[S_STOP] = 1.0;
        *stop = 1;
      }
      break;
    case FIN_RZ:     // a = r.z at the start
      s[S_RZ] = a;
      s[S_BAD] = 0.0;
      s[S_ITS] = 0.0;
      s[S_STOP] = 0.0;
      *stop = 0;
      break;
    case FIN_RR:
      s[S_RR] = a;
      break;
    case FIN_BB:
      s[S_BB] = a;
      break;
  }
}

// Streaming vector kernels: kVec elements per thread (coalesced per element
// slot), one partial per block, no grid-stride loop.
constexpr int kVec = 4;
inline int vec_blocks(int64_t n) {
  const int64_t per_block = (int64_t)kBlock * kVec;
  return (int)std::max<int64_t>(1, (n + per_block - 1) / per_block);
}
#define RT_VEC_LOOP(i)                                                                  \
  for (int _u = 0; _u < kVec; ++_u)                                                     \
    for (int64_t i = (int64_t)blockIdx.x * kBlock * kVec + (int64_t)_u * kBlock + threadIdx.x; \
         i < n; i = n)

// second reduction level: nb2 blocks each sum a contiguous chunk of pa (and pb)
__global__ void __launch_bounds__(kBlock)
k_partial_reduce(int np, int chunk, const double* __restrict__ pa, const double* __restrict__ pb,
                 double* __restrict__ out, const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (stop && *stop) return;
  const int lo = blockIdx.x * chunk;
  const int hi = lo + chunk < np ? lo + chunk : np;
  double a = 0.0, b = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kBlock) {
    a += pa[i];
    if (pb) b += pb[i];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = a;
    out[gridDim.x + blockIdx.x] = b;
  }
}

// p = M r for Jacobi (M = diag^-1), part = r.p
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_init_jacobi(int64_t n, const T* __restrict__ dinv, const T* __restrict__ r, T* __restrict__ p,
              double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  double acc = 0.0;
  RT_VEC_LOOP(i) {
    const T z = dinv[i] * r[i];
    p[i] = z;
    acc += (double)r[i] * (double)z;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// p = z, part = r.z
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_copy_dot(int64_t n, const T* __restrict__ r, const T* __restrict__ z, T* __restrict__ p,
           double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  double acc = 0.0;
  RT_VEC_LOOP(i) {
    p[i] = z[i];
    acc += (double)r[i] * (double)z[i];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_dot(int64_t n, const T* __restrict__ a, const T* __restrict__ b, double* __restrict__ part,
      const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (stop && *stop) return;
  double acc = 0.0;
  RT_VEC_LOOP(i) acc += (double)a[i] * (double)b[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// x += alpha p; r -= alpha q; partA = r.r; (Jacobi) partB = r.(dinv r)
template <typename T, bool JAC>
__global__ void __launch_bounds__(kBlock)
k_update(int64_t n, const double* __restrict__ s, T* __restrict__ x, T* __restrict__ r,
         const T* __restrict__ p, const T* __restrict__ q, const T* __restrict__ dinv,
         double* __restrict__ partA, double* __restrict__ partB, const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (*stop) return;
  const T alpha = (T)s[S_ALPHA];
  double rr = 0.0, rz = 0.0;
  RT_VEC_LOOP(i) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += (double)ri * (double)ri;
    if (JAC) rz += (double)ri * (double)(dinv[i] * ri);
  }
  rr = block_sum(rr, red);
  if (JAC) rz = block_sum(rz, red);
  if (threadIdx.x == 0) {
    partA[blockIdx.x] = rr;
    if (JAC) partB[blockIdx.x] = rz;
  }
}

// p = z + beta p, with z = dinv r (Jacobi) or the preconditioned vector
template <typename T, bool JAC>
__global__ void __launch_bounds__(kBlock)
k_pupdate(int64_t n, const double* __restrict__ s, const T* __restrict__ r,
          const T* __restrict__ dinv, const T* __restrict__ z, T* __restrict__ p,
          const int32_t* __restrict__ stop) {
  if (*stop) return;
  const T beta = (T)s[S_BETA];
  RT_VEC_LOOP(i) {
    const T zi = JAC ? dinv[i] * r[i] : z[i];
    p[i] = zi + beta * p[i];
  }
}

// Initial residual from the previous one: for the same matrix and x, b - A x =
// (b_prev - A x) + (b - b_prev).  r = r + (b - b_prev) (r32: its FP32 copy),
// partA = r.r, partB = b.b.
__global__ void __launch_bounds__(kBlock)
k_resid_shift(int64_t n, const double* __restrict__ b, const double* __restrict__ b_prev,
              double* __restrict__ r, float* __restrict__ r32, double* __restrict__ partA,
              double* __restrict__ partB) {
  __shared__ double red[kBlock / kWave];
  double rr = 0.0, bb = 0.0;
  RT_VEC_LOOP(i) {
    const double bi = b[i];
    const double ri = r[i] + (bi - b_prev[i]);
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  rr = block_sum(rr, red);
  bb = block_sum(bb, red);
  if (threadIdx.x == 0) {
    partA[blockIdx.x] = rr;
    partB[blockIdx.x] = bb;
  }
}

__global__ void k_add_f32(int64_t n, const float* __restrict__ d, double* __restrict__ x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += (double)d[i];
}

template <typename T>
__global__ void k_zero(int64_t n, T* __restrict__ x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ in,
                         double* __restrict__ out) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < n) out[s] = in[perm[s]];
}

__global__ void k_scatter(int64_t n, const int32_t* __restrict__ perm,
                          const double* __restrict__ in, double* __restrict__ out) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < n) out[perm[s]] = in[s];
}

struct Prof {
  rt_ctx* ctx;
  int kind;
  size_t a = 0;
  Prof(rt_ctx* c, int k) : ctx(c), kind(k) {}
  int begin() { return ctx->profiling ? ctx->prof_mark(&a) : RT_OK; }
  int end() {
    if (!ctx->profiling) return RT_OK;
    size_t b;
    RT_CHECK(ctx->prof_mark(&b));
    ctx->prof_spans.push_back({kind, a, b});
    return RT_OK;
  }
};

template <typename T> struct Sel;
template <> struct Sel<double> {
  static const double* val(const Level& L) { return L.val64.p; }
  static const double* diag(const Level& L) { return L.diag64.p; }
  static const double* dinv(const Level& L) { return L.dinv64.p; }
  static double* p(rt_matrix* A) { return A->p64.p; }
  static double* q(rt_matrix* A) { return A->q64.p; }
  static double* z(rt_matrix* A) { return A->z64.p; }
  static constexpr int kind = PROF_SPMV64;
};
template <> struct Sel<float> {
  static const float* val(const Level& L) { return L.val32.p; }
  static const float* diag(const Level& L) { return L.diag32.p; }
  static const float* dinv(const Level& L) { return L.dinv32.p; }
  static float* p(rt_matrix* A) { return A->p32.p; }
  static float* q(rt_matrix* A) { return A->q32.p; }
  static float* z(rt_matrix* A) { return A->z32.p; }
  static constexpr int kind = PROF_SPMV32;
};

int read_scalar(rt_ctx* ctx, rt_matrix* A, int idx, double* out) {
  RT_CHECK(ctx->sync_read(A->scal.p + idx, sizeof(double)));
  *out = ctx->host[0];
  return RT_OK;
}

// partial counts above which a second reduction level runs first
#ifndef RT_PARTIAL_FOLD_MIN
#define RT_PARTIAL_FOLD_MIN (4 * kMaxPartials)
#endif

int finalize(rt_ctx* ctx, rt_matrix* A, int op, int np, const double* pa, const double* pb,
             double thr2 = 0.0) {
  const bool in_loop = op == FIN_ALPHA || op == FIN_BETA;
  if (np > RT_PARTIAL_FOLD_MIN) {
    // first fold the partials into at most kMaxPartials values per array
    const int nb2 = std::min(kMaxPartials, std::max(1, np / 8));
    const int chunk = (np + nb2 - 1) / nb2;
    hipLaunchKernelGGL(k_partial_reduce, dim3(nb2), dim3(kBlock), 0, ctx->stream, np, chunk, pa,
                       pb, A->partC.p, in_loop ? A->stop.p : nullptr);
    RT_LAUNCH_CHECK();
    pa = A->partC.p;
    pb = pb ? A->partC.p + nb2 : nullptr;
    np = nb2;
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, ctx->stream, op, np, pa, pb,
                     A->scal.p, A->stop.p, thr2);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// One PCG iteration, queued; a no-op on the device once the stop flag is set.
template <typename T>
int pcg_iteration(rt_ctx* ctx, rt_matrix* A, bool amg, T* x, T* r, double thr2) {
  using S = Sel<T>;
  hipStream_t st = ctx->stream;
  const Level& L = A->levels[0];
  const int64_t n = L.n;
  T* p = S::p(A);
  T* q = S::q(A);
  T* z = S::z(A);
  const int32_t* stop = A->stop.p;
  const int gv = vec_blocks(n);
  int nbk = 0;
  Prof pf(ctx, S::kind);
  RT_CHECK(pf.begin());
  RT_CHECK((launch_spmv_level<T, SP_DOT>(st, L, S::val(L), S::diag(L), p, nullptr, nullptr, q,
                                         nullptr, A->partA.p, &nbk, level_shape<T>(L), nullptr,
                                         stop)));
  RT_CHECK(pf.end());
  RT_CHECK(finalize(ctx, A, FIN_ALPHA, nbk, A->partA.p, nullptr));
  if (amg) {
    hipLaunchKernelGGL((k_update<T, false>), dim3(gv), dim3(kBlock), 0, st, n, A->scal.p, x, r, p,
                       q, nullptr, A->partA.p, nullptr, stop);
    RT_LAUNCH_CHECK();
    RT_CHECK(vcycle<T>(ctx, A, r, z, stop));
    hipLaunchKernelGGL(k_dot<T>, dim3(gv), dim3(kBlock), 0, st, n, r, z, A->partB.p, stop);
  } else {
    hipLaunchKernelGGL((k_update<T, true>), dim3(gv), dim3(kBlock), 0, st, n, A->scal.p, x, r, p,
                       q, S::dinv(L), A->partA.p, A->partB.p, stop);
  }
  RT_LAUNCH_CHECK();
  RT_CHECK(finalize(ctx, A, FIN_BETA, gv, A->partA.p, A->partB.p, thr2));
  if (amg)
    hipLaunchKernelGGL((k_pupdate<T, false>), dim3(gv), dim3(kBlock), 0, st, n, A->scal.p, r,
                       nullptr, z, p, stop);
  else
    hipLaunchKernelGGL((k_pupdate<T, true>), dim3(gv), dim3(kBlock), 0, st, n, A->scal.p, r,
                       S::dinv(L), nullptr, p, stop);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// Iterations to queue before the next read of the state, from the decrease
// of ||r||^2 since the last read: three quarters of the estimated remaining
// count (at least one, at most 64); one while there is no decrease to go by.
int next_chunk(double rr_prev, int its_prev, double rr, int its, double thr2) {
  if (!(its > its_prev) || !(rr > 0.0) || !(rr < rr_prev) || !(thr2 > 0.0)) return 1;
  const double per_it = std::log(rr / rr_prev) / (its - its_prev);   // < 0
  const double need = std::log(thr2 / rr) / per_it;                  // > 0
  if (!std::isfinite(need)) return 1;
  return (int)std::min(64.0, std::max(1.0, std::floor(0.75 * need)));
}

// PCG iterations on A x = b given r = b - A x and s[S_RR] = ||r||^2 on entry.
// Stops when ||r||^2 <= thr2 or after max_it iterations.
template <typename T>
int pcg_core(rt_ctx* ctx, rt_matrix* A, bool amg, T* x, T* r, double rr0, double thr2,
             int max_it, int* its_out, double* rr_out) {
  using S = Sel<T>;
  hipStream_t st = ctx->stream;
  const Level& L = A->levels[0];
  const int64_t n = L.n;
  T* p = S::p(A);
  T* z = S::z(A);
  const int gv = vec_blocks(n);
  *its_out = 0;
  *rr_out = rr0;
  if (rr0 <= thr2 || max_it <= 0) return RT_OK;
  if (amg) {
    RT_CHECK(vcycle<T>(ctx, A, r, z));
    hipLaunchKernelGGL(k_copy_dot<T>, dim3(gv), dim3(kBlock), 0, st, n, r, z, p, A->partB.p);
  } else {
    hipLaunchKernelGGL(k_init_jacobi<T>, dim3(gv), dim3(kBlock), 0, st, n, S::dinv(L), r, p,
                       A->partB.p);
  }
  RT_LAUNCH_CHECK();
  RT_CHECK(finalize(ctx, A, FIN_RZ, gv, A->partB.p, nullptr));   // clears the stop flag
  const size_t spans0 = ctx->prof_spans.size();
  double rr = rr0, rr_prev = rr0;
  int its = 0, its_prev = 0, queued = 0, chunk = 1;
  bool stopped = false, bad = false;
  while (queued < max_it) {
    const int k = std::min(chunk, max_it - queued);
    for (int j = 0; j < k; ++j) RT_CHECK(pcg_iteration<T>(ctx, A, amg, x, r, thr2));
    queued += k;
    RT_CHECK(ctx->sync_read(A->scal.p, sizeof(double) * S_COUNT));
    const double* hs = ctx->host;
    rr = hs[S_RR];
    its = (int)hs[S_ITS];
    stopped = hs[S_STOP] != 0.0;
    bad = hs[S_BAD] != 0.0;
    if (its > 0 && !std::isfinite(rr)) {
      set_error("PCG breakdown: non-finite residual");
      *its_out = its;
      *rr_out = rr;
      return RT_E_DEVICE;
    }
    if (stopped) break;
    chunk = next_chunk(rr_prev, its_prev, rr, its, thr2);
    rr_prev = rr;
    its_prev = its;
  }
  if (its == 0) rr = rr0;
  if (bad && rr > thr2) set_error("PCG breakdown: p.Ap not positive after %d iterations", its);
  // product timings of queued iterations that did not run are dropped
  if (ctx->profiling && ctx->prof_spans.size() > spans0 + (size_t)its)
    ctx->prof_spans.resize(spans0 + (size_t)its);
  *its_out = its;
  *rr_out = rr;
  return RT_OK;
}

int ensure_work(rt_matrix* A, bool mixed) {
  const int64_t n = A->n;
  for (auto* b : {&A->r64, &A->p64, &A->q64, &A->z64}) RT_CHECK(b->reserve(n));
  RT_CHECK(A->partA.reserve(max_partials(n)));
  RT_CHECK(A->partB.reserve(max_partials(n)));
  RT_CHECK(A->partC.reserve(2 * kMaxPartials));
  RT_CHECK(A->scal.reserve(S_COUNT));
  RT_CHECK(A->stop.reserve(1));
  if (mixed)
    for (auto* b : {&A->r32, &A->p32, &A->q32, &A->z32, &A->d32}) RT_CHECK(b->reserve(n));
  return RT_OK;
}

// r = b - A x in FP64 (optionally also r32), returns ||r||^2
int residual64(rt_ctx* ctx, rt_matrix* A, const double* b, const double* x, float* r32,
               double* rr) {
  const Level& L = A->levels[0];
  int nbk = 0;
  Prof pf(ctx, PROF_RESID64);
  RT_CHECK(pf.begin());
  RT_CHECK((launch_spmv_level<double, SP_RESID>(ctx->stream, L, L.val64.p, L.diag64.p, x, b,
                                                nullptr, A->r64.p, r32, A->partA.p, &nbk,
                                                L.shape64)));
  RT_CHECK(pf.end());
  RT_CHECK(finalize(ctx, A, FIN_RR, nbk, A->partA.p, nullptr));
  return read_scalar(ctx, A, S_RR, rr);
}

}  // namespace

int solve_sorted(rt_ctx* ctx, rt_matrix* A, const double* b, double* x, const rt_solve_opts* o,
                 rt_solve_stats* stt, const double* b_prev, const int32_t* mismatch) {
  hipStream_t st = ctx->stream;
  const int64_t n = A->n;
  const bool mixed = o->precision == RT_PREC_MIXED;
  A->r64_valid = false;
  if (mixed && !A->has_fp32) {
    set_error("rt_solve: mixed precision needs a matrix assembled with build_fp32 = 1");
    return RT_E_STATE;
  }
  const bool amg = o->precond == 1 && A->levels.size() > 1;
  RT_CHECK(ensure_work(A, mixed));
  *stt = rt_solve_stats{};
  if (n == 0) return RT_OK;
  const int gv = vec_blocks(n);
  double bb = 0.0, rr = 0.0;
  bool have_r = false;   // r64 (and r32) hold b - A x, rr = ||r||^2
  if (b_prev) {
    hipLaunchKernelGGL(k_resid_shift, dim3(gv), dim3(kBlock), 0, st, n, b, b_prev, A->r64.p,
                       mixed ? A->r32.p : nullptr, A->partA.p, A->partB.p);
    RT_LAUNCH_CHECK();
    RT_CHECK(finalize(ctx, A, FIN_RR, gv, A->partA.p, nullptr));
    RT_CHECK(finalize(ctx, A, FIN_BB, gv, A->partB.p, nullptr));
    RT_CHECK_HIP(hipMemcpyAsync(ctx->host + S_COUNT, mismatch, sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
    RT_CHECK(ctx->sync_read(A->scal.p, sizeof(double) * S_COUNT));
    int32_t mis = 0;
    std::memcpy(&mis, ctx->host + S_COUNT, sizeof(int32_t));
    bb = ctx->host[S_BB];
    rr = ctx->host[S_RR];
    have_r = mis == 0;
  } else {
    hipLaunchKernelGGL(k_dot<double>, dim3(gv), dim3(kBlock), 0, st, n, b, b, A->partB.p,
                       nullptr);
    RT_LAUNCH_CHECK();
    RT_CHECK(finalize(ctx, A, FIN_BB, gv, A->partB.p, nullptr));
    RT_CHECK(read_scalar(ctx, A, S_BB, &bb));
  }
  if (!std::isfinite(bb)) {
    set_error("rt_solve: right-hand side is not finite");
    return RT_E_ARG;
  }
  if (bb == 0.0) {
    hipLaunchKernelGGL(k_zero<double>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, x);
    RT_LAUNCH_CHECK();
    return RT_OK;
  }
  const double thr2 = o->tol * o->tol * bb;
  int status = RT_OK;
  if (!mixed) {
    if (!have_r) RT_CHECK(residual64(ctx, A, b, x, nullptr, &rr));
    int its = 0;
    RT_CHECK(pcg_core<double>(ctx, A, amg, x, A->r64.p, rr, thr2, o->max_iter, &its, &rr));
    stt->iterations = its;
    if (rr > thr2) status = RT_NOT_CONVERGED;
  } else {
    if (!have_r) RT_CHECK(residual64(ctx, A, b, x, A->r32.p, &rr));
    int total = 0, refine = 0;
    while (rr > thr2 && total < o->max_iter && refine < o->max_refine) {
      // reduce by inner_tol, or just enough (with margin) to reach tol
      double red = std::max(o->inner_tol, 0.3 * std::sqrt(thr2 / rr));
      hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, A->d32.p);
      RT_LAUNCH_CHECK();
      int its = 0;
      double rr_in = 0.0;
      RT_CHECK(pcg_core<float>(ctx, A, amg, A->d32.p, A->r32.p, rr, red * red * rr,
                               o->max_iter - total, &its, &rr_in));
      total += its;
      hipLaunchKernelGGL(k_add_f32, dim3(grid_for(n)), dim3(kBlock), 0, st, n, A->d32.p, x);
      RT_LAUNCH_CHECK();
      RT_CHECK(residual64(ctx, A, b, x, A->r32.p, &rr));
      ++refine;
      if (its == 0) break;
    }
    stt->iterations = total;
    stt->refinements = refine;
    if (rr > thr2) status = RT_NOT_CONVERGED;
  }
  stt->rel_residual = std::sqrt(rr / bb);
  A->r64_valid = true;
  if (status == RT_NOT_CONVERGED)
    set_error("rt_solve: relative residual %.3e above tolerance %.3e", stt->rel_residual, o->tol);
  return status;
}

int collect_profile(rt_ctx* ctx, rt_solve_stats* s) {
  if (!ctx->profiling) return RT_OK;
  double sec[PROF_KINDS];
  int calls[PROF_KINDS];
  RT_CHECK(ctx->prof_collect(sec, calls, PROF_KINDS));
  s->spmv_calls = calls[PROF_SPMV64];
  s->spmv_seconds = sec[PROF_SPMV64];
  s->spmv32_calls = calls[PROF_SPMV32];
  s->spmv32_seconds = sec[PROF_SPMV32];
  return RT_OK;
}

int gather_sorted(rt_ctx* ctx, const rt_neighbors* nb, int64_t n, const double* user,
                  double* sorted) {
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, n, nb->perm.p,
                     user, sorted);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

int scatter_user(rt_ctx* ctx, const rt_neighbors* nb, int64_t n, const double* sorted,
                 double* user) {
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, n, nb->perm.p,
                     sorted, user);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

int check_solve_opts(const rt_solve_opts* o) {
  if (!o) {
    set_error("solve options are NULL");
    return RT_E_ARG;
  }
  if (o->precision != RT_PREC_FP64 && o->precision != RT_PREC_MIXED) {
    set_error("unknown precision %d", o->precision);
    return RT_E_ARG;
  }
  if (o->precond != 0 && o->precond != 1) {
    set_error("unknown preconditioner %d", o->precond);
    return RT_E_ARG;
  }
  if (!(o->tol >= 0.0) || o->max_iter < 0 ||
      (o->precision == RT_PREC_MIXED && (!(o->inner_tol > 0.0) || o->inner_tol >= 1.0))) {
    set_error("invalid tolerance or iteration limit");
    return RT_E_ARG;
  }
  return RT_OK;
}

}  // namespace rt

extern "C" int rt_solve(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                        const rt_solve_opts* opts, rt_solve_stats* stats) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || (A->n > 0 && (!b || !x))) {
    set_error("rt_solve: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK(check_solve_opts(opts));
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  auto t0 = std::chrono::steady_clock::now();
  rt_solve_stats local{};
  rt_solve_stats* stt = stats ? stats : &local;
  A->resid_ok = false;   // bs, xs and r64 are overwritten here
  RT_CHECK(A->xs.reserve(A->n));
  RT_CHECK(A->bs.reserve(A->n));
  RT_CHECK(gather_sorted(ctx, A->nb, A->n, b, A->bs.p));
  RT_CHECK(gather_sorted(ctx, A->nb, A->n, x, A->xs.p));
  int s = solve_sorted(ctx, A, A->bs.p, A->xs.p, opts, stt);
  if (s < 0) return s;
  RT_CHECK(scatter_user(ctx, A->nb, A->n, A->xs.p, x));
  RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  RT_CHECK(collect_profile(ctx, stt));
  stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

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
// Componentwise test (cw_tol > 0): both precisions also require
// max_i |r_i| / (a_ii |x_i|) <= cw_tol, the largest relative change of one
// unknown that a Jacobi sweep would still make.  A normwise test alone is
// blind to unknowns many decades below the largest: on a radiation front E
// spans eight decades, and rows near 1e-8 can keep relative errors of 1e-9
// under ||r|| <= 1e-14 ||b||.  The FP32 inner solve then measures its
// residual with the weights 1/(a_ii |x_i|) of the refinement's start.
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

enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_RR0, S_BB, S_BAD, S_ITS, S_STOP, S_CW, S_RZ_PREV,
       S_COUNT };
// componentwise measure of the update kernel: none, |r_i| w_i / |x_i| with
// w = 1/diag (the iterate's own measure), or |r_i| w_i with fixed weights
enum { CW_NONE = 0, CW_X = 1, CW_W = 2 };
enum { FIN_ALPHA = 0, FIN_BETA, FIN_RZ, FIN_RR, FIN_BB, FIN_RESUME };
enum { PROF_SPMV64 = 0, PROF_SPMV32 = 1, PROF_RESID64 = 2, PROF_KINDS = 3 };

// One block: combine the partials and update the scalars.  In the loop
// (FIN_ALPHA, FIN_BETA) nothing happens once *stop is set; FIN_BETA counts the
// iteration and sets *stop when ||r||^2 <= thr2 (or is not a number);
// FIN_ALPHA sets it on breakdown (p.Ap not positive).  FIN_RZ starts a loop.
__global__ void __launch_bounds__(kBlock)
k_finalize(int op, int np, const double* __restrict__ pa, const double* __restrict__ pb,
           const double* __restrict__ pc, double* __restrict__ s, int32_t* __restrict__ stop,
           double thr2, double cwthr) {
  __shared__ double red[kBlock / kWave];
  if ((op == FIN_ALPHA || op == FIN_BETA) && *stop) return;
  // pc (else NULL): block maxima of the componentwise measure
  double c = 0.0;
  if (pc) {
    for (int k = threadIdx.x; k < np; k += kBlock) c = fmax(c, pc[k]);
    c = block_max(c, red);
  }
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
    case FIN_BETA:   // a = ||r||^2, b = r.z (new), c = componentwise measure
      s[S_RR] = a;
      s[S_BETA] = b / s[S_RZ];
      s[S_RZ_PREV] = s[S_RZ];
      s[S_RZ] = b;
      s[S_ITS] += 1.0;
      if (pc) s[S_CW] = c;
      if (!(a > thr2) && (!pc || !(c > cwthr))) {
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
      if (pc) s[S_CW] = c;
      break;
    case FIN_BB:
      s[S_BB] = a;
      break;
    case FIN_RESUME:   // a = r.z of a residual that replaced the recursive one
      // The loop that stopped kept its last search direction and, in
      // S_RZ_PREV, the r.z it was formed with: beta continues from it, but
      // only while the replacement agrees with the recursion (S_RZ, the
      // recursive r.z it stopped at, within 25%).  The FP32 operator's own
      // error can make the two differ by far more than rounding; then
      // beta = 0, a restart (p = z).
      s[S_BETA] = s[S_RZ_PREV] > 0.0 && isfinite(s[S_RZ_PREV]) && a >= 0.75 * s[S_RZ] &&
                          a <= 1.25 * s[S_RZ]
                      ? a / s[S_RZ_PREV]
                      : 0.0;
      s[S_RZ] = a;
      s[S_BAD] = 0.0;
      s[S_ITS] = 0.0;
      s[S_STOP] = 0.0;
      *stop = 0;
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
                 const double* __restrict__ pc, double* __restrict__ out,
                 const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (stop && *stop) return;
  const int lo = blockIdx.x * chunk;
  const int hi = lo + chunk < np ? lo + chunk : np;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += kBlock) {
    a += pa[i];
    if (pb) b += pb[i];
    if (pc) c = fmax(c, pc[i]);
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (pc) c = block_max(c, red);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = a;
    out[gridDim.x + blockIdx.x] = b;
    out[2 * gridDim.x + blockIdx.x] = c;
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

// part = r.(D^-1 r): the r.z of a Jacobi-preconditioned residual
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_rz_jacobi(int64_t n, const T* __restrict__ dinv, const T* __restrict__ r,
            double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  double acc = 0.0;
  RT_VEC_LOOP(i) acc += (double)r[i] * (double)(dinv[i] * r[i]);
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

// x += alpha p; r -= alpha q; partA = r.r; (Jacobi) partB = r.(dinv r);
// CW != CW_NONE: partC = the block maximum of the componentwise measure, with
// w = dinv (CW_X: |r_i| w_i / |x_i| of the updated x) or fixed weights (CW_W)
template <typename T, bool JAC, int CW>
__global__ void __launch_bounds__(kBlock)
k_update(int64_t n, const double* __restrict__ s, T* __restrict__ x, T* __restrict__ r,
         const T* __restrict__ p, const T* __restrict__ q, const T* __restrict__ dinv,
         const T* __restrict__ w, double* __restrict__ partA, double* __restrict__ partB,
         double* __restrict__ partC, const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (*stop) return;
  const T alpha = (T)s[S_ALPHA];
  double rr = 0.0, rz = 0.0, cw = 0.0;
  RT_VEC_LOOP(i) {
    const T xi = x[i] + alpha * p[i];
    x[i] = xi;
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += (double)ri * (double)ri;
    if (JAC) rz += (double)ri * (double)(dinv[i] * ri);
    if (CW == CW_X) {
      const double ax = fabs((double)xi);
      const double t = fabs((double)ri) * (double)w[i];
      cw = fmax(cw, ax > 0.0 ? t / ax : (ri == T(0) ? 0.0 : INFINITY));
    } else if (CW == CW_W) {
      cw = fmax(cw, fabs((double)ri) * (double)w[i]);
    }
  }
  rr = block_sum(rr, red);
  if (JAC) rz = block_sum(rz, red);
  if (CW != CW_NONE) cw = block_max(cw, red);
  if (threadIdx.x == 0) {
    partA[blockIdx.x] = rr;
    if (JAC) partB[blockIdx.x] = rz;
    if (CW != CW_NONE) partC[blockIdx.x] = cw;
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
// partA = r.r, partB = b.b, partC = the block maximum of the componentwise
// measure |r_i| / (a_ii |x_i|) (x, diag), w32 (else NULL) its weights.
__global__ void __launch_bounds__(kBlock)
k_resid_shift(int64_t n, const double* __restrict__ b, const double* __restrict__ b_prev,
              const double* __restrict__ x, const double* __restrict__ diag,
              double* __restrict__ r, float* __restrict__ r32, float* __restrict__ w32,
              double* __restrict__ partA, double* __restrict__ partB,
              double* __restrict__ partC) {
  __shared__ double red[kBlock / kWave];
  double rr = 0.0, bb = 0.0, cw = 0.0;
  RT_VEC_LOOP(i) {
    const double bi = b[i];
    const double ri = r[i] + (bi - b_prev[i]);
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
    rr += ri * ri;
    bb += bi * bi;
    const double xi = x[i], di = diag[i];
    cw = fmax(cw, cw_term(ri, di, xi));
    if (w32) w32[i] = cw_weight(di, xi);
  }
  rr = block_sum(rr, red);
  bb = block_sum(bb, red);
  cw = block_max(cw, red);
  if (threadIdx.x == 0) {
    partA[blockIdx.x] = rr;
    partB[blockIdx.x] = bb;
    partC[blockIdx.x] = cw;
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

// Device buffers of one solve: work vectors of the fine level (n entries
// each; the FP32 ones only for mixed precision), block partials, the Krylov
// scalars and the stop flag.
struct Work {
  double *r64 = nullptr, *p64 = nullptr, *q64 = nullptr, *z64 = nullptr;
  float *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *z32 = nullptr, *d32 = nullptr,
        *w32 = nullptr;
  double *partA = nullptr, *partB = nullptr, *partC = nullptr, *partF = nullptr, *scal = nullptr;
  int32_t* stop = nullptr;
};

template <typename T> struct Sel;
template <> struct Sel<double> {
  static const double* val(const Level& L) { return L.val64.p; }
  static const double* diag(const Level& L) { return L.diag64.p; }
  static const double* dinv(const Level& L) { return L.dinv64.p; }
  static double* p(const Work& W) { return W.p64; }
  static double* q(const Work& W) { return W.q64; }
  static double* z(const Work& W) { return W.z64; }
  static constexpr int kind = PROF_SPMV64;
};
template <> struct Sel<float> {
  static const float* val(const Level& L) { return L.val32.p; }
  static const float* diag(const Level& L) { return L.diag32.p; }
  static const float* dinv(const Level& L) { return L.dinv32.p; }
  static float* p(const Work& W) { return W.p32; }
  static float* q(const Work& W) { return W.q32; }
  static float* z(const Work& W) { return W.z32; }
  static constexpr int kind = PROF_SPMV32;
};

int read_scalar(rt_ctx* ctx, const Work& W, int idx, double* out) {
  RT_CHECK(ctx->sync_read(W.scal + idx, sizeof(double)));
  *out = ctx->host[0];
  return RT_OK;
}

// partial counts above which a second reduction level runs first
#ifndef RT_PARTIAL_FOLD_MIN
#define RT_PARTIAL_FOLD_MIN (4 * kMaxPartials)
#endif

// pc (else NULL): block maxima of the componentwise measure; the loop stops
// only when it is <= cwthr as well
int finalize(rt_ctx* ctx, const Work& W, int op, int np, const double* pa, const double* pb,
             double thr2 = 0.0, const double* pc = nullptr, double cwthr = 0.0) {
  const bool in_loop = op == FIN_ALPHA || op == FIN_BETA;
  if (np > RT_PARTIAL_FOLD_MIN) {
    // first fold the partials into at most kMaxPartials values per array
    const int nb2 = std::min(kMaxPartials, std::max(1, np / 8));
    const int chunk = (np + nb2 - 1) / nb2;
    hipLaunchKernelGGL(k_partial_reduce, dim3(nb2), dim3(kBlock), 0, ctx->stream, np, chunk, pa,
                       pb, pc, W.partF, in_loop ? W.stop : nullptr);
    RT_LAUNCH_CHECK();
    pa = W.partF;
    pb = pb ? W.partF + nb2 : nullptr;
    pc = pc ? W.partF + 2 * nb2 : nullptr;
    np = nb2;
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, ctx->stream, op, np, pa, pb, pc,
                     W.scal, W.stop, thr2, cwthr);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// Componentwise test of a PCG loop: the update kernel's measure (mode), its
// weights and the threshold (infinity: measured, never binding).
struct CwTest {
  int mode = CW_NONE;
  const void* w = nullptr;
  double thr = INFINITY;
};

// One PCG iteration, queued; a no-op on the device once the stop flag is set.
template <typename T>
int pcg_iteration(rt_ctx* ctx, rt_matrix* A, const Work& W, bool amg, T* x, T* r, double thr2, const CwTest& cw) {
  using S = Sel<T>;
  hipStream_t st = ctx->stream;
  const Level& L = A->levels[0];
  const int64_t n = L.n;
  T* p = S::p(W);
  T* q = S::q(W);
  T* z = S::z(W);
  const int32_t* stop = W.stop;
  const int gv = vec_blocks(n);
  int nbk = 0;
  Prof pf(ctx, S::kind);
  RT_CHECK(pf.begin());
  RT_CHECK((launch_spmv_level<T, SP_DOT>(st, L, S::val(L), S::diag(L), p, nullptr, nullptr, q,
                                         nullptr, W.partA, &nbk, level_shape<T>(L), nullptr,
                                         stop)));
  RT_CHECK(pf.end());
  RT_CHECK(finalize(ctx, W, FIN_ALPHA, nbk, W.partA, nullptr));
  const T* w = static_cast<const T*>(cw.w);
  double* pc = cw.mode == CW_NONE ? nullptr : W.partC;
#define RT_UPD(JAC_, CW_)                                                                      \
  hipLaunchKernelGGL((k_update<T, JAC_, CW_>), dim3(gv), dim3(kBlock), 0, st, n, W.scal, x, r, \
                     p, q, JAC_ ? S::dinv(L) : nullptr, w, W.partA,                          \
                     JAC_ ? W.partB : nullptr, pc, stop)
  if (amg) {
    if (cw.mode == CW_X) RT_UPD(false, CW_X);
    else if (cw.mode == CW_W) RT_UPD(false, CW_W);
    else RT_UPD(false, CW_NONE);
    RT_LAUNCH_CHECK();
    RT_CHECK(vcycle<T>(ctx, A, r, z, stop));
    hipLaunchKernelGGL(k_dot<T>, dim3(gv), dim3(kBlock), 0, st, n, r, z, W.partB, stop);
  } else {
    if (cw.mode == CW_X) RT_UPD(true, CW_X);
    else if (cw.mode == CW_W) RT_UPD(true, CW_W);
    else RT_UPD(true, CW_NONE);
  }
#undef RT_UPD
  RT_LAUNCH_CHECK();
  RT_CHECK(finalize(ctx, W, FIN_BETA, gv, W.partA, W.partB, thr2, pc, cw.thr));
  if (amg)
    hipLaunchKernelGGL((k_pupdate<T, false>), dim3(gv), dim3(kBlock), 0, st, n, W.scal, r,
                       nullptr, z, p, stop);
  else
    hipLaunchKernelGGL((k_pupdate<T, true>), dim3(gv), dim3(kBlock), 0, st, n, W.scal, r,
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
// Stops when ||r||^2 <= thr2 (and the componentwise measure, cw0 on entry,
// is <= cw.thr) or after max_it iterations; *cw_out: the measure at the end.
template <typename T>
int pcg_core(rt_ctx* ctx, rt_matrix* A, const Work& W, bool amg, T* x, T* r, double rr0, double thr2,
             int max_it, int* its_out, double* rr_out, const CwTest& cw = CwTest{},
             double cw0 = 0.0, double* cw_out = nullptr, bool resume = false) {
  using S = Sel<T>;
  hipStream_t st = ctx->stream;
  const Level& L = A->levels[0];
  const int64_t n = L.n;
  T* p = S::p(W);
  T* z = S::z(W);
  const int gv = vec_blocks(n);
  *its_out = 0;
  *rr_out = rr0;
  if (cw_out) *cw_out = cw0;
  if ((rr0 <= thr2 && !(cw0 > cw.thr)) || max_it <= 0) return RT_OK;
  if (resume) {
    // the last loop on this system ended at a residual replacement: its
    // search direction p carries over, p = z + beta p with the new r.z
    if (amg) {
      RT_CHECK(vcycle<T>(ctx, A, r, z));
      hipLaunchKernelGGL(k_dot<T>, dim3(gv), dim3(kBlock), 0, st, n, r, z, W.partB, nullptr);
    } else {
      hipLaunchKernelGGL(k_rz_jacobi<T>, dim3(gv), dim3(kBlock), 0, st, n, S::dinv(L), r,
                         W.partB);
    }
    RT_LAUNCH_CHECK();
    RT_CHECK(finalize(ctx, W, FIN_RESUME, gv, W.partB, nullptr));   // clears the stop flag
    if (amg)
      hipLaunchKernelGGL((k_pupdate<T, false>), dim3(gv), dim3(kBlock), 0, st, n, W.scal, r,
                         nullptr, z, p, W.stop);
    else
      hipLaunchKernelGGL((k_pupdate<T, true>), dim3(gv), dim3(kBlock), 0, st, n, W.scal, r,
                         S::dinv(L), nullptr, p, W.stop);
  } else if (amg) {
    RT_CHECK(vcycle<T>(ctx, A, r, z));
    hipLaunchKernelGGL(k_copy_dot<T>, dim3(gv), dim3(kBlock), 0, st, n, r, z, p, W.partB);
  } else {
    hipLaunchKernelGGL(k_init_jacobi<T>, dim3(gv), dim3(kBlock), 0, st, n, S::dinv(L), r, p,
                       W.partB);
  }
  RT_LAUNCH_CHECK();
  if (!resume) RT_CHECK(finalize(ctx, W, FIN_RZ, gv, W.partB, nullptr));   // clears the stop flag
  const size_t spans0 = ctx->prof_spans.size();
  double rr = rr0, rr_prev = rr0;
  int its = 0, its_prev = 0, queued = 0, chunk = 1;
  bool stopped = false, bad = false;
  while (queued < max_it) {
    const int k = std::min(chunk, max_it - queued);
    for (int j = 0; j < k; ++j) RT_CHECK(pcg_iteration<T>(ctx, A, W, amg, x, r, thr2, cw));
    queued += k;
    RT_CHECK(ctx->sync_read(W.scal, sizeof(double) * S_COUNT));
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
    if (cw_out && its > 0) *cw_out = hs[S_CW];
    if (stopped) break;
    // while the componentwise test still binds, go by one iteration at a time
    chunk = rr > thr2 ? next_chunk(rr_prev, its_prev, rr, its, thr2) : 1;
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
  RT_CHECK(A->partC.reserve(max_partials(n)));
  RT_CHECK(A->partF.reserve(3 * kMaxPartials));
  RT_CHECK(A->scal.reserve(S_COUNT));
  RT_CHECK(A->stop.reserve(1));
  if (mixed)
    for (auto* b : {&A->r32, &A->p32, &A->q32, &A->z32, &A->d32, &A->w32}) RT_CHECK(b->reserve(n));
  return RT_OK;
}

// The matrix's own work buffers (after ensure_work)
Work work_of(rt_matrix* A) {
  Work W;
  W.r64 = A->r64.p;
  W.p64 = A->p64.p;
  W.q64 = A->q64.p;
  W.z64 = A->z64.p;
  W.r32 = A->r32.p;
  W.p32 = A->p32.p;
  W.q32 = A->q32.p;
  W.z32 = A->z32.p;
  W.d32 = A->d32.p;
  W.w32 = A->w32.p;
  W.partA = A->partA.p;
  W.partB = A->partB.p;
  W.partC = A->partC.p;
  W.partF = A->partF.p;
  W.scal = A->scal.p;
  W.stop = A->stop.p;
  return W;
}

// r = b - A x in FP64 (optionally also r32 and the componentwise weights w32);
// returns ||r||^2 and the componentwise measure max_i |r_i| / (a_ii |x_i|)
int residual64(rt_ctx* ctx, rt_matrix* A, const Work& W, const double* b, const double* x, float* r32,
               float* w32, double* rr, double* cw) {
  const Level& L = A->levels[0];
  int nbk = 0;
  Prof pf(ctx, PROF_RESID64);
  RT_CHECK(pf.begin());
  RT_CHECK((launch_spmv_level<double, SP_RESID>(ctx->stream, L, L.val64.p, L.diag64.p, x, b,
                                                nullptr, W.r64, r32, W.partA, &nbk,
                                                resid_shape(L), nullptr, nullptr, W.partC, w32)));
  RT_CHECK(pf.end());
  RT_CHECK(finalize(ctx, W, FIN_RR, nbk, W.partA, nullptr, 0.0, W.partC));
  RT_CHECK(ctx->sync_read(W.scal, sizeof(double) * S_COUNT));
  *rr = ctx->host[S_RR];
  *cw = ctx->host[S_CW];
  return RT_OK;
}

// FP64 CG steps after which the recursive residual is replaced by a
// computed one: the recursion's drift from b - A x grows with the steps
// taken (and carried between outer iterations); one product per 32 steps
// keeps it at rounding level for about 3% more products on long solves.
constexpr int kReplaceSteps = 32;

// The solve on sorted vectors with the buffers of W (see solve_sorted);
// *resid_valid: W.r64 holds b - A x on return.  *rec_steps: on entry, the
// CG steps the residual carried in W.r64 (with b_prev) has been updated by
// recursion since a product formed it; on return, the same for W.r64.
int solve_work(rt_ctx* ctx, rt_matrix* A, const Work& W, const double* b, double* x,
               const rt_solve_opts* o, rt_solve_stats* stt, const double* b_prev,
               const int32_t* mismatch, bool* resid_valid, int* rec_steps) {
  hipStream_t st = ctx->stream;
  const int64_t n = A->n;
  const bool mixed = o->precision == RT_PREC_MIXED;
  *resid_valid = false;
  const bool amg = o->precond == 1 && cycle_depth(A) > 1;
  *stt = rt_solve_stats{};
  if (n == 0) return RT_OK;
  const int gv = vec_blocks(n);
  const Level& L0 = A->levels[0];
  // componentwise test: its threshold, infinity when only measured
  const bool use_cw = o->cw_tol > 0.0;
  const double cwthr = use_cw ? o->cw_tol : INFINITY;
  float* w32 = mixed && use_cw ? W.w32 : nullptr;
  double bb = 0.0, rr = 0.0, cw = 0.0;
  bool have_r = false;   // r64 (and r32) hold b - A x, rr = ||r||^2, cw its measure
  if (b_prev) {
    hipLaunchKernelGGL(k_resid_shift, dim3(gv), dim3(kBlock), 0, st, n, b, b_prev, x,
                       L0.diag64.p, W.r64, mixed ? W.r32 : nullptr, w32, W.partA,
                       W.partB, W.partC);
    RT_LAUNCH_CHECK();
    RT_CHECK(finalize(ctx, W, FIN_RR, gv, W.partA, nullptr, 0.0, W.partC));
    RT_CHECK(finalize(ctx, W, FIN_BB, gv, W.partB, nullptr));
    RT_CHECK_HIP(hipMemcpyAsync(ctx->host + S_COUNT, mismatch, sizeof(int32_t),
                                hipMemcpyDeviceToHost, st));
    RT_CHECK(ctx->sync_read(W.scal, sizeof(double) * S_COUNT));
    int32_t mis = 0;
    std::memcpy(&mis, ctx->host + S_COUNT, sizeof(int32_t));
    bb = ctx->host[S_BB];
    rr = ctx->host[S_RR];
    cw = ctx->host[S_CW];
    have_r = mis == 0;
  } else {
    hipLaunchKernelGGL(k_dot<double>, dim3(gv), dim3(kBlock), 0, st, n, b, b, W.partB,
                       nullptr);
    RT_LAUNCH_CHECK();
    RT_CHECK(finalize(ctx, W, FIN_BB, gv, W.partB, nullptr));
    RT_CHECK(read_scalar(ctx, W, S_BB, &bb));
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
    int rec = have_r ? *rec_steps : 0;
    if (!have_r) RT_CHECK(residual64(ctx, A, W, b, x, nullptr, nullptr, &rr, &cw));
    stt->init_rel_residual = std::sqrt(rr / bb);
    const CwTest t{CW_X, L0.dinv64.p, cwthr};
    int total = 0;
    for (int pass = 0;; ++pass) {
      int its = 0;
      RT_CHECK(pcg_core<double>(ctx, A, W, amg, x, W.r64, rr, thr2, o->max_iter - total, &its,
                                &rr, t, cw, &cw));
      total += its;
      rec += its;
      if (rec <= kReplaceSteps || pass == 2) break;
      // residual replacement; CG restarts from the computed residual if it
      // misses the tolerance
      RT_CHECK(residual64(ctx, A, W, b, x, nullptr, nullptr, &rr, &cw));
      rec = 0;
      ++stt->replacements;
      if (!(rr > thr2 || cw > cwthr) || total >= o->max_iter) break;
    }
    stt->iterations = total;
    *rec_steps = rec;
  } else {
    if (!have_r) RT_CHECK(residual64(ctx, A, W, b, x, W.r32, w32, &rr, &cw));
    stt->init_rel_residual = std::sqrt(rr / bb);
    *rec_steps = 0;
    int total = 0, refine = 0;
    // After the first inner solve each one continues the last: the FP64
    // residual replaces CG's recursive one (reliable update) and the search
    // direction carries over, so the refinements do not restart the Krylov
    // space.
    bool resume = false;
    while ((rr > thr2 || cw > cwthr) && total < o->max_iter && refine < o->max_refine) {
      // reduce by inner_tol, or just enough (with margin) to reach tol; the
      // same for the componentwise measure when it is tested
      const double red = std::max(o->inner_tol, 0.3 * std::sqrt(thr2 / rr));
      CwTest t{};
      if (use_cw) t = CwTest{CW_W, w32, std::max(o->inner_tol, 0.3 * cwthr / cw) * cw};
      hipLaunchKernelGGL(k_zero<float>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, W.d32);
      RT_LAUNCH_CHECK();
      int its = 0;
      double rr_in = 0.0;
      RT_CHECK(pcg_core<float>(ctx, A, W, amg, W.d32, W.r32, rr, red * red * rr,
                               o->max_iter - total, &its, &rr_in, t, cw, nullptr, resume));
      total += its;
      resume = its > 0;
      hipLaunchKernelGGL(k_add_f32, dim3(grid_for(n)), dim3(kBlock), 0, st, n, W.d32, x);
      RT_LAUNCH_CHECK();
      RT_CHECK(residual64(ctx, A, W, b, x, W.r32, w32, &rr, &cw));
      ++refine;
      if (its == 0) break;
    }
    stt->iterations = total;
    stt->refinements = refine;
  }
  if (rr > thr2 || cw > cwthr) status = RT_NOT_CONVERGED;
  stt->rel_residual = std::sqrt(rr / bb);
  stt->cw_residual = cw;
  // r64 now holds b - A x: the residual of an FP64 product (mixed), or the
  // recursive residual of CG (FP64), which differs from it by rounding only
  *resid_valid = true;
  if (status == RT_NOT_CONVERGED)
    set_error("rt_solve: relative residual %.3e (componentwise %.3e) above tolerance %.3e "
              "(componentwise %.3e)", stt->rel_residual, cw, o->tol, o->cw_tol);
  return status;
}

}  // namespace

int residual_norms(rt_ctx* ctx, rt_matrix* A, const double* b, const double* x, double* rr,
                   double* bb) {
  A->resid_ok = false;
  A->r64_valid = false;
  RT_CHECK(ensure_work(A, false));
  const Work W = work_of(A);
  double cw = 0.0;
  RT_CHECK(residual64(ctx, A, W, b, x, nullptr, nullptr, rr, &cw));
  const int gv = vec_blocks(A->n);
  hipLaunchKernelGGL(k_dot<double>, dim3(gv), dim3(kBlock), 0, ctx->stream, A->n, b, b, W.partB,
                     nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK(finalize(ctx, W, FIN_BB, gv, W.partB, nullptr));
  return read_scalar(ctx, W, S_BB, bb);
}

int solve_sorted(rt_ctx* ctx, rt_matrix* A, const double* b, double* x, const rt_solve_opts* o,
                 rt_solve_stats* stt, const double* b_prev, const int32_t* mismatch) {
  const bool mixed = o->precision == RT_PREC_MIXED;
  A->r64_valid = false;
  if (mixed && !A->has_fp32) {
    set_error("rt_solve: mixed precision needs a matrix assembled with build_fp32 = 1");
    return RT_E_STATE;
  }
  RT_CHECK(ensure_work(A, mixed));
  bool valid = false;
  int rec = A->rec_steps;
  const int s = solve_work(ctx, A, work_of(A), b, x, o, stt, b_prev, mismatch, &valid, &rec);
  A->r64_valid = valid;
  A->rec_steps = rec;
  return s;
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
  s->resid_calls = calls[PROF_RESID64];
  s->resid_seconds = sec[PROF_RESID64];
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
  if (!(o->tol >= 0.0) || o->max_iter < 0 || !(o->cw_tol >= 0.0) ||
      (o->precision == RT_PREC_MIXED && (!(o->inner_tol > 0.0) || o->inner_tol >= 1.0))) {
    set_error("invalid tolerance or iteration limit");
    return RT_E_ARG;
  }
  return RT_OK;
}

}  // namespace rt

namespace rt {
namespace {

// Bytes of scratch the no-allocation solve carves for n unknowns: the gathered
// b and x, four FP64 work vectors (six FP32 ones in mixed precision), three
// arrays of block partials, the fold buffer, the scalars and the stop flag,
// each piece 256-byte aligned.
struct Carve {
  char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    used = (used + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += (count ? count : 1) * sizeof(T);
    return p;
  }
};

Work carve_work(Carve& c, int64_t n, bool mixed, double** bs, double** xs) {
  Work W;
  *bs = c.take<double>(n);
  *xs = c.take<double>(n);
  W.r64 = c.take<double>(n);
  W.p64 = c.take<double>(n);
  W.q64 = c.take<double>(n);
  W.z64 = c.take<double>(n);
  if (mixed) {
    W.r32 = c.take<float>(n);
    W.p32 = c.take<float>(n);
    W.q32 = c.take<float>(n);
    W.z32 = c.take<float>(n);
    W.d32 = c.take<float>(n);
    W.w32 = c.take<float>(n);
  }
  W.partA = c.take<double>(max_partials(n));
  W.partB = c.take<double>(max_partials(n));
  W.partC = c.take<double>(max_partials(n));
  W.partF = c.take<double>(3 * kMaxPartials);
  W.scal = c.take<double>(S_COUNT);
  W.stop = c.take<int32_t>(1);
  return W;
}

}  // namespace
}  // namespace rt

// rt_solve for callers that cannot allocate: every buffer of the solve comes
// from the device's scratch array; the matrix's own work buffers and the
// residual it carries between outer iterations are left untouched.
extern "C" int rt_solve_noalloc(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                                const rt_solve_opts* opts, rt_solve_stats* stats) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || (A->n > 0 && (!b || !x))) {
    set_error("rt_solve_noalloc: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK(check_solve_opts(opts));
  if (A->levels.empty()) {
    set_error("rt_solve_noalloc: matrix not assembled");
    return RT_E_STATE;
  }
  const bool mixed = opts->precision == RT_PREC_MIXED;
  if (mixed && !A->has_fp32) {
    set_error("rt_solve_noalloc: mixed precision needs a matrix assembled with build_fp32 = 1");
    return RT_E_STATE;
  }
  const int64_t n = A->n;
  Carve size{nullptr};
  double *bs = nullptr, *xs = nullptr;
  (void)carve_work(size, n, mixed, &bs, &xs);
  if (size.used > kScratchBytes) {
    set_error("rt_solve_noalloc: %lld unknowns need %zu bytes of scratch in %s, above the "
              "%zu-byte scratch array", (long long)n, size.used,
              mixed ? "mixed precision" : "FP64", kScratchBytes);
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  char* base = static_cast<char*>(scratch_base(ctx->device));
  if (!base) {
    set_error("rt_solve_noalloc: no scratch address for device %d", ctx->device);
    return RT_E_STATE;
  }
  auto t0 = std::chrono::steady_clock::now();
  rt_solve_stats local{};
  rt_solve_stats* stt = stats ? stats : &local;
  *stt = rt_solve_stats{};
  if (n == 0) return RT_OK;
  Carve carve{base};
  const Work W = carve_work(carve, n, mixed, &bs, &xs);
  // no event timings: recording them would create events
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  int s = gather_sorted(ctx, A->nb, n, b, bs);
  if (s == RT_OK) s = gather_sorted(ctx, A->nb, n, x, xs);
  bool valid = false;
  int rec = 0;
  if (s == RT_OK) s = solve_work(ctx, A, W, bs, xs, opts, stt, nullptr, nullptr, &valid, &rec);
  ctx->profiling = prof;
  if (s < 0) return s;
  RT_CHECK(scatter_user(ctx, A->nb, n, xs, x));
  RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

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

// Aggregation multigrid preconditioner (gfx950).
//
// The paper preconditions its Krylov solve with algebraic multigrid, set up
// once per time step and reused for every outer iteration (Sec. 3.2); it
// fixes no AMG parameters.  This hierarchy uses unsmoothed aggregation with
// aggregates taken from the neighbour-search grid: level 1 aggregates the
// interior particles of one cell, level l+1 aggregates the 2^dim cells of a
// Morton block of level l.  Because particles are sorted by Morton cell key,
// every aggregate is a contiguous run of rows at every level, so restriction
// is a segmented sum, prolongation a broadcast, and a coarse row has at most
// 3^dim entries.  The coarse operators are Galerkin products P^T A P with the
// piecewise-constant P (sums of fine entries by aggregate pair), computed
// with a fixed summation order.
//
// V-cycle (symmetric, so it is a valid CG preconditioner): pre-smoothing
// from zero, residual, restriction, coarse correction, prolongation,
// post-smoothing with the same smoother.  The l1 diagonal
// D1_ii = a_ii + sum_j |a_ij| bounds A from above (D1 - A is diagonally
// dominant), so the spectrum of D1^-1 A lies in (0, 1] and neither smoother
// needs an eigenvalue estimate: one l1-Jacobi sweep, or a Chebyshev
// polynomial in D1^-1 A on [1/4, 1] (the three-term recurrence of Chebyshev
// acceleration, Saad, Iterative Methods for Sparse Linear Systems, Sec. 12.3,
// with the residual recomputed as b - A x at every step).  The coarsest level is solved with a dense
// FP64 inverse (Gauss-Jordan at setup) when small enough, otherwise with four
// l1-Jacobi sweeps.
#include <climits>
#include <cstring>

#include "internal.h"
#include "prim.h"
#include "reduce.h"
#include "spmv.h"

namespace rt {
namespace {

constexpr int64_t kDenseMax = 1024;

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T w = __shfl_xor(v, o, kWave);
    v = v < w ? v : w;
  }
  return v;
}

// new-aggregate flags: level 0 groups equal cell codes, coarser levels equal
// parent codes (code >> dim)
__global__ void k_agg_flags(int64_t n, int shift, const uint64_t* __restrict__ code,
                            int32_t* __restrict__ flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (code[i] >> shift) != (code[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_agg_finish(int64_t n, int shift, const uint64_t* __restrict__ code,
                             const int32_t* __restrict__ flag, int32_t* __restrict__ pmap,
                             int32_t* __restrict__ crange, uint64_t* __restrict__ ccode,
                             int64_t nc) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t I = pmap[i] - 1;      // inclusive scan -> 0-based
  pmap[i] = I;
  if (flag[i]) {
    crange[I] = (int32_t)i;
    ccode[I] = code[i] >> shift;
  }
  if (i == n - 1) crange[nc] = (int32_t)n;
}

template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_galerkin(int64_t nc, const int32_t* __restrict__ crange, const int64_t* __restrict__ rp,
           const int32_t* __restrict__ col, const double* __restrict__ val,
           const double* __restrict__ diag, const int32_t* __restrict__ pmap,
           int64_t* __restrict__ cnt, const int64_t* __restrict__ crp, int32_t* __restrict__ ccol,
           double* __restrict__ cval, double* __restrict__ cdiag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  if (I >= nc) return;   // whole wavefront exits together
  const int64_t f0 = crange[I], f1 = crange[I + 1];
  const int64_t e0 = rp[f0], e1 = rp[f1];
  double dsum = 0.0;
  if (FILL) {
    for (int64_t i = f0 + lane; i < f1; i += kWave) dsum += diag[i];
    dsum = group_sum<kWave>(dsum);
  }
  int32_t last = -1;
  int64_t out = FILL ? crp[I] : 0;
  int64_t count = 0;
  while (true) {
    int32_t m = INT_MAX;
    for (int64_t k = e0 + lane; k < e1; k += kWave) {
      const int32_t pc = pmap[col[k]];
      if (pc > last && pc < m) m = pc;
    }
    m = wave_min(m);
    if (m == INT_MAX) break;
    if (FILL) {
      double sum = 0.0;
      for (int64_t k = e0 + lane; k < e1; k += kWave)
        if (pmap[col[k]] == m) sum += val[k];
      sum = group_sum<kWave>(sum);
      if (m == (int32_t)I) {
        dsum += sum;
      } else {
        if (lane == 0) {
          ccol[out] = m;
          cval[out] = sum;
        }
        ++out;
      }
    } else if (m != (int32_t)I) {
      ++count;
    }
    last = m;
  }
  if (lane == 0) {
    if (FILL) cdiag[I] = dsum;
    else cnt[I] = count;
  }
}

// l1-Jacobi smoother scaling and Jacobi inverse diagonal of a coarse level,
// plus FP32 copies; 8 lanes per row (coarse rows hold at most 3^dim entries).
__global__ void __launch_bounds__(kBlock)
k_smoother(int64_t n, const int64_t* __restrict__ rp, const double* __restrict__ val,
           const double* __restrict__ diag, double* __restrict__ sinv, double* __restrict__ dinv,
           float* __restrict__ sinv32, float* __restrict__ dinv32) {
  constexpr int G = 8;
  const int lane = threadIdx.x & (G - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  if (i >= n) return;   // the whole group leaves together
  double l1 = 0.0;
  for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += G) l1 += fabs(val[k]);
  l1 = group_sum<G>(l1) + diag[i];
  if (lane == 0) {
    sinv[i] = 1.0 / l1;
    dinv[i] = 1.0 / diag[i];
    if (sinv32) {
      sinv32[i] = (float)(1.0 / l1);
      dinv32[i] = (float)(1.0 / diag[i]);
    }
  }
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_dense_zero(int64_t nn, double* __restrict__ M) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nn) M[i] = 0.0;
}

__global__ void k_dense_fill(int64_t n, const int64_t* __restrict__ rp,
                             const int32_t* __restrict__ col, const double* __restrict__ val,
                             const double* __restrict__ diag, double* __restrict__ M) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  M[i * n + i] = diag[i];
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) M[i * n + col[k]] = val[k];
}

// In-place Gauss-Jordan inversion of an SPD matrix (positive pivots, no
// pivoting needed), one workgroup, n <= kDenseMax; colk holds column k of the step.
__global__ void __launch_bounds__(1024) k_gauss_jordan(int n, double* __restrict__ M) {
  __shared__ double colk[kDenseMax];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    const double piv = 1.0 / M[(int64_t)k * n + k];
    for (int i = tid; i < n; i += nt) colk[i] = M[(int64_t)i * n + k];
    __syncthreads();
    for (int j = tid; j < n; j += nt)
      if (j != k) M[(int64_t)k * n + j] *= piv;
    __syncthreads();
    const int64_t nn = (int64_t)n * n;
    for (int64_t idx = tid; idx < nn; idx += nt) {
      const int i = (int)(idx / n), j = (int)(idx % n);
      if (i == k) continue;
      if (j == k) M[idx] = -colk[i] * piv;
      else M[idx] -= colk[i] * M[(int64_t)k * n + j];
    }
    if (tid == 0) M[(int64_t)k * n + k] = piv;
    __syncthreads();
  }
}

// x = M b with the dense FP64 inverse; one wavefront per row.
template <typename T>
__global__ void k_coarse_solve(int64_t n, const double* __restrict__ M, const T* __restrict__ b,
                               T* __restrict__ x, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += kWave) s += M[i * n + j] * (double)b[j];
  s = group_sum<kWave>(s);
  if (lane == 0) x[i] = (T)s;
}

template <typename T>
__global__ void k_scale(int64_t n, const T* __restrict__ s, const T* __restrict__ b,
                        T* __restrict__ x, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = s[i] * b[i];
}

template <typename T>
__global__ void k_restrict(int64_t nc, const int32_t* __restrict__ crange, const T* __restrict__ r,
                           T* __restrict__ bc, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (I >= nc) return;
  T s = 0;
  for (int32_t i = crange[I]; i < crange[I + 1]; ++i) s += r[i];
  bc[I] = s;
}

template <typename T>
__global__ void k_prolong(int64_t n, const int32_t* __restrict__ pmap, const T* __restrict__ xc,
                          T* __restrict__ x, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += xc[pmap[i]];
}

// Chebyshev step: d = c1 d + c2 D1^-1 r (c1 = 0 on the first step), then
// xout = xin + d (xin NULL: from zero).  xin and xout may alias.
template <typename T>
__global__ void k_cheb(int64_t n, T c1, T c2, const T* __restrict__ s, const T* __restrict__ r,
                       T* __restrict__ d, const T* xin, T* xout,
                       const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T di = (c1 != T(0) ? c1 * d[i] : T(0)) + c2 * s[i] * r[i];
  d[i] = di;
  xout[i] = (xin ? xin[i] : T(0)) + di;
}

template <typename T> struct LevelBufs;
template <> struct LevelBufs<double> {
  static const double* val(const Level& L) { return L.val64.p; }
  static const double* diag(const Level& L) { return L.diag64.p; }
  static const double* sinv(const Level& L) { return L.sinv64.p; }
  static double* b(Level& L) { return L.b64.p; }
  static double* x(Level& L) { return L.x64.p; }
  static double* t(Level& L) { return L.t64.p; }
  static double* r(Level& L) { return L.r64.p; }
  static double* d(Level& L) { return L.d64.p; }
};
template <> struct LevelBufs<float> {
  static const float* val(const Level& L) { return L.val32.p; }
  static const float* diag(const Level& L) { return L.diag32.p; }
  static const float* sinv(const Level& L) { return L.sinv32.p; }
  static float* b(Level& L) { return L.b32.p; }
  static float* x(Level& L) { return L.x32.p; }
  static float* t(Level& L) { return L.t32.p; }
  static float* r(Level& L) { return L.r32.p; }
  static float* d(Level& L) { return L.d32.p; }
};

// Values (and columns) of the coarse level C = P^T F P.
int galerkin_fill(rt_ctx* ctx, const Level& F, Level& C) {
  hipLaunchKernelGGL((k_galerkin<true>), dim3(grid_for(C.n * kWave)), dim3(kBlock), 0,
                     ctx->stream, C.n, F.crange.p, F.rp.p, F.col.p, F.val64.p, F.diag64.p,
                     F.pmap.p, nullptr, C.rp.p, C.col.p, C.val64.p, C.diag64.p);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// Build level l+1 from level l: aggregation maps, coarse CSR structure, and
// the coarse columns and values, so that the new level is complete before it
// serves as the fine level of the next one.
int build_next_level(rt_ctx* ctx, rt_matrix* A, int l, int dim) {
  hipStream_t st = ctx->stream;
  Level& L = A->levels[l];
  const int64_t n = L.n;
  const int shift = l == 0 ? 0 : dim;
  DevBuf<int32_t> flag;
  RT_CHECK(flag.reserve(n));
  RT_CHECK(L.pmap.reserve(n));
  hipLaunchKernelGGL(k_agg_flags, dim3(grid_for(n)), dim3(kBlock), 0, st, n, shift, L.code.p,
                     flag.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int32_t, int32_t>(ctx, flag.p, L.pmap.p, n, true)));
  RT_CHECK(ctx->sync_read(L.pmap.p + n - 1, sizeof(int32_t)));
  int32_t nc32 = 0;
  std::memcpy(&nc32, ctx->host, sizeof(int32_t));
  const int64_t nc = nc32;
  A->levels.emplace_back();
  Level& C = A->levels.back();
  Level& Lr = A->levels[l];   // re-fetch after emplace_back
  C.n = nc;
  RT_CHECK(Lr.crange.reserve(nc + 1));
  RT_CHECK(C.code.reserve(nc));
  hipLaunchKernelGGL(k_agg_finish, dim3(grid_for(n)), dim3(kBlock), 0, st, n, shift, Lr.code.p,
                     flag.p, Lr.pmap.p, Lr.crange.p, C.code.p, nc);
  RT_LAUNCH_CHECK();
  // coarse structure: count, scan
  DevBuf<int64_t> cnt;
  RT_CHECK(cnt.reserve(nc + 1));
  RT_CHECK_HIP(hipMemsetAsync(cnt.p + nc, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL((k_galerkin<false>), dim3(grid_for(nc * kWave)), dim3(kBlock), 0, st, nc,
                     Lr.crange.p, Lr.rp.p, Lr.col.p, nullptr, nullptr, Lr.pmap.p, cnt.p, nullptr,
                     nullptr, nullptr, nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK(C.rp.reserve(nc + 1));
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, C.rp.p, nc + 1, false)));
  RT_CHECK(ctx->sync_read(C.rp.p + nc, sizeof(int64_t)));
  int64_t nnz = 0;
  std::memcpy(&nnz, ctx->host, sizeof(int64_t));
  C.nnz = nnz;
  RT_CHECK(max_nonneg<int64_t>(ctx, cnt.p, nc, &C.max_row));
  RT_CHECK(C.col.reserve(nnz));
  RT_CHECK(C.val64.reserve(nnz + kSpmvPad));
  RT_CHECK(C.diag64.reserve(nc));
  return galerkin_fill(ctx, A->levels[l], C);
}

int level_vectors(Level& L, bool fp32) {
  for (auto* b : {&L.b64, &L.x64, &L.t64, &L.r64, &L.d64, &L.sinv64, &L.dinv64})
    RT_CHECK(b->reserve(L.n));
  if (fp32) {
    for (auto* b : {&L.b32, &L.x32, &L.t32, &L.r32, &L.d32, &L.sinv32, &L.dinv32})
      RT_CHECK(b->reserve(L.n));
    RT_CHECK(L.val32.reserve(L.nnz + kSpmvPad));
    RT_CHECK(L.diag32.reserve(L.n));
  }
  return RT_OK;
}

}  // namespace

int amg_setup(rt_ctx* ctx, rt_matrix* A) {
  hipStream_t st = ctx->stream;
  const rt_neighbors* nb = A->nb;
  const bool fp32 = A->has_fp32;
  if (A->n == 0) return RT_OK;
  // structure (depends only on the neighbour object): built on first use
  if (A->levels.size() == 1 && A->amg.max_levels > 1 && A->levels[0].code.n == 0) {
    Level& L0 = A->levels[0];
    RT_CHECK(L0.code.reserve(L0.n));
    RT_CHECK_HIP(hipMemcpyAsync(L0.code.p, nb->skeys.p, sizeof(uint64_t) * L0.n,
                                hipMemcpyDeviceToDevice, st));
    for (int l = 0; (int)A->levels.size() < A->amg.max_levels; ++l) {
      const int64_t n = A->levels[l].n;
      if (n <= A->amg.coarse_size) break;
      RT_CHECK(build_next_level(ctx, A, l, nb->dim));
      const int64_t nc = A->levels.back().n;
      if (nc * 10 > n * 9 || nc == 0) {   // coarsening stalled: drop the level
        A->levels.pop_back();
        break;
      }
      if (A->amg.tiled_spmv) RT_CHECK(build_tiles(ctx, A->levels.back()));
    }
  }
  for (Level& L : A->levels) RT_CHECK(level_vectors(L, fp32));
  // numeric: Galerkin products down the hierarchy, smoother scalings
  for (size_t l = 0; l < A->levels.size(); ++l) {
    Level& L = A->levels[l];
    if (l > 0) {
      RT_CHECK(galerkin_fill(ctx, A->levels[l - 1], L));
      if (fp32) {
        if (L.nnz > 0)
          hipLaunchKernelGGL(k_to_f32, dim3(grid_for(L.nnz)), dim3(kBlock), 0, st, L.nnz,
                             L.val64.p, L.val32.p);
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(L.n)), dim3(kBlock), 0, st, L.n, L.diag64.p,
                           L.diag32.p);
        RT_LAUNCH_CHECK();
      }
      hipLaunchKernelGGL(k_smoother, dim3(grid_for(L.n * 8)), dim3(kBlock), 0, st, L.n, L.rp.p,
                         L.val64.p, L.diag64.p, L.sinv64.p, L.dinv64.p,
                         fp32 ? L.sinv32.p : nullptr, fp32 ? L.dinv32.p : nullptr);
      RT_LAUNCH_CHECK();
    }   // level 0: the assembly kernel wrote its scalings
  }
  // coarsest level: dense inverse when small
  Level& Lc = A->levels.back();
  A->coarse_direct = A->levels.size() > 1 && Lc.n <= kDenseMax;
  if (A->coarse_direct) {
    const int64_t nn = Lc.n * Lc.n;
    RT_CHECK(A->coarse_inv.reserve(nn));
    hipLaunchKernelGGL(k_dense_zero, dim3(grid_for(nn)), dim3(kBlock), 0, st, nn,
                       A->coarse_inv.p);
    hipLaunchKernelGGL(k_dense_fill, dim3(grid_for(Lc.n)), dim3(kBlock), 0, st, Lc.n, Lc.rp.p,
                       Lc.col.p, Lc.val64.p, Lc.diag64.p, A->coarse_inv.p);
    hipLaunchKernelGGL(k_gauss_jordan, dim3(1), dim3(1024), 0, st, (int)Lc.n, A->coarse_inv.p);
    RT_LAUNCH_CHECK();
  }
  return RT_OK;
}

// Chebyshev smoothing of A x = b on level L, degree steps: from zero into x
// (xin NULL), or from xin into x.  Each step after a start from zero costs
// one residual product.
template <typename T>
static int cheb_smooth(hipStream_t st, rt_matrix* A, Level& L, int degree, const T* b,
                       const T* xin, T* x, const int32_t* stop) {
  using B = LevelBufs<T>;
  const int64_t n = L.n;
  const double hi = 1.0, lo = 0.25;   // interval of D1^-1 A to damp
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  T* r = B::r(L);
  const T* r0 = b;   // residual of the zero start
  if (xin) {
    RT_CHECK((launch_spmv_level<T, SP_RESID>(st, L, B::val(L), B::diag(L), xin, b, nullptr, r,
                                             nullptr, nullptr, nullptr, level_shape<T>(L),
                                             nullptr, stop)));
    r0 = r;
  }
  hipLaunchKernelGGL(k_cheb<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, T(0),
                     (T)(1.0 / theta), B::sinv(L), r0, B::d(L), xin, x, stop);
  RT_LAUNCH_CHECK();
  for (int k = 1; k < degree; ++k) {
    RT_CHECK((launch_spmv_level<T, SP_RESID>(st, L, B::val(L), B::diag(L), x, b, nullptr, r,
                                             nullptr, nullptr, nullptr, level_shape<T>(L),
                                             nullptr, stop)));
    const double rho_next = 1.0 / (2.0 * sigma - rho);
    hipLaunchKernelGGL(k_cheb<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n,
                       (T)(rho_next * rho), (T)(2.0 * rho_next / delta), B::sinv(L), r, B::d(L),
                       x, x, stop);
    RT_LAUNCH_CHECK();
    rho = rho_next;
  }
  return RT_OK;
}

template <typename T>
static int vcycle_level(rt_ctx* ctx, rt_matrix* A, size_t l, const T* b, T* out,
                        const int32_t* stop) {
  using B = LevelBufs<T>;
  hipStream_t st = ctx->stream;
  Level& L = A->levels[l];
  const int64_t n = L.n;
  if (l + 1 == A->levels.size()) {
    if (A->coarse_direct) {
      hipLaunchKernelGGL(k_coarse_solve<T>, dim3(grid_for(n * kWave)), dim3(kBlock), 0, st, n,
                         A->coarse_inv.p, b, out, stop);
      RT_LAUNCH_CHECK();
      return RT_OK;
    }
    // four l1-Jacobi sweeps from zero (a symmetric positive-definite operator)
    T* t = B::t(L);
    hipLaunchKernelGGL(k_scale<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B::sinv(L), b, t,
                       stop);
    RT_LAUNCH_CHECK();
    T* src = t;
    T* dst = out;
    for (int sweep = 0; sweep < 3; ++sweep) {
      RT_CHECK((launch_spmv_level<T, SP_SMOOTH>(st, L, B::val(L), B::diag(L), src, b, B::sinv(L),
                                                dst, nullptr, nullptr, nullptr,
                                                level_shape<T>(L), nullptr, stop)));
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    if (src != out)
      RT_CHECK_HIP(hipMemcpyAsync(out, src, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
    return RT_OK;
  }
  Level& C = A->levels[l + 1];
  T* t = B::t(L);
  T* r = B::r(L);
  const bool cheb = A->amg.smoother == RT_SMOOTHER_CHEBYSHEV;
  if (cheb) {
    RT_CHECK(cheb_smooth<T>(st, A, L, A->amg.smoother_degree, b, nullptr, t, stop));
  } else {
    hipLaunchKernelGGL(k_scale<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B::sinv(L), b, t,
                       stop);
    RT_LAUNCH_CHECK();
  }
  RT_CHECK((launch_spmv_level<T, SP_RESID>(st, L, B::val(L), B::diag(L), t, b, nullptr, r,
                                           nullptr, nullptr, nullptr, level_shape<T>(L),
                                           nullptr, stop)));
  hipLaunchKernelGGL(k_restrict<T>, dim3(grid_for(C.n)), dim3(kBlock), 0, st, C.n, L.crange.p,
                     r, B::b(C), stop);
  RT_LAUNCH_CHECK();
  RT_CHECK(vcycle_level<T>(ctx, A, l + 1, B::b(C), B::x(C), stop));
  hipLaunchKernelGGL(k_prolong<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, L.pmap.p, B::x(C),
                     t, stop);
  RT_LAUNCH_CHECK();
  if (cheb) return cheb_smooth<T>(st, A, L, A->amg.smoother_degree, b, t, out, stop);
  RT_CHECK((launch_spmv_level<T, SP_SMOOTH>(st, L, B::val(L), B::diag(L), t, b, B::sinv(L), out,
                                            nullptr, nullptr, nullptr, level_shape<T>(L),
                                            nullptr, stop)));
  return RT_OK;
}

template <typename T>
int vcycle(rt_ctx* ctx, rt_matrix* A, const T* b, T* z, const int32_t* stop) {
  return vcycle_level<T>(ctx, A, 0, b, z, stop);
}

template int vcycle<double>(rt_ctx*, rt_matrix*, const double*, double*, const int32_t*);
template int vcycle<float>(rt_ctx*, rt_matrix*, const float*, float*, const int32_t*);

}  // namespace rt

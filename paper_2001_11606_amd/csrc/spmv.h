// Sparse matrix-vector kernels over (diagonal + off-diagonal CSR) on gfx950.
//
// One group of G lanes (G in {4, 8, 16, 32, 64}, about four entries per lane)
// per row and 256/G rows per block, with no grid-stride loop: the launch
// covers every row once, so the hardware keeps as many waves resident as the
// register file allows and each wave has one short dependency chain
// (row pointers -> values/columns -> x gathers).  Each lane issues up to four
// independent value/column loads before it consumes them, and values and
// columns are streamed with non-temporal loads so that L2 keeps the gathered
// x.  Blocks are renumbered so that each of the eight XCDs (which receive
// blocks round-robin) works on one contiguous eighth of the rows and its L2
// sees the x-neighbourhood of those rows.  Accumulation is in the value type
// T (FP32 in the mixed-precision inner solve, FP64 otherwise); per-block dot
// products are combined in FP64 in a fixed order, so results are
// deterministic run to run.
#pragma once

#include "internal.h"
#include "reduce.h"

namespace rt {

enum SpmvMode {
  SP_PLAIN = 0,   // y = A x
  SP_DOT = 1,     // y = A x, part[block] = sum x.y
  SP_RESID = 2,   // y = b - A x (optionally y32 = (float) y), part[block] = sum y.y
  SP_SMOOTH = 3,  // y = x + s (b - A x)
};

constexpr int kXcd = 8;

// physical block -> logical block, so that XCD k (blocks k, k+8, ...) gets the
// contiguous logical range [k*per, (k+1)*per)
__device__ __forceinline__ int xcd_block(int per) {
  const int p = blockIdx.x;
  return (p % kXcd) * per + p / kXcd;
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock)
k_spmv(int64_t n, int per, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
       const T* __restrict__ val, const T* __restrict__ diag, const T* __restrict__ x,
       const T* __restrict__ b, const T* __restrict__ s, T* __restrict__ y,
       float* __restrict__ y32, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  constexpr int RPB = kBlock / G;
  const int lb = xcd_block(per);
  const int lane = threadIdx.x & (G - 1);
  const int64_t i = (int64_t)lb * RPB + threadIdx.x / G;
  double acc = 0.0;
  if (i < n) {
    const int64_t k1 = rp[i + 1];
    int64_t k = rp[i] + lane;
    T sum = 0;
    for (; k + 3 * G < k1; k += 4 * G) {
      const int32_t c0 = stream_load(col + k), c1 = stream_load(col + k + G);
      const int32_t c2 = stream_load(col + k + 2 * G), c3 = stream_load(col + k + 3 * G);
      const T v0 = stream_load(val + k), v1 = stream_load(val + k + G);
      const T v2 = stream_load(val + k + 2 * G), v3 = stream_load(val + k + 3 * G);
      sum += v0 * x[c0];
      sum += v1 * x[c1];
      sum += v2 * x[c2];
      sum += v3 * x[c3];
    }
    for (; k < k1; k += G) sum += stream_load(val + k) * x[stream_load(col + k)];
    sum = group_sum<G>(sum);
    if (lane == 0) {
      const T xi = x[i];
      const T ax = diag[i] * xi + sum;
      if (MODE == SP_PLAIN) {
        y[i] = ax;
      } else if (MODE == SP_DOT) {
        y[i] = ax;
        acc = (double)xi * (double)ax;
      } else if (MODE == SP_RESID) {
        const T r = b[i] - ax;
        y[i] = r;
        if (y32) y32[i] = (float)r;
        acc = (double)r * (double)r;
      } else {
        y[i] = xi + s[i] * (b[i] - ax);
      }
    }
  }
  if (MODE == SP_DOT || MODE == SP_RESID) {
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0 && part) part[lb] = t;
  }
}

// about four entries per lane
inline int spmv_group(double avg_row) {
  if (avg_row > 192) return 64;
  if (avg_row > 48) return 16;
  if (avg_row > 20) return 8;
  return 4;
}

// Blocks (= partials written) of an SpMV over n rows with group size G.
inline int spmv_blocks(int64_t n, int G) {
  const int64_t rpb = kBlock / G;
  const int64_t nblk = (n + rpb - 1) / rpb;
  const int64_t per = (nblk + kXcd - 1) / kXcd;
  return (int)(per * kXcd);
}

// Launch helper; *nparts receives the number of partials written.
template <typename T, int MODE>
int launch_spmv(hipStream_t st, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                const T* val, const T* diag, const T* x, const T* b, const T* s, T* y,
                float* y32, double* part, int* nparts) {
  const int G = spmv_group(n ? (double)nnz / (double)n : 0.0);
  const int grid = spmv_blocks(n, G);
  const int per = grid / kXcd;
  if (nparts) *nparts = grid;
  if (n == 0) return RT_OK;
#define RT_SPMV_G(G_)                                                                        \
  hipLaunchKernelGGL((k_spmv<T, G_, MODE>), dim3(grid), dim3(kBlock), 0, st, n, per, rp, col, \
                     val, diag, x, b, s, y, y32, part)
  switch (G) {
    case 64: RT_SPMV_G(64); break;
    case 16: RT_SPMV_G(16); break;
    case 8: RT_SPMV_G(8); break;
    default: RT_SPMV_G(4); break;
  }
#undef RT_SPMV_G
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// Upper bound on the partials any kernel of the solver writes for n rows.
inline int64_t max_partials(int64_t n) { return (int64_t)spmv_blocks(n, 64) + 2 * kMaxPartials; }

}  // namespace rt

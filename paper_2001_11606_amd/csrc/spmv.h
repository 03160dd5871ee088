// Sparse matrix-vector kernels over (diagonal + off-diagonal CSR) on gfx950.
//
// One group of G lanes (G in {8, 16, 32, 64}) per row: the lanes stream the
// row's values and int32 columns contiguously, gather x through the caches,
// and combine their partial sums with lane shuffles.  Rows are assigned
// grid-stride; the per-row result is written by the group's first lane.
// Accumulation is in the value type T (FP32 in the mixed-precision path,
// FP64 otherwise); block partials of dot products are combined in FP64 with
// a fixed order.
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

template <typename T, int G, int MODE>
__global__ void __launch_bounds__(kBlock)
k_spmv(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
       const T* __restrict__ val, const T* __restrict__ diag, const T* __restrict__ x,
       const T* __restrict__ b, const T* __restrict__ s, T* __restrict__ y,
       float* __restrict__ y32, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  const int lane = threadIdx.x & (G - 1);
  const int64_t grp = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / G;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / G;
  double acc = 0.0;
  for (int64_t i = grp; i < n; i += ngrp) {
    const int64_t k1 = rp[i + 1];
    T sum = 0;
    for (int64_t k = rp[i] + lane; k < k1; k += G) sum += val[k] * x[col[k]];
    sum = group_sum<G>(sum);
    if (lane == 0) {
      const T xi = x[i];
      const T ax = diag[i] * xi + sum;
      if (MODE == SP_PLAIN) {
        y[i] = ax;
      } else if (MODE == SP_DOT) {
        y[i] = ax;
        acc += (double)xi * (double)ax;
      } else if (MODE == SP_RESID) {
        const T r = b[i] - ax;
        y[i] = r;
        if (y32) y32[i] = (float)r;
        acc += (double)r * (double)r;
      } else {
        y[i] = xi + s[i] * (b[i] - ax);
      }
    }
  }
  if (MODE == SP_DOT || MODE == SP_RESID) {
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0 && part) part[blockIdx.x] = t;
  }
}

inline int spmv_group(double avg_row) {
  if (avg_row > 40) return 64;
  if (avg_row > 18) return 32;
  if (avg_row > 8) return 16;
  return 8;
}

// Launch helper; returns the number of blocks (= partials written).
template <typename T, int MODE>
int launch_spmv(hipStream_t st, int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                const T* val, const T* diag, const T* x, const T* b, const T* s, T* y,
                float* y32, double* part, int* nblocks) {
  const int G = spmv_group(n ? (double)nnz / (double)n : 0.0);
  const int cap = (MODE == SP_DOT || MODE == SP_RESID) ? kMaxPartials : (1 << 20);
  const int grid = grid_for(n * (int64_t)G, kBlock, cap);
  if (nblocks) *nblocks = grid;
#define RT_SPMV_G(G_)                                                                       \
  hipLaunchKernelGGL((k_spmv<T, G_, MODE>), dim3(grid), dim3(kBlock), 0, st, n, rp, col, val, \
                     diag, x, b, s, y, y32, part)
  switch (G) {
    case 64: RT_SPMV_G(64); break;
    case 32: RT_SPMV_G(32); break;
    case 16: RT_SPMV_G(16); break;
    default: RT_SPMV_G(8); break;
  }
#undef RT_SPMV_G
  RT_LAUNCH_CHECK();
  return RT_OK;
}

}  // namespace rt

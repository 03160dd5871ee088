// Sparse matrix-vector kernels over (diagonal + off-diagonal CSR) on gfx950.
//
// A group of G lanes works on one row and each lane owns ENT entries of it
// (entries lane, lane + G, ..., lane + (ENT-1) G of the row), so a row of up
// to G*ENT entries is covered by one pass and 256/G rows share a block.  The
// kernel is built so that a wave waits on memory exactly three times:
//   1. row bounds and the row's own diagonal, x_i, b_i, s_i (independent loads),
//   2. all ENT column indices and values of the lane (issued back to back;
//      slots beyond the row end re-read the row's last entry, which is a cache
//      hit, and are weighted by zero),
//   3. all ENT gathers of x.
// Longer rows repeat steps 2-3.  With no serial chain inside a row, the bytes
// a wave has in flight scale with G*ENT*(rows per wave), which is what an
// HBM-bound sweep needs.  There is no grid-stride loop: the launch covers
// every row once.  Values and columns are streamed with non-temporal loads so
// that L2 keeps the gathered x.  Blocks are renumbered so that each of the
// eight XCDs (which receive blocks round-robin) works on one contiguous eighth
// of the rows and its L2 sees the x-neighbourhood of those rows.
// Accumulation is in the value type T (FP32 in the mixed-precision inner
// solve, FP64 otherwise); per-block dot products are combined in FP64 in a
// fixed order, so results are deterministic run to run.
#pragma once

#include "internal.h"
#include "reduce.h"

namespace rt {

enum SpmvMode {
  SP_PLAIN = 0,   // y = A x
  SP_DOT = 1,     // y = A x, part[block] = sum x.y
  SP_RESID = 2,   // y = b - A x (optionally y32 = (float) y), part[block] = sum y.y;
                  // optionally pmax[block] = max_i |y_i| / (a_ii |x_i|) and
                  // w32 = 1 / (a_ii |x_i|) (see cw_term)
  SP_SMOOTH = 3,  // y = x + s (b - A x)
};

// Componentwise residual measure of row i: |r_i| / (a_ii |x_i|), the relative
// change of x_i that one Jacobi sweep would make.  A row with x_i = 0 counts
// as converged when r_i = 0 and as unconverged (infinity) otherwise.
__device__ __forceinline__ double cw_term(double r, double aii, double x) {
  const double ax = aii * fabs(x);
  return ax > 0.0 ? fabs(r) / ax : (r == 0.0 ? 0.0 : INFINITY);
}
// Weight w_i with |r_i| w_i = cw_term for a fixed x (the FP32 inner solve of
// the refinement loop measures its own residual with it); 0 where x_i = 0,
// whose rows the FP64 test above still covers.
__device__ __forceinline__ float cw_weight(double aii, double x) {
  const double ax = aii * fabs(x);
  return ax > 0.0 ? (float)fmin(1.0 / ax, 3.0e38) : 0.0f;
}

constexpr int kXcd = 8;

// physical block -> logical block, so that XCD k (blocks k, k+8, ...) gets the
// contiguous logical range [k*per, (k+1)*per)
__device__ __forceinline__ int xcd_block(int per) {
  const int p = blockIdx.x;
  return (p % kXcd) * per + p / kXcd;
}

#ifndef RT_SPMV_STAGE
#define RT_SPMV_STAGE 8
#endif
#ifndef RT_SPMV_EAGER_TAIL
#define RT_SPMV_EAGER_TAIL 1
#endif
#ifndef RT_SPMV_NT_STORE
#define RT_SPMV_NT_STORE 1
#endif

// a product's per-row output, written once and read by a later kernel
template <typename T>
__device__ __forceinline__ void out_store(T* p, T v) {
#if RT_SPMV_NT_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

template <typename T, int G, int ENT, int MODE>
__global__ void __launch_bounds__(kBlock)
k_spmv(int64_t n, int per, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
       const T* __restrict__ val, const T* __restrict__ diag, const T* __restrict__ x,
       const T* __restrict__ b, const T* __restrict__ s, T* __restrict__ y,
       float* __restrict__ y32, double* __restrict__ part, const int32_t* __restrict__ tprob,
       const int32_t* __restrict__ skip, double* __restrict__ pmax, float* __restrict__ w32) {
  __shared__ double red[kBlock / kWave];
  constexpr int RPB = kBlock / G;
  const int lb = xcd_block(per);
  if (skip) {   // rows of a finished problem are left as they are
    const int64_t rb = (int64_t)lb * RPB;
    if (rb < n && skip[tprob ? tprob[rb / kTileRows] : 0]) return;
  }
  const int lane = threadIdx.x & (G - 1);
  const int64_t i = (int64_t)lb * RPB + threadIdx.x / G;
  double acc = 0.0, cwm = 0.0;
  if (i < n) {
    const int64_t k0 = rp[i], k1 = rp[i + 1];
    const T xi = x[i];
    const T di = diag[i];
    T bi = 0, si = 0;
    if (MODE == SP_RESID || MODE == SP_SMOOTH) bi = b[i];
    if (MODE == SP_SMOOTH) si = s[i];
    T sum = 0;
    for (int64_t base = k0 + lane; base < k1; base += G * ENT) {
      int32_t c[ENT];
      T v[ENT];
#pragma unroll
      for (int e = 0; e < ENT; ++e) {
        const int64_t k = base + e * G;
        const int64_t kc = k < k1 ? k : k1 - 1;
        c[e] = stream_load(col + kc);
        const T w = stream_load(val + kc);
        v[e] = k < k1 ? w : T(0);
      }
      T xv[ENT];
#pragma unroll
      for (int e = 0; e < ENT; ++e) xv[e] = x[c[e]];
#pragma unroll
      for (int e = 0; e < ENT; ++e) sum += v[e] * xv[e];
    }
    sum = group_sum<G>(sum);
    if (lane == 0) {
      const T ax = di * xi + sum;
      if (MODE == SP_PLAIN) {
        y[i] = ax;
      } else if (MODE == SP_DOT) {
        y[i] = ax;
        acc = (double)xi * (double)ax;
      } else if (MODE == SP_RESID) {
        const T r = bi - ax;
        y[i] = r;
        if (y32) y32[i] = (float)r;
        acc = (double)r * (double)r;
        if (pmax) cwm = cw_term((double)r, (double)di, (double)xi);
        if (w32) w32[i] = cw_weight((double)di, (double)xi);
      } else {
        y[i] = xi + si * (bi - ax);
      }
    }
  }
  if (MODE == SP_DOT || MODE == SP_RESID) {
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0 && part) part[lb] = t;
  }
  if (MODE == SP_RESID && pmax) {
    const double m = block_max(cwm, red);
    if (threadIdx.x == 0) pmax[lb] = m;
  }
}

// A lane's four entries of one pass over a row (a pass covers the 4G
// entries from a 4-aligned base gb).  Every load instruction of a group of G
// lanes reads one contiguous run: FP32 lanes hold four consecutive entries
// (16 bytes at 4 lane); FP64 lanes hold two pairs, entries 2 lane and
// 2G + 2 lane (16 bytes each), so that each 16-byte load is contiguous across
// the lanes rather than strided by 32 bytes.  Loads of entries at or past
// the row's end k1 are skipped; dot() adds only entries in [k0, k1).
typedef float rt_f32x4 __attribute__((vector_size(16)));
typedef double rt_f64x2 __attribute__((vector_size(16)));
typedef unsigned short rt_u16x4 __attribute__((vector_size(8)));
typedef unsigned short rt_u16x2 __attribute__((vector_size(4)));

template <typename T, int G>
struct LaneSeg;
template <int G>
struct LaneSeg<float, G> {
  rt_f32x4 v;
  rt_u16x4 c;
  int k;   // first entry
  __device__ __forceinline__ void load(const float* vt, const uint16_t* lt, int gb, int lane,
                                       int k1) {
    k = gb + 4 * lane;
    if (k < k1) {
      v = stream_load(reinterpret_cast<const rt_f32x4*>(vt + k));
      c = stream_load(reinterpret_cast<const rt_u16x4*>(lt + k));
    }
  }
  __device__ __forceinline__ float dot(int k0, int k1, const float* xs) const {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool in = k + j >= k0 && k + j < k1;
      s += in ? v[j] * xs[in ? c[j] : 0] : 0.f;   // (the index of an unloaded entry is not read)
    }
    return s;
  }
};
template <int G>
struct LaneSeg<double, G> {
  rt_f64x2 a, b;
  rt_u16x2 ca, cb;
  int k;   // first entry of the first pair; the second starts at k + 2G
  __device__ __forceinline__ void load(const double* vt, const uint16_t* lt, int gb, int lane,
                                       int k1) {
    k = gb + 2 * lane;
    if (k < k1) {
      a = stream_load(reinterpret_cast<const rt_f64x2*>(vt + k));
      ca = stream_load(reinterpret_cast<const rt_u16x2*>(lt + k));
    }
    if (k + 2 * G < k1) {
      b = stream_load(reinterpret_cast<const rt_f64x2*>(vt + k + 2 * G));
      cb = stream_load(reinterpret_cast<const rt_u16x2*>(lt + k + 2 * G));
    }
  }
  __device__ __forceinline__ double dot(int k0, int k1, const double* xs) const {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const bool in = k + j >= k0 && k + j < k1;
      s += in ? a[j] * xs[in ? ca[j] : 0] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int e = k + 2 * G + j;
      const bool in = e >= k0 && e < k1;
      s += in ? b[j] * xs[in ? cb[j] : 0] : 0.0;
    }
    return s;
  }
};

// Tiled product: one block per tile of kTileRows rows (one row per thread for
// the row data and the output).  The tile's distinct columns are staged from
// x into LDS, then groups of G lanes walk the rows, UNR rows per group at a
// time (their loads all in flight together), in passes of 4G entries from
// the 4-aligned base (k0 & ~3), each lane holding four entries of a pass
// (values and 16-bit local columns, laid out by LaneSeg); entries outside
// the row add nothing.  Row sums go through LDS so that the
// output and the dot-product terms are written by one thread per row.
#ifdef RT_SPMV_WAVES
#define RT_SPMV_OCC __attribute__((amdgpu_waves_per_eu(RT_SPMV_WAVES)))
#else
#define RT_SPMV_OCC
#endif
template <typename T, int G, int UNR, int MODE>
__global__ void __launch_bounds__(kBlock) RT_SPMV_OCC
k_spmv_tiled(int64_t n, int per, const int64_t* __restrict__ rp, const uint16_t* __restrict__ lcol,
             const T* __restrict__ val, const T* __restrict__ diag,
             const int64_t* __restrict__ toff, const int32_t* __restrict__ tcols,
             const T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ s,
             T* __restrict__ y, float* __restrict__ y32, double* __restrict__ part,
             const int32_t* __restrict__ tprob, const int32_t* __restrict__ skip,
             double* __restrict__ pmax, float* __restrict__ w32) {
  RT_DYNAMIC_LDS(dyn_lds);
  T* xs = reinterpret_cast<T*>(dyn_lds);
  __shared__ int srp[kTileRows + 1];      // row bounds relative to the tile's aligned base
  __shared__ int64_t sbase;
  __shared__ T sy[kTileRows];
  constexpr bool kNeedB = MODE == SP_RESID || MODE == SP_SMOOTH;
  // the rows' own data, fetched while the columns are staged
  __shared__ T sdx[(kNeedB ? 3 : 2) + (MODE == SP_SMOOTH ? 1 : 0)][kTileRows];
  __shared__ double red[kBlock / kWave];
  constexpr int NG = kBlock / G;   // row groups per block; UNR rows per group in flight
  static_assert(kTileRows % (NG * UNR) == 0, "tile rows must split evenly over the groups");
  const int t = xcd_block(per);
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)t * kTileRows;
  const int64_t i = r0 + tid;
  if (skip && r0 < n && skip[tprob ? tprob[t] : 0]) return;   // a finished problem's tile
  const bool live = i < n;   // grids are padded to a multiple of the XCD count
  if (tid == 0) sbase = r0 < n ? rp[r0] & ~(int64_t)3 : 0;
  __syncthreads();
  const int64_t base_e = sbase;   // entries of a tile number far below 2^31
  if (r0 < n) {
    srp[tid] = (int)(rp[live ? i : n] - base_e);
    if (tid == 0) srp[kTileRows] = (int)(rp[r0 + kTileRows < n ? r0 + kTileRows : n] - base_e);
    if (live) {
      sdx[0][tid] = diag[i];
      sdx[1][tid] = x[i];
      if (kNeedB) sdx[2][tid] = b[i];
      if (MODE == SP_SMOOTH) sdx[kNeedB ? 3 : 2][tid] = s[i];
    }
    // columns staged kStage per thread at a time: all index loads, then all
    // gathers, so that a thread keeps kStage gathers in flight
    constexpr int kStage = RT_SPMV_STAGE;
    const int64_t u0 = toff[t];
    const int cnt = (int)(toff[t + 1] - u0);
    for (int k0 = 0; k0 < cnt; k0 += kStage * kBlock) {
      int32_t c[kStage];
#pragma unroll
      for (int q = 0; q < kStage; ++q) {
        const int k = k0 + q * kBlock + tid;
        c[q] = k < cnt ? tcols[u0 + k] : -1;
      }
      T xv[kStage];
#pragma unroll
      for (int q = 0; q < kStage; ++q) xv[q] = c[q] >= 0 ? x[c[q]] : T(0);
#pragma unroll
      for (int q = 0; q < kStage; ++q) {
        const int k = k0 + q * kBlock + tid;
        if (k < cnt) xs[k] = xv[q];
      }
    }
  } else {
    srp[tid] = 0;
    if (tid == 0) srp[kTileRows] = 0;
  }
  __syncthreads();
  const int grp = tid / G, lane = tid & (G - 1);
  const T* vt = val + base_e;
  const uint16_t* lt = lcol + base_e;
  for (int base = 0; base < kTileRows; base += NG * UNR) {
    int k0[UNR], k1[UNR], gb[UNR];
    LaneSeg<T, G> v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int rr = base + u * NG + grp;
      k0[u] = srp[rr];
      k1[u] = srp[rr + 1];
      gb[u] = k0[u] & ~3;   // the group's pass base (4-aligned)
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) v[u].load(vt, lt, gb[u], lane, k1[u]);
#if RT_SPMV_EAGER_TAIL
    // the second pass of every row in flight with the first
    LaneSeg<T, G> v2[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (gb[u] + 4 * G < k1[u]) v2[u].load(vt, lt, gb[u] + 4 * G, lane, k1[u]);
    constexpr int kFirstTail = 2;
#else
    constexpr int kFirstTail = 1;
#endif
    T sum[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) sum[u] = v[u].dot(k0[u], k1[u], xs);
#if RT_SPMV_EAGER_TAIL
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (gb[u] + 4 * G < k1[u]) sum[u] += v2[u].dot(k0[u], k1[u], xs);
#endif
    // rows longer than the passes above
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      for (int pb = gb[u] + kFirstTail * 4 * G; pb < k1[u]; pb += 4 * G) {
        LaneSeg<T, G> w;
        w.load(vt, lt, pb, lane, k1[u]);
        sum[u] += w.dot(k0[u], k1[u], xs);
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const T r = group_sum<G>(sum[u]);
      if (lane == 0) sy[base + u * NG + grp] = r;
    }
  }
  __syncthreads();
  double acc = 0.0, cwm = 0.0;
  if (live) {
    const T di = sdx[0][tid];
    const T xi = sdx[1][tid];
    T bi = 0, si = 0;
    if (kNeedB) bi = sdx[2][tid];
    if (MODE == SP_SMOOTH) si = sdx[kNeedB ? 3 : 2][tid];
    const T ax = di * xi + sy[tid];
    if (MODE == SP_PLAIN) {
      out_store(y + i, ax);
    } else if (MODE == SP_DOT) {
      out_store(y + i, ax);
      acc = (double)xi * (double)ax;
    } else if (MODE == SP_RESID) {
      const T r = bi - ax;
      out_store(y + i, r);
      if (y32) out_store(y32 + i, (float)r);
      acc = (double)r * (double)r;
      if (pmax) cwm = cw_term((double)r, (double)di, (double)xi);
      if (w32) out_store(w32 + i, cw_weight((double)di, (double)xi));
    } else {
      out_store(y + i, xi + si * (bi - ax));
    }
  }
  if (MODE == SP_DOT || MODE == SP_RESID) {
    const double tsum = block_sum(acc, red);
    if (tid == 0 && part) part[t] = tsum;
  }
  if (MODE == SP_RESID && pmax) {
    const double m = block_max(cwm, red);
    if (tid == 0) pmax[t] = m;
  }
}

// Product shapes: plain ones (G lanes per row, E entries per lane, global x
// gathers) and tiled ones (G lanes per row, four-entry chunks, x from LDS,
// E rows per lane group in flight).
struct SpmvShape {
  int g, ent;
  bool tiled;
};
constexpr SpmvShape kSpmvShapes[] = {{4, 4, false},  {4, 8, false},  {8, 8, false},
                                     {8, 12, false}, {16, 6, false}, {32, 6, false},
                                     {64, 4, false}, {4, 4, true},   {8, 4, true},
                                     {16, 4, true},  {32, 4, true},  {64, 4, true},
                                     {8, 2, true},   {16, 2, true},  {32, 2, true},
                                     {8, 1, true},   {16, 1, true},  {32, 1, true}};
constexpr int kNumSpmvShapes = sizeof(kSpmvShapes) / sizeof(kSpmvShapes[0]);
constexpr int kFirstTiledShape = 7;

// the smallest plain shape whose one pass covers the longest row (else the widest)
inline int spmv_plain_shape_for(int64_t max_row) {
  for (int s = 0; s < kFirstTiledShape; ++s)
    if ((int64_t)kSpmvShapes[s].g * kSpmvShapes[s].ent >= max_row) return s;
  return kFirstTiledShape - 1;
}
// default tiled shape: two rows in flight per lane group (fewer registers
// than four, which measured faster on the 3-D workloads), lanes per row so
// that a row takes at most two passes; very short rows: four lanes, four rows
inline int spmv_tiled_shape_for(int64_t max_row) {
  if (max_row <= 13) return kFirstTiledShape;        // (4, 4)
  if (max_row <= 2 * (4 * 8 - 3)) return 12;        // (8, 2)
  if (max_row <= 2 * (4 * 16 - 3)) return 13;        // (16, 2)
  if (max_row <= 2 * (4 * 32 - 3)) return 14;        // (32, 2)
  return kFirstTiledShape + 4;                        // (64, 4)
}
// the shape a product over L runs with, given the requested one (-1: default)
inline int spmv_effective_shape(const Level& L, int shape) {
  if (shape >= 0 && shape < kNumSpmvShapes && (!kSpmvShapes[shape].tiled || L.tiled)) return shape;
  return L.tiled ? spmv_tiled_shape_for(L.max_row) : spmv_plain_shape_for(L.max_row);
}

// Blocks (= partials written) of a product over n rows, rows_per_block rows
// per block, padded to a multiple of the XCD count.
inline int spmv_blocks_rows(int64_t n, int64_t rows_per_block) {
  const int64_t nblk = (n + rows_per_block - 1) / rows_per_block;
  const int64_t per = (nblk + kXcd - 1) / kXcd;
  return (int)(per * kXcd);
}
inline int spmv_blocks(int64_t n, int G) { return spmv_blocks_rows(n, kBlock / G); }

// Product over level L in the precision of T; *nparts receives the number of
// partials written.  shape: index into kSpmvShapes, -1 = the level's default.
// Rows per block (= per partial) of a product over L with the given shape.
inline int spmv_rows_per_block(const Level& L, int shape) {
  const SpmvShape sh = kSpmvShapes[spmv_effective_shape(L, shape)];
  return sh.tiled ? kTileRows : kBlock / sh.g;
}

// skip (else NULL): per-problem stop flags; blocks whose problem is flagged
// do nothing.  tprob: the problem of every 256-row tile (batched systems), or
// NULL for one problem (flag skip[0]).
// pmax, w32 (SP_RESID only, else NULL): per-block maxima of the componentwise
// residual measure and the per-row weights of cw_weight.
template <typename T, int MODE>
int launch_spmv_level(hipStream_t st, const Level& L, const T* val, const T* diag, const T* x,
                      const T* b, const T* s, T* y, float* y32, double* part, int* nparts,
                      int shape = -1, const int32_t* tprob = nullptr,
                      const int32_t* skip = nullptr, double* pmax = nullptr,
                      float* w32 = nullptr) {
  const int64_t n = L.n;
  shape = spmv_effective_shape(L, shape);
  const SpmvShape sh = kSpmvShapes[shape];
  const int grid = sh.tiled ? spmv_blocks_rows(n, kTileRows) : spmv_blocks(n, sh.g);
  const int per = grid / kXcd;
  if (nparts) *nparts = grid;
  if (n == 0) return RT_OK;
  if (sh.tiled) {
    const size_t lds = sizeof(T) * (size_t)(L.max_tile_cols > 0 ? L.max_tile_cols : 1);
#define RT_SPMV_T(G_, U_)                                                                     \
  hipLaunchKernelGGL((k_spmv_tiled<T, G_, U_, MODE>), dim3(grid), dim3(kBlock), lds, st, n, per, \
                     L.rp.p, L.lcol.p, val, diag, L.tile_off.p, L.tile_cols.p, x, b, s, y, y32,  \
                     part, tprob, skip, pmax, w32)
    switch (shape) {
      case 7: RT_SPMV_T(4, 4); break;
      case 8: RT_SPMV_T(8, 4); break;
      case 9: RT_SPMV_T(16, 4); break;
      case 10: RT_SPMV_T(32, 4); break;
      case 11: RT_SPMV_T(64, 4); break;
      case 12: RT_SPMV_T(8, 2); break;
      case 13: RT_SPMV_T(16, 2); break;
      case 14: RT_SPMV_T(32, 2); break;
      case 15: RT_SPMV_T(8, 1); break;
      case 16: RT_SPMV_T(16, 1); break;
      default: RT_SPMV_T(32, 1); break;
    }
#undef RT_SPMV_T
  } else {
#define RT_SPMV_S(G_, E_)                                                                       \
  hipLaunchKernelGGL((k_spmv<T, G_, E_, MODE>), dim3(grid), dim3(kBlock), 0, st, n, per, L.rp.p, \
                     L.col.p, val, diag, x, b, s, y, y32, part, tprob, skip, pmax, w32)
    switch (shape) {
      case 0: RT_SPMV_S(4, 4); break;
      case 1: RT_SPMV_S(4, 8); break;
      case 2: RT_SPMV_S(8, 8); break;
      case 3: RT_SPMV_S(8, 12); break;
      case 4: RT_SPMV_S(16, 6); break;
      case 5: RT_SPMV_S(32, 6); break;
      default: RT_SPMV_S(64, 4); break;
    }
#undef RT_SPMV_S
  }
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// Upper bound on the partials any kernel of the solver writes for n rows.
inline int64_t max_partials(int64_t n) { return (int64_t)spmv_blocks(n, 64) + 2 * kMaxPartials; }

}  // namespace rt

// Device primitives of the set-up paths: prefix sums, a stable radix sort of
// (key, value) pairs and a per-row sort.  They run once per neighbour build,
// matrix structure or hierarchy set-up, never inside the Krylov loop, so
// they favour simplicity over speed: a three-phase tiled scan, a one-bit LSD
// split sort built on that scan (stable by construction), and an insertion
// sort per row for the short rows of the neighbour and matrix exports.
#include "prim.h"

#include <cstring>

#include "reduce.h"

namespace rt {
namespace {

constexpr int kScanItems = 8;                       // items per thread
constexpr int kScanTile = kBlock * kScanItems;      // items per block

// block-wide exclusive scan of one value per thread (Hillis-Steele in LDS)
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* buf, T* total) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    T add = t >= o ? buf[t - o] : T(0);
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  const T incl = buf[t];
  *total = buf[kBlock - 1];
  __syncthreads();
  return incl - v;
}

template <typename In, typename Out>
__global__ void __launch_bounds__(kBlock)
k_scan_reduce(int64_t n, const In* __restrict__ in, Out* __restrict__ sums) {
  __shared__ Out red[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Out s = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += (Out)in[base + k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// exclusive scan of the block sums in one block, chunk by chunk
template <typename Out>
__global__ void __launch_bounds__(kBlock) k_scan_sums(int64_t nb, Out* __restrict__ sums) {
  __shared__ Out buf[kBlock];
  __shared__ Out carry_sh;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += kBlock) {
    const int64_t i = c0 + threadIdx.x;
    const Out v = i < nb ? sums[i] : Out(0);
    Out total;
    const Out ex = block_exclusive_scan(v, buf, &total);
    const Out carry = carry_sh;
    if (i < nb) sums[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry_sh = carry + total;
    __syncthreads();
  }
}

template <typename In, typename Out, bool INCLUSIVE>
__global__ void __launch_bounds__(kBlock)
k_scan_apply(int64_t n, const In* __restrict__ in, const Out* __restrict__ sums,
             Out* __restrict__ out) {
  __shared__ Out buf[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  Out v[kScanItems];
  Out s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? (Out)in[base + k] : Out(0);
    s += v[k];
  }
  Out total;
  Out run = block_exclusive_scan(s, buf, &total) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (INCLUSIVE) run += v[k];
    if (base + k < n) out[base + k] = run;
    if (!INCLUSIVE) run += v[k];
  }
}

__global__ void k_split_flags(int64_t n, int bit, const uint64_t* __restrict__ keys,
                              int32_t* __restrict__ zero) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) zero[i] = ((keys[i] >> bit) & 1) ? 0 : 1;
}

// stable partition by one key bit: zeros keep their order in front, ones after
__global__ void k_split_scatter(int64_t n, int bit, const uint64_t* __restrict__ kin,
                                const int32_t* __restrict__ vin, const int32_t* __restrict__ zero,
                                const int64_t* __restrict__ zpos, uint64_t* __restrict__ kout,
                                int32_t* __restrict__ vout) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t nz = zpos[n - 1] + zero[n - 1];
  const int64_t d = zero[i] ? zpos[i] : nz + (i - zpos[i]);
  kout[d] = kin[i];
  vout[d] = vin[i];
}

template <typename K, typename V>
__global__ void k_row_sort(int64_t nseg, const int64_t* __restrict__ off, K* __restrict__ keys,
                           V* __restrict__ vals) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int64_t a = off[s], b = off[s + 1];
  for (int64_t i = a + 1; i < b; ++i) {
    const K k = keys[i];
    V v{};
    if (vals) v = vals[i];
    int64_t j = i - 1;
    while (j >= a && keys[j] > k) {
      keys[j + 1] = keys[j];
      if (vals) vals[j + 1] = vals[j];
      --j;
    }
    keys[j + 1] = k;
    if (vals) vals[j + 1] = v;
  }
}

// counting sort: bucket sizes, then every item to its bucket's next free slot
__global__ void k_bucket_count(int64_t n, const uint64_t* __restrict__ keys,
                               int32_t* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[keys[i]], 1);
}

__global__ void k_bucket_scatter(int64_t n, const uint64_t* __restrict__ kin,
                                 const int32_t* __restrict__ vin, int32_t* __restrict__ cur,
                                 uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t k = kin[i];
  const int32_t d = atomicAdd(&cur[k], 1);
  kout[d] = k;
  vout[d] = vin[i];
}

__global__ void k_fill_i32(int64_t n, int32_t* __restrict__ p, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_set_last(int64_t* p, int64_t v) { *p = v; }

// per-block maximum of non-negative values (grid-stride)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_max_partial(int64_t n, const T* __restrict__ in, T* __restrict__ part) {
  __shared__ T red[kBlock / kWave];
  T m = 0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    m = in[i] > m ? in[i] : m;
  m = block_max(m, red);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

}  // namespace

template <typename T>
int max_nonneg(rt_ctx* ctx, const T* in, int64_t n, T* out) {
  *out = 0;
  if (n <= 0) return RT_OK;
  const int g = grid_for(n, kBlock, kMaxPartials);
  DevBuf<T> part;
  RT_CHECK(part.reserve(g + 1));
  hipLaunchKernelGGL((k_max_partial<T>), dim3(g), dim3(kBlock), 0, ctx->stream, n, in, part.p);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_max_partial<T>), dim3(1), dim3(kBlock), 0, ctx->stream, (int64_t)g, part.p,
                     part.p + g);
  RT_LAUNCH_CHECK();
  RT_CHECK(ctx->sync_read(part.p + g, sizeof(T)));
  std::memcpy(out, ctx->host, sizeof(T));
  return RT_OK;
}

template int max_nonneg<int64_t>(rt_ctx*, const int64_t*, int64_t, int64_t*);
template int max_nonneg<int32_t>(rt_ctx*, const int32_t*, int64_t, int32_t*);

int bucket_sort_pairs(rt_ctx* ctx, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                      int32_t* vout, int64_t n, int key_bits, bool* done) {
  *done = false;
  if (key_bits > kBucketSortMaxBits || n <= 0 || n >= ((int64_t)1 << 31)) return RT_OK;
  hipStream_t st = ctx->stream;
  const int64_t nb = (int64_t)1 << key_bits;
  DevBuf<int32_t> cnt, cur;
  DevBuf<int64_t> off;
  RT_CHECK(cnt.reserve(nb));
  RT_CHECK(cur.reserve(nb));
  RT_CHECK(off.reserve(nb + 1));
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nb)), dim3(kBlock), 0, st, nb, cnt.p, 0);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bucket_count, dim3(grid_for(n)), dim3(kBlock), 0, st, n, kin, cnt.p);
  RT_LAUNCH_CHECK();
  int32_t maxb = 0;
  RT_CHECK(max_nonneg<int32_t>(ctx, cnt.p, nb, &maxb));
  if (maxb > kBucketSortMaxBucket) return RT_OK;   // long buckets: the split sort does better
  RT_CHECK((scan<int32_t, int32_t>(ctx, cnt.p, cur.p, nb, false)));
  RT_CHECK((scan<int32_t, int64_t>(ctx, cnt.p, off.p, nb, false)));
  hipLaunchKernelGGL(k_bucket_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, n, kin, vin, cur.p,
                     kout, vout);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_set_last, dim3(1), dim3(1), 0, st, off.p + nb, n);
  RT_LAUNCH_CHECK();
  // the scatter order within a bucket is arbitrary: restore the input order
  RT_CHECK((row_sort<int32_t, int32_t>(ctx, off.p, vout, nullptr, nb)));
  RT_CHECK_HIP(hipStreamSynchronize(st));   // the temporaries are freed on return
  *done = true;
  return RT_OK;
}

template <typename In, typename Out>
int scan(rt_ctx* ctx, const In* in, Out* out, int64_t n, bool inclusive) {
  if (n <= 0) return RT_OK;
  hipStream_t st = ctx->stream;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  DevBuf<Out> sums;
  RT_CHECK(sums.reserve(nb));
  hipLaunchKernelGGL((k_scan_reduce<In, Out>), dim3(nb), dim3(kBlock), 0, st, n, in, sums.p);
  hipLaunchKernelGGL((k_scan_sums<Out>), dim3(1), dim3(kBlock), 0, st, nb, sums.p);
  if (inclusive)
    hipLaunchKernelGGL((k_scan_apply<In, Out, true>), dim3(nb), dim3(kBlock), 0, st, n, in, sums.p,
                       out);
  else
    hipLaunchKernelGGL((k_scan_apply<In, Out, false>), dim3(nb), dim3(kBlock), 0, st, n, in,
                       sums.p, out);
  RT_LAUNCH_CHECK();
  // `sums` is released (after a device-wide wait) when this returns
  return RT_OK;
}

template int scan<int64_t, int64_t>(rt_ctx*, const int64_t*, int64_t*, int64_t, bool);
template int scan<int32_t, int64_t>(rt_ctx*, const int32_t*, int64_t*, int64_t, bool);
template int scan<int32_t, int32_t>(rt_ctx*, const int32_t*, int32_t*, int64_t, bool);

int radix_sort_pairs(rt_ctx* ctx, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                     int32_t* vout, int64_t n, int end_bit) {
  hipStream_t st = ctx->stream;
  if (n <= 0) return RT_OK;
  DevBuf<uint64_t> k2;
  DevBuf<int32_t> v2, zero;
  DevBuf<int64_t> zpos;
  RT_CHECK(k2.reserve(n));
  RT_CHECK(v2.reserve(n));
  RT_CHECK(zero.reserve(n));
  RT_CHECK(zpos.reserve(n));
  // ping-pong between (kout, vout) and (k2, v2); the first pass reads the input
  const uint64_t* ksrc = kin;
  const int32_t* vsrc = vin;
  uint64_t* kdst = (end_bit % 2 == 1) ? kout : k2.p;
  int32_t* vdst = (end_bit % 2 == 1) ? vout : v2.p;
  for (int bit = 0; bit < end_bit; ++bit) {
    hipLaunchKernelGGL(k_split_flags, dim3(grid_for(n)), dim3(kBlock), 0, st, n, bit, ksrc,
                       zero.p);
    RT_LAUNCH_CHECK();
    RT_CHECK((scan<int32_t, int64_t>(ctx, zero.p, zpos.p, n, false)));
    hipLaunchKernelGGL(k_split_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, n, bit, ksrc, vsrc,
                       zero.p, zpos.p, kdst, vdst);
    RT_LAUNCH_CHECK();
    ksrc = kdst;
    vsrc = vdst;
    kdst = (kdst == kout) ? k2.p : kout;
    vdst = (vdst == vout) ? v2.p : vout;
  }
  if (end_bit == 0) {
    RT_CHECK_HIP(hipMemcpyAsync(kout, kin, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st));
    RT_CHECK_HIP(hipMemcpyAsync(vout, vin, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  }
  return RT_OK;
}

template <typename K, typename V>
int row_sort(rt_ctx* ctx, const int64_t* off, K* keys, V* vals, int64_t nseg) {
  if (nseg <= 0) return RT_OK;
  hipLaunchKernelGGL((k_row_sort<K, V>), dim3(grid_for(nseg)), dim3(kBlock), 0, ctx->stream, nseg,
                     off, keys, vals);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

template int row_sort<int32_t, double>(rt_ctx*, const int64_t*, int32_t*, double*, int64_t);
template int row_sort<int32_t, int32_t>(rt_ctx*, const int64_t*, int32_t*, int32_t*, int64_t);

}  // namespace rt

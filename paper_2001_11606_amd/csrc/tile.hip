// Tiled form of a CSR level for the LDS-staged sparse products.
//
// Rows are cut into tiles of kTileRows consecutive rows.  For each tile the
// set of distinct columns its entries reference is found with an
// open-addressing hash set in LDS and written out as the tile's column list,
// in slot order; each entry's column is then replaced by its 16-bit position
// in that list.  A product over a tile first loads x[tile_cols] into LDS
// (one read per distinct column instead of one gather per entry) and reads x
// from there.  Since particles are sorted by cell and rows couple only
// neighbouring cells, a tile of 256 rows references about one to two
// thousand distinct columns, in runs of consecutive indices (one run per
// adjacent cell).  The table is 256 buckets of 16 slots: column c probes the
// buckets h(c / 16), h(c / 16) + 1, ... at the in-bucket offset c mod 16, so
// the columns of one aligned block of 16 land in one bucket in ascending
// order, and compaction in slot order keeps every such block contiguous in
// the list -- the staging reads stay coalesced without sorting.  The order
// of a list does not change any product (each entry still reads its own
// column's value); where two columns race for a slot the list order may
// differ between builds, the products do not.  A probe that visits every
// bucket marks the tile as overflowing (the level then stays untiled), so
// insertion ends for any input.  Built once per matrix structure: one pass
// writes each tile's list into room for kTileMaxCols columns and counts it,
// then the lists are packed after a scan of the counts.
#include <climits>
#include <cstring>

#include "internal.h"
#include "prim.h"
#include "reduce.h"

namespace rt {
namespace {

constexpr int kHashBits = 12;
constexpr int kHash = 1 << kHashBits;   // slots; > kTileMaxCols + kBlock, so never full
static_assert(kHash >= kTileMaxCols + kBlock, "hash set must have room for in-flight inserts");
static_assert(kTileRows == kBlock, "one tile per block, one row per thread");
static_assert(kTileMaxCols <= 65536, "positions in a tile's list are 16-bit");

constexpr int kBucket = 16;                   // slots per bucket = columns per block
constexpr int kBuckets = kHash / kBucket;

// first bucket probed by column c
__device__ __forceinline__ int first_bucket(int32_t c) {
  return (int)((((uint32_t)c >> 4) * 2654435761u) >> 24) & (kBuckets - 1);
}

// Insert column c into keys (empty = -1); *count is the number of distinct
// columns inserted; *overflow is set once it reaches kTileMaxCols or a probe
// finds no free slot.
__device__ __forceinline__ void tile_insert_one(int c, int* keys, int* count, int* overflow) {
  const int off = c & (kBucket - 1);
  int b = first_bucket(c);
  bool placed = false;
  for (int step = 0; step < kBuckets && !placed; ++step, b = (b + 1) & (kBuckets - 1)) {
    const int s = b * kBucket + off;
    const int cur = ((volatile int*)keys)[s];
    if (cur == c) {
      placed = true;
    } else if (cur == -1) {
      const int prev = atomicCAS(&keys[s], -1, c);
      if (prev == -1) {
        if (atomicAdd(count, 1) + 1 >= kTileMaxCols) *(volatile int*)overflow = 1;
        placed = true;
      } else if (prev == c) {
        placed = true;
      }
    }
  }
  if (!placed) *(volatile int*)overflow = 1;
}

// Insert the columns of entries [e0, e1) (insertion stops at an overflow).
// A thread requests kTileBatch columns, one per block-wide stride, before it
// hashes any of them: a tile's entries are then read in a few round trips
// to memory rather than one per entry.
constexpr int kTileBatch = 8;

__device__ void tile_insert(int64_t e0, int64_t e1, const int32_t* __restrict__ col, int* keys,
                            int* count, int* overflow) {
  for (int64_t kb = e0 + threadIdx.x; kb < e1; kb += (int64_t)kBlock * kTileBatch) {
    if (*(volatile int*)overflow) break;
    int c[kTileBatch];
#pragma unroll
    for (int e = 0; e < kTileBatch; ++e) {
      const int64_t k = kb + (int64_t)e * kBlock;
      c[e] = k < e1 ? col[k] : -1;   // columns are >= 0
    }
#pragma unroll
    for (int e = 0; e < kTileBatch; ++e)
      if (c[e] >= 0) tile_insert_one(c[e], keys, count, overflow);
  }
}

// slot of a column that was inserted
__device__ __forceinline__ int tile_find(const int* keys, int c) {
  const int off = c & (kBucket - 1);
  int b = first_bucket(c);
  while (keys[b * kBucket + off] != c) b = (b + 1) & (kBuckets - 1);
  return b * kBucket + off;
}

__device__ __forceinline__ void tile_rows(int64_t n, int64_t t, const int64_t* rp, int64_t* e0,
                                          int64_t* e1) {
  const int64_t r0 = t * kTileRows;
  const int64_t r1 = r0 + kTileRows < n ? r0 + kTileRows : n;
  *e0 = rp[r0];
  *e1 = rp[r1];
}

// Distinct columns of every tile in slot order, into a padded list (tile t
// at t * kTileMaxCols), their number, and each entry's position among them.
// A tile that overflows writes count 0 and sets *flag; its entries are left.
__global__ void __launch_bounds__(kBlock)
k_tile_fill(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
            int32_t* __restrict__ tpad, int64_t* __restrict__ cnt, uint16_t* __restrict__ lcol,
            int* __restrict__ flag) {
  constexpr int PER = kHash / kBlock;   // consecutive slots per thread
  __shared__ int keys[kHash];
  __shared__ uint16_t pos[kHash];   // positions < kTileMaxCols: 16 bits, so six blocks fit a CU
  __shared__ int wsum[kBlock / kWave];
  __shared__ int count, overflow;
  for (int s = threadIdx.x; s < kHash; s += kBlock) keys[s] = -1;
  if (threadIdx.x == 0) {
    count = 0;
    overflow = 0;
  }
  __syncthreads();
  int64_t e0, e1;
  tile_rows(n, blockIdx.x, rp, &e0, &e1);
  tile_insert(e0, e1, col, keys, &count, &overflow);
  __syncthreads();
  if (overflow) {   // uniform over the block
    if (threadIdx.x == 0) {
      cnt[blockIdx.x] = 0;
      flag[0] = 1;
    }
    return;
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = count;
  // positions = exclusive prefix count of occupied slots (block scan)
  const int s0 = threadIdx.x * PER;
  int own = 0;
  for (int q = 0; q < PER; ++q) own += keys[s0 + q] != -1;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int incl = own;
  for (int o = 1; o < kWave; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int base = incl - own;
  for (int q = 0; q < w; ++q) base += wsum[q];
  int32_t* out = tpad + (int64_t)blockIdx.x * kTileMaxCols;
  for (int q = 0; q < PER; ++q) {
    const int c = keys[s0 + q];
    if (c != -1) {
      pos[s0 + q] = base;
      out[base] = c;   // base < count < kTileMaxCols (no overflow)
      ++base;
    }
  }
  __syncthreads();
  for (int64_t kb = e0 + threadIdx.x; kb < e1; kb += (int64_t)kBlock * kTileBatch) {
    int c[kTileBatch];
#pragma unroll
    for (int e = 0; e < kTileBatch; ++e) {
      const int64_t k = kb + (int64_t)e * kBlock;
      c[e] = k < e1 ? col[k] : -1;
    }
#pragma unroll
    for (int e = 0; e < kTileBatch; ++e)
      if (c[e] >= 0) lcol[kb + (int64_t)e * kBlock] = (uint16_t)pos[tile_find(keys, c[e])];
  }
}

// padded lists -> contiguous tile_cols (tile t at off[t])
__global__ void __launch_bounds__(kBlock)
k_tile_compact(const int32_t* __restrict__ tpad, const int64_t* __restrict__ off,
               int32_t* __restrict__ tcols) {
  const int64_t o = off[blockIdx.x];
  const int c = (int)(off[blockIdx.x + 1] - o);
  const int32_t* in = tpad + (int64_t)blockIdx.x * kTileMaxCols;
  for (int k = threadIdx.x; k < c; k += kBlock) tcols[o + k] = in[k];
}

}  // namespace

int build_tiles(rt_ctx* ctx, Level& L) {
  hipStream_t st = ctx->stream;
  L.tiled = false;
  L.ntiles = 0;
  L.tile_cols_total = 0;
  L.max_tile_cols = 0;
  const int64_t n = L.n;
  if (n == 0) return RT_OK;
  const int64_t nt = (n + kTileRows - 1) / kTileRows;
  if (nt > INT_MAX) return RT_OK;
  DevBuf<int64_t> cnt;
  DevBuf<int> flag;
  DevBuf<int32_t> tpad;   // kTileMaxCols columns of room per tile
  RT_CHECK(cnt.reserve(nt + 1));
  RT_CHECK(flag.reserve(1));
  RT_CHECK(tpad.reserve((size_t)nt * kTileMaxCols));
  RT_CHECK(L.lcol.reserve(L.nnz + kSpmvPad));
  RT_CHECK_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
  RT_CHECK_HIP(hipMemsetAsync(cnt.p + nt, 0, sizeof(int64_t), st));
  RT_CHECK_HIP(hipMemsetAsync(L.lcol.p + L.nnz, 0, sizeof(uint16_t) * kSpmvPad, st));
  hipLaunchKernelGGL(k_tile_fill, dim3((unsigned)nt), dim3(kBlock), 0, st, n, L.rp.p, L.col.p,
                     tpad.p, cnt.p, L.lcol.p, flag.p);
  RT_LAUNCH_CHECK();
  RT_CHECK(ctx->sync_read(flag.p, sizeof(int)));
  int overflow = 0;
  std::memcpy(&overflow, ctx->host, sizeof(int));
  if (overflow) return RT_OK;   // lcol is unused by untiled products
  int64_t maxc = 0;
  RT_CHECK(max_nonneg<int64_t>(ctx, cnt.p, nt, &maxc));
  RT_CHECK(L.tile_off.reserve(nt + 1));
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, L.tile_off.p, nt + 1, false)));
  RT_CHECK(ctx->sync_read(L.tile_off.p + nt, sizeof(int64_t)));
  int64_t total = 0;
  std::memcpy(&total, ctx->host, sizeof(int64_t));
  RT_CHECK(L.tile_cols.reserve(total));
  hipLaunchKernelGGL(k_tile_compact, dim3((unsigned)nt), dim3(kBlock), 0, st, tpad.p,
                     L.tile_off.p, L.tile_cols.p);
  RT_LAUNCH_CHECK();
  L.tiled = true;
  L.ntiles = nt;
  L.tile_cols_total = total;
  L.max_tile_cols = (int)maxc;
  return RT_OK;
}

}  // namespace rt

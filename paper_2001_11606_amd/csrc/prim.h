// Device primitives of the set-up paths (see prim.hip).
#pragma once

#include "internal.h"

namespace rt {

// out[i] = sum of in[0..i) (exclusive) or in[0..i] (inclusive), n items.
template <typename In, typename Out>
int scan(rt_ctx* ctx, const In* in, Out* out, int64_t n, bool inclusive);

// *out = max(0, in[0..n)) on the host (synchronises the stream).
template <typename T>
int max_nonneg(rt_ctx* ctx, const T* in, int64_t n, T* out);

// Stable sort of (key, value) pairs by key for keys below 2^key_bits whose
// values are the items' input positions in ascending order (so sorting a
// bucket by value restores input order): counting sort.  *done = false (and
// nothing written) when key_bits exceeds kBucketSortMaxBits or a bucket holds
// more than kBucketSortMaxBucket items; the caller then uses radix_sort_pairs.
constexpr int kBucketSortMaxBits = 24;
constexpr int kBucketSortMaxBucket = 1024;
int bucket_sort_pairs(rt_ctx* ctx, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                      int32_t* vout, int64_t n, int key_bits, bool* done);

// Stable sort of (key, value) pairs by the low end_bit bits of the key.
int radix_sort_pairs(rt_ctx* ctx, const uint64_t* kin, uint64_t* kout, const int32_t* vin,
                     int32_t* vout, int64_t n, int end_bit);

// In-place ascending sort of every row [off[s], off[s+1]) of keys (and the
// matching vals, if not NULL); meant for short rows.
template <typename K, typename V>
int row_sort(rt_ctx* ctx, const int64_t* off, K* keys, V* vals, int64_t nseg);

}  // namespace rt

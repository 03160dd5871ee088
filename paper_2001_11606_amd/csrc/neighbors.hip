// Cell-list neighbour search over cell-sorted particles (gfx950).
//
// 1. bounding box and largest smoothing length (block reduction);
// 2. uniform grid of cells no smaller than the largest support;
// 3. stable radix sort of (key, user index) with key = ghost flag above the
//    Morton code of the cell: interior particles first, cells in Morton order
//    (spatially compact runs of rows for every later gather, and 2^dim-aligned
//    blocks of cells contiguous at every level of the aggregation hierarchy);
//    gather sorted positions and smoothing lengths (SoA);
// 4. table of [start, end) per (flag, row-major cell index);
// 5. list of occupied cells (runs of equal keys);
// 6. count pass, scan, fill pass: one block per occupied cell stages the
//    candidates of the 3^dim adjacent cells (interior cells first, then ghost
//    cells; cells in z, y, x order; ascending index within a cell) in LDS,
//    and each wave tests one row of the cell against 64 candidates at a time,
//    compacting the hits with a ballot so that a row's neighbours are written
//    as contiguous runs.  The candidate order makes the interior neighbours of
//    every row a prefix of the row.
//
// The predicate r^2 < (kappa * max(h_i, h_j))^2 is evaluated in FP64 with
// r^2 accumulated in axis order and contraction to FMA disabled, so that it
// decides exactly as a separately-rounded evaluation does.
//
// Periodic axes (the periodic box of the manufactured problem of Sec. 4.3):
// the grid covers [0, L) with a whole number (at least 3) of cells no smaller
// than the largest support, adjacent-cell offsets wrap around, and every
// displacement is reduced to its nearest image before it is squared.  With
// the period at least three supports long, this yields the pairs that copies
// of the boundary points placed across the boundary would (Sec. 3.1), with
// each pair coupled to the node itself.
#include <cmath>
#include <cstring>
#include <algorithm>

#include "internal.h"
#include "prim.h"
#include "reduce.h"

#pragma clang fp contract(off)

namespace rt {
namespace {

template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_bbox(int64_t n, const double* __restrict__ pos, const double* __restrict__ h,
       double* __restrict__ part) {
  __shared__ double red[8][kBlock];
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double hmax = 0.0, bad = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double x = pos[a * n + i];
      if (!isfinite(x)) {
        bad += 1.0;
      } else {
        lo[a] = fmin(lo[a], x);
        hi[a] = fmax(hi[a], x);
      }
    }
    const double hh = h[i];
    if (!(hh > 0.0) || !isfinite(hh)) bad += 1.0;
    else hmax = fmax(hmax, hh);
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    red[a][t] = lo[a];
    red[3 + a][t] = hi[a];
  }
  red[6][t] = hmax;
  red[7][t] = bad;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        red[a][t] = fmin(red[a][t], red[a][t + s]);
        red[3 + a][t] = fmax(red[3 + a][t], red[3 + a][t + s]);
      }
      red[6][t] = fmax(red[6][t], red[6][t + s]);
      red[7][t] = red[7][t] + red[7][t + s];
    }
    __syncthreads();
  }
  if (t < 8) part[blockIdx.x * 8 + t] = red[t][0];
}

template <int DIM>
__device__ __forceinline__ uint64_t morton(int bits, const int* c) {
  uint64_t code = 0;
  for (int b = 0; b < bits; ++b)
#pragma unroll
    for (int a = 0; a < DIM; ++a) code |= (uint64_t)((c[a] >> b) & 1) << (DIM * b + a);
  return code;
}

template <int DIM>
__device__ __forceinline__ void demorton(int bits, uint64_t code, int* c) {
  c[0] = c[1] = c[2] = 0;
  for (int b = 0; b < bits; ++b)
#pragma unroll
    for (int a = 0; a < DIM; ++a) c[a] |= (int)((code >> (DIM * b + a)) & 1) << b;
}

template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_keys(int bits, int64_t n, int64_t nin, const double* __restrict__ pos, double lo0, double lo1,
       double lo2, double cs0, double cs1, double cs2, int nc0, int nc1, int nc2,
       uint64_t* __restrict__ keys, int32_t* __restrict__ ids) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {lo0, lo1, lo2};
  const double cs[3] = {cs0, cs1, cs2};
  const int nc[3] = {nc0, nc1, nc2};
  int c[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    const double q = floor((pos[a * n + i] - lo[a]) / cs[a]);
    int ci = (int)q;
    ci = ci < 0 ? 0 : (ci >= nc[a] ? nc[a] - 1 : ci);
    c[a] = ci;
  }
  const uint64_t flag = i >= nin ? 1 : 0;
  keys[i] = (flag << (DIM * bits)) | morton<DIM>(bits, c);
  ids[i] = (int32_t)i;
}

// (x, y, z, h) of every particle in user order, read coalesced from the
// caller's arrays into one 32-byte record each (z = 0 in 2-D).
__global__ void k_pack_pos(int dim, int64_t n, const double* __restrict__ pos,
                           const double* __restrict__ h, double* __restrict__ rec) {
  int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  rt_f64x2_t* out = reinterpret_cast<rt_f64x2_t*>(rec + 4 * u);
  out[0] = rt_f64x2_t{pos[u], pos[n + u]};
  out[1] = rt_f64x2_t{dim == 3 ? pos[2 * n + u] : 0.0, h[u]};
}

// Sorted records: one gathered per particle; iperm = inverse of perm.
__global__ void k_gather_sorted(int64_t n, const int32_t* __restrict__ perm,
                                const double* __restrict__ rec, double* __restrict__ sp4,
                                int32_t* __restrict__ iperm) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t u = perm[s];
  const Rec4 q = load_rec4(rec, u);
  rt_f64x2_t* o = reinterpret_cast<rt_f64x2_t*>(sp4 + 4 * s);
  o[0] = rt_f64x2_t{q.x, q.y};
  o[1] = rt_f64x2_t{q.z, q.h};
  iperm[u] = (int32_t)s;
}

// Range table: start/end of the sorted particles of every (flag, row-major cell).
template <int DIM>
__global__ void __launch_bounds__(kBlock)
k_cell_table(int bits, int64_t n, int nc0, int nc1, int64_t ncells,
             const uint64_t* __restrict__ skeys, int32_t* __restrict__ cstart,
             int32_t* __restrict__ cend) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint64_t key = skeys[s];
  const bool first = s == 0 || skeys[s - 1] != key;
  const bool last = s == n - 1 || skeys[s + 1] != key;
  if (!first && !last) return;
  const uint64_t mask = ((uint64_t)1 << (DIM * bits)) - 1;
  int c[3];
  demorton<DIM>(bits, key & mask, c);
  const int64_t flag = (int64_t)(key >> (DIM * bits));
  const int64_t t = flag * ncells + ((int64_t)c[2] * nc1 + c[1]) * nc0 + c[0];
  if (first) cstart[t] = (int32_t)s;
  if (last) cend[t] = (int32_t)(s + 1);
}

// first sorted position of every run of equal keys; runs[nruns] = n
__global__ void k_run_flags(int64_t n, const uint64_t* __restrict__ skeys,
                            int32_t* __restrict__ flags) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < n) flags[s] = (s == 0 || skeys[s] != skeys[s - 1]) ? 1 : 0;
}

__global__ void k_run_starts(int64_t n, const int32_t* __restrict__ flags,
                             const int32_t* __restrict__ rid, const uint64_t* __restrict__ skeys,
                             int32_t* __restrict__ runs, uint64_t* __restrict__ runkey) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (flags[s]) {
    runs[rid[s] - 1] = (int32_t)s;
    runkey[rid[s] - 1] = skeys[s];
  }
  if (s == n - 1) runs[rid[s]] = (int32_t)n;
}

constexpr int kNbrCand = 512;   // candidates staged in LDS per pass
constexpr int kNbrRows = 512;   // rows of one cell handled per pass
constexpr int kCountRows = 8;   // count pass: rows tested against a wave's candidates in turn
constexpr double kNbrMaskBytes = 4.0e9;   // largest hit-mask buffer kept between the passes

// Adjacent cell x + o on an axis of nc cells: wraps on a periodic axis
// (nc >= 3, so the three offsets reach three distinct cells), else false
// outside the grid.
__device__ __forceinline__ bool adjacent(int& x, int nc, bool periodic) {
  if (x < 0) {
    if (!periodic) return false;
    x += nc;
  } else if (x >= nc) {
    if (!periodic) return false;
    x -= nc;
  }
  return true;
}

// Component a of a displacement; PER: nearest image on the box's periodic axes.
template <bool PER>
__device__ __forceinline__ double axis_disp(double d, const PeriodicBox& box, int a) {
  return PER ? periodic_disp(d, box, a) : d;
}

// Candidates of a cell: the particle count of its 2 * 3^DIM adjacent-cell slots.
template <int DIM>
__global__ void k_cell_candidates(int64_t nruns, int bits, int64_t ncells, int nc0, int nc1,
                                  int nc2, int pmask, const int32_t* __restrict__ runs,
                                  const uint64_t* __restrict__ skeys,
                                  const int32_t* __restrict__ cstart,
                                  const int32_t* __restrict__ cend, int32_t* __restrict__ m) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nruns) return;
  const uint64_t mask = ((uint64_t)1 << (DIM * bits)) - 1;
  int c[3];
  demorton<DIM>(bits, skeys[runs[q]] & mask, c);
  int32_t total = 0;
  for (int flag = 0; flag < 2; ++flag)
    for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int x = c[0] + ox, y = c[1] + oy, z = c[2] + oz;
          if (!adjacent(x, nc0, pmask & 1) || !adjacent(y, nc1, pmask & 2) ||
              !adjacent(z, nc2, pmask & 4))
            continue;
          const int64_t cell = flag * ncells + ((int64_t)z * nc1 + y) * nc0 + x;
          total += cend[cell] - cstart[cell];
        }
  m[q] = total;
}

// FILL = false: count neighbours per row and, when masks is not NULL, store
// every 64-candidate hit mask (row s, candidate chunk q at masks[s*mstride+q]).
// FILL = true, FROM_MASK = true: write the lists from those masks (no distance
// tests, no staged positions); FROM_MASK = false: test the pairs again.
template <int DIM, bool FILL, bool FROM_MASK, bool PER>
__global__ void __launch_bounds__(kBlock)
k_nbr_cells(int64_t n, int64_t nin, int bits, int64_t ncells, int nc0, int nc1, int nc2,
            PeriodicBox box, double kappa, const int32_t* __restrict__ runs, const uint64_t* __restrict__ runkey,
            const double* __restrict__ sp4, const int32_t* __restrict__ cstart,
            const int32_t* __restrict__ cend,
            int64_t* __restrict__ cnt, const int64_t* __restrict__ ptr, int32_t* __restrict__ idx,
            int32_t* __restrict__ n_int_nbrs, uint64_t* __restrict__ masks, int mstride) {
  constexpr int NB = DIM == 3 ? 27 : 9;   // adjacent cells per flag
  // candidates' positions and squared support radii (kappa h)^2
  __shared__ double cx[kNbrCand], cy[kNbrCand], cz[kNbrCand], ch[kNbrCand];
  __shared__ int32_t ct[kNbrCand];
  __shared__ int32_t rlo[2 * NB], roff[2 * NB + 1];
  __shared__ int32_t rcount[kNbrRows], rint[kNbrRows];
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid & (kWave - 1);
  const int64_t r0 = runs[blockIdx.x], r1 = runs[blockIdx.x + 1];
  // candidate ranges: slot = flag * NB + (z, y, x offset), empty when outside the grid
  static_assert(2 * NB <= kWave, "the slot scan runs in one wave");
  if (tid < kWave) {   // wave 0: slot ranges and their prefix sum
    const uint64_t key = runkey[blockIdx.x];
    const uint64_t mask = ((uint64_t)1 << (DIM * bits)) - 1;
    int c[3];
    demorton<DIM>(bits, key & mask, c);
    const int flag = tid / NB, o = tid % NB;
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
    int x = c[0] + ox, y = c[1] + oy, z = c[2] + oz;
    int32_t lo = 0, len = 0;
    if (tid < 2 * NB && adjacent(x, nc0, box.mask & 1) && adjacent(y, nc1, box.mask & 2) &&
        adjacent(z, nc2, box.mask & 4)) {
      const int64_t cell = flag * ncells + ((int64_t)z * nc1 + y) * nc0 + x;
      lo = cstart[cell];
      len = cend[cell] - lo;
    }
    int32_t incl = len;
    for (int d = 1; d < kWave; d <<= 1) {
      const int32_t v = __shfl_up(incl, d);
      if (tid >= d) incl += v;
    }
    if (tid < 2 * NB) {
      rlo[tid] = lo;
      roff[tid + 1] = incl;
    }
    if (tid == 0) roff[0] = 0;
  }
  __syncthreads();
  const int m = roff[2 * NB];
  for (int64_t rb = r0; rb < r1; rb += kNbrRows) {
    const int nrows = (int)(r1 - rb < kNbrRows ? r1 - rb : kNbrRows);
    for (int r = tid; r < nrows; r += kBlock) {
      rcount[r] = 0;
      rint[r] = 0;
    }
    for (int c0 = 0; c0 < m; c0 += kNbrCand) {
      const int mc = m - c0 < kNbrCand ? m - c0 : kNbrCand;
      __syncthreads();   // the previous chunk is consumed, row counters are set
      for (int k = tid; k < mc; k += kBlock) {
        const int kk = c0 + k;
        int lo = 0, hi = 2 * NB;   // roff[lo] <= kk < roff[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (roff[mid] <= kk) lo = mid;
          else hi = mid;
        }
        const int32_t t = rlo[lo] + (kk - roff[lo]);
        ct[k] = t;
        if (!FROM_MASK) {
          const Rec4 q = load_rec4(sp4, t);
          cx[k] = q.x;
          cy[k] = q.y;
          cz[k] = q.z;
          const double kq = kappa * q.h;
          ch[k] = kq * kq;
        }
      }
      __syncthreads();
      // the block's own cell is the centre slot of its flag: its rows are candidates too
      const int cslot = (r0 >= nin ? NB : 0) + NB / 2;
      if (!FILL && !FROM_MASK) {
        // Count pass: a wave holds one word of 64 candidates in registers and
        // tests up to kCountRows rows against it, the row read by all lanes
        // at once; work items are (candidate word, row group) pairs.
        const int nwords = RT_UNIFORM((mc + kWave - 1) / kWave);
        const int ngroups = RT_UNIFORM((nrows + kCountRows - 1) / kCountRows);
        // item = g * nwords + w, stepped by the wave count without dividing
        // (mc >= 1 inside the chunk loop, so nwords >= 1)
        int w = wave, g = nwords > 0 ? 0 : ngroups;
        while (g < ngroups && w >= nwords) {
          w -= nwords;
          ++g;
        }
        for (; g < ngroups; w += kBlock / kWave) {
          while (w >= nwords) {
            w -= nwords;
            ++g;
          }
          if (g >= ngroups) break;
          const int k = w * kWave + lane;
          // The pair test r^2 < (kappa max(h_i, h_j))^2 as max((kappa h_i)^2,
          // (kappa h_j)^2): rounding is monotone, so both give the same bits;
          // each squared radius is formed once, when its particle is staged.
          // An empty lane has NaN coordinates: its r^2 never tests true.
          double qx = __builtin_nan(""), qy = qx, qz = qx, tq = 0.0;
          if (k < mc) {
            qx = cx[k];
            qy = cy[k];
            qz = cz[k];
            tq = ch[k];
          }
          const int ra = g * kCountRows;
          const int nr = RT_UNIFORM(nrows - ra < kCountRows ? nrows - ra : kCountRows);
          const int32_t s0 = (int32_t)(rb + ra);   // particle indices fit in int32
          const int ks0 = RT_UNIFORM(roff[cslot] + (s0 - rlo[cslot]) - c0);
          const bool staged = ks0 >= 0 && ks0 + nr <= mc;   // the rows are candidates here
          unsigned long long mine = 0ull;   // lane r keeps the mask word of row ra + r
          for (int r = 0; r < nr; ++r) {
            const int32_t s = s0 + r;
            double xi, yi, zi, ti;
            if (staged) {
              xi = cx[ks0 + r];
              yi = cy[ks0 + r];
              zi = cz[ks0 + r];
              ti = ch[ks0 + r];
            } else {
              const Rec4 q = load_rec4(sp4, s);
              xi = q.x;
              yi = q.y;
              zi = q.z;
              const double ki = kappa * q.h;
              ti = ki * ki;
            }
            double d = axis_disp<PER>(xi - qx, box, 0);
            double r2 = d * d;
            d = axis_disp<PER>(yi - qy, box, 1);
            r2 = r2 + d * d;
            if (DIM == 3) {
              d = axis_disp<PER>(zi - qz, box, 2);
              r2 = r2 + d * d;
            }
            const double th2 = fmax(ti, tq);
            unsigned long long bm = __ballot(r2 < th2);
            // the row itself is candidate ks0 + r of the chunk (its own cell's
            // slot): its bit is cleared here rather than tested in every lane
            const int kself = RT_UNIFORM(ks0 + r - w * kWave);
            if (kself >= 0 && kself < kWave) bm &= ~(1ull << kself);
            if (lane == r) mine = bm;
          }
          if (lane < nr) {
            if (masks) masks[(int64_t)(s0 + lane) * mstride + c0 / kWave + w] = mine;
            atomicAdd(&rcount[ra + lane], (int)__popcll(mine));
          }
        }
        continue;   // next chunk of candidates
      }
      for (int r = wave; r < nrows; r += kBlock / kWave) {
        const int64_t s = rb + r;
        const int ks = roff[cslot] + (int)(s - rlo[cslot]) - c0;
        double xi = 0.0, yi = 0.0, zi = 0.0, ti = 0.0;
        if (FROM_MASK) {
          // positions are not needed
        } else if (ks >= 0 && ks < mc) {
          xi = cx[ks];
          yi = cy[ks];
          zi = cz[ks];
          ti = ch[ks];
        } else {
          const Rec4 q = load_rec4(sp4, s);
          xi = q.x;
          yi = q.y;
          zi = q.z;
          const double ki = kappa * q.h;
          ti = ki * ki;
        }
        int found = 0, fint = 0;
        int64_t out = FILL ? ptr[s] + rcount[r] : 0;
        for (int k = lane; k - lane < mc; k += kWave) {
          bool hit = false;
          int32_t t = -1;
          if (FROM_MASK) {
            const uint64_t mk = masks[s * mstride + (c0 + k - lane) / kWave];
            if (k < mc) {
              t = ct[k];
              hit = (mk >> lane) & 1ull;
            }
          } else if (k < mc) {
            t = ct[k];
            if (t != s) {
              double d = axis_disp<PER>(xi - cx[k], box, 0);
              double r2 = d * d;
              d = axis_disp<PER>(yi - cy[k], box, 1);
              r2 = r2 + d * d;
              if (DIM == 3) {
                d = axis_disp<PER>(zi - cz[k], box, 2);
                r2 = r2 + d * d;
              }
              hit = r2 < fmax(ti, ch[k]);   // the count pass's test, bit for bit
            }
          }
          const unsigned long long bm = __ballot(hit);
          const unsigned long long bi = __ballot(hit && t < nin);
          if (!FILL && masks && lane == 0) masks[s * mstride + (c0 + k) / kWave] = bm;
          if (FILL && hit) {
            const unsigned long long below = lane ? (bm & (~0ull >> (kWave - lane))) : 0ull;
            idx[out + __popcll(below)] = t;
          }
          out += __popcll(bm);
          found += __popcll(bm);
          fint += __popcll(bi);
        }
        if (lane == 0) {
          rcount[r] += found;
          rint[r] += fint;
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < nrows; r += kBlock) {
      if (!FILL) cnt[rb + r] = rcount[r];
      else n_int_nbrs[rb + r] = rint[r];
    }
    __syncthreads();
  }
}

// Fill pass from the count pass's hit masks, for cells whose candidates span
// at most kMaskWords mask words per staged chunk: each lane expands one mask
// word of one row (kMaskWords lanes per row, 64 / kMaskWords rows per wave at a
// time), so the work follows the hits, not the candidates.
constexpr int kMaskWords = kNbrCand / kWave;   // mask words per staged chunk (8)
#ifndef RT_FILL_BLOCK
#define RT_FILL_BLOCK 128
#endif
// threads per block of the fill pass: a cell holds about 15 rows in 3-D, 8 rows
// per wave step, so two waves are all a block's rows keep busy
constexpr int kFillBlock = RT_FILL_BLOCK;

template <int DIM>
__global__ void __launch_bounds__(kFillBlock)
k_nbr_fill_masks(int64_t n, int64_t nin, int bits, int64_t ncells, int nc0, int nc1, int nc2,
                 PeriodicBox box, const int32_t* __restrict__ runs, const uint64_t* __restrict__ runkey,
                 const int32_t* __restrict__ cstart, const int32_t* __restrict__ cend,
                 const int64_t* __restrict__ ptr, int32_t* __restrict__ idx,
                 int32_t* __restrict__ n_int_nbrs, const uint64_t* __restrict__ masks,
                 int mstride) {
  constexpr int NB = DIM == 3 ? 27 : 9;
  constexpr int RPW = kWave / kMaskWords;   // rows per wave per step
  __shared__ int32_t ct[kNbrCand];
  __shared__ int32_t rlo[2 * NB], roff[2 * NB + 1];
  __shared__ int32_t rcount[kNbrRows], rint[kNbrRows];
  const int tid = threadIdx.x;
  const int wave = tid / kWave, lane = tid & (kWave - 1);
  const int64_t r0 = runs[blockIdx.x], r1 = runs[blockIdx.x + 1];
  static_assert(2 * NB <= kWave, "the slot scan runs in one wave");
  if (tid < kWave) {
    const uint64_t key = runkey[blockIdx.x];
    const uint64_t mask = ((uint64_t)1 << (DIM * bits)) - 1;
    int c[3];
    demorton<DIM>(bits, key & mask, c);
    const int flag = tid / NB, o = tid % NB;
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = DIM == 3 ? o / 9 - 1 : 0;
    int x = c[0] + ox, y = c[1] + oy, z = c[2] + oz;
    int32_t lo = 0, len = 0;
    if (tid < 2 * NB && adjacent(x, nc0, box.mask & 1) && adjacent(y, nc1, box.mask & 2) &&
        adjacent(z, nc2, box.mask & 4)) {
      const int64_t cell = flag * ncells + ((int64_t)z * nc1 + y) * nc0 + x;
      lo = cstart[cell];
      len = cend[cell] - lo;
    }
    int32_t incl = len;
    for (int d = 1; d < kWave; d <<= 1) {
      const int32_t v = __shfl_up(incl, d);
      if (tid >= d) incl += v;
    }
    if (tid < 2 * NB) {
      rlo[tid] = lo;
      roff[tid + 1] = incl;
    }
    if (tid == 0) roff[0] = 0;
  }
  __syncthreads();
  const int m = roff[2 * NB];
  const int rr = lane / kMaskWords, q = lane % kMaskWords;
  for (int64_t rb = r0; rb < r1; rb += kNbrRows) {
    const int nrows = (int)(r1 - rb < kNbrRows ? r1 - rb : kNbrRows);
    for (int r = tid; r < nrows; r += kFillBlock) {
      rcount[r] = 0;
      rint[r] = 0;
    }
    for (int c0 = 0; c0 < m; c0 += kNbrCand) {
      const int mc = m - c0 < kNbrCand ? m - c0 : kNbrCand;
      __syncthreads();
      for (int k = tid; k < mc; k += kFillBlock) {
        const int kk = c0 + k;
        int lo = 0, hi = 2 * NB;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (roff[mid] <= kk) lo = mid;
          else hi = mid;
        }
        ct[k] = rlo[lo] + (kk - roff[lo]);
      }
      __syncthreads();
      const int words = (mc + kWave - 1) / kWave;
      for (int base = wave * RPW; base < nrows; base += (kFillBlock / kWave) * RPW) {
        const int r = base + rr;
        const bool live = r < nrows && q < words;
        const int64_t s = rb + r;
        const uint64_t mk = live ? masks[s * mstride + c0 / kWave + q] : 0ull;
        const int cntw = __popcll(mk);
        int incl = cntw;   // prefix over the words of this row
        for (int d = 1; d < kMaskWords; d <<= 1) {
          const int v = __shfl_up(incl, d, kMaskWords);
          if (q >= d) incl += v;
        }
        int interior = 0;
        if (live && mk) {
          int64_t out = ptr[s] + rcount[r] + (incl - cntw);
          uint64_t bitsleft = mk;
          while (bitsleft) {
            const int b = __builtin_ctzll(bitsleft);
            bitsleft &= bitsleft - 1;
            const int32_t t = ct[q * kWave + b];
            idx[out++] = t;
            interior += t < nin;
          }
        }
        for (int d = kMaskWords / 2; d > 0; d >>= 1) interior += __shfl_xor(interior, d, kMaskWords);
        const int total = __shfl(incl, kMaskWords - 1, kMaskWords);
        // rows belong to one wave per chunk, and the reads above precede this
        // write in the wave's instruction stream
        if (q == 0 && r < nrows) {
          rcount[r] += total;
          rint[r] += interior;
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < nrows; r += kFillBlock) n_int_nbrs[rb + r] = rint[r];
    __syncthreads();
  }
}

// user-order export: scatter mapped rows, then sort each row
__global__ void k_user_counts(int64_t n, const int32_t* __restrict__ iperm,
                              const int64_t* __restrict__ ptr, int64_t* __restrict__ ucnt) {
  int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  int32_t s = iperm[u];
  ucnt[u] = ptr[s + 1] - ptr[s];
}

__global__ void k_user_scatter(int64_t n, const int32_t* __restrict__ perm,
                               const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                               const int64_t* __restrict__ uptr, int32_t* __restrict__ uidx) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  int64_t o = uptr[perm[s]];
  for (int64_t k = ptr[s]; k < ptr[s + 1]; ++k) uidx[o++] = perm[idx[k]];
}

}  // namespace

int build_neighbors(rt_ctx* ctx, int dim, int64_t n, int64_t nin, const double* pos,
                    const double* h, int kernel, const double* period, rt_neighbors* nb) {
  hipStream_t st = ctx->stream;
  nb->dim = dim;
  nb->kernel = kernel;
  nb->kappa = kernel == RT_KERNEL_CUBIC_SPLINE ? 2.0 : 1.0;
  nb->n_total = n;
  nb->n_interior = nin;
  PeriodicBox box{{0.0, 0.0, 0.0}, 0};
  for (int a = 0; period && a < dim; ++a) {
    if (period[a] == 0.0) continue;
    if (!(period[a] > 0.0) || !std::isfinite(period[a])) {
      set_error("rt_build_neighbors: period %g along axis %d is not a positive finite length",
                period[a], a);
      return RT_E_ARG;
    }
    box.len[a] = period[a];
    box.mask |= 1 << a;
  }
  nb->box = box;

  // 1. bounding box
  int gb = grid_for(n, kBlock, 1024);
  DevBuf<double> part;
  RT_CHECK(part.reserve((size_t)gb * 8));
  if (dim == 3) hipLaunchKernelGGL(k_bbox<3>, dim3(gb), dim3(kBlock), 0, st, n, pos, h, part.p);
  else hipLaunchKernelGGL(k_bbox<2>, dim3(gb), dim3(kBlock), 0, st, n, pos, h, part.p);
  RT_LAUNCH_CHECK();
  std::vector<double> hp((size_t)gb * 8);
  RT_CHECK_HIP(hipMemcpyAsync(hp.data(), part.p, hp.size() * sizeof(double),
                              hipMemcpyDeviceToHost, st));
  RT_CHECK_HIP(hipStreamSynchronize(st));
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double hmax = 0, bad = 0;
  for (int b = 0; b < gb; ++b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(lo[a], hp[b * 8 + a]);
      hi[a] = std::fmax(hi[a], hp[b * 8 + 3 + a]);
    }
    hmax = std::fmax(hmax, hp[b * 8 + 6]);
    bad += hp[b * 8 + 7];
  }
  if (bad > 0) {
    set_error("rt_build_neighbors: %.0f non-finite positions or non-positive/non-finite h", bad);
    return RT_E_ARG;
  }
  // cells at least as large as the largest support, with a relative margin
  // far above the rounding of (x - lo)/cs, so adjacent cells hold every pair
  const double cs = nb->kappa * hmax * (1.0 + 1e-6);
  double width[3] = {cs, cs, cs};
  int64_t ncells = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < dim && ((box.mask >> a) & 1)) {
      // a whole number of cells tiles the period; three or more keep the
      // nearest image the only image inside any support
      const double L = box.len[a];
      if (!(lo[a] >= 0.0) || !(hi[a] < L)) {
        set_error("rt_build_neighbors: positions along periodic axis %d span [%g, %g], "
                  "outside [0, %g)", a, lo[a], hi[a], L);
        return RT_E_ARG;
      }
      const double cnt = std::floor(L / cs);
      if (cnt < 3.0) {
        set_error("rt_build_neighbors: period %g along axis %d is shorter than three "
                  "supports (%g)", L, a, cs);
        return RT_E_ARG;
      }
      if (cnt > 2.0e9) {
        set_error("rt_build_neighbors: grid too large along axis %d", a);
        return RT_E_ARG;
      }
      nb->nc[a] = (int)cnt;
      nb->lo[a] = 0.0;
      width[a] = L / cnt;
    } else if (a < dim) {
      double cnt = std::floor((hi[a] - lo[a]) / cs) + 1.0;
      if (cnt > 2.0e9) {
        set_error("rt_build_neighbors: grid too large along axis %d", a);
        return RT_E_ARG;
      }
      nb->nc[a] = (int)cnt;
      nb->lo[a] = lo[a];
    } else {
      nb->nc[a] = 1;
      nb->lo[a] = 0.0;
    }
    ncells *= nb->nc[a];
  }
  // the cell table holds 2 * ncells int32 pairs: bound it by the
  // particle count so that widely separated clusters fail loudly
  if (ncells > std::max<int64_t>(16 * n, (int64_t)1 << 24)) {
    set_error("rt_build_neighbors: %lld cells for %lld particles exceed the cell-table bound",
              (long long)ncells, (long long)n);
    return RT_E_ARG;
  }
  nb->ncells = ncells;
  nb->cell_size = cs;

  // Morton bits per axis
  int bits = 1;
  for (int a = 0; a < dim; ++a)
    while (((int64_t)1 << bits) < nb->nc[a]) ++bits;
  if (dim * bits > 62) {
    set_error("rt_build_neighbors: grid of %d x %d x %d cells needs more than 62 key bits",
              nb->nc[0], nb->nc[1], nb->nc[2]);
    return RT_E_ARG;
  }
  nb->bits = bits;

  // 2-3. keys and stable sort
  DevBuf<uint64_t> keys;
  DevBuf<int32_t> ids;
  RT_CHECK(keys.reserve(n));
  RT_CHECK(nb->skeys.reserve(n));
  RT_CHECK(ids.reserve(n));
  RT_CHECK(nb->perm.reserve(n));
  RT_CHECK(nb->iperm.reserve(n));
  RT_CHECK(nb->sp4.reserve((size_t)4 * n));
#define RT_KEYS(D_)                                                                            \
  hipLaunchKernelGGL(k_keys<D_>, dim3(grid_for(n)), dim3(kBlock), 0, st, bits, n, nin, pos,     \
                     nb->lo[0], nb->lo[1], nb->lo[2], width[0], width[1], width[2], nb->nc[0],  \
                     nb->nc[1], nb->nc[2], keys.p, ids.p)
  if (dim == 3) RT_KEYS(3);
  else RT_KEYS(2);
#undef RT_KEYS
  RT_LAUNCH_CHECK();
  const int end_bit = dim * bits + 1;
  bool sorted = false;
  RT_CHECK(bucket_sort_pairs(ctx, keys.p, nb->skeys.p, ids.p, nb->perm.p, n, end_bit, &sorted));
  if (!sorted) RT_CHECK(radix_sort_pairs(ctx, keys.p, nb->skeys.p, ids.p, nb->perm.p, n, end_bit));
  keys.release();
  ids.release();
  {
    DevBuf<double> rec;
    RT_CHECK(rec.reserve((size_t)4 * n));
    hipLaunchKernelGGL(k_pack_pos, dim3(grid_for(n)), dim3(kBlock), 0, st, dim, n, pos, h, rec.p);
    hipLaunchKernelGGL(k_gather_sorted, dim3(grid_for(n)), dim3(kBlock), 0, st, n, nb->perm.p,
                       rec.p, nb->sp4.p, nb->iperm.p);
    RT_LAUNCH_CHECK();
  }

  // 4. [start, end) per (flag, row-major cell); empty cells stay [0, 0)
  DevBuf<int32_t> cstart, cend;
  RT_CHECK(cstart.reserve((size_t)(2 * ncells)));
  RT_CHECK(cend.reserve((size_t)(2 * ncells)));
  RT_CHECK_HIP(hipMemsetAsync(cstart.p, 0, sizeof(int32_t) * 2 * ncells, st));
  RT_CHECK_HIP(hipMemsetAsync(cend.p, 0, sizeof(int32_t) * 2 * ncells, st));
  if (dim == 3)
    hipLaunchKernelGGL(k_cell_table<3>, dim3(grid_for(n)), dim3(kBlock), 0, st, bits, n,
                       nb->nc[0], nb->nc[1], ncells, nb->skeys.p, cstart.p, cend.p);
  else
    hipLaunchKernelGGL(k_cell_table<2>, dim3(grid_for(n)), dim3(kBlock), 0, st, bits, n,
                       nb->nc[0], nb->nc[1], ncells, nb->skeys.p, cstart.p, cend.p);
  RT_LAUNCH_CHECK();

  // 5. occupied cells
  DevBuf<int32_t> rflag, rid, runs;
  DevBuf<uint64_t> runkey;
  RT_CHECK(rflag.reserve(n));
  RT_CHECK(rid.reserve(n));
  hipLaunchKernelGGL(k_run_flags, dim3(grid_for(n)), dim3(kBlock), 0, st, n, nb->skeys.p, rflag.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int32_t, int32_t>(ctx, rflag.p, rid.p, n, true)));
  RT_CHECK(ctx->sync_read(rid.p + n - 1, sizeof(int32_t)));
  int32_t nruns = 0;
  std::memcpy(&nruns, ctx->host, sizeof(int32_t));
  RT_CHECK(runs.reserve((size_t)nruns + 1));
  RT_CHECK(runkey.reserve((size_t)nruns));
  hipLaunchKernelGGL(k_run_starts, dim3(grid_for(n)), dim3(kBlock), 0, st, n, rflag.p, rid.p,
                     nb->skeys.p, runs.p, runkey.p);
  RT_LAUNCH_CHECK();

  // 6. hit masks of the count pass are kept for the fill pass when they fit
  DevBuf<int32_t> mcell;
  RT_CHECK(mcell.reserve((size_t)nruns));
  if (dim == 3)
    hipLaunchKernelGGL(k_cell_candidates<3>, dim3(grid_for(nruns)), dim3(kBlock), 0, st, nruns,
                       bits, ncells, nb->nc[0], nb->nc[1], nb->nc[2], box.mask, runs.p, nb->skeys.p,
                       cstart.p,
                       cend.p, mcell.p);
  else
    hipLaunchKernelGGL(k_cell_candidates<2>, dim3(grid_for(nruns)), dim3(kBlock), 0, st, nruns,
                       bits, ncells, nb->nc[0], nb->nc[1], nb->nc[2], box.mask, runs.p, nb->skeys.p,
                       cstart.p,
                       cend.p, mcell.p);
  RT_LAUNCH_CHECK();
  int32_t mmax = 0;
  RT_CHECK(max_nonneg<int32_t>(ctx, mcell.p, nruns, &mmax));
  const int mstride = (mmax + kWave - 1) / kWave;
  DevBuf<uint64_t> masks;
  const bool use_masks = mstride > 0 && (double)n * mstride * 8.0 <= kNbrMaskBytes &&
                         masks.reserve((size_t)n * mstride) == RT_OK;
  if (!use_masks) {
    (void)hipGetLastError();
    clear_error();
  }

  // 7. count, scan, fill
  DevBuf<int64_t> cnt;
  RT_CHECK(cnt.reserve(n + 1));
  RT_CHECK(nb->ptr.reserve(n + 1));
  RT_CHECK(nb->n_int_nbrs.reserve(n));
  RT_CHECK_HIP(hipMemsetAsync(cnt.p + n, 0, sizeof(int64_t), st));
#define RT_NBR1(D_, F_, M_, P_)                                                                  \
  hipLaunchKernelGGL((k_nbr_cells<D_, F_, M_, P_>), dim3(nruns), dim3(kBlock), 0, st, n, nin,    \
                     bits, ncells, nb->nc[0], nb->nc[1], nb->nc[2], box, nb->kappa, runs.p,      \
                     runkey.p,                                                                   \
                     nb->sp4.p, cstart.p, cend.p, cnt.p, nb->ptr.p, nb->idx.p, nb->n_int_nbrs.p, \
                     use_masks ? masks.p : nullptr, mstride)
#define RT_NBR(D_, F_, M_)                                                                      \
  do {                                                                                          \
    if (box.mask) RT_NBR1(D_, F_, M_, true);                                                    \
    else RT_NBR1(D_, F_, M_, false);                                                            \
  } while (0)
  if (dim == 3) RT_NBR(3, false, false);
  else RT_NBR(2, false, false);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, nb->ptr.p, n + 1, false)));
  RT_CHECK(ctx->sync_read(nb->ptr.p + n, sizeof(int64_t)));
  int64_t npairs = 0;
  std::memcpy(&npairs, ctx->host, sizeof(int64_t));
  if (npairs >= ((int64_t)1 << 31)) {
    set_error("rt_build_neighbors: %lld pairs exceed the int32 index range", (long long)npairs);
    return RT_E_ARG;
  }
  nb->npairs = npairs;
  RT_CHECK(nb->idx.reserve((size_t)npairs));
  if (use_masks) {
#define RT_FILLM(D_)                                                                             \
  hipLaunchKernelGGL((k_nbr_fill_masks<D_>), dim3(nruns), dim3(kFillBlock), 0, st, n, nin, bits, ncells, \
                     nb->nc[0], nb->nc[1], nb->nc[2], box, runs.p, runkey.p, cstart.p, cend.p,    \
                     nb->ptr.p, nb->idx.p, nb->n_int_nbrs.p, masks.p, mstride)
    if (dim == 3) RT_FILLM(3);
    else RT_FILLM(2);
#undef RT_FILLM
  } else {
    if (dim == 3) RT_NBR(3, true, false);
    else RT_NBR(2, true, false);
  }
#undef RT_NBR
#undef RT_NBR1
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipStreamSynchronize(st));
  return RT_OK;
}

}  // namespace rt

extern "C" {

int rt_build_neighbors(rt_ctx* ctx, int dim, int64_t n_total, int64_t n_interior,
                       const double* pos, const double* h, int kernel, rt_neighbors** out) {
  return rt_build_neighbors_periodic(ctx, dim, n_total, n_interior, pos, h, kernel, nullptr, out);
}

int rt_build_neighbors_periodic(rt_ctx* ctx, int dim, int64_t n_total, int64_t n_interior,
                                const double* pos, const double* h, int kernel,
                                const double* period, rt_neighbors** out) {
  rt::clear_error();
  if (!ctx || !out || !pos || !h) {
    rt::set_error("rt_build_neighbors: NULL argument");
    return RT_E_ARG;
  }
  *out = nullptr;
  if (dim != 2 && dim != 3) {
    rt::set_error("rt_build_neighbors: dim must be 2 or 3 (got %d)", dim);
    return RT_E_ARG;
  }
  if (n_total < 1 || n_total >= ((int64_t)1 << 31) || n_interior < 0 || n_interior > n_total) {
    rt::set_error("rt_build_neighbors: bad sizes n_total=%lld n_interior=%lld",
                  (long long)n_total, (long long)n_interior);
    return RT_E_ARG;
  }
  if (kernel != RT_KERNEL_CUBIC_SPLINE && kernel != RT_KERNEL_WENDLAND_C4) {
    rt::set_error("rt_build_neighbors: unknown kernel %d", kernel);
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  rt_neighbors* nb = new rt_neighbors();
  int s = rt::build_neighbors(ctx, dim, n_total, n_interior, pos, h, kernel, period, nb);
  if (s < 0) {
    delete nb;
    return s;
  }
  *out = nb;
  return RT_OK;
}

int rt_neighbors_get_info(const rt_neighbors* nb, rt_neighbors_info* info) {
  if (!nb || !info) {
    rt::set_error("rt_neighbors_get_info: NULL argument");
    return RT_E_ARG;
  }
  info->dim = nb->dim;
  info->kernel = nb->kernel;
  info->n_total = nb->n_total;
  info->n_interior = nb->n_interior;
  info->npairs = nb->npairs;
  info->ncells = nb->ncells;
  info->cell_size = nb->cell_size;
  return RT_OK;
}

int rt_neighbors_order(rt_ctx* ctx, const rt_neighbors* nb, int32_t* perm) {
  if (!ctx || !nb || !perm) {
    rt::set_error("rt_neighbors_order: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipMemcpyAsync(perm, nb->perm.p, sizeof(int32_t) * nb->n_total,
                              hipMemcpyDeviceToDevice, ctx->stream));
  RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return RT_OK;
}

int rt_neighbors_export(rt_ctx* ctx, const rt_neighbors* nb, int64_t* nbr_ptr, int32_t* nbr_idx) {
  using namespace rt;
  clear_error();
  if (!ctx || !nb || !nbr_ptr || (!nbr_idx && nb->npairs > 0)) {
    set_error("rt_neighbors_export: NULL argument");
    return RT_E_ARG;
  }
  const int64_t n = nb->n_total;
  hipStream_t st = ctx->stream;
  DevBuf<int64_t> ucnt;
  RT_CHECK(ucnt.reserve(n + 1));
  RT_CHECK_HIP(hipMemsetAsync(ucnt.p + n, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL(k_user_counts, dim3(grid_for(n)), dim3(kBlock), 0, st, n, nb->iperm.p,
                     nb->ptr.p, ucnt.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int64_t, int64_t>(ctx, ucnt.p, nbr_ptr, n + 1, false)));
  if (nb->npairs == 0) return RT_OK;
  hipLaunchKernelGGL(k_user_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, n, nb->perm.p,
                     nb->ptr.p, nb->idx.p, nbr_ptr, nbr_idx);
  RT_LAUNCH_CHECK();
  RT_CHECK((row_sort<int32_t, int32_t>(ctx, nbr_ptr, nbr_idx, nullptr, n)));
  RT_CHECK_HIP(hipStreamSynchronize(st));
  return RT_OK;
}

void rt_neighbors_free(rt_neighbors* nb) {
  if (!nb) return;
  rt::IdleScope idle;   // one wait for the device, then every buffer goes back to the cache
  delete nb;
}

}  // extern "C"

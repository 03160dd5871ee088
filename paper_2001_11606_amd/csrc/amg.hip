// Aggregation multigrid preconditioner (gfx950).
//
// The paper preconditions its Krylov solve with algebraic multigrid, set up
// once per time step and reused for every outer iteration (Sec. 3.2); it
// fixes no AMG parameters.  This hierarchy uses aggregation (unsmoothed
// piecewise-constant prolongation) built from the strength of the couplings:
//
//   strength: a_ij couples i and j strongly when
//       |a_ij| >= theta sqrt(m_i m_j),   m_i = max_k |a_ik| (off-diagonal),
//     the classical relative measure made symmetric; a row whose
//     off-diagonal sum is below kCoupled a_ii is left out of the coarse space
//     (one Jacobi sweep already reduces its error by more than 1/kCoupled), so
//     a system dominated by its diagonal, such as cold material at a
//     radiation front, is not coarsened at all;
//   aggregates: candidate blocks are the neighbour-search cells on the fine
//     level and Morton blocks of 2^dim cells on coarser ones.  In each of
//     kAggRounds rounds every block elects as a root its first unassigned
//     node with no strongly coupled assigned neighbour, and unassigned nodes
//     join the strongest strongly coupled new root; then, twice, unassigned
//     nodes join the aggregate of their strongest strongly coupled assigned
//     neighbour, and the rest form their own.
//     With theta <= 0 each candidate block is one aggregate (geometric
//     aggregation).
//
// Aggregates are numbered in the order of their first (root) node, so coarse
// levels keep the Morton locality; the members of every aggregate are listed
// in ascending order, and restriction, the Galerkin products P^T A P (sums of
// fine entries by aggregate pair) and the coarse diagonals are sums in that
// fixed order.
//
// Smoothed aggregation (option): P = (I - 4/3 D1^-1 A) P0 smooths the
// piecewise-constant P0 by one damped l1-Jacobi step, and the coarse
// operator is the Galerkin product P^T (A P), both sparse products formed
// by merging sorted rows over a wavefront in a fixed order.
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
#include <algorithm>
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

constexpr double kCoupled = 0.05;   // off-diagonal row sum / a_ii below which a row stays fine
constexpr int kAggRounds = 6;       // root elections per level
constexpr int kStrG = 16;           // lanes per row of the strength kernels

// candidate-block starts: level 0 groups equal cell codes, coarser levels
// equal parent codes (code >> dim)
__global__ void k_agg_flags(int64_t n, int shift, const uint64_t* __restrict__ code,
                            int32_t* __restrict__ flag) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (code[i] >> shift) != (code[i - 1] >> shift)) ? 1 : 0;
}

__device__ __forceinline__ bool strong_pair(double aij, double mi, double mj, double theta) {
  return aij > 0.0 && aij >= theta * sqrt(mi * mj);
}

// m_i = max_k |a_ik| and whether row i takes part in the coarse space
__global__ void __launch_bounds__(kBlock)
k_row_strength(int64_t n, const int64_t* __restrict__ rp, const double* __restrict__ val,
               const double* __restrict__ diag, double* __restrict__ mrow,
               int32_t* __restrict__ coupled) {
  const int lane = threadIdx.x & (kStrG - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kStrG;
  if (i >= n) return;   // whole groups leave together
  double m = 0.0, sum = 0.0;
  for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kStrG) {
    const double a = fabs(val[k]);
    m = fmax(m, a);
    sum += a;
  }
  m = group_max<kStrG>(m);
  sum = group_sum<kStrG>(sum);
  if (lane == 0) {
    mrow[i] = m;
    coupled[i] = sum >= kCoupled * diag[i] ? 1 : 0;
  }
}

// aggregation state: -2 left out, -1 unassigned, else the aggregate's root node.
// A row starts unassigned when it takes part and has a strong coupling.
__global__ void __launch_bounds__(kBlock)
k_agg_init(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
           const double* __restrict__ val, const double* __restrict__ mrow,
           const int32_t* __restrict__ coupled, double theta, int32_t* __restrict__ agg) {
  const int lane = threadIdx.x & (kStrG - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kStrG;
  if (i >= n) return;
  int cnt = 0;
  if (coupled[i]) {
    const double mi = mrow[i];
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kStrG) {
      const int32_t j = col[k];
      if (coupled[j] && strong_pair(fabs(val[k]), mi, mrow[j], theta)) ++cnt;
    }
  }
  cnt = group_sum<kStrG>(cnt);
  if (lane == 0) agg[i] = cnt > 0 ? -1 : -2;
}

__global__ void k_fill_i32v(int64_t n, int32_t* __restrict__ p, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// every candidate block elects its first unassigned node none of whose strong
// neighbours is assigned yet, so that a new aggregate does not start at the
// edge of an existing one (the minimum is the same whatever the order of the
// atomics); geometric: the block's first node
__global__ void __launch_bounds__(kBlock)
k_agg_elect(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
            const double* __restrict__ val, const double* __restrict__ mrow,
            const int32_t* __restrict__ coupled, const int32_t* __restrict__ bid,
            const int32_t* __restrict__ agg, double theta, int geometric,
            int32_t* __restrict__ root) {
  const int lane = threadIdx.x & (kStrG - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kStrG;
  if (i >= n || agg[i] != -1) return;   // uniform over the group
  int busy = 0;
  if (!geometric) {
    const double mi = mrow[i];
    for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kStrG) {
      const int32_t j = col[k];
      if (agg[j] >= 0 && coupled[j] && strong_pair(fabs(val[k]), mi, mrow[j], theta)) busy = 1;
    }
    busy = group_max<kStrG>(busy);
  }
  if (lane == 0 && !busy) atomicMin(&root[bid[i] - 1], (int32_t)i);
}

// the strongest candidate over a group: larger coupling, then smaller index
template <int G>
__device__ __forceinline__ void group_best(double& v, int32_t& j) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const double w = __shfl_xor(v, o, G);
    const int32_t q = __shfl_xor(j, o, G);
    if (w > v || (w == v && q >= 0 && (j < 0 || q < j))) {
      v = w;
      j = q;
    }
  }
}

// one round: a new root forms its aggregate; an unassigned node joins the
// strongest strongly coupled new root (geometric: its own block's root)
__global__ void __launch_bounds__(kBlock)
k_agg_assign(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
             const double* __restrict__ val, const double* __restrict__ mrow,
             const int32_t* __restrict__ coupled, const int32_t* __restrict__ bid,
             const int32_t* __restrict__ root, double theta, int geometric,
             int32_t* __restrict__ agg) {
  const int lane = threadIdx.x & (kStrG - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kStrG;
  if (i >= n) return;
  if (agg[i] != -1) return;   // uniform over the group
  const int32_t ri = root[bid[i] - 1];
  if (ri == (int32_t)i || geometric) {
    if (lane == 0) agg[i] = ri;
    return;
  }
  const double mi = mrow[i];
  double bv = -1.0;
  int32_t bj = -1;
  for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kStrG) {
    const int32_t j = col[k];
    const double a = fabs(val[k]);
    if (root[bid[j] - 1] == j && coupled[j] && strong_pair(a, mi, mrow[j], theta) &&
        (a > bv || (a == bv && j < bj))) {
      bv = a;
      bj = j;
    }
  }
  group_best<kStrG>(bv, bj);
  if (lane == 0 && bj >= 0) agg[i] = bj;
}

// after the rounds: an unassigned node joins the aggregate of its strongest
// strongly coupled assigned neighbour (as assigned before this pass); if it
// has none it stays unassigned (last pass: forms its own)
__global__ void __launch_bounds__(kBlock)
k_agg_join(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
           const double* __restrict__ val, const double* __restrict__ mrow,
           const int32_t* __restrict__ coupled, double theta, int last,
           const int32_t* __restrict__ agg_in, int32_t* __restrict__ agg_out) {
  const int lane = threadIdx.x & (kStrG - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kStrG;
  if (i >= n) return;
  const int32_t ai = agg_in[i];
  if (ai != -1) {
    if (lane == 0) agg_out[i] = ai;
    return;
  }
  const double mi = mrow[i];
  double bv = -1.0;
  int32_t bj = -1;
  for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kStrG) {
    const int32_t j = col[k];
    const double a = fabs(val[k]);
    if (agg_in[j] >= 0 && coupled[j] && strong_pair(a, mi, mrow[j], theta) &&
        (a > bv || (a == bv && j < bj))) {
      bv = a;
      bj = j;
    }
  }
  group_best<kStrG>(bv, bj);
  if (lane == 0) agg_out[i] = bj >= 0 ? agg_in[bj] : (last ? (int32_t)i : -1);
}

// aggregates numbered by their root node: lead = root flags; rank (inclusive
// scan of lead) gives the number; the coarse node takes its root's code
__global__ void k_agg_lead(int64_t n, const int32_t* __restrict__ agg, int32_t* __restrict__ lead) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) lead[i] = agg[i] == (int32_t)i ? 1 : 0;
}

__global__ void k_agg_number(int64_t n, int shift, const int32_t* __restrict__ agg,
                             const int32_t* __restrict__ rank, const uint64_t* __restrict__ code,
                             int32_t* __restrict__ pmap, uint64_t* __restrict__ ccode,
                             int32_t* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = agg[i];
  const int32_t I = a >= 0 ? rank[a] - 1 : -1;
  pmap[i] = I;
  if (a == (int32_t)i) ccode[I] = code[i] >> shift;
  if (I >= 0) atomicAdd(&cnt[I], 1);
}

__global__ void k_agg_members(int64_t n, const int32_t* __restrict__ pmap,
                              int32_t* __restrict__ cur, int32_t* __restrict__ amem) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t I = pmap[i];
  if (I >= 0) amem[atomicAdd(&cur[I], 1)] = (int32_t)i;
}

__global__ void k_i64_to_i32(int64_t n, const int64_t* __restrict__ a, int32_t* __restrict__ b) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

// Coarse row I = sum over the members of aggregate I (one wavefront per
// coarse row, members in ascending order): the distinct coarse columns in
// ascending order, each the sum of the members' entries mapping to it; the
// entries mapping to I itself and the members' diagonals form the coarse
// diagonal.  Entries of rows left out of the coarse space (pmap -1) drop out.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_galerkin(int64_t nc, const int64_t* __restrict__ crange, const int32_t* __restrict__ amem,
           const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
           const double* __restrict__ val, const double* __restrict__ diag,
           const int32_t* __restrict__ pmap, int64_t* __restrict__ cnt,
           const int64_t* __restrict__ crp, int32_t* __restrict__ ccol,
           double* __restrict__ cval, double* __restrict__ cdiag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  if (I >= nc) return;   // whole wavefront exits together
  const int64_t m0 = crange[I], m1 = crange[I + 1];
  double dsum = 0.0;
  if (FILL) {
    for (int64_t q = m0 + lane; q < m1; q += kWave) dsum += diag[amem[q]];
    dsum = group_sum<kWave>(dsum);
  }
  int32_t last = -1;
  int64_t out = FILL ? crp[I] : 0;
  int64_t count = 0;
  while (true) {
    int32_t m = INT_MAX;
    for (int64_t q = m0; q < m1; ++q) {
      const int32_t i = amem[q];
      for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kWave) {
        const int32_t pc = pmap[col[k]];
        if (pc > last && pc < m) m = pc;
      }
    }
    m = wave_min(m);
    if (m == INT_MAX) break;
    if (FILL) {
      double sum = 0.0;
      for (int64_t q = m0; q < m1; ++q) {
        const int32_t i = amem[q];
        for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += kWave)
          if (pmap[col[k]] == m) sum += val[k];
      }
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

// ---- smoothed aggregation ----------------------------------------------------
// P = (I - omega D1^-1 A) P0 with the l1 diagonal D1: the spectrum of
// D1^-1 A lies in (0, 1], so omega = 4/3 (the usual 4/(3 lambda_max) with the
// bound lambda_max <= 1) damps the high end without an eigenvalue estimate.
constexpr double kSaOmega = 4.0 / 3.0;
constexpr int kMergeK = 16;   // input rows per lane of a merged row sum

// Row i of P over the coarse-space rows: the distinct aggregates of i and its
// neighbours, ascending, each with the value
//   [J == pmap_i] (1 - omega s_i a_ii) - omega s_i sum_{k: pmap_k == J} a_ik,
// s = 1/D1; a row left out of the coarse space (pmap_i < 0) stays empty.
// One wavefront per row.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_sa_prolong(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
             const double* __restrict__ val, const double* __restrict__ diag,
             const double* __restrict__ sinv, const int32_t* __restrict__ pmap,
             int64_t* __restrict__ cnt, const int64_t* __restrict__ prp,
             int32_t* __restrict__ pcol, double* __restrict__ pval) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  if (i >= n) return;   // whole wavefront exits together
  const int32_t pi = pmap[i];
  if (pi < 0) {
    if (!FILL && lane == 0) cnt[i] = 0;
    return;
  }
  const double w = kSaOmega * sinv[i];
  const int64_t k0 = rp[i], k1 = rp[i + 1];
  int32_t last = -1;
  int64_t out = FILL ? prp[i] : 0;
  int64_t count = 0;
  while (true) {
    int32_t m = pi > last ? pi : INT_MAX;
    for (int64_t k = k0 + lane; k < k1; k += kWave) {
      const int32_t J = pmap[col[k]];
      if (J > last && J < m) m = J;
    }
    m = wave_min(m);
    if (m == INT_MAX) break;
    if (FILL) {
      double s = 0.0;
      for (int64_t k = k0 + lane; k < k1; k += kWave)
        if (pmap[col[k]] == m) s -= w * val[k];
      s = group_sum<kWave>(s);
      if (m == pi) s += 1.0 - w * diag[i];
      if (lane == 0) {
        pcol[out] = m;
        pval[out] = s;
      }
      ++out;
    } else {
      ++count;
    }
    last = m;
  }
  if (!FILL && lane == 0) cnt[i] = count;
}

// Merged weighted sum of sorted sparse rows over a wavefront: the lane holds
// up to kMergeK input rows (cursor cur[q] up to e[q], weight w[q]).  Each step
// takes the smallest head column over the wavefront and adds every head at
// that column (a row holds a column once), lanes combined in a fixed order;
// the sum at column dcol (if >= 0) goes to *dsum instead of the output.
// Counts the output columns (FILL false) or writes them from `out` on.
template <bool FILL>
__device__ __forceinline__ void merge_rows(int nq, const double* w, int64_t* cur, const int64_t* e,
                                           const int32_t* __restrict__ col,
                                           const double* __restrict__ val, int32_t dcol,
                                           int64_t out, int32_t* __restrict__ ocol,
                                           double* __restrict__ oval, int64_t* count,
                                           double* dsum) {
  const int lane = threadIdx.x & (kWave - 1);
  int64_t c = 0;
  double d = 0.0;
  while (true) {
    int32_t m = INT_MAX;
#pragma unroll
    for (int q = 0; q < kMergeK; ++q)
      if (q < nq && cur[q] < e[q]) {
        const int32_t cq = col[cur[q]];
        m = cq < m ? cq : m;
      }
    m = wave_min(m);
    if (m == INT_MAX) break;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kMergeK; ++q)
      if (q < nq && cur[q] < e[q] && col[cur[q]] == m) {
        if (FILL) s += w[q] * val[cur[q]];
        ++cur[q];
      }
    if (FILL) s = group_sum<kWave>(s);
    if (m == dcol) {
      d += s;
    } else {
      if (FILL && lane == 0) {
        ocol[out] = m;
        oval[out] = s;
      }
      ++out;
      ++c;
    }
  }
  *count = c;
  *dsum = d;
}

// Row i of A P = a_ii P_i + sum_k a_ik P_k (rows outside the coarse space,
// unused by the coarse operator, stay empty).  Lane l takes the row's
// entries l, l + 64, ... with the diagonal as entry number len.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_sa_ap(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
        const double* __restrict__ val, const double* __restrict__ diag,
        const int32_t* __restrict__ pmap, const int64_t* __restrict__ prp,
        const int32_t* __restrict__ pcol, const double* __restrict__ pval,
        int64_t* __restrict__ cnt, const int64_t* __restrict__ aprp,
        int32_t* __restrict__ apcol, double* __restrict__ apval) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  if (i >= n) return;
  if (pmap[i] < 0) {
    if (!FILL && lane == 0) cnt[i] = 0;
    return;
  }
  const int64_t k0 = rp[i];
  const int len = (int)(rp[i + 1] - k0);
  double w[kMergeK];
  int64_t cur[kMergeK], e[kMergeK];
  int nq = 0;
#pragma unroll
  for (int q = 0; q < kMergeK; ++q) {
    const int t = lane + q * kWave;
    w[q] = 0.0;
    cur[q] = e[q] = 0;
    if (t <= len) {
      const int32_t k = t < len ? col[k0 + t] : (int32_t)i;
      w[q] = t < len ? val[k0 + t] : diag[i];
      cur[q] = prp[k];
      e[q] = prp[k + 1];
      nq = q + 1;
    }
  }
  int64_t count = 0;
  double dsum = 0.0;
  merge_rows<FILL>(nq, w, cur, e, pcol, pval, -1, FILL ? aprp[i] : 0, apcol, apval, &count,
                   &dsum);
  if (!FILL && lane == 0) cnt[i] = count;
}

// Coarse row I of P^T (A P): the rows of A P listed in column I of P (its
// transpose's row I), weighted by P's entries; the coarse diagonal apart.
template <bool FILL>
__global__ void __launch_bounds__(kBlock)
k_sa_rap(int64_t nc, const int64_t* __restrict__ ptrp, const int32_t* __restrict__ ptrow,
         const double* __restrict__ ptval, const int64_t* __restrict__ aprp,
         const int32_t* __restrict__ apcol, const double* __restrict__ apval,
         int64_t* __restrict__ cnt, const int64_t* __restrict__ crp, int32_t* __restrict__ ccol,
         double* __restrict__ cval, double* __restrict__ cdiag) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  if (I >= nc) return;
  const int64_t t0 = ptrp[I];
  const int len = (int)(ptrp[I + 1] - t0);
  double w[kMergeK];
  int64_t cur[kMergeK], e[kMergeK];
  int nq = 0;
#pragma unroll
  for (int q = 0; q < kMergeK; ++q) {
    const int t = lane + q * kWave;
    w[q] = 0.0;
    cur[q] = e[q] = 0;
    if (t < len) {
      const int32_t i = ptrow[t0 + t];
      w[q] = ptval[t0 + t];
      cur[q] = aprp[i];
      e[q] = aprp[i + 1];
      nq = q + 1;
    }
  }
  int64_t count = 0;
  double dsum = 0.0;
  merge_rows<FILL>(nq, w, cur, e, apcol, apval, (int32_t)I, FILL ? crp[I] : 0, ccol, cval,
                   &count, &dsum);
  if (lane == 0) {
    if (FILL) cdiag[I] = dsum;
    else cnt[I] = count;
  }
}

// column counts of P, then its entries moved to their column's next slot
__global__ void k_pt_count(int64_t n, const int64_t* __restrict__ prp,
                           const int32_t* __restrict__ pcol, int32_t* __restrict__ cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t q = prp[i]; q < prp[i + 1]; ++q) atomicAdd(&cnt[pcol[q]], 1);
}

__global__ void k_pt_fill(int64_t n, const int64_t* __restrict__ prp,
                          const int32_t* __restrict__ pcol, const double* __restrict__ pval,
                          int32_t* __restrict__ cur, int32_t* __restrict__ ptrow,
                          double* __restrict__ ptval) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t q = prp[i]; q < prp[i + 1]; ++q) {
    const int32_t slot = atomicAdd(&cur[pcol[q]], 1);
    ptrow[slot] = (int32_t)i;
    ptval[slot] = pval[q];
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

// The vector passes below take one row per thread; stop (else NULL) holds
// the flag of the block's 256-row chunk at tp[block] (tp NULL: one flag).
template <typename T>
__global__ void k_scale(int64_t n, const T* __restrict__ s, const T* __restrict__ b,
                        T* __restrict__ x, const int32_t* __restrict__ tp,
                        const int32_t* __restrict__ stop) {
  if (stop && stop[tp ? tp[blockIdx.x] : 0]) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = s[i] * b[i];
}

// bc[I] = sum of r over the members of aggregate I, in ascending order
template <typename T>
__global__ void k_restrict(int64_t nc, const int64_t* __restrict__ crange,
                           const int32_t* __restrict__ amem, const T* __restrict__ r,
                           T* __restrict__ bc, const int32_t* __restrict__ tp,
                           const int32_t* __restrict__ stop) {
  if (stop && stop[tp ? tp[blockIdx.x] : 0]) return;
  int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (I >= nc) return;
  T s = 0;
  for (int64_t q = crange[I]; q < crange[I + 1]; ++q) s += r[amem[q]];
  bc[I] = s;
}

// bc = P^T r with the transpose's rows (fine rows ascending)
template <typename T, typename PV>
__global__ void k_restrict_p(int64_t nc, const int64_t* __restrict__ ptrp,
                             const int32_t* __restrict__ ptrow, const PV* __restrict__ ptv,
                             const T* __restrict__ r, T* __restrict__ bc,
                             const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (I >= nc) return;
  T s = 0;
  for (int64_t t = ptrp[I]; t < ptrp[I + 1]; ++t) s += (T)ptv[t] * r[ptrow[t]];
  bc[I] = s;
}

// x += P xc
template <typename T, typename PV>
__global__ void k_prolong_p(int64_t n, const int64_t* __restrict__ prp,
                            const int32_t* __restrict__ pcol, const PV* __restrict__ pv,
                            const T* __restrict__ xc, T* __restrict__ x,
                            const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = 0;
  for (int64_t q = prp[i]; q < prp[i + 1]; ++q) s += (T)pv[q] * xc[pcol[q]];
  x[i] += s;
}

// x += y
template <typename T>
__global__ void k_axpy1(int64_t n, const T* __restrict__ y, T* __restrict__ x,
                        const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += y[i];
}

// x += P xc (rows left out of the coarse space get nothing)
template <typename T>
__global__ void k_prolong(int64_t n, const int32_t* __restrict__ pmap, const T* __restrict__ xc,
                          T* __restrict__ x, const int32_t* __restrict__ tp,
                          const int32_t* __restrict__ stop) {
  if (stop && stop[tp ? tp[blockIdx.x] : 0]) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t I = pmap[i];
    if (I >= 0) x[i] += xc[I];
  }
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

// ---- K-cycle -------------------------------------------------------------------
// Krylov-accelerated coarse correction: on a level C that is not the
// coarsest, the correction from its right-hand side r is two steps of a
// flexible conjugate-gradient iteration on A_C preconditioned by the cycle of
// the levels below:
//   v1 = cycle(r), rho1 = v1.r, alpha1 = v1.A v1, rt = r - (rho1/alpha1) A v1,
//   v2 = cycle(rt), gamma = v2.A v1, beta = v2.A v2, rho2 = v2.rt,
//   alpha2 = beta - gamma^2/alpha1,
//   x = (rho1/alpha1 - gamma rho2/(alpha1 alpha2)) v1 + (rho2/alpha2) v2,
// the second direction being v2 made A-orthogonal to v1.  The inner products
// are formed and turned into weights on the device.
constexpr int kKdotBlocks = 128;

// Block partials (double) of u.a, u.b and u.c over [0, n) at part[blk],
// part[nb + blk] and part[2 nb + blk], nb = gridDim.x; b, c NULL: zero.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_kdots(int64_t n, const T* __restrict__ u, const T* __restrict__ a, const T* __restrict__ b,
        const T* __restrict__ c, double* __restrict__ part, const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (stop && *stop) return;
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double ui = (double)u[i];
    sa += ui * (double)a[i];
    if (b) sb += ui * (double)b[i];
    if (c) sc += ui * (double)c[i];
  }
  sa = block_sum(sa, red);
  sb = block_sum(sb, red);
  sc = block_sum(sc, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sa;
    part[gridDim.x + blockIdx.x] = sb;
    part[2 * gridDim.x + blockIdx.x] = sc;
  }
}

// One block: the K-cycle weights from nb block partials of three inner
// products.  Phase 1 (rho1, alpha1): kc[0] = rho1, kc[1] = alpha1,
// kc[2] = rho1/alpha1 (0 unless alpha1 > 0).  Phase 2 (gamma, beta, rho2):
// kc[3], kc[4] = the weights of v1 and v2; when alpha2 is not positive
// against beta (v2 A-parallel to v1 within rounding) the second direction is
// dropped.
__global__ void __launch_bounds__(kBlock)
k_kcoef(int phase, int nb, const double* __restrict__ part, double* __restrict__ kc,
        const int32_t* __restrict__ stop) {
  __shared__ double red[kBlock / kWave];
  if (stop && *stop) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < nb; k += kBlock) {
    s0 += part[k];
    s1 += part[nb + k];
    s2 += part[2 * nb + k];
  }
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x != 0) return;
  if (phase == 1) {
    kc[0] = s0;
    kc[1] = s1;
    kc[2] = (s1 > 0.0 && isfinite(s1) && isfinite(s0)) ? s0 / s1 : 0.0;
  } else {
    const double rho1 = kc[0], a1 = kc[1], gam = s0, beta = s1, rho2 = s2;
    double c1 = kc[2], c2 = 0.0;
    if (a1 > 0.0 && isfinite(a1)) {
      const double a2 = beta - gam * gam / a1;
      if (a2 > 1e-12 * beta && isfinite(a2) && isfinite(rho2)) {
        c2 = rho2 / a2;
        c1 = rho1 / a1 - gam * c2 / a1;
      }
    }
    kc[3] = c1;
    kc[4] = c2;
  }
}

// out = r - kc[2] w
template <typename T>
__global__ void k_kresid(int64_t n, const double* __restrict__ kc, const T* __restrict__ r,
                         const T* __restrict__ w, T* __restrict__ out,
                         const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = r[i] - (T)kc[2] * w[i];
}

// x = kc[3] v1 + kc[4] v2 (x may alias v1)
template <typename T>
__global__ void k_kcomb(int64_t n, const double* __restrict__ kc, const T* v1,
                        const T* __restrict__ v2, T* x, const int32_t* __restrict__ stop) {
  if (stop && *stop) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = (T)kc[3] * v1[i] + (T)kc[4] * v2[i];
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
  static double* wr(Level& L) { return L.wr64.p; }
  static double* wx(Level& L) { return L.wx64.p; }
  static double* kw(Level& L) { return L.kw64.p; }
  static const double* pv(const Level& L) { return L.p_val.p; }
  static const double* ptv(const Level& L) { return L.pt_val.p; }
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
  static float* wr(Level& L) { return L.wr32.p; }
  static float* wx(Level& L) { return L.wx32.p; }
  static float* kw(Level& L) { return L.kw32.p; }
  static const float* pv(const Level& L) { return L.p_val32.p; }
  static const float* ptv(const Level& L) { return L.pt_val32.p; }
};

// Values (and columns) of the coarse level C = P^T F P.
int galerkin_fill(rt_ctx* ctx, const Level& F, Level& C) {
  hipLaunchKernelGGL((k_galerkin<true>), dim3(grid_for(C.n * kWave)), dim3(kBlock), 0,
                     ctx->stream, C.n, F.crange.p, F.amem.p, F.rp.p, F.col.p, F.val64.p,
                     F.diag64.p, F.pmap.p, nullptr, C.rp.p, C.col.p, C.val64.p, C.diag64.p);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// Aggregates of level l (L.pmap, L.crange, L.amem) and the codes of their
// coarse nodes; returns the number of aggregates.
int aggregate(rt_ctx* ctx, Level& L, int shift, double theta, DevBuf<uint64_t>& ccode,
              int64_t* nc_out) {
  hipStream_t st = ctx->stream;
  const int64_t n = L.n;
  const bool geometric = !(theta > 0.0);
  DevBuf<int32_t> flag, bid, coupled, agg, agg2, root;
  DevBuf<double> mrow;
  for (auto* b : {&flag, &bid, &coupled, &agg, &agg2}) RT_CHECK(b->reserve(n));
  RT_CHECK(mrow.reserve(n));
  RT_CHECK(L.pmap.reserve(n));
  // candidate blocks: bid = 1-based block number of every node
  hipLaunchKernelGGL(k_agg_flags, dim3(grid_for(n)), dim3(kBlock), 0, st, n, shift, L.code.p,
                     flag.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int32_t, int32_t>(ctx, flag.p, bid.p, n, true)));
  RT_CHECK(ctx->sync_read(bid.p + n - 1, sizeof(int32_t)));
  int32_t nblk = 0;
  std::memcpy(&nblk, ctx->host, sizeof(int32_t));
  RT_CHECK(root.reserve(nblk));
  const int gs = grid_for(n * (int64_t)kStrG);
  if (geometric) {
    hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(n)), dim3(kBlock), 0, st, n, agg.p, -1);
  } else {
    hipLaunchKernelGGL(k_row_strength, dim3(gs), dim3(kBlock), 0, st, n, L.rp.p, L.val64.p,
                       L.diag64.p, mrow.p, coupled.p);
    RT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_agg_init, dim3(gs), dim3(kBlock), 0, st, n, L.rp.p, L.col.p, L.val64.p,
                       mrow.p, coupled.p, theta, agg.p);
  }
  RT_LAUNCH_CHECK();
  for (int round = 0; round < (geometric ? 1 : kAggRounds); ++round) {
    hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(nblk)), dim3(kBlock), 0, st, (int64_t)nblk,
                       root.p, INT_MAX);
    hipLaunchKernelGGL(k_agg_elect, dim3(gs), dim3(kBlock), 0, st, n, L.rp.p, L.col.p, L.val64.p,
                       mrow.p, coupled.p, bid.p, agg.p, theta, geometric ? 1 : 0, root.p);
    hipLaunchKernelGGL(k_agg_assign, dim3(gs), dim3(kBlock), 0, st, n, L.rp.p, L.col.p,
                       L.val64.p, mrow.p, coupled.p, bid.p, root.p, theta, geometric ? 1 : 0,
                       agg.p);
    RT_LAUNCH_CHECK();
  }
  int32_t* final_agg = agg.p;
  if (!geometric) {   // two join passes reach nodes up to two strong couplings away
    hipLaunchKernelGGL(k_agg_join, dim3(gs), dim3(kBlock), 0, st, n, L.rp.p, L.col.p, L.val64.p,
                       mrow.p, coupled.p, theta, 0, agg.p, agg2.p);
    hipLaunchKernelGGL(k_agg_join, dim3(gs), dim3(kBlock), 0, st, n, L.rp.p, L.col.p, L.val64.p,
                       mrow.p, coupled.p, theta, 1, agg2.p, agg.p);
    RT_LAUNCH_CHECK();
  }
  // numbering by root node, member counts
  hipLaunchKernelGGL(k_agg_lead, dim3(grid_for(n)), dim3(kBlock), 0, st, n, final_agg, flag.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int32_t, int32_t>(ctx, flag.p, bid.p, n, true)));   // bid now holds the ranks
  RT_CHECK(ctx->sync_read(bid.p + n - 1, sizeof(int32_t)));
  int32_t nc32 = 0;
  std::memcpy(&nc32, ctx->host, sizeof(int32_t));
  const int64_t nc = nc32;
  *nc_out = nc;
  if (nc == 0) return RT_OK;
  DevBuf<int32_t> cnt;
  DevBuf<int64_t> cnt64;
  RT_CHECK(cnt.reserve(nc + 1));
  RT_CHECK(cnt64.reserve(nc + 1));
  RT_CHECK(ccode.reserve(nc));
  hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(nc + 1)), dim3(kBlock), 0, st, nc + 1, cnt.p, 0);
  hipLaunchKernelGGL(k_agg_number, dim3(grid_for(n)), dim3(kBlock), 0, st, n, shift, final_agg,
                     bid.p, L.code.p, L.pmap.p, ccode.p, cnt.p);
  RT_LAUNCH_CHECK();
  // member lists: offsets (exclusive scan of the counts), then every member
  // at its aggregate's next slot, then each list sorted ascending
  RT_CHECK(L.crange.reserve(nc + 1));
  RT_CHECK((scan<int32_t, int64_t>(ctx, cnt.p, L.crange.p, nc + 1, false)));
  RT_CHECK(ctx->sync_read(L.crange.p + nc, sizeof(int64_t)));
  int64_t nmem = 0;
  std::memcpy(&nmem, ctx->host, sizeof(int64_t));
  RT_CHECK(L.amem.reserve(std::max<int64_t>(nmem, 1)));
  hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(nc)), dim3(kBlock), 0, st, nc, L.crange.p,
                     cnt.p);   // cnt = next free slot per aggregate
  hipLaunchKernelGGL(k_agg_members, dim3(grid_for(n)), dim3(kBlock), 0, st, n, L.pmap.p, cnt.p,
                     L.amem.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((row_sort<int32_t, int32_t>(ctx, L.crange.p, L.amem.p, nullptr, nc)));
  return RT_OK;
}

// Smoothed prolongation from F to C (aggregates already in F.pmap, nc of
// them) and the coarse operator P^T A P into C.  *ok = false (nothing
// changed in C) when a row of F or a column of P is longer than the merged
// sums take (64 kMergeK entries); the caller then keeps P piecewise constant.
int build_smoothed(rt_ctx* ctx, Level& F, Level& C, int64_t nc, bool* ok) {
  hipStream_t st = ctx->stream;
  const int64_t n = F.n;
  *ok = false;
  if (F.max_row + 1 > (int64_t)kWave * kMergeK) return RT_OK;
  // P: count, offsets, fill
  DevBuf<int64_t> cnt;
  RT_CHECK(cnt.reserve(n + 1));
  RT_CHECK_HIP(hipMemsetAsync(cnt.p + n, 0, sizeof(int64_t), st));
  const int gw = grid_for(n * (int64_t)kWave);
  hipLaunchKernelGGL((k_sa_prolong<false>), dim3(gw), dim3(kBlock), 0, st, n, F.rp.p, F.col.p,
                     F.val64.p, F.diag64.p, F.sinv64.p, F.pmap.p, cnt.p, nullptr, nullptr,
                     nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK(F.p_rp.reserve(n + 1));
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, F.p_rp.p, n + 1, false)));
  RT_CHECK(ctx->sync_read(F.p_rp.p + n, sizeof(int64_t)));
  int64_t nnzp = 0;
  std::memcpy(&nnzp, ctx->host, sizeof(int64_t));
  F.p_nnz = nnzp;
  RT_CHECK(F.p_col.reserve(std::max<int64_t>(nnzp, 1)));
  RT_CHECK(F.p_val.reserve(std::max<int64_t>(nnzp, 1)));
  hipLaunchKernelGGL((k_sa_prolong<true>), dim3(gw), dim3(kBlock), 0, st, n, F.rp.p, F.col.p,
                     F.val64.p, F.diag64.p, F.sinv64.p, F.pmap.p, nullptr, F.p_rp.p, F.p_col.p,
                     F.p_val.p);
  RT_LAUNCH_CHECK();
  // P^T: column counts, offsets, entries by atomic slots, then each column
  // sorted by fine row (a fixed order)
  DevBuf<int32_t> ccnt;
  RT_CHECK(ccnt.reserve(nc + 1));
  hipLaunchKernelGGL(k_fill_i32v, dim3(grid_for(nc + 1)), dim3(kBlock), 0, st, nc + 1, ccnt.p, 0);
  hipLaunchKernelGGL(k_pt_count, dim3(grid_for(n)), dim3(kBlock), 0, st, n, F.p_rp.p, F.p_col.p,
                     ccnt.p);
  RT_LAUNCH_CHECK();
  int32_t maxcol = 0;
  RT_CHECK(max_nonneg<int32_t>(ctx, ccnt.p, nc, &maxcol));
  if ((int64_t)maxcol > (int64_t)kWave * kMergeK) return RT_OK;
  RT_CHECK(F.pt_rp.reserve(nc + 1));
  RT_CHECK((scan<int32_t, int64_t>(ctx, ccnt.p, F.pt_rp.p, nc + 1, false)));
  RT_CHECK(F.pt_row.reserve(std::max<int64_t>(nnzp, 1)));
  RT_CHECK(F.pt_val.reserve(std::max<int64_t>(nnzp, 1)));
  hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(nc)), dim3(kBlock), 0, st, nc, F.pt_rp.p,
                     ccnt.p);   // ccnt = next free slot per column
  hipLaunchKernelGGL(k_pt_fill, dim3(grid_for(n)), dim3(kBlock), 0, st, n, F.p_rp.p, F.p_col.p,
                     F.p_val.p, ccnt.p, F.pt_row.p, F.pt_val.p);
  RT_LAUNCH_CHECK();
  RT_CHECK((row_sort<int32_t, double>(ctx, F.pt_rp.p, F.pt_row.p, F.pt_val.p, nc)));
  // A P (temporary)
  DevBuf<int64_t> aprp;
  DevBuf<int32_t> apcol;
  DevBuf<double> apval;
  RT_CHECK(aprp.reserve(n + 1));
  hipLaunchKernelGGL((k_sa_ap<false>), dim3(gw), dim3(kBlock), 0, st, n, F.rp.p, F.col.p,
                     F.val64.p, F.diag64.p, F.pmap.p, F.p_rp.p, F.p_col.p, F.p_val.p, cnt.p,
                     nullptr, nullptr, nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, aprp.p, n + 1, false)));
  RT_CHECK(ctx->sync_read(aprp.p + n, sizeof(int64_t)));
  int64_t nnzap = 0;
  std::memcpy(&nnzap, ctx->host, sizeof(int64_t));
  RT_CHECK(apcol.reserve(std::max<int64_t>(nnzap, 1)));
  RT_CHECK(apval.reserve(std::max<int64_t>(nnzap, 1)));
  hipLaunchKernelGGL((k_sa_ap<true>), dim3(gw), dim3(kBlock), 0, st, n, F.rp.p, F.col.p,
                     F.val64.p, F.diag64.p, F.pmap.p, F.p_rp.p, F.p_col.p, F.p_val.p, nullptr,
                     aprp.p, apcol.p, apval.p);
  RT_LAUNCH_CHECK();
  // P^T (A P): the coarse rows
  DevBuf<int64_t> rcnt;
  RT_CHECK(rcnt.reserve(nc + 1));
  RT_CHECK_HIP(hipMemsetAsync(rcnt.p + nc, 0, sizeof(int64_t), st));
  const int gc = grid_for(nc * (int64_t)kWave);
  hipLaunchKernelGGL((k_sa_rap<false>), dim3(gc), dim3(kBlock), 0, st, nc, F.pt_rp.p, F.pt_row.p,
                     F.pt_val.p, aprp.p, apcol.p, apval.p, rcnt.p, nullptr, nullptr, nullptr,
                     nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK(C.rp.reserve(nc + 1));
  RT_CHECK((scan<int64_t, int64_t>(ctx, rcnt.p, C.rp.p, nc + 1, false)));
  RT_CHECK(ctx->sync_read(C.rp.p + nc, sizeof(int64_t)));
  int64_t nnz = 0;
  std::memcpy(&nnz, ctx->host, sizeof(int64_t));
  C.nnz = nnz;
  RT_CHECK(max_nonneg<int64_t>(ctx, rcnt.p, nc, &C.max_row));
  RT_CHECK(C.col.reserve(std::max<int64_t>(nnz, 1)));
  RT_CHECK(C.val64.reserve(nnz + kSpmvPad));
  RT_CHECK(C.diag64.reserve(nc));
  hipLaunchKernelGGL((k_sa_rap<true>), dim3(gc), dim3(kBlock), 0, st, nc, F.pt_rp.p, F.pt_row.p,
                     F.pt_val.p, aprp.p, apcol.p, apval.p, nullptr, C.rp.p, C.col.p, C.val64.p,
                     C.diag64.p);
  RT_LAUNCH_CHECK();
  *ok = true;
  return RT_OK;
}

// Build level l+1 from level l: aggregates, coarse CSR structure, and the
// coarse columns and values, so that the new level is complete before it
// serves as the fine level of the next one.  *stalled: the aggregation left
// no coarse space or coarsened too little (no level added).
int build_next_level(rt_ctx* ctx, rt_matrix* A, int l, int dim, bool* stalled) {
  hipStream_t st = ctx->stream;
  const int shift = l == 0 ? 0 : dim;
  DevBuf<uint64_t> ccode;
  int64_t nc = 0;
  RT_CHECK(aggregate(ctx, A->levels[l], shift, A->amg.strength, ccode, &nc));
  const int64_t n = A->levels[l].n;
  *stalled = nc == 0 || nc * 10 > n * 9;
  if (*stalled) return RT_OK;
  A->levels.emplace_back();
  Level& C = A->levels.back();
  Level& Lr = A->levels[l];   // re-fetch after emplace_back
  C.n = nc;
  C.code = std::move(ccode);
  Lr.smoothed = false;
  if (A->amg.prolongation == RT_PROLONG_SMOOTHED) {
    bool ok = false;
    RT_CHECK(build_smoothed(ctx, Lr, C, nc, &ok));
    Lr.smoothed = ok;
    if (ok) return RT_OK;
  }
  // piecewise-constant prolongation: coarse structure: count, scan
  DevBuf<int64_t> cnt;
  RT_CHECK(cnt.reserve(nc + 1));
  RT_CHECK_HIP(hipMemsetAsync(cnt.p + nc, 0, sizeof(int64_t), st));
  hipLaunchKernelGGL((k_galerkin<false>), dim3(grid_for(nc * kWave)), dim3(kBlock), 0, st, nc,
                     Lr.crange.p, Lr.amem.p, Lr.rp.p, Lr.col.p, nullptr, nullptr, Lr.pmap.p,
                     cnt.p, nullptr, nullptr, nullptr, nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK(C.rp.reserve(nc + 1));
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, C.rp.p, nc + 1, false)));
  RT_CHECK(ctx->sync_read(C.rp.p + nc, sizeof(int64_t)));
  int64_t nnz = 0;
  std::memcpy(&nnz, ctx->host, sizeof(int64_t));
  C.nnz = nnz;
  RT_CHECK(max_nonneg<int64_t>(ctx, cnt.p, nc, &C.max_row));
  RT_CHECK(C.col.reserve(std::max<int64_t>(nnz, 1)));
  RT_CHECK(C.val64.reserve(nnz + kSpmvPad));
  RT_CHECK(C.diag64.reserve(nc));
  return galerkin_fill(ctx, A->levels[l], C);
}

// Work vectors of a level; cycle 2 (W) adds the second visit's residual and
// correction, cycle 3 (K) also A v1 and the inner products' partials.
int level_vectors(Level& L, bool fp32, int cycle) {
  for (auto* b : {&L.b64, &L.x64, &L.t64, &L.r64, &L.d64, &L.sinv64, &L.dinv64})
    RT_CHECK(b->reserve(L.n));
  if (cycle >= 2)
    for (auto* b : {&L.wr64, &L.wx64}) RT_CHECK(b->reserve(L.n));
  if (cycle == 3) {
    RT_CHECK(L.kw64.reserve(L.n));
    RT_CHECK(L.kpart.reserve(3 * kKdotBlocks));
    RT_CHECK(L.kc.reserve(8));
  }
  if (fp32) {
    for (auto* b : {&L.b32, &L.x32, &L.t32, &L.r32, &L.d32, &L.sinv32, &L.dinv32})
      RT_CHECK(b->reserve(L.n));
    if (cycle >= 2)
      for (auto* b : {&L.wr32, &L.wx32}) RT_CHECK(b->reserve(L.n));
    if (cycle == 3) RT_CHECK(L.kw32.reserve(L.n));
    RT_CHECK(L.val32.reserve(L.nnz + kSpmvPad));
    RT_CHECK(L.diag32.reserve(L.n));
  }
  return RT_OK;
}

}  // namespace

int amg_level_vectors(Level& L, bool fp32, int cycle) { return level_vectors(L, fp32, cycle); }

int amg_setup(rt_ctx* ctx, rt_matrix* A) {
  hipStream_t st = ctx->stream;
  const rt_neighbors* nb = A->nb;
  const bool fp32 = A->has_fp32;
  if (A->n == 0) return RT_OK;
  // The aggregates depend on the values (strength of the couplings), so the
  // hierarchy is rebuilt with every assembly: once per time step.
  A->levels.resize(1);
  Level& L0 = A->levels[0];
  if (A->amg.max_levels > 1 && L0.code.n == 0) {   // cell codes of the fine level
    RT_CHECK(L0.code.reserve(L0.n));
    RT_CHECK_HIP(hipMemcpyAsync(L0.code.p, nb->skeys.p, sizeof(uint64_t) * L0.n,
                                hipMemcpyDeviceToDevice, st));
  }
  RT_CHECK(level_vectors(L0, fp32, A->amg.cycle));   // level 0: assembly wrote its scalings
  for (int l = 0; (int)A->levels.size() < A->amg.max_levels; ++l) {
    if (A->levels[l].n <= A->amg.coarse_size) break;
    bool stalled = false;
    RT_CHECK(build_next_level(ctx, A, l, nb->dim, &stalled));
    if (stalled) break;
    Level& L = A->levels.back();
    if (A->amg.tiled_spmv) RT_CHECK(build_tiles(ctx, L));
    // vectors, FP32 copy and smoother scalings of the new level now: the
    // smoothed prolongation out of it reads its l1 scaling
    RT_CHECK(level_vectors(L, fp32, A->amg.cycle));
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
  }
  for (Level& L : A->levels) {
    if (fp32 && L.smoothed) {   // FP32 copies of P and P^T for the FP32 V-cycle
      const int64_t np = std::max<int64_t>(L.p_nnz, 1);
      RT_CHECK(L.p_val32.reserve(np));
      RT_CHECK(L.pt_val32.reserve(np));
      hipLaunchKernelGGL(k_to_f32, dim3(grid_for(np)), dim3(kBlock), 0, st, np, L.p_val.p,
                         L.p_val32.p);
      hipLaunchKernelGGL(k_to_f32, dim3(grid_for(np)), dim3(kBlock), 0, st, np, L.pt_val.p,
                         L.pt_val32.p);
      RT_LAUNCH_CHECK();
    }
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
                        const int32_t* stop);

// The K-cycle's coarse correction on level c (not the coarsest): from b(c)
// into x(c).  wr, wx hold the second visit's residual and correction, kw the
// product A v1; t(c) is free between the visits and takes A v2.
template <typename T>
static int kcycle_correct(rt_ctx* ctx, rt_matrix* A, size_t c, const int32_t* stop) {
  using B = LevelBufs<T>;
  hipStream_t st = ctx->stream;
  Level& C = A->levels[c];
  const int64_t n = C.n;
  const int nb = std::min<int>(kKdotBlocks, std::max(1, grid_for(n)));
  RT_CHECK(vcycle_level<T>(ctx, A, c, B::b(C), B::x(C), stop));
  RT_CHECK((launch_spmv_level<T, SP_PLAIN>(st, C, B::val(C), B::diag(C), B::x(C), nullptr,
                                           nullptr, B::kw(C), nullptr, nullptr, nullptr,
                                           level_shape<T>(C), nullptr, stop)));
  hipLaunchKernelGGL(k_kdots<T>, dim3(nb), dim3(kBlock), 0, st, n, B::x(C), B::b(C), B::kw(C),
                     nullptr, C.kpart.p, stop);
  hipLaunchKernelGGL(k_kcoef, dim3(1), dim3(kBlock), 0, st, 1, nb, C.kpart.p, C.kc.p, stop);
  hipLaunchKernelGGL(k_kresid<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, C.kc.p, B::b(C),
                     B::kw(C), B::wr(C), stop);
  RT_LAUNCH_CHECK();
  RT_CHECK(vcycle_level<T>(ctx, A, c, B::wr(C), B::wx(C), stop));
  RT_CHECK((launch_spmv_level<T, SP_PLAIN>(st, C, B::val(C), B::diag(C), B::wx(C), nullptr,
                                           nullptr, B::t(C), nullptr, nullptr, nullptr,
                                           level_shape<T>(C), nullptr, stop)));
  hipLaunchKernelGGL(k_kdots<T>, dim3(nb), dim3(kBlock), 0, st, n, B::wx(C), B::kw(C), B::t(C),
                     B::wr(C), C.kpart.p, stop);
  hipLaunchKernelGGL(k_kcoef, dim3(1), dim3(kBlock), 0, st, 2, nb, C.kpart.p, C.kc.p, stop);
  hipLaunchKernelGGL(k_kcomb<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, C.kc.p, B::x(C),
                     B::wx(C), B::x(C), stop);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

template <typename T>
static int vcycle_level(rt_ctx* ctx, rt_matrix* A, size_t l, const T* b, T* out,
                        const int32_t* stop) {
  using B = LevelBufs<T>;
  hipStream_t st = ctx->stream;
  Level& L = A->levels[l];
  const int64_t n = L.n;
  const size_t nl = cycle_depth(A);
  // a batch's levels: the products and vector passes skip the chunks of
  // stopped problems
  const bool bskip = l < A->lvl_skip.size();
  const int32_t* tp = bskip ? A->lvl_tprob[l] : nullptr;
  const int32_t* sk = bskip ? A->lvl_skip[l] : stop;
  if (l + 1 == nl) {
    if (A->coarse_direct && nl == A->levels.size()) {
      hipLaunchKernelGGL(k_coarse_solve<T>, dim3(grid_for(n * kWave)), dim3(kBlock), 0, st, n,
                         A->coarse_inv.p, b, out, stop);
      RT_LAUNCH_CHECK();
      return RT_OK;
    }
    // four l1-Jacobi sweeps from zero (a symmetric positive-definite operator)
    T* t = B::t(L);
    hipLaunchKernelGGL(k_scale<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B::sinv(L), b, t,
                       tp, sk);
    RT_LAUNCH_CHECK();
    T* src = t;
    T* dst = out;
    for (int sweep = 0; sweep < 3; ++sweep) {
      RT_CHECK((launch_spmv_level<T, SP_SMOOTH>(st, L, B::val(L), B::diag(L), src, b, B::sinv(L),
                                                dst, nullptr, nullptr, nullptr,
                                                level_shape<T>(L), tp, sk)));
      T* tmp = src;
      src = dst;
      dst = tmp;
    }
    if (src != out)
      RT_CHECK_HIP(hipMemcpyAsync(out, src, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
    return RT_OK;
  }
  Level& C = A->levels[l + 1];
  const bool cskip = l + 1 < A->lvl_skip.size();
  const int32_t* tpc = cskip ? A->lvl_tprob[l + 1] : nullptr;
  const int32_t* skc = cskip ? A->lvl_skip[l + 1] : stop;
  T* t = B::t(L);
  T* r = B::r(L);
  const bool cheb = A->amg.smoother == RT_SMOOTHER_CHEBYSHEV;
  if (cheb) {
    RT_CHECK(cheb_smooth<T>(st, A, L, A->amg.smoother_degree, b, nullptr, t, stop));
  } else {
    hipLaunchKernelGGL(k_scale<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B::sinv(L), b, t,
                       tp, sk);
    RT_LAUNCH_CHECK();
  }
  RT_CHECK((launch_spmv_level<T, SP_RESID>(st, L, B::val(L), B::diag(L), t, b, nullptr, r,
                                           nullptr, nullptr, nullptr, level_shape<T>(L),
                                           tp, sk)));
  if (L.smoothed)
    hipLaunchKernelGGL((k_restrict_p<T, T>), dim3(grid_for(C.n)), dim3(kBlock), 0, st, C.n,
                       L.pt_rp.p, L.pt_row.p, B::ptv(L), r, B::b(C), stop);
  else
    hipLaunchKernelGGL(k_restrict<T>, dim3(grid_for(C.n)), dim3(kBlock), 0, st, C.n, L.crange.p,
                       L.amem.p, r, B::b(C), tpc, skc);
  RT_LAUNCH_CHECK();
  if (A->amg.cycle == 3 && l + 2 < nl)
    RT_CHECK(kcycle_correct<T>(ctx, A, l + 1, stop));
  else
    RT_CHECK(vcycle_level<T>(ctx, A, l + 1, B::b(C), B::x(C), stop));
  if (A->amg.cycle == 2 && l + 2 < nl) {
    // W-cycle: a second coarse correction from the residual of the first
    RT_CHECK((launch_spmv_level<T, SP_RESID>(st, C, B::val(C), B::diag(C), B::x(C), B::b(C),
                                             nullptr, B::wr(C), nullptr, nullptr, nullptr,
                                             level_shape<T>(C), nullptr, stop)));
    RT_CHECK(vcycle_level<T>(ctx, A, l + 1, B::wr(C), B::wx(C), stop));
    hipLaunchKernelGGL(k_axpy1<T>, dim3(grid_for(C.n)), dim3(kBlock), 0, st, C.n, B::wx(C),
                       B::x(C), stop);
    RT_LAUNCH_CHECK();
  }
  if (L.smoothed)
    hipLaunchKernelGGL((k_prolong_p<T, T>), dim3(grid_for(n)), dim3(kBlock), 0, st, n, L.p_rp.p,
                       L.p_col.p, B::pv(L), B::x(C), t, stop);
  else
    hipLaunchKernelGGL(k_prolong<T>, dim3(grid_for(n)), dim3(kBlock), 0, st, n, L.pmap.p,
                       B::x(C), t, tp, sk);
  RT_LAUNCH_CHECK();
  if (cheb) return cheb_smooth<T>(st, A, L, A->amg.smoother_degree, b, t, out, stop);
  RT_CHECK((launch_spmv_level<T, SP_SMOOTH>(st, L, B::val(L), B::diag(L), t, b, B::sinv(L), out,
                                            nullptr, nullptr, nullptr, level_shape<T>(L),
                                            tp, sk)));
  return RT_OK;
}

template <typename T>
int vcycle(rt_ctx* ctx, rt_matrix* A, const T* b, T* z, const int32_t* stop) {
  return vcycle_level<T>(ctx, A, 0, b, z, stop);
}

template int vcycle<double>(rt_ctx*, rt_matrix*, const double*, double*, const int32_t*);
template int vcycle<float>(rt_ctx*, rt_matrix*, const float*, float*, const int32_t*);

}  // namespace rt

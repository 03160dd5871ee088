// Ensembles of independent problems solved together.
//
// rt_batch_create concatenates the assembled fine-level systems of nprob
// problems into one block-diagonal system.  Problem p owns rows
// [row_off[p], row_off[p] + n_p): its range starts on a 256-row tile
// boundary and is padded to the next one with identity rows (diagonal 1, no
// off-diagonal entries, right-hand side 0), so every tile -- and every block
// of every product and vector kernel -- belongs to exactly one problem.
// Each launch then covers the whole ensemble: one product, one vector update,
// one material pass for all problems.  The Krylov scalars are per problem
// (alpha_p, beta_p, r_p.z_p, ||r_p||), kept on the device; the block partials
// of a problem are combined by one block per problem in a fixed order.  A
// problem that meets its own tolerance is flagged, and the blocks of flagged
// problems return at once, so the others keep iterating undisturbed.  Since
// a flagged problem is left as it is, extra iterations are no-ops: the PCG
// iterations can be replayed as HIP graphs of K iterations with a single
// host read of the flags per graph.  Preconditioner: Jacobi.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"
#include "material.h"
#include "prim.h"
#include "reduce.h"
#include "spmv.h"

namespace rt {
namespace {

enum { B_RZ = 0, B_PQ, B_ALPHA, B_BETA, B_RR, B_THR, B_BB, B_THR2, B_COUNT };
enum { F_INNER = 0, F_OUTER, F_ITS, F_REFINE, F_COUNT };
enum { BOP_BB = 0, BOP_OUTER, BOP_RZ, BOP_ALPHA, BOP_BETA };
enum { M_DE = 0, M_DEE, M_ITS, M_BAD, M_NONPHYS, M_EN, M_EN0, M_WIDTH };

inline int64_t pad_rows(int64_t n) { return (n + kTileRows - 1) / kTileRows * kTileRows; }

}  // namespace
}  // namespace rt

struct rt_batch {
  int nprob = 0;
  std::vector<rt_matrix*> mats;
  std::vector<int64_t> row_off, uoff;   // host: padded row offsets, user offsets (nprob + 1)
  int64_t n = 0, nuser = 0, ntiles = 0;
  bool fp32 = false;
  // The batch's hierarchy: level 0 the concatenated fine level, level l >= 1
  // the problems' level l concatenated (a problem whose hierarchy is shorter
  // has no rows there); the V-cycle runs on it as on one matrix.  Its level
  // vector never grows past RT_MAX_LEVELS, so L stays valid.
  std::unique_ptr<rt_matrix> H;
  rt::Level& L;                         // the concatenated fine level (H->levels[0])
  rt::DevBuf<double> z64;               // V-cycle output of the batched AMG PCG
  rt::DevBuf<float> z32;
  rt_batch() : H(make_h()), L(H->levels[0]) {}
  static rt_matrix* make_h() {
    rt_matrix* h = new rt_matrix();
    h->levels.reserve(RT_MAX_LEVELS);
    h->levels.resize(1);
    return h;
  }
  rt::DevBuf<int64_t> d_row_off;
  rt::DevBuf<int32_t> tprob;            // problem of every tile
  // coarse levels of the hierarchy, per 256-row chunk (levels concatenated):
  // first and last problem with rows in it, and whether all of them stopped
  rt::DevBuf<int32_t> crng, cdone, ciota;
  int64_t nchunks = 0;
  rt::DevBuf<int32_t> perm;             // row -> concatenated user index (-1: padding)
  rt::DevBuf<double> pdt, pc, pa;       // per-problem dt, c, a
  rt::DevBuf<double> V, sa, f, rho, cv, m, e_prev, E_prev, Qe, QE, g;
  rt::DevBuf<double> ecur, Ecur, enew, xs, bs, r64, p64, q64;
  rt::DevBuf<float> r32, p32, q32, d32;
  rt::DevBuf<double> partA, partB, ps, mres;
  rt::DevBuf<int32_t> flags;            // F_COUNT x nprob
  hipStream_t cap = nullptr;            // stream the graphs are captured on
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // [FP64, FP32] PCG iterations
  int graph_k[2] = {0, 0};
  bool graph_amg[2] = {false, false};              // the iterations captured are V-cycle ones
  ~rt_batch() {
    for (auto& gx : graph)
      if (gx) (void)hipGraphExecDestroy(gx);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace rt {
namespace {

struct CopyArgs {
  // source problem (sorted order)
  const int64_t* rp;
  const double *diag64, *dinv64, *V, *sa, *f, *rho, *cv, *m, *e_prev, *E_prev, *Qe, *QE, *g;
  const float *diag32, *dinv32;
  const int32_t* perm;
  int64_t nin, nrows, row0, nnz0, nnz_end, user0;
  // destination (concatenated)
  int64_t* rp_d;
  double *diag64_d, *dinv64_d, *V_d, *sa_d, *f_d, *rho_d, *cv_d, *m_d, *e_prev_d, *E_prev_d,
      *Qe_d, *QE_d, *g_d;
  float *diag32_d, *dinv32_d;
  int32_t* perm_d;
};

// rows of one problem (padding rows: identity, zero data)
__global__ void k_b_copy_rows(CopyArgs A) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= A.nrows) return;
  const int64_t i = A.row0 + s;
  if (s < A.nin) {
    A.rp_d[i] = A.nnz0 + A.rp[s];
    A.diag64_d[i] = A.diag64[s];
    A.dinv64_d[i] = A.dinv64[s];
    if (A.diag32_d) {
      A.diag32_d[i] = A.diag32[s];
      A.dinv32_d[i] = A.dinv32[s];
    }
    A.V_d[i] = A.V[s];
    A.sa_d[i] = A.sa[s];
    A.f_d[i] = A.f[s];
    A.rho_d[i] = A.rho[s];
    A.cv_d[i] = A.cv[s];
    A.m_d[i] = A.m[s];
    A.e_prev_d[i] = A.e_prev[s];
    A.E_prev_d[i] = A.E_prev[s];
    A.Qe_d[i] = A.Qe[s];
    A.QE_d[i] = A.QE[s];
    A.g_d[i] = A.g[s];
    A.perm_d[i] = (int32_t)(A.user0 + A.perm[s]);
  } else {
    A.rp_d[i] = A.nnz_end;
    A.diag64_d[i] = 1.0;
    A.dinv64_d[i] = 1.0;
    if (A.diag32_d) {
      A.diag32_d[i] = 1.0f;
      A.dinv32_d[i] = 1.0f;
    }
    A.V_d[i] = 0.0;
    A.sa_d[i] = 0.0;
    A.f_d[i] = 1.0;
    A.rho_d[i] = 1.0;
    A.cv_d[i] = 1.0;
    A.m_d[i] = 0.0;
    A.e_prev_d[i] = 0.0;
    A.E_prev_d[i] = 0.0;
    A.Qe_d[i] = 0.0;
    A.QE_d[i] = 0.0;
    A.g_d[i] = 0.0;
    A.perm_d[i] = -1;
  }
}

__global__ void k_b_copy_cols(int64_t nnz, const int32_t* __restrict__ col, int64_t nnz0,
                              int64_t row0, int32_t* __restrict__ col_d) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nnz) col_d[nnz0 + k] = (int32_t)(row0 + col[k]);
}

__global__ void k_b_set_i64(int64_t* p, int64_t v) { *p = v; }

// ---- the batch hierarchy: a problem's level copied in with offsets ----------
__global__ void k_bh_rp(int64_t n, const int64_t* __restrict__ rp, int64_t eoff,
                        int64_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = rp[i] + eoff;
}
// aggregate of a fine row on the batch's next level (-1 stays: no aggregate)
__global__ void k_bh_pmap(int64_t n, const int32_t* __restrict__ src, int64_t coff,
                          int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = src[i] >= 0 ? (int32_t)(src[i] + coff) : -1;
}
__global__ void k_bh_crange(int64_t nc, const int64_t* __restrict__ src, int64_t moff,
                            int64_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nc) out[i] = src[i] + moff;
}
template <typename T>
__global__ void k_bh_fill(int64_t n, T* __restrict__ p, T v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_b_iota(int64_t n, int32_t* __restrict__ p) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// chunk c is skipped when every problem from crng[2c] to crng[2c + 1] stopped
__global__ void k_b_chunk_done(int64_t nch, const int32_t* __restrict__ crng,
                               const int32_t* __restrict__ done, int32_t* __restrict__ cdone) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nch) return;
  int all = 1;
  for (int p = crng[2 * c]; p <= crng[2 * c + 1] && all; ++p) all = done[p] != 0;
  cdone[c] = all;
}

__global__ void k_b_fill_i32(int64_t n, int32_t* __restrict__ p, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ void k_b_zero(int64_t n, T* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

__global__ void k_b_add_f32(int64_t n, const float* __restrict__ d, double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += (double)d[i];
}

// ---- per-problem reductions ----------------------------------------------
// part[t] over 256-row tiles (one block per tile, one row per thread)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_b_dot(int64_t n, const T* __restrict__ a, const T* __restrict__ b, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const double v = i < n ? (double)a[i] * (double)b[i] : 0.0;
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// One block per problem: sum the partials of the problem's blocks (rpb rows
// each) in a fixed order and apply op to its scalars.
__global__ void __launch_bounds__(kBlock)
k_b_seg(int op, int nprob, const int64_t* __restrict__ row_off, int rpb,
        const double* __restrict__ pa, const double* __restrict__ pb, double* __restrict__ ps,
        int32_t* __restrict__ flags, double tol2, int mixed, double inner_tol) {
  __shared__ double red[kBlock / kWave];
  const int p = blockIdx.x;
  int32_t* inner = flags + F_INNER * nprob;
  int32_t* outer = flags + F_OUTER * nprob;
  if ((op == BOP_RZ || op == BOP_ALPHA || op == BOP_BETA) && inner[p]) return;
  // a problem that met its tolerance keeps its residual (its product blocks were skipped)
  if (op == BOP_OUTER && outer[p]) return;
  const int64_t b0 = row_off[p] / rpb, b1 = row_off[p + 1] / rpb;
  double a = 0.0, b = 0.0;
  for (int64_t q = b0 + threadIdx.x; q < b1; q += kBlock) {
    a += pa[q];
    if (pb) b += pb[q];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x != 0) return;
  double* s = ps;
#define PS(k) s[(k) * nprob + p]
  switch (op) {
    case BOP_BB:
      PS(B_BB) = a;
      PS(B_THR2) = tol2 * a;
      break;
    case BOP_OUTER: {   // a = ||b - A x||^2 of the current iterate
      PS(B_RR) = a;
      const bool done = !(a > PS(B_THR2)) || PS(B_BB) == 0.0 || !isfinite(a);
      outer[p] = done ? 1 : 0;
      inner[p] = done ? 1 : 0;
      if (mixed) {
        const double red_p = fmax(inner_tol, 0.3 * sqrt(PS(B_THR2) / a));
        PS(B_THR) = red_p * red_p * a;
        if (!done) flags[F_REFINE * nprob + p] += 1;
      } else {
        PS(B_THR) = PS(B_THR2);
      }
      break;
    }
    case BOP_RZ:
      PS(B_RZ) = a;
      break;
    case BOP_ALPHA:
      PS(B_PQ) = a;
      if (a > 0.0 && isfinite(a)) {
        PS(B_ALPHA) = PS(B_RZ) / a;
      } else {   // breakdown: stop this problem
        PS(B_ALPHA) = 0.0;
        inner[p] = 1;
      }
      break;
    case BOP_BETA:
      PS(B_RR) = a;
      PS(B_BETA) = b / PS(B_RZ);
      PS(B_RZ) = b;
      flags[F_ITS * nprob + p] += 1;
      if (!(a > PS(B_THR)) || !isfinite(a)) inner[p] = 1;
      break;
  }
#undef PS
}

// ---- batched Jacobi-PCG vector kernels (one block per tile) ----------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_b_init_jacobi(int64_t n, const int32_t* __restrict__ tprob, const int32_t* __restrict__ done,
                const T* __restrict__ dinv, const T* __restrict__ r, T* __restrict__ p,
                double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  if (done[tprob[blockIdx.x]]) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    const T z = dinv[i] * r[i];
    p[i] = z;
    acc = (double)r[i] * (double)z;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_b_update(int64_t n, int nprob, const int32_t* __restrict__ tprob,
           const int32_t* __restrict__ done, const double* __restrict__ ps, T* __restrict__ x,
           T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
           const T* __restrict__ dinv, double* __restrict__ partA, double* __restrict__ partB) {
  __shared__ double red[kBlock / kWave];
  const int pr = tprob[blockIdx.x];
  if (done[pr]) return;
  const T alpha = (T)ps[B_ALPHA * nprob + pr];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double rr = 0.0, rz = 0.0;
  if (i < n) {
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr = (double)ri * (double)ri;
    if (dinv) rz = (double)ri * (double)(dinv[i] * ri);
  }
  rr = block_sum(rr, red);
  rz = block_sum(rz, red);
  if (threadIdx.x == 0) {
    partA[blockIdx.x] = rr;
    partB[blockIdx.x] = rz;
  }
}

// p = z + beta p, z = D^-1 r (Jacobi) or the given z (the V-cycle's)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_b_pupdate(int64_t n, int nprob, const int32_t* __restrict__ tprob,
            const int32_t* __restrict__ done, const double* __restrict__ ps,
            const T* __restrict__ r, const T* __restrict__ dinv, const T* __restrict__ z,
            T* __restrict__ p) {
  const int pr = tprob[blockIdx.x];
  if (done[pr]) return;
  const T beta = (T)ps[B_BETA * nprob + pr];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = (z ? z[i] : dinv[i] * r[i]) + beta * p[i];
}

// tile partials of r.z for the problems not done; with p (else NULL) also p = z
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_b_rz(int64_t n, const int32_t* __restrict__ tprob, const int32_t* __restrict__ done,
       const T* __restrict__ r, const T* __restrict__ z, T* __restrict__ p,
       double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  if (done[tprob[blockIdx.x]]) return;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    acc = (double)r[i] * (double)z[i];
    if (p) p[i] = z[i];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// ---- Newton-step kernels -----------------------------------------------------
__global__ void k_b_gather(int64_t n, const int32_t* __restrict__ perm,
                           const double* __restrict__ user, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t u = perm[i];
  out[i] = u >= 0 ? user[u] : 0.0;
}

__global__ void k_b_scatter(int64_t n, const int32_t* __restrict__ perm,
                            const double* __restrict__ in, double* __restrict__ user) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t u = perm[i];
  if (u >= 0) user[u] = in[i];
}

struct BRhs {
  const int32_t* tprob;
  const double *dt, *c, *a;
  const double *V, *sa, *f, *cv, *E_prev, *QE, *g, *e_l, *E_l;
  double* b;
};

__global__ void k_b_rhs(int64_t n, BRhs A) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = A.tprob[i / kTileRows];
  const double dt = A.dt[p], c = A.c[p], a = A.a[p];
  const double T = A.e_l[i] / A.cv[i];
  const double T2 = T * T;
  const double ca = c * A.sa[i];
  const double P = A.E_prev[i] / dt + ca * (a * (T2 * T2)) - (1.0 - A.f[i]) * ca * A.E_l[i] +
                   A.QE[i];
  A.b[i] = A.V[i] * P + A.g[i];
}

struct BMat {
  const int32_t *tprob, *perm;
  const double *dt, *c, *a;
  const double *e_prev, *rho, *cv, *sa, *Qe, *m, *V, *E_prev;
  const double *E_new, *E_old, *e_start;
  double* e_out;
  double tol;
  int max_iter;
};

// one block per tile; partials [tile][M_WIDTH]
__global__ void __launch_bounds__(kBlock) k_b_material(int64_t n, BMat A, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  const int p = A.tprob[blockIdx.x];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double de = 0.0, dE = 0.0, its = 0.0, bad = 0.0, nonphys = 0.0, en = 0.0, en0 = 0.0;
  if (i < n && A.perm[i] >= 0) {
    const double Enew = A.E_new[i];
    const MaterialResult mr =
        material_solve(A.rho[i], A.cv[i], A.sa[i], A.e_prev[i], A.Qe[i], Enew, A.e_start[i],
                       A.dt[p], A.c[p], A.a[p], A.tol, A.max_iter);
    const double e = mr.e;
    if (mr.nonphysical) nonphys = 1.0;
    if (!mr.converged) bad = 1.0;
    A.e_out[i] = e;
    de = fabs(e - A.e_start[i]) / fabs(e);
    dE = fabs(Enew - A.E_old[i]) / fabs(Enew);
    its = (double)mr.iterations;
    en = A.m[i] * e + A.V[i] * Enew;
    en0 = A.m[i] * A.e_prev[i] + A.V[i] * A.E_prev[i];
  } else if (i < n) {
    A.e_out[i] = 0.0;
  }
  de = block_max(de, red);
  dE = block_max(dE, red);
  its = block_max(its, red);
  bad = block_sum(bad, red);
  nonphys = block_sum(nonphys, red);
  en = block_sum(en, red);
  en0 = block_sum(en0, red);
  if (threadIdx.x == 0) {
    double* o = part + (int64_t)blockIdx.x * M_WIDTH;
    o[M_DE] = de;
    o[M_DEE] = dE;
    o[M_ITS] = its;
    o[M_BAD] = bad;
    o[M_NONPHYS] = nonphys;
    o[M_EN] = en;
    o[M_EN0] = en0;
  }
}

// one block per problem: column-wise max (first three) / sum (rest) over its tiles
__global__ void __launch_bounds__(kBlock)
k_b_material_seg(int nprob, const int64_t* __restrict__ row_off, const double* __restrict__ part,
                 double* __restrict__ out) {
  __shared__ double red[kBlock / kWave];
  const int p = blockIdx.x;
  const int64_t t0 = row_off[p] / kTileRows, t1 = row_off[p + 1] / kTileRows;
  for (int c = 0; c < M_WIDTH; ++c) {
    const bool is_max = c <= M_ITS;
    double v = 0.0;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kBlock) {
      const double x = part[t * M_WIDTH + c];
      v = is_max ? fmax(v, x) : v + x;
    }
    v = is_max ? block_max(v, red) : block_sum(v, red);
    if (threadIdx.x == 0) out[(int64_t)p * M_WIDTH + c] = v;
  }
}

// ---- host side -----------------------------------------------------------------
int b_seg(rt_ctx* ctx, rt_batch* B, int op, int rpb, const double* pa, const double* pb,
          double tol2 = 0.0, int mixed = 0, double inner_tol = 0.0) {
  hipLaunchKernelGGL(k_b_seg, dim3(B->nprob), dim3(kBlock), 0, ctx->stream, op, B->nprob,
                     B->d_row_off.p, rpb, pa, pb, B->ps.p, B->flags.p, tol2, mixed, inner_tol);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// flags of kind k to the host; *all = every problem flagged
int b_read_flags(rt_ctx* ctx, rt_batch* B, int kind, std::vector<int32_t>* out, bool* all) {
  out->resize(B->nprob);
  RT_CHECK_HIP(hipMemcpyAsync(out->data(), B->flags.p + (int64_t)kind * B->nprob,
                              sizeof(int32_t) * B->nprob, hipMemcpyDeviceToHost, ctx->stream));
  RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  *all = std::all_of(out->begin(), out->end(), [](int32_t v) { return v != 0; });
  return RT_OK;
}

template <typename T>
struct BSel;
template <>
struct BSel<double> {
  static const double* val(const Level& L) { return L.val64.p; }
  static const double* diag(const Level& L) { return L.diag64.p; }
  static const double* dinv(const Level& L) { return L.dinv64.p; }
  static double* p(rt_batch* B) { return B->p64.p; }
  static double* q(rt_batch* B) { return B->q64.p; }
  static double* z(rt_batch* B) { return B->z64.p; }
  static int shape(const Level& L) { return L.shape64; }
  static constexpr int slot = 0;
};
template <>
struct BSel<float> {
  static const float* val(const Level& L) { return L.val32.p; }
  static const float* diag(const Level& L) { return L.diag32.p; }
  static const float* dinv(const Level& L) { return L.dinv32.p; }
  static float* p(rt_batch* B) { return B->p32.p; }
  static float* q(rt_batch* B) { return B->q32.p; }
  static float* z(rt_batch* B) { return B->z32.p; }
  static int shape(const Level& L) { return L.shape32; }
  static constexpr int slot = 1;
};

// the coarse-level chunk flags from the problems' inner flags
static int b_chunk_flags(hipStream_t st, rt_batch* B) {
  if (B->nchunks == 0) return RT_OK;
  hipLaunchKernelGGL(k_b_chunk_done, dim3(grid_for(B->nchunks)), dim3(kBlock), 0, st, B->nchunks,
                     B->crng.p, B->flags.p + F_INNER * B->nprob, B->cdone.p);
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// one PCG iteration for every problem not flagged done (kernels only); amg:
// preconditioned by the V-cycle of the batch hierarchy (on the context's
// stream, which st must then be)
template <typename T>
int b_iteration(rt_ctx* ctx, hipStream_t st, rt_batch* B, T* x, T* r, bool amg = false) {
  using S = BSel<T>;
  const Level& L = B->L;
  const int32_t* done = B->flags.p + F_INNER * B->nprob;
  const int shape = S::shape(L);
  const int rpb = spmv_rows_per_block(L, shape);
  RT_CHECK((launch_spmv_level<T, SP_DOT>(st, L, S::val(L), S::diag(L), S::p(B), nullptr, nullptr,
                                         S::q(B), nullptr, B->partA.p, nullptr, shape,
                                         B->tprob.p, done)));
  hipLaunchKernelGGL(k_b_seg, dim3(B->nprob), dim3(kBlock), 0, st, (int)BOP_ALPHA, B->nprob,
                     B->d_row_off.p, rpb, B->partA.p, (const double*)nullptr, B->ps.p,
                     B->flags.p, 0.0, 0, 0.0);
  RT_LAUNCH_CHECK();
  const unsigned nt = (unsigned)B->ntiles;
  hipLaunchKernelGGL((k_b_update<T>), dim3(nt), dim3(kBlock), 0, st, B->n, B->nprob, B->tprob.p,
                     done, B->ps.p, x, r, S::p(B), S::q(B), amg ? nullptr : S::dinv(L),
                     B->partA.p, B->partB.p);
  RT_LAUNCH_CHECK();
  if (amg) {
    RT_CHECK(b_chunk_flags(st, B));
    RT_CHECK(vcycle<T>(ctx, B->H.get(), r, S::z(B)));
    hipLaunchKernelGGL((k_b_rz<T>), dim3(nt), dim3(kBlock), 0, st, B->n, B->tprob.p, done, r,
                       S::z(B), (T*)nullptr, B->partB.p);
    RT_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_b_seg, dim3(B->nprob), dim3(kBlock), 0, st, (int)BOP_BETA, B->nprob,
                     B->d_row_off.p, kTileRows, B->partA.p, B->partB.p, B->ps.p, B->flags.p, 0.0,
                     0, 0.0);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_b_pupdate<T>), dim3(nt), dim3(kBlock), 0, st, B->n, B->nprob, B->tprob.p,
                     done, B->ps.p, r, S::dinv(L), amg ? S::z(B) : (const T*)nullptr, S::p(B));
  RT_LAUNCH_CHECK();
  return RT_OK;
}

// PCG (Jacobi, or amg: the batch hierarchy's V-cycle) on every problem whose
// inner flag is clear; on entry r = b - A x and the per-problem thresholds
// are set.  graph_k > 0 replays graphs of graph_k iterations between host
// reads of the flags.
template <typename T>
int b_pcg(rt_ctx* ctx, rt_batch* B, T* x, T* r, int max_it, int graph_k, bool amg = false) {
  using S = BSel<T>;
  hipStream_t st = ctx->stream;
  const Level& L = B->L;
  const int32_t* done = B->flags.p + F_INNER * B->nprob;
  if (amg) {
    RT_CHECK(b_chunk_flags(st, B));
    RT_CHECK(vcycle<T>(ctx, B->H.get(), r, S::z(B)));
    hipLaunchKernelGGL((k_b_rz<T>), dim3((unsigned)B->ntiles), dim3(kBlock), 0, st, B->n,
                       B->tprob.p, done, r, S::z(B), S::p(B), B->partB.p);
  } else {
    hipLaunchKernelGGL((k_b_init_jacobi<T>), dim3((unsigned)B->ntiles), dim3(kBlock), 0, st, B->n,
                       B->tprob.p, done, S::dinv(L), r, S::p(B), B->partB.p);
  }
  RT_LAUNCH_CHECK();
  RT_CHECK(b_seg(ctx, B, BOP_RZ, kTileRows, B->partB.p, nullptr));
  std::vector<int32_t> fl;
  bool all = false;
  RT_CHECK(b_read_flags(ctx, B, F_INNER, &fl, &all));
  int launched = 0;
  while (!all && launched < max_it) {
    if (graph_k > 0 && launched + graph_k <= max_it) {
      const int slot = S::slot;
      if (!B->graph[slot] || B->graph_k[slot] != graph_k || B->graph_amg[slot] != amg) {
        if (B->graph[slot]) {
          RT_CHECK_HIP(hipGraphExecDestroy(B->graph[slot]));
          B->graph[slot] = nullptr;
        }
        if (!B->cap) RT_CHECK_HIP(hipStreamCreate(&B->cap));
        hipGraph_t g = nullptr;
        RT_CHECK_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
        // the V-cycle launches on the context's stream: the capture stream
        // stands in for it while the iterations are recorded
        hipStream_t own = ctx->stream;
        ctx->stream = B->cap;
        int cs = RT_OK;
        for (int k = 0; k < graph_k && cs == RT_OK; ++k)
          cs = b_iteration<T>(ctx, B->cap, B, x, r, amg);
        ctx->stream = own;
        const hipError_t ce = hipStreamEndCapture(B->cap, &g);
        if (cs != RT_OK) {
          if (g) (void)hipGraphDestroy(g);
          return cs;
        }
        RT_CHECK_HIP(ce);
        const hipError_t ie = hipGraphInstantiate(&B->graph[slot], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        RT_CHECK_HIP(ie);
        B->graph_k[slot] = graph_k;
        B->graph_amg[slot] = amg;
      }
      RT_CHECK_HIP(hipGraphLaunch(B->graph[slot], st));
      launched += graph_k;
    } else {
      RT_CHECK(b_iteration<T>(ctx, st, B, x, r, amg));
      launched += 1;
    }
    RT_CHECK(b_read_flags(ctx, B, F_INNER, &fl, &all));
  }
  return RT_OK;
}

// solve A x = b for every problem (sorted, concatenated vectors in xs / bs)
int b_solve(rt_ctx* ctx, rt_batch* B, const rt_solve_opts* o, int graph_k, rt_solve_stats* stats) {
  hipStream_t st = ctx->stream;
  const int64_t n = B->n;
  const int np = B->nprob;
  const bool mixed = o->precision == RT_PREC_MIXED;
  // the V-cycle when asked for and the batch's depth is above 1 (else Jacobi)
  const bool amg = o->precond == 1 && cycle_depth(B->H.get()) > 1;
  const Level& L = B->L;
  hipLaunchKernelGGL(k_b_fill_i32, dim3(grid_for((int64_t)F_COUNT * np)), dim3(kBlock), 0, st,
                     (int64_t)F_COUNT * np, B->flags.p, 0);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_b_dot<double>), dim3((unsigned)B->ntiles), dim3(kBlock), 0, st, n,
                     B->bs.p, B->bs.p, B->partA.p);
  RT_LAUNCH_CHECK();
  RT_CHECK(b_seg(ctx, B, BOP_BB, kTileRows, B->partA.p, nullptr, o->tol * o->tol));
  const int32_t* outer_done = B->flags.p + F_OUTER * np;
  const int rpb64 = spmv_rows_per_block(L, resid_shape(L));
  std::vector<int32_t> fl;
  bool all = false;
  int refine = 0;
  for (;;) {
    RT_CHECK((launch_spmv_level<double, SP_RESID>(st, L, L.val64.p, L.diag64.p, B->xs.p, B->bs.p,
                                                  nullptr, B->r64.p, mixed ? B->r32.p : nullptr,
                                                  B->partA.p, nullptr, resid_shape(L), B->tprob.p,
                                                  refine > 0 ? outer_done : nullptr)));
    RT_CHECK(b_seg(ctx, B, BOP_OUTER, rpb64, B->partA.p, nullptr, 0.0, mixed ? 1 : 0,
                   o->inner_tol));
    RT_CHECK(b_read_flags(ctx, B, F_OUTER, &fl, &all));
    if (all) break;
    if (!mixed) {
      RT_CHECK(b_pcg<double>(ctx, B, B->xs.p, B->r64.p, o->max_iter, graph_k, amg));
      break;   // the recursive residual decided convergence
    }
    if (refine >= o->max_refine) break;
    hipLaunchKernelGGL((k_b_zero<float>), dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->d32.p);
    RT_LAUNCH_CHECK();
    RT_CHECK(b_pcg<float>(ctx, B, B->d32.p, B->r32.p, o->max_iter, graph_k, amg));
    hipLaunchKernelGGL(k_b_add_f32, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->d32.p, B->xs.p);
    RT_LAUNCH_CHECK();
    ++refine;
  }
  // per-problem statistics
  std::vector<double> ps((size_t)B_COUNT * np);
  std::vector<int32_t> fh((size_t)F_COUNT * np);
  RT_CHECK_HIP(hipMemcpyAsync(ps.data(), B->ps.p, sizeof(double) * ps.size(),
                              hipMemcpyDeviceToHost, st));
  RT_CHECK_HIP(hipMemcpyAsync(fh.data(), B->flags.p, sizeof(int32_t) * fh.size(),
                              hipMemcpyDeviceToHost, st));
  RT_CHECK_HIP(hipStreamSynchronize(st));
  int status = RT_OK;
  for (int p = 0; p < np; ++p) {
    const double bb = ps[(size_t)B_BB * np + p], rr = ps[(size_t)B_RR * np + p];
    const bool conv = bb == 0.0 || rr <= ps[(size_t)B_THR2 * np + p];
    if (!conv) status = RT_NOT_CONVERGED;
    if (stats) {
      stats[p] = rt_solve_stats{};
      stats[p].iterations = fh[(size_t)F_ITS * np + p];
      stats[p].refinements = fh[(size_t)F_REFINE * np + p];
      stats[p].rel_residual = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    }
  }
  return status;
}

// The batch hierarchy from the problems' hierarchies (see rt_batch): level
// l >= 1 concatenates every problem's level l; level 0 (the batch's padded
// fine level) gains the l1 smoother scalings and, like every level above the
// last, the aggregate maps to the next (a problem whose hierarchy ends at l
// maps nothing: its rows there are smoothed only).  Built only when every
// problem's prolongations are piecewise constant; otherwise the batch keeps
// one level and its V-cycle is Jacobi.
int build_hierarchy(rt_ctx* ctx, rt_batch* B) {
  hipStream_t st = ctx->stream;
  const int np = B->nprob;
  rt_matrix* H = B->H.get();
  H->n = B->n;
  H->has_fp32 = B->fp32;
  // each problem contributes the levels its own V-cycle uses (its depth, as
  // set or tuned on its matrix), and is smoothed on the last of them
  int D = 1;
  for (rt_matrix* A : B->mats) {
    const int la = std::min<int>((int)cycle_depth(A), RT_MAX_LEVELS);
    for (int l = 0; l + 1 < la; ++l)
      if (A->levels[l].smoothed) return RT_OK;
    D = std::max(D, la);
  }
  H->amg = rt_amg_opts{D, 0, 0.0, B->fp32 ? 1 : 0, 0, RT_SMOOTHER_L1_JACOBI, 2, 1,
                       RT_PROLONG_PIECEWISE};
  H->coarse_direct = false;
  if (D == 1) return RT_OK;
  const bool fp32 = B->fp32;
  auto has = [&](int p, int l) { return (int)cycle_depth(B->mats[p]) > l; };
  // row and entry offsets per level (level 0: the padded fine rows)
  std::vector<std::vector<int64_t>> off(D, std::vector<int64_t>(np + 1, 0)),
      eoff(D, std::vector<int64_t>(np + 1, 0));
  off[0] = B->row_off;
  for (int l = 1; l < D; ++l)
    for (int p = 0; p < np; ++p) {
      off[l][p + 1] = off[l][p] + (has(p, l) ? B->mats[p]->levels[l].n : 0);
      eoff[l][p + 1] = eoff[l][p] + (has(p, l) ? B->mats[p]->levels[l].nnz : 0);
    }
  // level 0: l1 scalings (padding rows: 1, their residual is 0)
  Level& L0 = B->L;
  RT_CHECK(L0.sinv64.reserve(B->n));
  hipLaunchKernelGGL(k_bh_fill<double>, dim3(grid_for(B->n)), dim3(kBlock), 0, st, B->n,
                     L0.sinv64.p, 1.0);
  if (fp32) {
    RT_CHECK(L0.sinv32.reserve(B->n));
    hipLaunchKernelGGL(k_bh_fill<float>, dim3(grid_for(B->n)), dim3(kBlock), 0, st, B->n,
                       L0.sinv32.p, 1.0f);
  }
  RT_LAUNCH_CHECK();
  for (int p = 0; p < np; ++p) {
    const Level& S = B->mats[p]->levels[0];
    RT_CHECK_HIP(hipMemcpyAsync(L0.sinv64.p + off[0][p], S.sinv64.p, sizeof(double) * S.n,
                                hipMemcpyDeviceToDevice, st));
    if (fp32)
      RT_CHECK_HIP(hipMemcpyAsync(L0.sinv32.p + off[0][p], S.sinv32.p, sizeof(float) * S.n,
                                  hipMemcpyDeviceToDevice, st));
  }
  // coarse levels
  for (int l = 1; l < D; ++l) {
    H->levels.emplace_back();
    Level& C = H->levels.back();
    C.n = off[l][np];
    C.nnz = eoff[l][np];
    for (int p = 0; p < np; ++p)
      if (has(p, l)) C.max_row = std::max(C.max_row, B->mats[p]->levels[l].max_row);
    RT_CHECK(C.rp.reserve(C.n + 1));
    RT_CHECK(C.col.reserve(std::max<int64_t>(C.nnz, 1)));
    RT_CHECK(C.val64.reserve(C.nnz + kSpmvPad));
    for (auto* b : {&C.diag64, &C.sinv64, &C.dinv64}) RT_CHECK(b->reserve(C.n));
    if (fp32) {
      RT_CHECK(C.val32.reserve(C.nnz + kSpmvPad));
      for (auto* b : {&C.diag32, &C.sinv32, &C.dinv32}) RT_CHECK(b->reserve(C.n));
    }
    for (int p = 0; p < np; ++p) {
      if (!has(p, l)) continue;
      const Level& S = B->mats[p]->levels[l];
      const int64_t r0 = off[l][p], e0 = eoff[l][p];
      if (S.n > 0)
        hipLaunchKernelGGL(k_bh_rp, dim3(grid_for(S.n)), dim3(kBlock), 0, st, S.n, S.rp.p, e0,
                           C.rp.p + r0);
      if (S.nnz > 0)
        hipLaunchKernelGGL(k_b_copy_cols, dim3(grid_for(S.nnz)), dim3(kBlock), 0, st, S.nnz,
                           S.col.p, e0, r0, C.col.p);
      RT_LAUNCH_CHECK();
      auto cp = [&](void* dst, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
      };
      RT_CHECK_HIP(cp(C.val64.p + e0, S.val64.p, sizeof(double) * S.nnz));
      RT_CHECK_HIP(cp(C.diag64.p + r0, S.diag64.p, sizeof(double) * S.n));
      RT_CHECK_HIP(cp(C.sinv64.p + r0, S.sinv64.p, sizeof(double) * S.n));
      RT_CHECK_HIP(cp(C.dinv64.p + r0, S.dinv64.p, sizeof(double) * S.n));
      if (fp32) {
        RT_CHECK_HIP(cp(C.val32.p + e0, S.val32.p, sizeof(float) * S.nnz));
        RT_CHECK_HIP(cp(C.diag32.p + r0, S.diag32.p, sizeof(float) * S.n));
        RT_CHECK_HIP(cp(C.sinv32.p + r0, S.sinv32.p, sizeof(float) * S.n));
        RT_CHECK_HIP(cp(C.dinv32.p + r0, S.dinv32.p, sizeof(float) * S.n));
      }
    }
    hipLaunchKernelGGL(k_b_set_i64, dim3(1), dim3(1), 0, st, C.rp.p + C.n, C.nnz);
    RT_LAUNCH_CHECK();
  }
  // aggregate maps from level l to l + 1
  for (int l = 0; l + 1 < D; ++l) {
    Level& F = H->levels[l];
    const int64_t nc = H->levels[l + 1].n;
    RT_CHECK(F.pmap.reserve(std::max<int64_t>(F.n, 1)));
    hipLaunchKernelGGL(k_b_fill_i32, dim3(grid_for(F.n)), dim3(kBlock), 0, st, F.n, F.pmap.p, -1);
    RT_LAUNCH_CHECK();
    // members per problem: the last offset of its own map
    std::vector<int64_t> members(np, 0), moff(np + 1, 0);
    for (int p = 0; p < np; ++p) {
      if (has(p, l + 1)) {
        const Level& S = B->mats[p]->levels[l];
        RT_CHECK(ctx->sync_read(S.crange.p + B->mats[p]->levels[l + 1].n, sizeof(int64_t)));
        std::memcpy(&members[p], ctx->host, sizeof(int64_t));
      }
      moff[p + 1] = moff[p] + members[p];
    }
    RT_CHECK(F.crange.reserve(nc + 1));
    RT_CHECK(F.amem.reserve(std::max<int64_t>(moff[np], 1)));
    for (int p = 0; p < np; ++p) {
      if (!has(p, l + 1)) continue;
      const Level& S = B->mats[p]->levels[l];
      const int64_t ncp = B->mats[p]->levels[l + 1].n;
      if (S.n > 0)
        hipLaunchKernelGGL(k_bh_pmap, dim3(grid_for(S.n)), dim3(kBlock), 0, st, S.n, S.pmap.p,
                           off[l + 1][p], F.pmap.p + off[l][p]);
      if (ncp > 0)
        hipLaunchKernelGGL(k_bh_crange, dim3(grid_for(ncp)), dim3(kBlock), 0, st, ncp,
                           S.crange.p, moff[p], F.crange.p + off[l + 1][p]);
      if (members[p] > 0)
        hipLaunchKernelGGL(k_b_copy_cols, dim3(grid_for(members[p])), dim3(kBlock), 0, st,
                           members[p], S.amem.p, moff[p], off[l][p], F.amem.p);
      RT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_b_set_i64, dim3(1), dim3(1), 0, st, F.crange.p + nc, moff[np]);
    RT_LAUNCH_CHECK();
    F.smoothed = false;
  }
  for (Level& L : H->levels) RT_CHECK(amg_level_vectors(L, fp32, 1));
  RT_CHECK(B->z64.reserve(B->n));
  if (fp32) RT_CHECK(B->z32.reserve(B->n));
  // The V-cycle's products and vector passes skip the rows of problems whose
  // inner iteration has stopped: on the fine level by tile (one problem
  // each), on a coarse level by 256-row chunk once every problem with rows
  // in the chunk has stopped (k_b_chunk_done before each V-cycle).  Skipped
  // rows of a level's vectors keep the last value written (zero before the
  // first), and the levels, block-diagonal, carry them only into rows of the
  // same stopped problems, which no update reads.
  const int32_t* done = B->flags.p + F_INNER * np;
  std::vector<int32_t> rng;
  std::vector<int64_t> choff(D, 0);
  int64_t maxch = 0;
  for (int l = 1; l < D; ++l) {
    const int64_t n = H->levels[l].n, nch = (n + kTileRows - 1) / kTileRows;
    choff[l] = (int64_t)rng.size() / 2;
    maxch = std::max(maxch, nch);
    for (int64_t c = 0; c < nch; ++c) {
      // problems owning the chunk's first and last rows (empty ones own none)
      const int64_t a = c * kTileRows, z = std::min(n, a + kTileRows) - 1;
      const auto& o = off[l];
      rng.push_back((int32_t)(std::upper_bound(o.begin(), o.end(), a) - o.begin() - 1));
      rng.push_back((int32_t)(std::upper_bound(o.begin(), o.end(), z) - o.begin() - 1));
    }
  }
  B->nchunks = (int64_t)rng.size() / 2;
  RT_CHECK(B->crng.reserve(std::max<size_t>(rng.size(), 2)));
  RT_CHECK(B->cdone.reserve(std::max<int64_t>(B->nchunks, 1)));
  RT_CHECK(B->ciota.reserve(std::max<int64_t>(maxch, 1)));
  if (!rng.empty())
    RT_CHECK_HIP(hipMemcpyAsync(B->crng.p, rng.data(), sizeof(int32_t) * rng.size(),
                                hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_b_iota, dim3(grid_for(std::max<int64_t>(maxch, 1))), dim3(kBlock), 0, st,
                     maxch, B->ciota.p);
  hipLaunchKernelGGL(k_b_fill_i32, dim3(grid_for(std::max<int64_t>(B->nchunks, 1))), dim3(kBlock),
                     0, st, B->nchunks, B->cdone.p, 0);
  RT_LAUNCH_CHECK();
  H->lvl_tprob.assign(D, B->ciota.p);
  H->lvl_skip.assign(D, nullptr);
  H->lvl_tprob[0] = B->tprob.p;
  H->lvl_skip[0] = done;
  for (int l = 1; l < D; ++l) H->lvl_skip[l] = B->cdone.p + choff[l];
  for (int l = 0; l < D; ++l) {
    Level& V = H->levels[l];
    for (double* q : {V.r64.p, V.x64.p, V.t64.p, V.b64.p})
      hipLaunchKernelGGL(k_bh_fill<double>, dim3(grid_for(V.n)), dim3(kBlock), 0, st, V.n, q, 0.0);
    if (fp32)
      for (float* q : {V.r32.p, V.x32.p, V.t32.p, V.b32.p})
        hipLaunchKernelGGL(k_bh_fill<float>, dim3(grid_for(V.n)), dim3(kBlock), 0, st, V.n, q,
                           0.0f);
  }
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipStreamSynchronize(st));
  return RT_OK;
}

}  // namespace
}  // namespace rt

extern "C" {

int rt_batch_create(rt_ctx* ctx, int nprob, rt_matrix* const* mats, rt_batch** out) {
  using namespace rt;
  clear_error();
  if (!ctx || !out || nprob < 1 || !mats) {
    set_error("rt_batch_create: NULL argument or nprob < 1");
    return RT_E_ARG;
  }
  *out = nullptr;
  bool fp32 = true;
  for (int p = 0; p < nprob; ++p) {
    if (!mats[p] || mats[p]->levels.empty()) {
      set_error("rt_batch_create: matrix %d is NULL or not assembled", p);
      return RT_E_ARG;
    }
    fp32 = fp32 && mats[p]->has_fp32;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  hipStream_t st = ctx->stream;
  rt_batch* B = new rt_batch();
  B->nprob = nprob;
  B->mats.assign(mats, mats + nprob);
  B->fp32 = fp32;
  B->row_off.assign(nprob + 1, 0);
  B->uoff.assign(nprob + 1, 0);
  std::vector<int64_t> nnz_off(nprob + 1, 0);
  int64_t max_row = 0;
  for (int p = 0; p < nprob; ++p) {
    const rt_matrix* A = mats[p];
    B->row_off[p + 1] = B->row_off[p] + pad_rows(A->n);
    B->uoff[p + 1] = B->uoff[p] + A->n;
    nnz_off[p + 1] = nnz_off[p] + A->levels[0].nnz;
    max_row = std::max(max_row, A->levels[0].max_row);
  }
  B->n = B->row_off[nprob];
  B->nuser = B->uoff[nprob];
  B->ntiles = B->n / kTileRows;
  if (B->n >= ((int64_t)1 << 31) || nnz_off[nprob] >= ((int64_t)1 << 31)) {
    delete B;
    set_error("rt_batch_create: the ensemble exceeds the int32 index range");
    return RT_E_ARG;
  }
  Level& L = B->L;
  L.n = B->n;
  L.nnz = nnz_off[nprob];
  L.max_row = max_row;
  auto fail = [&](int s) {
    delete B;
    return s;
  };
  const int64_t n = B->n;
  int s = RT_OK;
#define RT_B(expr)      \
  do {                  \
    s = (expr);         \
    if (s < 0) return fail(s); \
  } while (0)
  RT_B(L.rp.reserve(n + 1));
  RT_B(L.col.reserve(std::max<int64_t>(L.nnz, 1)));
  RT_B(L.val64.reserve(L.nnz + kSpmvPad));
  RT_B(L.diag64.reserve(n));
  RT_B(L.dinv64.reserve(n));
  if (fp32) {
    RT_B(L.val32.reserve(L.nnz + kSpmvPad));
    RT_B(L.diag32.reserve(n));
    RT_B(L.dinv32.reserve(n));
  }
  for (auto* b : {&B->V, &B->sa, &B->f, &B->rho, &B->cv, &B->m, &B->e_prev, &B->E_prev, &B->Qe,
                  &B->QE, &B->g, &B->ecur, &B->Ecur, &B->enew, &B->xs, &B->bs, &B->r64, &B->p64,
                  &B->q64})
    RT_B(b->reserve(n));
  if (fp32)
    for (auto* b : {&B->r32, &B->p32, &B->q32, &B->d32}) RT_B(b->reserve(n));
  RT_B(B->perm.reserve(n));
  RT_B(B->tprob.reserve(B->ntiles));
  RT_B(B->d_row_off.reserve(nprob + 1));
  RT_B(B->partA.reserve(max_partials(n)));
  RT_B(B->partB.reserve(max_partials(n)));
  RT_B(B->ps.reserve((size_t)B_COUNT * nprob));
  RT_B(B->flags.reserve((size_t)F_COUNT * nprob));
  RT_B(B->mres.reserve(std::max<int64_t>((int64_t)M_WIDTH * B->ntiles, (int64_t)M_WIDTH * nprob)));
  RT_B(B->pdt.reserve(nprob));
  RT_B(B->pc.reserve(nprob));
  RT_B(B->pa.reserve(nprob));
  std::vector<int32_t> tp(B->ntiles);
  std::vector<double> hdt(nprob), hc(nprob), ha(nprob);
  for (int p = 0; p < nprob; ++p) {
    for (int64_t t = B->row_off[p] / kTileRows; t < B->row_off[p + 1] / kTileRows; ++t)
      tp[t] = p;
    hdt[p] = mats[p]->dt;
    hc[p] = mats[p]->c;
    ha[p] = mats[p]->a;
  }
  // host buffers must outlive the asynchronous copies: synchronise below
  if (hipMemcpyAsync(B->tprob.p, tp.data(), sizeof(int32_t) * tp.size(), hipMemcpyHostToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(B->d_row_off.p, B->row_off.data(), sizeof(int64_t) * (nprob + 1),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(B->pdt.p, hdt.data(), sizeof(double) * nprob, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(B->pc.p, hc.data(), sizeof(double) * nprob, hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(B->pa.p, ha.data(), sizeof(double) * nprob, hipMemcpyHostToDevice, st) !=
          hipSuccess) {
    set_error("rt_batch_create: host-to-device copy failed");
    return fail(RT_E_DEVICE);
  }
  for (int p = 0; p < nprob; ++p) {
    rt_matrix* A = mats[p];
    const Level& S = A->levels[0];
    CopyArgs ca{S.rp.p, S.diag64.p, S.dinv64.p, A->V.p, A->sa.p, A->f.p, A->rho.p, A->cv.p,
                A->m.p, A->e_prev.p, A->E_prev.p, A->Qe.p, A->QE.p, A->g.p,
                fp32 ? S.diag32.p : nullptr, fp32 ? S.dinv32.p : nullptr, A->nb->perm.p,
                A->n, B->row_off[p + 1] - B->row_off[p], B->row_off[p], nnz_off[p],
                nnz_off[p + 1], B->uoff[p], L.rp.p, L.diag64.p, L.dinv64.p, B->V.p, B->sa.p,
                B->f.p, B->rho.p, B->cv.p, B->m.p, B->e_prev.p, B->E_prev.p, B->Qe.p, B->QE.p,
                B->g.p, fp32 ? L.diag32.p : nullptr, fp32 ? L.dinv32.p : nullptr, B->perm.p};
    hipLaunchKernelGGL(k_b_copy_rows, dim3(grid_for(ca.nrows)), dim3(kBlock), 0, st, ca);
    if (hipGetLastError() != hipSuccess) {
      set_error("rt_batch_create: launch failed");
      return fail(RT_E_DEVICE);
    }
    if (S.nnz > 0) {
      hipLaunchKernelGGL(k_b_copy_cols, dim3(grid_for(S.nnz)), dim3(kBlock), 0, st, S.nnz,
                         S.col.p, nnz_off[p], B->row_off[p], L.col.p);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(L.val64.p + nnz_off[p], S.val64.p, sizeof(double) * S.nnz,
                         hipMemcpyDeviceToDevice, st) != hipSuccess ||
          (fp32 && hipMemcpyAsync(L.val32.p + nnz_off[p], S.val32.p, sizeof(float) * S.nnz,
                                  hipMemcpyDeviceToDevice, st) != hipSuccess)) {
        set_error("rt_batch_create: copy of problem %d failed", p);
        return fail(RT_E_DEVICE);
      }
    }
  }
  hipLaunchKernelGGL(k_b_set_i64, dim3(1), dim3(1), 0, st, L.rp.p + n, L.nnz);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    set_error("rt_batch_create: device error");
    return fail(RT_E_DEVICE);
  }
  RT_B(build_tiles(ctx, L));
  RT_B(build_hierarchy(ctx, B));
#undef RT_B
  *out = B;
  return RT_OK;
}

void rt_batch_free(rt_batch* B) {
  if (!B) return;
  rt::IdleScope idle;   // one wait for the device, then every buffer goes back to the cache
  delete B;
}

int rt_batch_get_info(const rt_batch* B, int64_t* rows, int64_t* nnz, int64_t* tile_cols) {
  rt::clear_error();
  if (!B) {
    rt::set_error("rt_batch_get_info: NULL batch");
    return RT_E_ARG;
  }
  if (rows) *rows = B->n;
  if (nnz) *nnz = B->L.nnz;
  if (tile_cols) *tile_cols = B->L.tiled ? B->L.tile_cols_total : 0;
  return RT_OK;
}

int rt_batch_tune(rt_ctx* ctx, rt_batch* B, int reps, rt_tune_report* rep) {
  rt::clear_error();
  if (!ctx || !B) {
    rt::set_error("rt_batch_tune: NULL argument");
    return RT_E_ARG;
  }
  // the batch's hierarchy is an ordinary operator: every level is tuned
  const int s = rt_matrix_tune(ctx, B->H.get(), reps, rep);
  for (auto& g : B->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  return s;
}

int rt_batch_set_spmv_shape(rt_batch* B, int precision, int shape) {
  using namespace rt;
  clear_error();
  if (!B || (precision != RT_PREC_FP64 && precision != RT_PREC_MIXED &&
             precision != RT_PRODUCT_RESIDUAL) || shape < -1 || shape >= kNumSpmvShapes) {
    set_error("rt_batch_set_spmv_shape: bad batch, precision or shape");
    return RT_E_ARG;
  }
  if (precision == RT_PRODUCT_RESIDUAL) {   // not part of the replayed PCG graphs
    B->L.shape_res = shape;
    return RT_OK;
  }
  (precision == RT_PREC_FP64 ? B->L.shape64 : B->L.shape32) = shape;
  const int slot = precision == RT_PREC_FP64 ? 0 : 1;
  if (B->graph[slot]) {   // the graph holds the launches of the previous shape
    (void)hipGraphExecDestroy(B->graph[slot]);
    B->graph[slot] = nullptr;
  }
  return RT_OK;
}

int rt_batch_set_cycle_depth(rt_batch* B, int depth) {
  rt::clear_error();
  if (!B || depth < 0) {
    rt::set_error("rt_batch_set_cycle_depth: NULL batch or negative depth");
    return RT_E_ARG;
  }
  B->H->cycle_levels = depth;
  for (auto& g : B->graph)   // graphs hold the launches of the previous depth
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  return RT_OK;
}

int rt_batch_tune_depth(rt_ctx* ctx, rt_batch* B, const double* b, const double* x0,
                        const rt_solve_opts* opts, int graph_iters, int reps,
                        rt_depth_report* rep) {
  using namespace rt;
  clear_error();
  if (!ctx || !B || !opts || !b || !x0 || reps < 1) {
    set_error("rt_batch_tune_depth: NULL argument or reps < 1");
    return RT_E_ARG;
  }
  if (opts->precond != 1) {
    set_error("rt_batch_tune_depth: the solve options must use the V-cycle (precond 1)");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt_depth_report local{};
  rt_depth_report* r = rep ? rep : &local;
  *r = rt_depth_report{};
  const int nl = std::min<int>((int)B->H->levels.size(), RT_MAX_LEVELS);
  r->depths = nl;
  r->chosen = nl;
  if (nl <= 1 || B->nuser == 0) return RT_OK;
  DevBuf<double> x;
  {
    rt::StreamScope scope(ctx->stream);
    RT_CHECK(x.reserve(B->nuser));
  }
  std::vector<rt_solve_stats> st(B->nprob);
  const int keep = B->H->cycle_levels;
  double best = 0.0;
  int arg = -1;
  for (int d = 1; d <= nl; ++d) {
    RT_CHECK(rt_batch_set_cycle_depth(B, d));
    double total = 0.0;
    int status = RT_OK, its = 0;
    for (int k = 0; k <= reps; ++k) {   // the first run (graph capture) is not timed
      RT_CHECK_HIP(hipMemcpyAsync(x.p, x0, sizeof(double) * B->nuser, hipMemcpyDeviceToDevice,
                                  ctx->stream));
      RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
      const auto t0 = std::chrono::steady_clock::now();
      const int s = rt_batch_solve(ctx, B, b, x.p, opts, graph_iters, st.data());
      RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
      const double sec =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (s < 0) {
        (void)rt_batch_set_cycle_depth(B, keep);
        return s;
      }
      if (k == 0) continue;
      if (s == RT_NOT_CONVERGED) status = RT_NOT_CONVERGED;
      total += sec;
      its = 0;
      for (const rt_solve_stats& q : st) its = std::max(its, q.iterations);
    }
    r->seconds[d - 1] = total / reps;
    r->iterations[d - 1] = its;
    r->status[d - 1] = status;
    if (status == RT_OK && (arg < 0 || r->seconds[d - 1] < best)) {
      best = r->seconds[d - 1];
      arg = d;
    }
  }
  clear_error();   // a depth that did not converge is only left out
  r->chosen = arg > 0 ? arg : nl;
  return rt_batch_set_cycle_depth(B, r->chosen == nl ? 0 : r->chosen);
}

int rt_batch_solve(rt_ctx* ctx, rt_batch* B, const double* b, double* x, const rt_solve_opts* opts,
                   int graph_iters, rt_solve_stats* stats) {
  using namespace rt;
  clear_error();
  if (!ctx || !B || !b || !x) {
    set_error("rt_batch_solve: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK(check_solve_opts(opts));
  if (opts->cw_tol != 0.0) {
    set_error("rt_batch_solve: batched solves use the normwise test only (cw_tol 0)");
    return RT_E_ARG;
  }
  if (opts->precision == RT_PREC_MIXED && !B->fp32) {
    set_error("rt_batch_solve: mixed precision needs FP32 copies in every matrix");
    return RT_E_STATE;
  }
  if (graph_iters < 0) {
    set_error("rt_batch_solve: graph_iters must be >= 0");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  hipStream_t st = ctx->stream;
  const int64_t n = B->n;
  hipLaunchKernelGGL(k_b_gather, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, b, B->bs.p);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_b_gather, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, x, B->xs.p);
  RT_LAUNCH_CHECK();
  const int s = b_solve(ctx, B, opts, graph_iters, stats);
  if (s < 0) return s;
  hipLaunchKernelGGL(k_b_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, B->xs.p, x);
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipStreamSynchronize(st));
  if (s == RT_NOT_CONVERGED) set_error("rt_batch_solve: a problem did not reach its tolerance");
  return s;
}

int rt_batch_newton_step(rt_ctx* ctx, rt_batch* B, double* e, double* E, int ell,
                         const rt_newton_opts* opts, int graph_iters, rt_newton_stats* stats) {
  using namespace rt;
  clear_error();
  if (!ctx || !B || !e || !E || !opts) {
    set_error("rt_batch_newton_step: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK(check_solve_opts(&opts->solve));
  if (opts->solve.cw_tol != 0.0) {
    set_error("rt_batch_newton_step: batched solves use the normwise test only (cw_tol 0)");
    return RT_E_ARG;
  }
  if (opts->solve.precision == RT_PREC_MIXED && !B->fp32) {
    set_error("rt_batch_newton_step: mixed precision needs FP32 copies in every matrix");
    return RT_E_STATE;
  }
  if (!(opts->material_tol > 0.0) || opts->material_max_iter < 1 || graph_iters < 0 ||
      opts->state_order != 0) {
    set_error("rt_batch_newton_step: invalid material options, graph_iters or state_order "
              "(batches take user order)");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  hipStream_t st = ctx->stream;
  const int64_t n = B->n;
  const int np = B->nprob;
  hipLaunchKernelGGL(k_b_gather, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, e, B->ecur.p);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_b_gather, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, E, B->Ecur.p);
  RT_LAUNCH_CHECK();
  const unsigned nt = (unsigned)B->ntiles;
  std::vector<double> res((size_t)M_WIDTH * np);
  std::vector<int> status_p(np, RT_OK);
  auto material = [&](const double* Enew, const double* Eold, const double* estart,
                      double* eout) -> int {
    BMat ma{B->tprob.p, B->perm.p, B->pdt.p, B->pc.p, B->pa.p, B->e_prev.p, B->rho.p, B->cv.p,
            B->sa.p, B->Qe.p, B->m.p, B->V.p, B->E_prev.p, Enew, Eold, estart, eout,
            opts->material_tol, opts->material_max_iter};
    hipLaunchKernelGGL(k_b_material, dim3(nt), dim3(kBlock), 0, st, n, ma, B->mres.p);
    RT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_b_material_seg, dim3(np), dim3(kBlock), 0, st, np, B->d_row_off.p,
                       B->mres.p, B->partB.p);
    RT_LAUNCH_CHECK();
    RT_CHECK_HIP(hipMemcpyAsync(res.data(), B->partB.p, sizeof(double) * res.size(),
                                hipMemcpyDeviceToHost, st));
    RT_CHECK_HIP(hipStreamSynchronize(st));
    return RT_OK;
  };
  if (ell == 0) {
    // initial material solve with E^{n,0} (Algorithm 1, before the loop)
    RT_CHECK(material(B->Ecur.p, B->Ecur.p, B->e_prev.p, B->ecur.p));
    for (int p = 0; p < np; ++p) {
      if (res[(size_t)p * M_WIDTH + M_BAD] > 0) status_p[p] = RT_NOT_CONVERGED;
      if (res[(size_t)p * M_WIDTH + M_NONPHYS] > 0) status_p[p] = RT_NONPHYSICAL;
    }
  }
  BRhs ra{B->tprob.p, B->pdt.p, B->pc.p, B->pa.p, B->V.p, B->sa.p, B->f.p, B->cv.p, B->E_prev.p,
          B->QE.p, B->g.p, B->ecur.p, B->Ecur.p, B->bs.p};
  hipLaunchKernelGGL(k_b_rhs, dim3(grid_for(n)), dim3(kBlock), 0, st, n, ra);
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipMemcpyAsync(B->xs.p, B->Ecur.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  std::vector<rt_solve_stats> sst(np);
  const int ss = b_solve(ctx, B, &opts->solve, graph_iters, sst.data());
  if (ss < 0) return ss;
  RT_CHECK(material(B->xs.p, B->Ecur.p, B->ecur.p, B->enew.p));
  hipLaunchKernelGGL(k_b_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, B->enew.p, e);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_b_scatter, dim3(grid_for(n)), dim3(kBlock), 0, st, n, B->perm.p, B->xs.p, E);
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipStreamSynchronize(st));
  int status = RT_OK;
  for (int p = 0; p < np; ++p) {
    const double* r = &res[(size_t)p * M_WIDTH];
    if (sst[p].rel_residual > opts->solve.tol && status_p[p] == RT_OK)
      status_p[p] = RT_NOT_CONVERGED;
    if (r[M_BAD] > 0 && status_p[p] == RT_OK) status_p[p] = RT_NOT_CONVERGED;
    if (r[M_NONPHYS] > 0) status_p[p] = RT_NONPHYSICAL;
    status = std::max(status, status_p[p]);
    if (stats) {
      stats[p] = rt_newton_stats{};
      stats[p].delta_e = r[M_DE];
      stats[p].delta_E = r[M_DEE];
      stats[p].material_iterations = (int)r[M_ITS];
      stats[p].nonphysical = (int64_t)r[M_NONPHYS];
      stats[p].energy = r[M_EN];
      stats[p].energy_prev = r[M_EN0];
      stats[p].solve = sst[p];
    }
  }
  if (status == RT_NONPHYSICAL) set_error("rt_batch_newton_step: negative material roots");
  else if (status == RT_NOT_CONVERGED)
    set_error("rt_batch_newton_step: a solve or material update did not converge");
  return status;
}

}  // extern "C"

// Per-step frozen data and assembly of the V-scaled Brookshaw diffusion system.
//
// Frozen data (Sec. 3.2: computed once at the start of the step), per sorted
// particle: T = e/c_v, sigma_a = sigma0_a T^p, sigma_t = sigma_a + sigma_s,
// Fleck factor f = 1/(1 + c sigma_a dt 4 a T^3/(rho c_v)) (Sec. 2.2),
// V = m/rho (Sec. 2.3), D = c lambda/sigma_t (Sec. 2.4).  With a flux limiter
// (Sec. 2.1) lambda of the interior particles uses R = |grad E|/(sigma_t E)
// with the SPH first derivative of E^{n-1} (Sec. 2.3).
//
// Matrix (the D^-1 operator of Sec. 3.2 with row i multiplied by V_i):
//   F_ij = -1/2 [W'(r,h_i) + W'(r,h_j)] / r,  a_ij = V_j (D_i + D_j) F_ij
//   A_ij = -(V_i V_j)(D_i + D_j) F_ij      (interior j, off-diagonal CSR)
//   A_ii = V_i (1/dt + c sigma_a,i f_i) + V_i sum_j a_ij
//   g_i  = V_i sum_{j ghost} a_ij E_j      (ghost coupling -> right-hand side)
// One group of G lanes per row: lanes walk the row's neighbours, so reads of
// the neighbour list and writes of the values are contiguous.
#include <cmath>
#include <cstring>

#include "internal.h"
#include "kernels_sph.h"
#include "prim.h"
#include "reduce.h"
#include "spmv.h"

namespace rt {
namespace {

struct FrozenArgs {
  const int32_t* perm;
  const double* rec;   // per-particle input records in user order (k_pack_inputs)
  const double* ss;
  double dt, c, a, p;
  double *V, *D, *sa, *st, *f, *Eall, *e_prev, *E_prev, *rho_s, *cv_s, *m_s, *Qe_s, *QE_s;
  double* VD;
};

// The caller's per-particle inputs, read in user order (coalesced) and
// packed into one 64-byte record per particle, (c_v, rho, e, E, sigma_0, m,
// Q_e, Q_E); the sorted-order pass then gathers one record instead of eight
// scattered values.
__global__ void k_pack_inputs(int64_t n, const double* __restrict__ cv,
                              const double* __restrict__ rho, const double* __restrict__ e,
                              const double* __restrict__ E, const double* __restrict__ s0,
                              const double* __restrict__ m, const double* __restrict__ Qe,
                              const double* __restrict__ Qn, double* __restrict__ rec) {
  int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= n) return;
  rt_f64x2_t* out = reinterpret_cast<rt_f64x2_t*>(rec + 8 * u);
  out[0] = rt_f64x2_t{cv[u], rho[u]};
  out[1] = rt_f64x2_t{e[u], E[u]};
  out[2] = rt_f64x2_t{s0[u], m[u]};
  out[3] = rt_f64x2_t{Qe ? Qe[u] : 0.0, Qn ? Qn[u] : 0.0};
}

__global__ void k_frozen(int64_t n, int64_t nin, FrozenArgs A) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t u = A.perm[s];
  const rt_f64x2_t* in = reinterpret_cast<const rt_f64x2_t*>(A.rec + 8 * (int64_t)u);
  const rt_f64x2_t r0 = in[0], r1 = in[1], r2 = in[2], r3 = in[3];
  const double cv = r0[0], rho = r0[1], e = r1[0], E = r1[1];
  const double s0 = r2[0], m = r2[1];
  const double T = e / cv;
  const double sa = A.p == 0.0 ? s0 : s0 * pow(T, A.p);
  const double st = sa + (A.ss ? A.ss[u] : 0.0);
  const double f = 1.0 / (1.0 + A.c * sa * A.dt * 4.0 * A.a * (T * T * T) / (rho * cv));
  const double V = m / rho;
  const double D = A.c * (1.0 / 3.0) / st;
  A.V[s] = V;
  A.sa[s] = sa;
  A.st[s] = st;
  A.f[s] = f;
  A.D[s] = D;
  A.VD[2 * s] = V;
  A.VD[2 * s + 1] = D;
  A.Eall[s] = E;
  if (s < nin) {
    A.e_prev[s] = e;
    A.E_prev[s] = E;
    A.rho_s[s] = rho;
    A.cv_s[s] = cv;
    A.m_s[s] = m;
    A.Qe_s[s] = r3[0];
    A.QE_s[s] = r3[1];
  }
}

// Flux-limited diffusion coefficient of interior particles.  One group of G
// lanes per row, ENT neighbour entries per lane requested before any
// arithmetic, and each XCD on one contiguous range of rows, as in the
// assembly; the gradient's three components are summed over the group.
template <int DIM, int G, int ENT>
__global__ void __launch_bounds__(kBlock)
k_limiter(int64_t nin, int kernel, int limiter, double lk, double c,
          const double* __restrict__ sp4, const int64_t* __restrict__ nptr,
          const int32_t* __restrict__ nidx, const double* __restrict__ V,
          const double* __restrict__ Eall, const double* __restrict__ st,
          double* __restrict__ D, double* __restrict__ VD, PeriodicBox box, int per) {
  const int lane = threadIdx.x & (G - 1);
  const int64_t i = ((int64_t)xcd_block(per) * kBlock + threadIdx.x) / G;
  if (i >= nin) return;   // whole groups leave together
  const Rec4 pi = load_rec4(sp4, i);
  const double xi = pi.x, yi = pi.y, zi = pi.z;
  const double hi = pi.h, Ei = Eall[i];
  const int64_t k0 = nptr[i], k1 = nptr[i + 1];
  double gx = 0, gy = 0, gz = 0;
  for (int64_t kb = k0 + lane; kb < k1; kb += G * ENT) {
    int32_t j[ENT];
#pragma unroll
    for (int e = 0; e < ENT; ++e) {
      const int64_t k = kb + e * G;
      j[e] = nidx[k < k1 ? k : k1 - 1];
    }
    Rec4 pj[ENT];
    double vj[ENT], ej[ENT];
#pragma unroll
    for (int e = 0; e < ENT; ++e) {
      pj[e] = load_rec4(sp4, j[e]);
      vj[e] = V[j[e]];
      ej[e] = Eall[j[e]];
    }
#pragma unroll
    for (int e = 0; e < ENT; ++e) {
      if (kb + e * G >= k1) break;
      // nearest images on periodic axes (the pair is within one support)
      const double dx = periodic_disp(xi - pj[e].x, box, 0);
      const double dy = periodic_disp(yi - pj[e].y, box, 1);
      const double dz = DIM == 3 ? periodic_disp(zi - pj[e].z, box, 2) : 0.0;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      // grad_i W_ij = 1/2 [W'(r,h_i) + W'(r,h_j)] x_ij / r
      const double w = vj[e] * (ej[e] - Ei) * 0.5 *
                       (sph_dwdr<DIM>(r, hi, kernel) + sph_dwdr<DIM>(r, pj[e].h, kernel)) / r;
      gx += w * dx;
      gy += w * dy;
      gz += w * dz;
    }
  }
  gx = group_sum<G>(gx);
  gy = group_sum<G>(gy);
  if (DIM == 3) gz = group_sum<G>(gz);
  if (lane != 0) return;
  // R = |grad E|/(sigma_t E); no gradient is the diffusion limit (R = 0, also
  // where E = 0), a gradient where E <= 0 the free-streaming limit (R = inf)
  const double gn = sqrt(gx * gx + gy * gy + gz * gz);
  const double den = st[i] * Ei;
  const double R = gn == 0.0 ? 0.0 : (den > 0.0 ? gn / den : INFINITY);
  double lam;
  if (limiter == RT_LIMITER_LARSEN) {
    lam = pow(pow(3.0, lk) + pow(R, lk), -1.0 / lk);
  } else if (R <= 1.0) {
    lam = (2.0 + R) / (6.0 + 3.0 * R + R * R);
  } else {   // the same quotient in u = 1/R, finite for any R
    const double u = 1.0 / R;
    lam = u * (1.0 + 2.0 * u) / (1.0 + 3.0 * u + 6.0 * u * u);
  }
  D[i] = c * lam / st[i];
  VD[2 * i + 1] = D[i];
}

__global__ void k_int_counts(int64_t nin, const int32_t* __restrict__ cnt32,
                             int64_t* __restrict__ cnt64) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nin) cnt64[i] = cnt32[i];
}

struct AsmArgs {
  const int64_t *nptr, *rp;
  const int32_t* nidx;
  const double *sp4, *VD, *sa, *f, *Eall;
  int32_t* col;                       // written when the structure is new, else NULL
  double *val64, *diag64, *dinv64, *sinv64, *g;
  float *val32, *diag32, *dinv32, *sinv32;
  PeriodicBox box;                    // periodic axes of the neighbour lists
};

// One group of G lanes per row, ENT neighbour entries per lane: the entry
// indices, the neighbours' (x, y, z, h) and (V, D) records of a lane are all
// requested before any arithmetic, so a row waits on memory about three
// times whatever its length (rows longer than G*ENT take further passes).
template <int DIM, int G, int ENT>
__global__ void __launch_bounds__(kBlock)
k_assemble(int64_t nin, int64_t n, int kernel, double dt, double c, AsmArgs A, int per) {
  const int lane = threadIdx.x & (G - 1);
  // each XCD takes one contiguous range of rows, so that the neighbour records
  // its rows gather stay in its own L2
  const int64_t i = ((int64_t)xcd_block(per) * kBlock + threadIdx.x) / G;
  if (i >= nin) return;   // whole groups leave together
  const Rec4 pi = load_rec4(A.sp4, i);
  const rt_f64x2_t vdi = load_pair(A.VD, i);
  const double xi = pi.x, yi = pi.y, zi = pi.z;
  const double hi = pi.h, Vi = vdi[0], Di = vdi[1];
  const int64_t k0 = A.nptr[i], k1 = A.nptr[i + 1], o = A.rp[i];
  double suma = 0.0, gsum = 0.0, absoff = 0.0;
  for (int64_t kb = k0 + lane; kb < k1; kb += G * ENT) {
    int32_t j[ENT];
#pragma unroll
    for (int e = 0; e < ENT; ++e) {
      const int64_t k = kb + e * G;
      j[e] = A.nidx[k < k1 ? k : k1 - 1];
    }
    Rec4 pj[ENT];
    rt_f64x2_t vdj[ENT];
#pragma unroll
    for (int e = 0; e < ENT; ++e) {
      pj[e] = load_rec4(A.sp4, j[e]);
      vdj[e] = load_pair(A.VD, j[e]);
    }
#pragma unroll
    for (int e = 0; e < ENT; ++e) {
      const int64_t k = kb + e * G;
      if (k >= k1) break;
      const double dx = periodic_disp(xi - pj[e].x, A.box, 0);
      const double dy = periodic_disp(yi - pj[e].y, A.box, 1);
      const double dz = DIM == 3 ? periodic_disp(zi - pj[e].z, A.box, 2) : 0.0;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      // equal smoothing lengths give equal kernel derivatives: evaluate once
      const double wi = sph_dwdr<DIM>(r, hi, kernel);
      const double wj = pj[e].h == hi ? wi : sph_dwdr<DIM>(r, pj[e].h, kernel);
      const double F = -0.5 * (wi + wj) / r;
      const double Dij = Di + vdj[e][1];
      const double aij = vdj[e][0] * Dij * F;
      suma += aij;
      if (j[e] < nin) {
        const double v = -(Vi * vdj[e][0]) * Dij * F;
        A.val64[o + (k - k0)] = v;
        if (A.val32) A.val32[o + (k - k0)] = (float)v;
        if (A.col) A.col[o + (k - k0)] = j[e];
        absoff += fabs(v);
      } else {
        gsum += aij * A.Eall[j[e]];
      }
    }
  }
  suma = group_sum<G>(suma);
  gsum = group_sum<G>(gsum);
  absoff = group_sum<G>(absoff);
  if (lane == 0) {
    const double d = Vi * (1.0 / dt + c * A.sa[i] * A.f[i]) + Vi * suma;
    A.diag64[i] = d;
    A.dinv64[i] = 1.0 / d;                 // Jacobi preconditioner
    A.sinv64[i] = 1.0 / (d + absoff);      // l1-Jacobi smoother of the V-cycle
    if (A.diag32) {
      A.diag32[i] = (float)d;
      A.dinv32[i] = (float)(1.0 / d);
      A.sinv32[i] = (float)(1.0 / (d + absoff));
    }
    A.g[i] = Vi * gsum;
  }
}

// export in user order: scatter (col, val) incl. diagonal, then sort rows
__global__ void k_export_counts(int64_t nin, const int32_t* __restrict__ iperm,
                                const int64_t* __restrict__ rp, int64_t* __restrict__ ucnt) {
  int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (u >= nin) return;
  const int32_t s = iperm[u];
  ucnt[u] = rp[s + 1] - rp[s] + 1;
}

__global__ void k_export_scatter(int64_t nin, const int32_t* __restrict__ perm,
                                 const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const double* __restrict__ val, const double* __restrict__ diag,
                                 const double* __restrict__ g, const int64_t* __restrict__ urp,
                                 int32_t* __restrict__ ucol, double* __restrict__ uval,
                                 double* __restrict__ ug) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= nin) return;
  const int32_t u = perm[s];
  int64_t o = urp[u];
  ucol[o] = u;
  uval[o] = diag[s];
  ++o;
  for (int64_t k = rp[s]; k < rp[s + 1]; ++k, ++o) {
    ucol[o] = perm[col[k]];
    uval[o] = val[k];
  }
  if (ug) ug[u] = g[s];
}

// lanes per row (four entries per lane)
int pick_group(double avg_row) {
  if (avg_row > 100) return 64;
  if (avg_row > 40) return 16;
  if (avg_row > 20) return 8;
  return 4;
}

}  // namespace

int assemble(rt_ctx* ctx, const rt_neighbors* nb, const rt_step_inputs* in, rt_matrix* A,
             bool new_structure) {
  hipStream_t st = ctx->stream;
  const int64_t n = nb->n_total, nin = nb->n_interior;
  A->nb = nb;
  A->n = nin;
  A->n_total = n;
  A->dt = in->dt;
  A->c = in->c;
  A->a = in->a;
  for (auto* b : {&A->V, &A->D, &A->sa, &A->f, &A->Eall}) RT_CHECK(b->reserve(n));
  RT_CHECK(A->VD.reserve((size_t)2 * n));
  for (auto* b : {&A->rho, &A->cv, &A->m, &A->e_prev, &A->E_prev, &A->Qe, &A->QE, &A->g})
    RT_CHECK(b->reserve(nin));
  DevBuf<double> sigt, rec;
  RT_CHECK(sigt.reserve(n));
  RT_CHECK(rec.reserve((size_t)8 * n));
  hipLaunchKernelGGL(k_pack_inputs, dim3(grid_for(n)), dim3(kBlock), 0, st, n, in->cv, in->rho,
                     in->e, in->E, in->sigma0_a, in->m, in->Q_e, in->Q_E, rec.p);
  RT_LAUNCH_CHECK();
  FrozenArgs fa{nb->perm.p, rec.p, in->sigma_s, in->dt, in->c, in->a, in->opacity_exponent,
                A->V.p, A->D.p, A->sa.p, sigt.p, A->f.p, A->Eall.p, A->e_prev.p, A->E_prev.p,
                A->rho.p, A->cv.p, A->m.p, A->Qe.p, A->QE.p, A->VD.p};
  hipLaunchKernelGGL(k_frozen, dim3(grid_for(n)), dim3(kBlock), 0, st, n, nin, fa);
  RT_LAUNCH_CHECK();
  if (in->limiter != RT_LIMITER_NONE && nin > 0) {
    const int G = pick_group(nin ? (double)nb->npairs / (double)n : 0.0);
    const int per = (grid_for(nin * (int64_t)G, kBlock) + kXcd - 1) / kXcd;
    const int grid = per * kXcd;
#define RT_LIM(D_, G_)                                                                      \
  hipLaunchKernelGGL((k_limiter<D_, G_, 4>), dim3(grid), dim3(kBlock), 0, st, nin, nb->kernel, \
                     in->limiter, in->limiter_k, in->c, nb->sp4.p, nb->ptr.p, nb->idx.p,      \
                     A->V.p, A->Eall.p, sigt.p, A->D.p, A->VD.p, nb->box, per)
    if (nb->dim == 3) {
      if (G == 64) RT_LIM(3, 64); else if (G == 16) RT_LIM(3, 16);
      else if (G == 8) RT_LIM(3, 8); else RT_LIM(3, 4);
    } else {
      if (G == 64) RT_LIM(2, 64); else if (G == 16) RT_LIM(2, 16);
      else if (G == 8) RT_LIM(2, 8); else RT_LIM(2, 4);
    }
#undef RT_LIM
    RT_LAUNCH_CHECK();
  }

  if (A->levels.empty()) A->levels.resize(1);
  Level& L = A->levels[0];
  if (new_structure) {
    L.n = nin;
    RT_CHECK(L.rp.reserve(nin + 1));
    DevBuf<int64_t> cnt;
    RT_CHECK(cnt.reserve(nin + 1));
    RT_CHECK_HIP(hipMemsetAsync(cnt.p + nin, 0, sizeof(int64_t), st));
    if (nin > 0) {
      hipLaunchKernelGGL(k_int_counts, dim3(grid_for(nin)), dim3(kBlock), 0, st, nin,
                         nb->n_int_nbrs.p, cnt.p);
      RT_LAUNCH_CHECK();
    }
    RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, L.rp.p, nin + 1, false)));
    RT_CHECK(ctx->sync_read(L.rp.p + nin, sizeof(int64_t)));
    int64_t nnz = 0;
    std::memcpy(&nnz, ctx->host, sizeof(int64_t));
    L.nnz = nnz;
    RT_CHECK(max_nonneg<int64_t>(ctx, cnt.p, nin, &L.max_row));
    RT_CHECK(L.col.reserve(nnz));
  }
  RT_CHECK(L.val64.reserve(L.nnz + kSpmvPad));
  for (auto* b : {&L.diag64, &L.dinv64, &L.sinv64}) RT_CHECK(b->reserve(nin));
  const bool fp32 = A->amg.build_fp32 != 0;
  if (fp32) {
    RT_CHECK(L.val32.reserve(L.nnz + kSpmvPad));
    for (auto* b : {&L.diag32, &L.dinv32, &L.sinv32}) RT_CHECK(b->reserve(nin));
  }
  A->has_fp32 = fp32;
  if (nin > 0) {
    AsmArgs aa{nb->ptr.p, L.rp.p, nb->idx.p, nb->sp4.p, A->VD.p, A->sa.p,
               A->f.p, A->Eall.p, new_structure ? L.col.p : nullptr, L.val64.p, L.diag64.p,
               L.dinv64.p, L.sinv64.p, A->g.p, fp32 ? L.val32.p : nullptr,
               fp32 ? L.diag32.p : nullptr, fp32 ? L.dinv32.p : nullptr,
               fp32 ? L.sinv32.p : nullptr, nb->box};
    const double avg = nin ? (double)nb->npairs / (double)n : 0.0;
    const int G = pick_group(avg);
    const int per = (grid_for(nin * (int64_t)G, kBlock) + kXcd - 1) / kXcd;
    const int grid = per * kXcd;
#define RT_ASM(D_, G_)                                                                           \
  hipLaunchKernelGGL((k_assemble<D_, G_, 4>), dim3(grid), dim3(kBlock), 0, st, nin, n, nb->kernel, \
                     in->dt, in->c, aa, per)
    if (nb->dim == 3) {
      if (G == 64) RT_ASM(3, 64); else if (G == 16) RT_ASM(3, 16);
      else if (G == 8) RT_ASM(3, 8); else RT_ASM(3, 4);
    } else {
      if (G == 64) RT_ASM(2, 64); else if (G == 16) RT_ASM(2, 16);
      else if (G == 8) RT_ASM(2, 8); else RT_ASM(2, 4);
    }
#undef RT_ASM
    RT_LAUNCH_CHECK();
  }
  if (new_structure && A->amg.tiled_spmv) RT_CHECK(build_tiles(ctx, L));
  return RT_OK;
}

int matrix_export(rt_ctx* ctx, const rt_matrix* A, int64_t* urp, int32_t* ucol, double* uval,
                  double* ug) {
  hipStream_t st = ctx->stream;
  const rt_neighbors* nb = A->nb;
  const Level& L = A->levels[0];
  const int64_t nin = A->n;
  DevBuf<int64_t> cnt;
  RT_CHECK(cnt.reserve(nin + 1));
  RT_CHECK_HIP(hipMemsetAsync(cnt.p + nin, 0, sizeof(int64_t), st));
  if (nin > 0) {
    hipLaunchKernelGGL(k_export_counts, dim3(grid_for(nin)), dim3(kBlock), 0, st, nin,
                       nb->iperm.p, L.rp.p, cnt.p);
    RT_LAUNCH_CHECK();
  }
  RT_CHECK((scan<int64_t, int64_t>(ctx, cnt.p, urp, nin + 1, false)));
  if (nin == 0) return RT_OK;
  hipLaunchKernelGGL(k_export_scatter, dim3(grid_for(nin)), dim3(kBlock), 0, st, nin,
                     nb->perm.p, L.rp.p, L.col.p, L.val64.p, L.diag64.p, A->g.p, urp, ucol, uval,
                     ug);
  RT_LAUNCH_CHECK();
  RT_CHECK((row_sort<int32_t, double>(ctx, urp, ucol, uval, nin)));
  RT_CHECK_HIP(hipStreamSynchronize(st));
  return RT_OK;
}

}  // namespace rt

extern "C" {

int rt_assemble(rt_ctx* ctx, const rt_neighbors* nb, const rt_step_inputs* in,
                const rt_amg_opts* amg, rt_matrix** A) {
  rt::clear_error();
  if (!ctx || !nb || !in || !A) {
    rt::set_error("rt_assemble: NULL argument");
    return RT_E_ARG;
  }
  if (!in->m || !in->rho || !in->cv || !in->sigma0_a || !in->e || !in->E) {
    rt::set_error("rt_assemble: a required per-particle array is NULL");
    return RT_E_ARG;
  }
  if (!(in->dt > 0.0) || !std::isfinite(in->dt) || !(in->c > 0.0) || !(in->a > 0.0)) {
    rt::set_error("rt_assemble: dt, c and a must be positive and finite");
    return RT_E_ARG;
  }
  if (in->limiter != RT_LIMITER_NONE && in->limiter != RT_LIMITER_LARSEN &&
      in->limiter != RT_LIMITER_LEVERMORE) {
    rt::set_error("rt_assemble: unknown limiter %d", in->limiter);
    return RT_E_ARG;
  }
  if (in->limiter == RT_LIMITER_LARSEN && !(in->limiter_k > 0.0)) {
    rt::set_error("rt_assemble: Larsen limiter needs k > 0");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  rt_matrix* M = *A;
  bool fresh = false;
  if (M && M->nb != nb) {
    rt::set_error("rt_assemble: matrix was built from another neighbour object");
    return RT_E_STATE;
  }
  if (!M) {
    M = new rt_matrix();
    fresh = true;
  }
  M->resid_ok = false;   // a new operator: no residual carries over
  rt_amg_opts d{8, 256, 0.25, 1, 1, RT_SMOOTHER_L1_JACOBI, 2, 1, RT_PROLONG_PIECEWISE};
  if (amg && (amg->smoother < RT_SMOOTHER_L1_JACOBI || amg->smoother > RT_SMOOTHER_CHEBYSHEV ||
              amg->smoother_degree < 1 || amg->smoother_degree > 8 || amg->cycle < 1 ||
              amg->cycle > 3 || amg->prolongation < RT_PROLONG_PIECEWISE ||
              amg->prolongation > RT_PROLONG_SMOOTHED)) {
    rt::set_error("rt_assemble: smoother %d of degree %d, cycle %d, prolongation %d (smoother 0 "
                  "or 1, degree 1..8, cycle 1, 2 or 3, prolongation 0 or 1)", amg->smoother,
                  amg->smoother_degree, amg->cycle, amg->prolongation);
    if (fresh) delete M;
    return RT_E_ARG;
  }
  M->amg = amg ? *amg : d;
  if (M->amg.max_levels < 1) M->amg.max_levels = 1;
  if (M->amg.max_levels > 16) M->amg.max_levels = 16;
  int s = rt::assemble(ctx, nb, in, M, fresh);
  if (s >= 0) s = rt::amg_setup(ctx, M);
  if (s < 0) {
    if (fresh) delete M;
    return s;
  }
  *A = M;
  return RT_OK;
}

int rt_matrix_get_info(const rt_matrix* A, rt_matrix_info* info) {
  if (!A || !info) {
    rt::set_error("rt_matrix_get_info: NULL argument");
    return RT_E_ARG;
  }
  *info = rt_matrix_info{};
  info->n = A->n;
  info->nnz = A->levels.empty() ? 0 : A->levels[0].nnz + A->n;
  info->levels = (int)A->levels.size();
  for (size_t l = 0; l < A->levels.size() && l < 16; ++l) {
    info->level_n[l] = A->levels[l].n;
    info->level_nnz[l] = A->levels[l].nnz + A->levels[l].n;
    info->level_tile_cols[l] = A->levels[l].tiled ? A->levels[l].tile_cols_total : 0;
    info->level_p_nnz[l] = A->levels[l].smoothed ? A->levels[l].p_nnz : 0;
  }
  return RT_OK;
}

int rt_matrix_export(rt_ctx* ctx, const rt_matrix* A, int64_t* row_ptr, int32_t* col,
                     double* val, double* ghost_rhs) {
  rt::clear_error();
  if (!ctx || !A || !row_ptr || (A->n > 0 && (!col || !val))) {
    rt::set_error("rt_matrix_export: NULL argument");
    return RT_E_ARG;
  }
  return rt::matrix_export(ctx, A, row_ptr, col, val, ghost_rhs);
}

void rt_matrix_free(rt_matrix* A) {
  if (!A) return;
  rt::IdleScope idle;   // one wait for the device, then every buffer goes back to the cache
  delete A;
}

}  // extern "C"

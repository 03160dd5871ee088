// One outer iteration of Algorithm 1 (nonlinear elimination), on the device.
//
// Right-hand side of the diffusion solve (Sec. 2.2, inexact Newton equation;
// operators S and N of Sec. 3.2), multiplied by V_i:
//   b_i = V_i [E_i^{n-1}/dt + c sigma_a,i a T_i^4 - (1 - f_i) c sigma_a,i E_i^l + Q_E,i] + g_i
// Material update, the operator M^-1 of Sec. 3.2: the per-particle bracketed
// Newton solve of material.h.
// Convergence measures (Sec. 2.2): max_i |e^{l+1} - e^l|/|e^{l+1}| and the
// same for E; energy (Sec. 2.5): sum_i (m_i e_i + V_i E_i).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <utility>
#include <vector>

#include "internal.h"
#include "material.h"
#include "reduce.h"
#include "spmv.h"

namespace rt {
namespace {

__global__ void k_rhs(int64_t n, double dt, double c, double a, const double* __restrict__ V,
                      const double* __restrict__ sa, const double* __restrict__ f,
                      const double* __restrict__ cv, const double* __restrict__ E_prev,
                      const double* __restrict__ QE, const double* __restrict__ g,
                      const double* __restrict__ e_l, const double* __restrict__ E_l,
                      double* __restrict__ b, const double* __restrict__ x_last,
                      int32_t* __restrict__ mismatch) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double T = e_l[i] / cv[i];
  const double T2 = T * T;
  const double ca = c * sa[i];
  const double El = E_l[i];
  const double P = E_prev[i] / dt + ca * (a * (T2 * T2)) - (1.0 - f[i]) * ca * El + QE[i];
  b[i] = V[i] * P + g[i];
  // the carried residual is valid only if E^l is the last solution, bit for bit
  if (x_last && El != x_last[i]) atomicAdd(mismatch, 1);
}

// Block maxima of the material residual of the backward-Euler system,
// |m_i| / (rho_i |e_i| / dt) with m_i = rho_i/dt (e_i - e_i^{n-1})
// + c sigma_a,i (a T_i^4 - E_i) - Q_e,i (Sec. 2.2); a row with e_i = 0
// counts |m_i| dt / rho_i.
__global__ void __launch_bounds__(kBlock)
k_mat_resid(int64_t n, double dt, double c, double a, const double* __restrict__ e,
            const double* __restrict__ E, const double* __restrict__ e_prev,
            const double* __restrict__ rho, const double* __restrict__ cv,
            const double* __restrict__ sa, const double* __restrict__ Qe,
            double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double T = e[i] / cv[i];
    const double T2 = T * T;
    const double m = rho[i] / dt * (e[i] - e_prev[i]) + c * sa[i] * (a * (T2 * T2) - E[i]) - Qe[i];
    const double scale = rho[i] / dt * (e[i] != 0.0 ? fabs(e[i]) : 1.0);
    v = fabs(m) / scale;
    if (!(v == v)) v = INFINITY;   // a NaN residual counts as unbounded
  }
  v = block_max(v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// one block: out[0] = the largest of np values
__global__ void __launch_bounds__(kBlock)
k_max_of(int np, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[kBlock / kWave];
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += kBlock) v = fmax(v, part[k]);
  v = block_max(v, red);
  if (threadIdx.x == 0) out[0] = v;
}

enum { R_DE = 0, R_DEE, R_ITS, R_BAD, R_NONPHYS, R_EN, R_EN0, R_WIDTH };

struct MatArgs {
  const double *e_prev, *rho, *cv, *sa, *Qe, *m, *V, *E_prev;
  const double *E_new, *E_old, *e_start;
  double* e_out;
  double dt, c, a, tol;
  int max_iter;
};

__global__ void __launch_bounds__(kBlock) k_material(int64_t n, MatArgs A, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  double de = 0.0, dE = 0.0, its_max = 0.0, bad = 0.0, nonphys = 0.0, en = 0.0, en0 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double ep = A.e_prev[i];
    const double Enew = A.E_new[i];
    const MaterialResult mr = material_solve(A.rho[i], A.cv[i], A.sa[i], ep, A.Qe[i], Enew,
                                             A.e_start[i], A.dt, A.c, A.a, A.tol, A.max_iter);
    const double e = mr.e;
    const int it = mr.iterations;
    if (mr.nonphysical) nonphys += 1.0;
    if (!mr.converged) bad += 1.0;
    A.e_out[i] = e;
    de = fmax(de, fabs(e - A.e_start[i]) / fabs(e));
    dE = fmax(dE, fabs(Enew - A.E_old[i]) / fabs(Enew));
    its_max = fmax(its_max, (double)it);
    en += A.m[i] * e + A.V[i] * Enew;
    en0 += A.m[i] * ep + A.V[i] * A.E_prev[i];
  }
  de = block_max(de, red);
  dE = block_max(dE, red);
  its_max = block_max(its_max, red);
  bad = block_sum(bad, red);
  nonphys = block_sum(nonphys, red);
  en = block_sum(en, red);
  en0 = block_sum(en0, red);
  if (threadIdx.x == 0) {
    double* o = part + (int64_t)blockIdx.x * R_WIDTH;
    o[R_DE] = de;
    o[R_DEE] = dE;
    o[R_ITS] = its_max;
    o[R_BAD] = bad;
    o[R_NONPHYS] = nonphys;
    o[R_EN] = en;
    o[R_EN0] = en0;
  }
}

// column-wise combination of the block partials (max for the first three
// columns, sum for the rest), one block, fixed order
__global__ void __launch_bounds__(kBlock) k_material_final(int np, const double* __restrict__ part,
                                                           double* __restrict__ out) {
  __shared__ double red[kBlock / kWave];
  for (int c = 0; c < R_WIDTH; ++c) {
    const bool is_max = c <= R_ITS;
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
      const double x = part[(int64_t)i * R_WIDTH + c];
      v = is_max ? fmax(v, x) : v + x;
    }
    v = is_max ? block_max(v, red) : block_sum(v, red);
    if (threadIdx.x == 0) out[c] = v;
  }
}

int material(rt_ctx* ctx, rt_matrix* A, const double* E_new, const double* E_old,
             const double* e_start, double* e_out, double tol, int max_iter, double* res) {
  const int64_t n = A->n;
  const int gv = grid_for(n, kBlock, kMaxPartials);
  RT_CHECK(A->partA.reserve(std::max<int64_t>((int64_t)kMaxPartials * R_WIDTH, max_partials(n))));
  RT_CHECK(A->scal.reserve(16));
  MatArgs ma{A->e_prev.p, A->rho.p, A->cv.p, A->sa.p, A->Qe.p, A->m.p, A->V.p, A->E_prev.p,
             E_new, E_old, e_start, e_out, A->dt, A->c, A->a, tol, max_iter};
  hipLaunchKernelGGL(k_material, dim3(gv), dim3(kBlock), 0, ctx->stream, n, ma, A->partA.p);
  RT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_material_final, dim3(1), dim3(kBlock), 0, ctx->stream, gv, A->partA.p,
                     A->scal.p + 8);
  RT_LAUNCH_CHECK();
  RT_CHECK(ctx->sync_read(A->scal.p + 8, sizeof(double) * R_WIDTH));
  for (int c = 0; c < R_WIDTH; ++c) res[c] = ctx->host[c];
  return RT_OK;
}

// pass 1: sums of e V, E V and V; pass 2: the largest fractional changes
__global__ void __launch_bounds__(kBlock)
k_frac_sums(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ V,
            const double* __restrict__ E, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  double sE = 0.0, sv = 0.0;
  for (int64_t s = blockIdx.x * (int64_t)kBlock + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kBlock) {
    sE += E[perm[s]] * V[s];
    sv += V[s];
  }
  sE = block_sum(sE, red);
  sv = block_sum(sv, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sE;
    part[2 * blockIdx.x + 1] = sv;
  }
}

__global__ void __launch_bounds__(kBlock)
k_frac_max(int64_t n, const double* __restrict__ e_new, const double* __restrict__ e_old,
           const double* __restrict__ E_new, const double* __restrict__ E_old, double pe,
           double pE, double tiny, double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  double me = 0.0, mE = 0.0;
  for (int64_t u = blockIdx.x * (int64_t)kBlock + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * kBlock) {
    me = fmax(me, fabs(e_new[u] - e_old[u]) / (e_new[u] + pe + tiny));
    mE = fmax(mE, fabs(E_new[u] - E_old[u]) / (E_new[u] + pE + tiny));
  }
  me = block_max(me, red);
  mE = block_max(mE, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = me;
    part[2 * blockIdx.x + 1] = mE;
  }
}

}  // namespace
}  // namespace rt

extern "C" int rt_fractional_change(rt_ctx* ctx, const rt_matrix* A, const double* e_new,
                                    const double* e_old, const double* E_new,
                                    const double* E_old, double eta_target, double tiny,
                                    double* eta) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || !eta || (A->n > 0 && (!e_new || !e_old || !E_new || !E_old))) {
    set_error("rt_fractional_change: NULL argument");
    return RT_E_ARG;
  }
  if (!(eta_target > 0.0) || !(tiny >= 0.0)) {
    set_error("rt_fractional_change: eta_target must be > 0 and tiny >= 0");
    return RT_E_ARG;
  }
  eta[0] = eta[1] = 0.0;
  const int64_t n = A->n;
  if (n == 0) return RT_OK;
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  hipStream_t st = ctx->stream;
  const int g = grid_for(n, kBlock, kMaxPartials);
  DevBuf<double> part;
  RT_CHECK(part.reserve((size_t)2 * g));
  std::vector<double> hp((size_t)2 * g);
  hipLaunchKernelGGL(k_frac_sums, dim3(g), dim3(kBlock), 0, st, n, A->nb->perm.p, A->V.p, E_new,
                     part.p);
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * 2 * g, hipMemcpyDeviceToHost, st));
  RT_CHECK_HIP(hipStreamSynchronize(st));
  double sE = 0.0, sv = 0.0;
  for (int b = 0; b < g; ++b) {
    sE += hp[2 * b];
    sv += hp[2 * b + 1];
  }
  // the floor of both fractional changes is the mean radiation energy (Sec. 3.3 as read)
  const double Ebar = sE / sv;
  hipLaunchKernelGGL(k_frac_max, dim3(g), dim3(kBlock), 0, st, n, e_new, e_old, E_new, E_old,
                     eta_target * Ebar, eta_target * Ebar, tiny, part.p);
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * 2 * g, hipMemcpyDeviceToHost, st));
  RT_CHECK_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < g; ++b) {
    eta[0] = std::max(eta[0], hp[2 * b]);
    eta[1] = std::max(eta[1], hp[2 * b + 1]);
  }
  return RT_OK;
}

extern "C" int rt_newton_step(rt_ctx* ctx, rt_matrix* A, double* e, double* E, int ell,
                              const rt_newton_opts* opts, rt_newton_stats* stats) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || !opts || (A->n > 0 && (!e || !E))) {
    set_error("rt_newton_step: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK(check_solve_opts(&opts->solve));
  if (!(opts->material_tol > 0.0) || opts->material_max_iter < 1 ||
      (opts->state_order != 0 && opts->state_order != 1) ||
      (opts->recompute_residual != 0 && opts->recompute_residual != 1)) {
    set_error("rt_newton_step: material_tol must be > 0, material_max_iter >= 1, state_order "
              "and recompute_residual 0 or 1");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  auto t0 = std::chrono::steady_clock::now();
  rt_newton_stats local{};
  rt_newton_stats* stt = stats ? stats : &local;
  *stt = rt_newton_stats{};
  const int64_t n = A->n;
  if (n == 0) return RT_OK;
  hipStream_t st = ctx->stream;
  for (auto* b : {&A->ecur, &A->Ecur, &A->enew, &A->xs, &A->bs}) RT_CHECK(b->reserve(n));
  const bool in_sorted = opts->state_order == 1;
  // the state in sorted order: the caller's arrays themselves, or gathered copies
  double* ecur = in_sorted ? e : A->ecur.p;
  double* Ecur = in_sorted ? E : A->Ecur.p;
  if (!in_sorted) {
    RT_CHECK(gather_sorted(ctx, A->nb, n, e, ecur));
    RT_CHECK(gather_sorted(ctx, A->nb, n, E, Ecur));
  }
  double res[8];
  int status = RT_OK;
  if (ell == 0) {
    // initial material solve with E^{n,0} from e^{n-1} (Algorithm 1, before the loop)
    RT_CHECK(material(ctx, A, Ecur, Ecur, A->e_prev.p, ecur, opts->material_tol,
                      opts->material_max_iter, res));
    if (res[3] > 0) status = RT_NOT_CONVERGED;
    if (res[4] > 0) status = RT_NONPHYSICAL;
  }
  // Outer iterations after the first start from the last solution with the
  // same matrix, so the last solve's residual b^l - A E^{l+1} turns into the
  // new initial residual by adding b^{l+1} - b^l: no product needed.
  const bool carry = ell > 0 && A->resid_ok && !opts->recompute_residual;
  A->resid_ok = false;
  if (carry) {
    std::swap(A->bs, A->bs_prev);   // bs_prev: the last right-hand side
    RT_CHECK(A->bs.reserve(n));
    RT_CHECK(A->xmis.reserve(1));
    RT_CHECK_HIP(hipMemsetAsync(A->xmis.p, 0, sizeof(int32_t), st));
  }
  hipLaunchKernelGGL(k_rhs, dim3(grid_for(n)), dim3(kBlock), 0, st, n, A->dt, A->c, A->a, A->V.p,
                     A->sa.p, A->f.p, A->cv.p, A->E_prev.p, A->QE.p, A->g.p, ecur, Ecur,
                     A->bs.p, carry ? A->xs.p : nullptr, carry ? A->xmis.p : nullptr);
  RT_LAUNCH_CHECK();
  RT_CHECK_HIP(hipMemcpyAsync(A->xs.p, Ecur, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  RT_CHECK_HIP(hipEventRecord(ctx->ev0, st));
  int s = solve_sorted(ctx, A, A->bs.p, A->xs.p, &opts->solve, &stt->solve,
                       carry ? A->bs_prev.p : nullptr, carry ? A->xmis.p : nullptr);
  if (s < 0) return s;
  const bool resid_after = A->r64_valid;
  RT_CHECK_HIP(hipEventRecord(ctx->ev1, st));
  if (s == RT_NOT_CONVERGED) status = RT_NOT_CONVERGED;
  RT_CHECK(material(ctx, A, A->xs.p, Ecur, ecur, A->enew.p, opts->material_tol,
                    opts->material_max_iter, res));
  stt->delta_e = res[0];
  stt->delta_E = res[1];
  stt->material_iterations = (int)res[2];
  stt->nonphysical = (int64_t)res[4];
  stt->energy = res[5];
  stt->energy_prev = res[6];
  if (res[3] > 0 && status == RT_OK) status = RT_NOT_CONVERGED;
  if (res[4] > 0) status = RT_NONPHYSICAL;
  if (in_sorted) {
    RT_CHECK_HIP(hipMemcpyAsync(e, A->enew.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    RT_CHECK_HIP(hipMemcpyAsync(E, A->xs.p, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  } else {
    RT_CHECK(scatter_user(ctx, A->nb, n, A->enew.p, e));
    RT_CHECK(scatter_user(ctx, A->nb, n, A->xs.p, E));
  }
  RT_CHECK_HIP(hipStreamSynchronize(st));
  float solve_ms = 0.f;
  RT_CHECK_HIP(hipEventElapsedTime(&solve_ms, ctx->ev0, ctx->ev1));
  stt->solve.seconds = 1e-3 * solve_ms;
  RT_CHECK(collect_profile(ctx, &stt->solve));
  stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  A->resid_ok = resid_after;
  if (status == RT_NONPHYSICAL) set_error("rt_newton_step: %lld negative material roots", (long long)stt->nonphysical);
  else if (status == RT_NOT_CONVERGED && rt_last_error()[0] == 0)
    set_error("rt_newton_step: a material solve did not converge");
  return status;
}

extern "C" int rt_newton_residual(rt_ctx* ctx, rt_matrix* A, const double* e, const double* E,
                                  int state_order, rt_be_residual* out) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || !out || (A->n > 0 && (!e || !E))) {
    set_error("rt_newton_residual: NULL argument");
    return RT_E_ARG;
  }
  if (state_order != 0 && state_order != 1) {
    set_error("rt_newton_residual: state_order must be 0 or 1");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);
  *out = rt_be_residual{};
  const int64_t n = A->n;
  if (n == 0) return RT_OK;
  hipStream_t st = ctx->stream;
  for (auto* b : {&A->ecur, &A->Ecur, &A->bs}) RT_CHECK(b->reserve(n));
  const double* es = e;
  const double* Es = E;
  if (state_order == 0) {
    RT_CHECK(gather_sorted(ctx, A->nb, n, e, A->ecur.p));
    RT_CHECK(gather_sorted(ctx, A->nb, n, E, A->Ecur.p));
    es = A->ecur.p;
    Es = A->Ecur.p;
  }
  // b(e, E): Algorithm 1's right-hand side at the state itself, so that
  // A E - b = V r (the f terms cancel)
  hipLaunchKernelGGL(k_rhs, dim3(grid_for(n)), dim3(kBlock), 0, st, n, A->dt, A->c, A->a, A->V.p,
                     A->sa.p, A->f.p, A->cv.p, A->E_prev.p, A->QE.p, A->g.p, es, Es, A->bs.p,
                     nullptr, nullptr);
  RT_LAUNCH_CHECK();
  double rr = 0.0, bb = 0.0;
  RT_CHECK(residual_norms(ctx, A, A->bs.p, Es, &rr, &bb));
  const int nbk = grid_for(n);
  DevBuf<double> part;
  RT_CHECK(part.reserve(nbk + 1));
  hipLaunchKernelGGL(k_mat_resid, dim3(nbk), dim3(kBlock), 0, st, n, A->dt, A->c, A->a, es, Es,
                     A->e_prev.p, A->rho.p, A->cv.p, A->sa.p, A->Qe.p, part.p);
  hipLaunchKernelGGL(k_max_of, dim3(1), dim3(kBlock), 0, st, nbk, part.p, part.p + nbk);
  RT_LAUNCH_CHECK();
  RT_CHECK(ctx->sync_read(part.p + nbk, sizeof(double)));
  out->rad_norm = std::sqrt(rr);
  out->rad_rel = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
  out->mat_rel = ctx->host[0];
  return RT_OK;
}

extern "C" int rt_to_sorted(rt_ctx* ctx, const rt_neighbors* nb, const double* user,
                            double* sorted) {
  using namespace rt;
  clear_error();
  if (!ctx || !nb || (nb->n_interior > 0 && (!user || !sorted))) {
    set_error("rt_to_sorted: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  if (nb->n_interior > 0) RT_CHECK(gather_sorted(ctx, nb, nb->n_interior, user, sorted));
  return RT_OK;
}

extern "C" int rt_to_user(rt_ctx* ctx, const rt_neighbors* nb, const double* sorted,
                          double* user) {
  using namespace rt;
  clear_error();
  if (!ctx || !nb || (nb->n_interior > 0 && (!user || !sorted))) {
    set_error("rt_to_user: NULL argument");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  if (nb->n_interior > 0) RT_CHECK(scatter_user(ctx, nb, nb->n_interior, sorted, user));
  return RT_OK;
}

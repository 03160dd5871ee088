// Restarted GMRES on the unscaled diffusion operator, as the paper solves the
// diffusion equation (Sec. 3.2, with a multigrid preconditioner).
//
// The library's main solver is CG on the V-scaled symmetric system A x = b
// (row i of the paper's operator multiplied by V_i).  This solver works on
// the paper's own, unscaled form U x = c with U = diag(V)^-1 A and
// c = diag(V)^-1 b, which has the same solution x.  U is not symmetric.
//
// Right-preconditioned GMRES(m): the Krylov space is built from U M^-1 and
// x = x0 + M^-1 (Z y), so the residual the method minimises is the true
// residual of U x = c.  The preconditioner approximates U^-1 = A^-1 diag(V):
//   Jacobi:  M^-1 v = diag(A)^-1 (V v)   (= diag(U)^-1 v)
//   AMG:     M^-1 v = Vcycle(V v)        (the V-cycle of A)
// Both are linear and fixed, so the correction is formed once per cycle from
// the combined basis vector.  The basis is orthogonalised by classical
// Gram-Schmidt applied twice, one multi-dot and one multi-axpy kernel per
// pass; the small Hessenberg least-squares problem is solved on the host
// with Givens rotations.  Stop when ||c - U x||_2 <= tol ||c||_2; the final
// relative residual is recomputed from a product, not taken from the
// recurrence.  FP64 throughout.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "reduce.h"
#include "spmv.h"

namespace rt {
namespace {

constexpr int kGmresMaxRestart = 64;
constexpr int kGmresBlocks = 512;   // most blocks (= partials per dot) of the reductions

// out[i] = in[i] / V[i]
__global__ void k_div_v(int64_t n, const double* __restrict__ in, const double* __restrict__ V,
                        double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] / V[i];
}

// out[i] = s[i] * V[i] * v[i]   (s = 1/diag(A) for Jacobi, else s = NULL)
__global__ void k_mul_v(int64_t n, const double* __restrict__ s, const double* __restrict__ V,
                        const double* __restrict__ v, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (s ? s[i] : 1.0) * (V[i] * v[i]);
}

// part[j * gridDim.x + block] = block's share of w . basis_j, j < J
__global__ void __launch_bounds__(kBlock)
k_mdot(int64_t n, int J, const double* __restrict__ basis, const double* __restrict__ w,
       double* __restrict__ part) {
  __shared__ double red[kBlock / kWave];
  for (int j = 0; j < J; ++j) {
    const double* bj = basis + (int64_t)j * n;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
      acc += w[i] * bj[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = acc;
  }
}

// w += sign * sum_{j<J} c[j] basis_j
__global__ void k_maxpy(int64_t n, int J, const double* __restrict__ basis,
                        const double* __restrict__ c, double sign, double* __restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < J; ++j) s += c[j] * basis[(int64_t)j * n + i];
  w[i] += sign * s;
}

// x += z
__global__ void k_add(int64_t n, const double* __restrict__ z, double* __restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += z[i];
}

__global__ void k_fill0(int64_t n, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = 0.0;
}

// out = in * a
__global__ void k_scal(int64_t n, double a, const double* __restrict__ in,
                       double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * in[i];
}

struct Gmres {
  rt_ctx* ctx;
  rt_matrix* A;
  int64_t n;
  int m;
  bool amg;
  DevBuf<double> basis, w, t, z, part, coef;
  std::vector<double> hpart;
  double* hcoef = nullptr;   // pinned staging of the coefficients sent to the device
  int nbl = 1;               // blocks of the reductions

  ~Gmres() {
    if (hcoef) (void)hipHostFree(hcoef);
  }
  int init() {
    RT_CHECK_HIP(hipHostMalloc((void**)&hcoef, sizeof(double) * (m + 1), hipHostMallocDefault));
    nbl = grid_for(n, kBlock, kGmresBlocks);
    RT_CHECK(basis.reserve((size_t)(m + 1) * n));
    for (auto* b : {&w, &t, &z}) RT_CHECK(b->reserve(n));
    RT_CHECK(part.reserve((size_t)(m + 1) * kGmresBlocks));
    RT_CHECK(coef.reserve(m + 1));
    hpart.resize((size_t)(m + 1) * kGmresBlocks);
    return RT_OK;
  }
  double* vec(int j) { return basis.p + (int64_t)j * n; }
  // coef[0..k) = c[0..k) on the device (stream-ordered; the staging buffer is
  // written again only after the next host wait, which follows this copy)
  int send(const double* c, int k) {
    std::memcpy(hcoef, c, sizeof(double) * k);
    RT_CHECK_HIP(hipMemcpyAsync(coef.p, hcoef, sizeof(double) * k, hipMemcpyHostToDevice,
                                ctx->stream));
    return RT_OK;
  }

  // dots[j] = w . basis_j for j < J, summed on the host in a fixed order
  int mdot(int J, const double* v, double* dots) {
    hipLaunchKernelGGL(k_mdot, dim3(nbl), dim3(kBlock), 0, ctx->stream, n, J, basis.p, v,
                       part.p);
    RT_LAUNCH_CHECK();
    RT_CHECK_HIP(hipMemcpyAsync(hpart.data(), part.p, sizeof(double) * J * nbl,
                                hipMemcpyDeviceToHost, ctx->stream));
    RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    for (int j = 0; j < J; ++j) {
      double s = 0.0;
      for (int b = 0; b < nbl; ++b) s += hpart[(size_t)j * nbl + b];
      dots[j] = s;
    }
    return RT_OK;
  }
  int norm(const double* v, double* out) {
    // the dot of v with itself, through a one-vector "basis"
    hipLaunchKernelGGL(k_mdot, dim3(nbl), dim3(kBlock), 0, ctx->stream, n, 1, v, v, part.p);
    RT_LAUNCH_CHECK();
    RT_CHECK_HIP(hipMemcpyAsync(hpart.data(), part.p, sizeof(double) * nbl,
                                hipMemcpyDeviceToHost, ctx->stream));
    RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0.0;
    for (int b = 0; b < nbl; ++b) s += hpart[b];
    *out = std::sqrt(s);
    return RT_OK;
  }
  // out = M^-1 v
  int precond(const double* v, double* out) {
    const Level& L = A->levels[0];
    if (amg) {
      hipLaunchKernelGGL(k_mul_v, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, n, nullptr,
                         A->V.p, v, t.p);
      RT_LAUNCH_CHECK();
      return vcycle<double>(ctx, A, t.p, out);
    }
    hipLaunchKernelGGL(k_mul_v, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, n, L.dinv64.p,
                       A->V.p, v, out);
    RT_LAUNCH_CHECK();
    return RT_OK;
  }
  // out = U v = (A v) / V
  int apply(const double* v, double* out) {
    const Level& L = A->levels[0];
    RT_CHECK((launch_spmv_level<double, SP_PLAIN>(ctx->stream, L, L.val64.p, L.diag64.p, v,
                                                  nullptr, nullptr, t.p, nullptr, nullptr,
                                                  nullptr, L.shape64)));
    hipLaunchKernelGGL(k_div_v, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, n, t.p, A->V.p,
                       out);
    RT_LAUNCH_CHECK();
    return RT_OK;
  }
  // out = c - U x = (b - A x) / V
  int residual(const double* b, const double* x, double* out) {
    const Level& L = A->levels[0];
    int nbk = 0;
    RT_CHECK((launch_spmv_level<double, SP_RESID>(ctx->stream, L, L.val64.p, L.diag64.p, x, b,
                                                  nullptr, t.p, nullptr, A->partA.p, &nbk,
                                                  L.shape64)));
    hipLaunchKernelGGL(k_div_v, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, n, t.p, A->V.p,
                       out);
    RT_LAUNCH_CHECK();
    return RT_OK;
  }
};

// Givens rotation zeroing b in (a, b)
void givens(double a, double b, double* c, double* s) {
  if (b == 0.0) {
    *c = 1.0;
    *s = 0.0;
  } else {
    const double r = std::hypot(a, b);
    *c = a / r;
    *s = b / r;
  }
}

int gmres_sorted(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                 const rt_gmres_opts* o, rt_solve_stats* stt) {
  hipStream_t st = ctx->stream;
  Gmres G{ctx, A, A->n, o->restart, o->precond == 1 && cycle_depth(A) > 1};
  RT_CHECK(A->partA.reserve(max_partials(A->n)));
  RT_CHECK(G.init());
  const int64_t n = A->n;
  const int m = G.m;
  // ||c||
  hipLaunchKernelGGL(k_div_v, dim3(grid_for(n)), dim3(kBlock), 0, st, n, b, A->V.p, G.w.p);
  RT_LAUNCH_CHECK();
  double cnorm = 0.0;
  RT_CHECK(G.norm(G.w.p, &cnorm));
  if (!std::isfinite(cnorm)) {
    set_error("rt_solve_gmres: right-hand side is not finite");
    return RT_E_ARG;
  }
  if (cnorm == 0.0) {
    hipLaunchKernelGGL(k_fill0, dim3(grid_for(n)), dim3(kBlock), 0, st, n, x);
    RT_LAUNCH_CHECK();
    stt->rel_residual = 0.0;
    return RT_OK;
  }
  const double target = o->tol * cnorm;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(m + 1), h2(m + 1);
  auto Hat = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  int total = 0;
  double beta = 0.0;
  RT_CHECK(G.residual(b, x, G.vec(0)));
  RT_CHECK(G.norm(G.vec(0), &beta));
  while (beta > target && total < o->max_iter) {
    if (!std::isfinite(beta)) {
      set_error("rt_solve_gmres: non-finite residual");
      return RT_E_DEVICE;
    }
    hipLaunchKernelGGL(k_scal, dim3(grid_for(n)), dim3(kBlock), 0, st, n, 1.0 / beta, G.vec(0),
                       G.vec(0));
    RT_LAUNCH_CHECK();
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;   // columns of this cycle
    double est = beta;
    while (k < m && total < o->max_iter) {
      // w = U M^-1 v_k
      RT_CHECK(G.precond(G.vec(k), G.z.p));
      RT_CHECK(G.apply(G.z.p, G.w.p));
      // two passes of classical Gram-Schmidt against v_0 .. v_k
      std::fill(h.begin(), h.end(), 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        RT_CHECK(G.mdot(k + 1, G.w.p, h2.data()));
        RT_CHECK(G.send(h2.data(), k + 1));
        hipLaunchKernelGGL(k_maxpy, dim3(grid_for(n)), dim3(kBlock), 0, st, n, k + 1, G.basis.p,
                           G.coef.p, -1.0, G.w.p);
        RT_LAUNCH_CHECK();
        for (int j = 0; j <= k; ++j) h[j] += h2[j];
      }
      double hn = 0.0;
      RT_CHECK(G.norm(G.w.p, &hn));
      ++total;
      for (int j = 0; j <= k; ++j) Hat(j, k) = h[j];
      Hat(k + 1, k) = hn;
      // apply the earlier rotations to the new column, then a new one
      for (int j = 0; j < k; ++j) {
        const double a = Hat(j, k), bb = Hat(j + 1, k);
        Hat(j, k) = cs[j] * a + sn[j] * bb;
        Hat(j + 1, k) = -sn[j] * a + cs[j] * bb;
      }
      givens(Hat(k, k), Hat(k + 1, k), &cs[k], &sn[k]);
      Hat(k, k) = cs[k] * Hat(k, k) + sn[k] * Hat(k + 1, k);
      Hat(k + 1, k) = 0.0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      est = std::fabs(g[k + 1]);
      ++k;
      if (est <= target || hn == 0.0 || !std::isfinite(hn)) break;
      hipLaunchKernelGGL(k_scal, dim3(grid_for(n)), dim3(kBlock), 0, st, n, 1.0 / hn, G.w.p,
                         G.vec(k));
      RT_LAUNCH_CHECK();
    }
    // y = R^-1 g (upper triangular k x k), x += M^-1 (V y)
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < k; ++j) s -= Hat(i, j) * y[j];
      y[i] = s / Hat(i, i);
    }
    RT_CHECK(G.send(y.data(), k));
    hipLaunchKernelGGL(k_fill0, dim3(grid_for(n)), dim3(kBlock), 0, st, n, G.w.p);
    hipLaunchKernelGGL(k_maxpy, dim3(grid_for(n)), dim3(kBlock), 0, st, n, k, G.basis.p,
                       G.coef.p, 1.0, G.w.p);
    RT_LAUNCH_CHECK();
    RT_CHECK(G.precond(G.w.p, G.z.p));
    hipLaunchKernelGGL(k_add, dim3(grid_for(n)), dim3(kBlock), 0, st, n, G.z.p, x);
    RT_LAUNCH_CHECK();
    // true residual for the next cycle (and the stopping test)
    RT_CHECK(G.residual(b, x, G.vec(0)));
    RT_CHECK(G.norm(G.vec(0), &beta));
  }
  stt->iterations = total;
  stt->rel_residual = beta / cnorm;
  if (!(beta <= target)) {
    set_error("rt_solve_gmres: relative residual %.3e above tolerance %.3e", beta / cnorm,
              o->tol);
    return RT_NOT_CONVERGED;
  }
  return RT_OK;
}

}  // namespace
}  // namespace rt

extern "C" int rt_solve_gmres(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                              const rt_gmres_opts* opts, rt_solve_stats* stats) {
  using namespace rt;
  clear_error();
  if (!ctx || !A || !opts || (A->n > 0 && (!b || !x))) {
    set_error("rt_solve_gmres: NULL argument");
    return RT_E_ARG;
  }
  if ((opts->precond != 0 && opts->precond != 1) || !(opts->tol >= 0.0) || opts->max_iter < 0 ||
      opts->restart < 1 || opts->restart > kGmresMaxRestart) {
    set_error("rt_solve_gmres: precond must be 0 or 1, tol >= 0, max_iter >= 0, "
              "1 <= restart <= %d", kGmresMaxRestart);
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  rt::StreamScope release_scope(ctx->stream);   // buffers released here are stream-ordered
  auto t0 = std::chrono::steady_clock::now();
  rt_solve_stats local{};
  rt_solve_stats* stt = stats ? stats : &local;
  *stt = rt_solve_stats{};
  if (A->n == 0) return RT_OK;
  A->resid_ok = false;   // bs, xs and the work vectors are overwritten here
  RT_CHECK(A->xs.reserve(A->n));
  RT_CHECK(A->bs.reserve(A->n));
  RT_CHECK(gather_sorted(ctx, A->nb, A->n, b, A->bs.p));
  RT_CHECK(gather_sorted(ctx, A->nb, A->n, x, A->xs.p));
  const int s = gmres_sorted(ctx, A, A->bs.p, A->xs.p, opts, stt);
  if (s < 0) return s;
  RT_CHECK(scatter_user(ctx, A->nb, A->n, A->xs.p, x));
  RT_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return s;
}

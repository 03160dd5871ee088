// Internal declarations of the MI355X radiation-diffusion library (gfx950).
//
// Device layout: every per-particle array lives in the library's cell-sorted
// order.  Interior particles occupy sorted positions [0, n_interior) and
// ghosts [n_interior, n_total); perm[s] maps a sorted position back to the
// caller's index.  The V-scaled diffusion matrix (rows and columns = sorted
// interior particles) is stored as a diagonal plus an off-diagonal CSR with
// int64 row pointers, int32 columns (ascending) and FP64 values, with FP32
// copies for the mixed-precision solver.  For the sparse products each level
// may also hold a tiled form of the same CSR: rows in tiles of kTileRows, the
// ascending distinct columns of each tile (tile_cols, offsets tile_off) and,
// per entry, the 16-bit position of its column in its tile's list (lcol).
// Value and lcol arrays carry kSpmvPad spare entries so that 16-byte chunk
// loads may run past the last entry.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/rt.h"

namespace rt {

void set_error(const char* fmt, ...);
void clear_error();

#define RT_CHECK_HIP(expr)                                                      \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess) {                                                     \
      ::rt::set_error("%s:%d: %s failed: %s", __FILE__, __LINE__, #expr,        \
                      hipGetErrorString(_e));                                   \
      return RT_E_DEVICE;                                                       \
    }                                                                           \
  } while (0)

#define RT_CHECK(expr)                                                          \
  do {                                                                          \
    int _s = (expr);                                                            \
    if (_s < 0) return _s;                                                      \
  } while (0)

#define RT_LAUNCH_CHECK() RT_CHECK_HIP(hipGetLastError())

// Device memory cache behind every buffer of the library.  A released block
// is kept for reuse instead of being freed; a request takes a cached block of
// the current device whose size is at least the request and at most about an
// eighth above it, else allocates.  When an allocation fails, the device's
// cached blocks are freed and the allocation is tried once more; blocks
// beyond kPoolCapBytes of cache are freed at once.  Repeated set-up of
// same-sized problems (a neighbour build and an assembly per time step) then
// makes no hipMalloc / hipFree calls, which map and unmap pages and stall
// the host for milliseconds at gigabyte sizes.
//
// Reuse is stream-ordered.  Inside a library call (a StreamScope for the
// context's stream) a released block is tagged with that stream and handed
// back without waiting: work queued later on the same stream runs after the
// work that used it.  A block taken by another stream first waits for the
// device.  Outside any scope, release waits for the device; an IdleScope
// waits once for a whole group of releases (freeing a handle).
constexpr size_t kPoolCapBytes = (size_t)96 << 30;
// *bytes: requested size in, size of the returned block out; *device: the
// device it belongs to.  NULL when the device is out of memory.
void* pool_get(size_t* bytes, int* device);
// idle: no queued work uses the block; else it was used on `stream` only
void pool_put(void* p, size_t bytes, int device, bool idle, hipStream_t stream);
void pool_trim(int device);   // free the cached blocks of a device (-1: all)
size_t pool_cached_bytes(int device);

// Release context of the calling thread (see above).
struct ReleaseState {
  int stream_scopes = 0;      // > 0 inside a library call
  hipStream_t stream = nullptr;
  int idle_scopes = 0;        // > 0 while the device is known to be idle
};
ReleaseState& release_state();
struct StreamScope {
  ReleaseState& st;
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : st(release_state()), prev(st.stream) {
    ++st.stream_scopes;
    st.stream = s;
  }
  ~StreamScope() {
    st.stream = prev;
    --st.stream_scopes;
  }
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};
struct IdleScope {
  ReleaseState& st;
  IdleScope() : st(release_state()) {
    (void)hipDeviceSynchronize();
    ++st.idle_scopes;
  }
  ~IdleScope() { --st.idle_scopes; }
  IdleScope(const IdleScope&) = delete;
  IdleScope& operator=(const IdleScope&) = delete;
};

// Owning device buffer.  Not copyable; grows on demand.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  size_t cap = 0;   // bytes of the block
  int dev = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), cap(o.cap), dev(o.dev) {
    o.p = nullptr;
    o.n = o.cap = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      dev = o.dev;
      o.p = nullptr;
      o.n = o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  // Frees happen only in set-up paths.  The block goes back to the cache,
  // stream-ordered inside a library call, else once queued work is done.
  void release() {
    if (p) {
      ReleaseState& rs = release_state();
      if (rs.idle_scopes > 0) {
        pool_put(p, cap, dev, true, nullptr);
      } else if (rs.stream_scopes > 0) {
        pool_put(p, cap, dev, false, rs.stream);
      } else {
        (void)hipDeviceSynchronize();
        pool_put(p, cap, dev, true, nullptr);
      }
    }
    p = nullptr;
    n = cap = 0;
  }
  // Ensure capacity for `count` elements (contents are not preserved).
  int reserve(size_t count) {
    if (count <= n && p) return RT_OK;
    release();
    size_t bytes = (count ? count : 1) * sizeof(T);
    void* q = pool_get(&bytes, &dev);
    if (!q) {
      set_error("device allocation of %zu bytes failed", bytes);
      return RT_E_OOM;
    }
    p = static_cast<T*>(q);
    n = count;
    cap = bytes;
    return RT_OK;
  }
};

// Device scratch of rt_solve_noalloc (context.hip): one array per GPU.
constexpr size_t kScratchBytes = (size_t)256 << 20;
int scratch_setup(int device);    // look up the array's address on a device (current)
void* scratch_base(int device);   // that address, NULL before scratch_setup

constexpr int kBlock = 256;            // threads per block (4 wavefronts)
constexpr int kMaxPartials = 2048;     // cap on blocks of reduction kernels
constexpr int kTileRows = kBlock;      // rows per tile of the tiled SpMV format
constexpr int kTileMaxCols = 3072;     // distinct columns a tile may have
constexpr int kSpmvPad = 8;            // spare entries after values / lcol

// Dynamic LDS of a kernel (bytes set at launch).
#ifndef RT_DYNAMIC_LDS
#define RT_DYNAMIC_LDS(name) extern __shared__ __attribute__((aligned(16))) unsigned char name[]
#endif
// A value the code knows to be equal in all lanes of the wave, moved to a
// scalar register so that loops and branches on it stay scalar.
#ifndef RT_UNIFORM
#define RT_UNIFORM(x) __builtin_amdgcn_readfirstlane(x)
#endif

// Per-particle records read by the pair loops with two 16-byte loads:
// (x, y, z, h) in 4 doubles (z = 0 in 2-D) and (V, D) in 2 doubles.
typedef double rt_f64x2_t __attribute__((vector_size(16)));
struct Rec4 {
  double x, y, z, h;
};
__device__ __forceinline__ Rec4 load_rec4(const double* __restrict__ p, int64_t i) {
  const rt_f64x2_t a = *reinterpret_cast<const rt_f64x2_t*>(p + 4 * i);
  const rt_f64x2_t b = *reinterpret_cast<const rt_f64x2_t*>(p + 4 * i + 2);
  return Rec4{a[0], a[1], b[0], b[1]};
}
__device__ __forceinline__ rt_f64x2_t load_pair(const double* __restrict__ p, int64_t i) {
  return *reinterpret_cast<const rt_f64x2_t*>(p + 2 * i);
}

inline int grid_for(int64_t work_items, int per_block = kBlock, int cap = 1 << 30) {
  int64_t g = (work_items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace rt

// ---------------------------------------------------------------------------
struct rt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool profiling = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // small pinned host staging area for scalar read-backs
  double* host = nullptr;     // 64 doubles
  int sync_read(const void* dev, size_t bytes);   // async copy to host + stream sync
  // profiling: events recorded around timed launches, resolved at the end of a call
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used = 0;
  struct Span { int kind; size_t a, b; };
  std::vector<Span> prof_spans;
  int prof_mark(size_t* idx);                      // record an event on the stream
  int prof_collect(double* seconds_by_kind, int* calls_by_kind, int nkinds);
  ~rt_ctx();
};

namespace rt {
// Periodic axes of a neighbour object: bit a of mask set means axis a has
// period len[a] (positions in [0, len[a])).
struct PeriodicBox {
  double len[3];
  int mask;
};
// x_i - x_j reduced to the nearest image on an axis of period L: one period
// off above L/2, one on below -L/2.
__device__ __forceinline__ double nearest_image(double d, double L) {
  const double half = 0.5 * L;
  return d > half ? d - L : (d < -half ? d + L : d);
}
// Component a of a displacement, reduced on the box's periodic axes.
__device__ __forceinline__ double periodic_disp(double d, const PeriodicBox& box, int a) {
  return ((box.mask >> a) & 1) ? nearest_image(d, box.len[a]) : d;
}
}  // namespace rt

struct rt_neighbors {
  int dim = 3;
  int kernel = RT_KERNEL_CUBIC_SPLINE;
  double kappa = 2.0;
  int64_t n_total = 0, n_interior = 0, npairs = 0;
  int nc[3] = {1, 1, 1};
  int bits = 1;                 // Morton bits per axis
  int64_t ncells = 0;
  double lo[3] = {0, 0, 0};
  double cell_size = 0;
  rt::PeriodicBox box{{0.0, 0.0, 0.0}, 0};   // periodic axes (mask 0: none)
  rt::DevBuf<uint64_t> skeys;   // sorted keys: ghost flag << (dim*bits) | Morton(cell)
  rt::DevBuf<int32_t> perm;     // sorted -> user
  rt::DevBuf<int32_t> iperm;    // user -> sorted
  rt::DevBuf<double> sp4;       // 4 x n_total: (x, y, z, h) per particle, sorted order
  rt::DevBuf<int64_t> ptr;      // n_total + 1, sorted order
  rt::DevBuf<int32_t> idx;      // npairs, sorted indices, ascending per row
  rt::DevBuf<int32_t> n_int_nbrs;  // interior neighbours per interior row
};

namespace rt {
// One level of the operator hierarchy.  Level 0 is the assembled fine system;
// level l+1 has one node per aggregate of level-l nodes: pmap maps a node to
// its aggregate (-1: left out of the coarse space), and the members of
// aggregate I are amem[crange[I] .. crange[I+1]) in ascending order.
struct Level {
  int64_t n = 0, nnz = 0;       // nnz = off-diagonal entries
  int64_t max_row = 0;          // longest off-diagonal row
  int shape64 = -1, shape32 = -1;   // SpMV row-group shape per precision (-1: by max_row)
  int shape_res = -1;               // shape of the FP64 residual product (-1: shape64)
  // tiled form (see the file comment); tiled == false: plain CSR products only
  bool tiled = false;
  int64_t ntiles = 0, tile_cols_total = 0;
  int max_tile_cols = 0;
  DevBuf<int64_t> tile_off;     // ntiles + 1
  DevBuf<int32_t> tile_cols;    // tile_cols_total
  DevBuf<uint16_t> lcol;        // nnz + kSpmvPad
  DevBuf<int64_t> rp;
  DevBuf<int32_t> col;
  DevBuf<double> val64, diag64, sinv64, dinv64;   // sinv = l1-Jacobi smoother, dinv = 1/diag
  DevBuf<float> val32, diag32, sinv32, dinv32;
  DevBuf<uint64_t> code;        // Morton code of each node's cell block (candidate blocks)
  DevBuf<int32_t> pmap;         // node -> aggregate on the next level (-1: none)
  DevBuf<int64_t> crange;       // next-level aggregate -> offset of its members (n_next + 1)
  DevBuf<int32_t> amem;         // members of the aggregates, ascending per aggregate
  // smoothed prolongation to the next level (smoothed == false: piecewise
  // constant over pmap): P in CSR (rows = nodes, ascending columns) and its
  // transpose (rows = next-level nodes, ascending fine rows), FP64 and FP32
  bool smoothed = false;
  int64_t p_nnz = 0;            // entries of P (and of P^T)
  DevBuf<int64_t> p_rp, pt_rp;
  DevBuf<int32_t> p_col, pt_row;
  DevBuf<double> p_val, pt_val;
  DevBuf<float> p_val32, pt_val32;
  // work vectors of this level (b: right-hand side, x: result, t, r: temporaries)
  DevBuf<double> b64, x64, t64, r64, d64;   // d: Chebyshev search direction
  DevBuf<float> b32, x32, t32, r32, d32;
  DevBuf<double> wr64, wx64;   // W- and K-cycle: residual and correction of the second visit
  DevBuf<float> wr32, wx32;
  DevBuf<double> kw64;         // K-cycle: A times the first correction
  DevBuf<float> kw32;
  DevBuf<double> kpart;        // K-cycle: block partials of its inner products
  DevBuf<double> kc;           // K-cycle: its inner products and weights
};
template <typename T>
inline int level_shape(const Level& L) {
  return sizeof(T) == sizeof(double) ? L.shape64 : L.shape32;
}
// shape of the FP64 residual product b - A x of the refinement loop
inline int resid_shape(const Level& L) { return L.shape_res >= 0 ? L.shape_res : L.shape64; }
}  // namespace rt

struct rt_matrix {
  const rt_neighbors* nb = nullptr;
  int64_t n = 0;          // interior unknowns
  int64_t n_total = 0;
  double dt = 0, c = 1, a = 1;
  bool has_fp32 = false;
  rt_amg_opts amg{};
  // frozen per-step data, sorted order
  rt::DevBuf<double> V, D, sa, f, rho, cv, m, e_prev, E_prev, Qe, QE, g;
  rt::DevBuf<double> VD;        // 2 x n_total: (V, D) per particle, sorted order
  rt::DevBuf<double> Eall;      // E^{n-1} / ghost data for all particles (sorted)
  // hierarchy: levels[0] is the fine operator
  std::vector<rt::Level> levels;
  bool coarse_direct = false;        // coarsest level solved with a dense inverse
  int cycle_levels = 0;              // levels the V-cycle uses (0: all; set by the depth tuner)
  // a batch's hierarchy, per level (else empty): the map from 256-row chunks
  // to flag slots and the flags themselves, set for chunks whose rows all
  // belong to problems whose iteration has stopped; the V-cycle's products
  // leave those chunks as they are
  std::vector<const int32_t*> lvl_tprob, lvl_skip;
  rt::DevBuf<double> coarse_inv;     // dense inverse of the coarsest operator (FP64)
  // Krylov work vectors (fine size)
  rt::DevBuf<double> r64, p64, q64, z64, xs, bs, ecur, Ecur, enew;
  rt::DevBuf<float> r32, p32, q32, z32, d32;
  rt::DevBuf<double> partA, partB;   // block partials of the reductions
  rt::DevBuf<double> partC;          // block maxima of the componentwise residual measure
  rt::DevBuf<double> partF;          // second level of the partial reductions
  rt::DevBuf<float> w32;             // weights 1/(a_ii |x_i|) of the FP32 inner solve
  rt::DevBuf<double> scal;           // device scalars (see solve.hip)
  rt::DevBuf<int32_t> stop;          // PCG stop flag: set on the device when the loop ends
  // Residual carried between outer iterations: after a Newton step, r64 holds
  // bs - A xs for the step's right-hand side bs and solution xs (resid_ok);
  // bs_prev keeps that right-hand side while the next step forms its own, and
  // xmis counts particles whose state differs from xs at the next step.
  rt::DevBuf<double> bs_prev;
  rt::DevBuf<int32_t> xmis;
  bool resid_ok = false;
  bool r64_valid = false;            // set by solve_sorted: r64 = b - A x on return (the
                                     // recursive residual after FP64 CG: equal up to rounding)
  int rec_steps = 0;                 // CG steps r64 has been carried by the recursion since
                                     // it was last formed by a product (FP64 path)
};

namespace rt {
// tiled SpMV form of a level whose rp/col are final (tile.hip); leaves the
// level untiled when a tile has more than kTileMaxCols distinct columns
int build_tiles(rt_ctx* ctx, Level& L);

// neighbours
int build_neighbors(rt_ctx* ctx, int dim, int64_t n_total, int64_t n_interior,
                    const double* pos, const double* h, int kernel, const double* period,
                    rt_neighbors* nb);
// solve helpers used by the Newton step
// b_prev (else NULL): r64 holds b_prev - A x on entry, unless *mismatch
// (device counter) is non-zero; the initial residual is then r64 + (b - b_prev)
// instead of a product.
int solve_sorted(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                 const rt_solve_opts* o, rt_solve_stats* st, const double* b_prev = nullptr,
                 const int32_t* mismatch = nullptr);
int amg_setup(rt_ctx* ctx, rt_matrix* A);
// work vectors of a level of a V-cycle (cycle: rt_amg_opts.cycle)
int amg_level_vectors(Level& L, bool fp32, int cycle);
// levels the V-cycle uses: all, or the tuned depth
inline size_t cycle_depth(const rt_matrix* A) {
  const size_t nl = A->levels.size();
  return A->cycle_levels > 0 && (size_t)A->cycle_levels < nl ? (size_t)A->cycle_levels : nl;
}
// ||b - A x||^2 (an FP64 product, into the matrix's r64) and ||b||^2; the
// residual the Newton step carries is dropped
int residual_norms(rt_ctx* ctx, rt_matrix* A, const double* b, const double* x, double* rr,
                   double* bb);
int check_solve_opts(const rt_solve_opts* o);
int collect_profile(rt_ctx* ctx, rt_solve_stats* s);
int gather_sorted(rt_ctx* ctx, const rt_neighbors* nb, int64_t n, const double* user,
                  double* sorted);
int scatter_user(rt_ctx* ctx, const rt_neighbors* nb, int64_t n, const double* sorted,
                 double* user);
// One V-cycle z = M^-1 b; every kernel does nothing once *stop is set (stop
// may be NULL).
template <typename T>
int vcycle(rt_ctx* ctx, rt_matrix* A, const T* b, T* z, const int32_t* stop = nullptr);
int assemble(rt_ctx* ctx, const rt_neighbors* nb, const rt_step_inputs* in, rt_matrix* A,
             bool new_structure);
}  // namespace rt

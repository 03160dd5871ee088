/*
 * rt.h -- C ABI of the MI355X (gfx950) implicit SPH radiation-diffusion library.
 *
 * Paper: Bassett, Owen & Brunner, "Efficient smoothed particle radiation
 * hydrodynamics I: Thermal radiative transfer", arXiv:2001.11606.
 *
 * The library implements one time step of the paper's implicit scheme for grey
 * thermal radiative transfer with a stationary material: the nonlinear
 * elimination iteration of Algorithm 1, in which every outer iteration solves
 * one linear SPH diffusion system for the radiation energy E (Sec. 3.2, the
 * diffusion-solve operator D^-1) and then a per-particle nonlinear equation
 * for the material energy e (Sec. 3.2, the material operator M^-1).
 *
 * Conventions (all entry points):
 *   - Array arguments are DEVICE pointers owned by the caller; the library
 *     never frees or retains them beyond the call.  double = IEEE binary64.
 *   - Particles are in the caller's ("user") order.  Interior particles are
 *     [0, n_interior); constant-value (Dirichlet) ghost particles, the
 *     boundary treatment of Sec. 3.1, are [n_interior, n_total).
 *   - Positions are structure-of-arrays: pos[alpha * n_total + i].
 *   - Library objects (rt_ctx, rt_neighbors, rt_matrix) are opaque handles,
 *     created by the library and released with the matching *_free/destroy.
 *   - Every call is ordered on the context's HIP stream.  Calls that return
 *     counts or statistics synchronise that stream before returning.
 *   - Return value: RT_OK (0); a positive soft status (outputs valid); or a
 *     negative hard error (outputs undefined).  rt_last_error() returns a
 *     message for the last failing call on the calling thread.
 *   - Nothing here allocates or frees caller memory; library-owned device
 *     memory is released by the *_free/destroy calls.
 */
#ifndef RT_H
#define RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RT_OK 0
#define RT_NOT_CONVERGED 1   /* tolerance not reached within max iterations  */
#define RT_NONPHYSICAL 2     /* a material root was negative (clamped to 0)  */
#define RT_E_ARG (-1)        /* invalid argument (null, size, NaN, option)   */
#define RT_E_OOM (-2)        /* device allocation failed                     */
#define RT_E_DEVICE (-3)     /* HIP runtime error                            */
#define RT_E_STATE (-4)      /* objects do not belong together               */

/* ---- kernels (Sec. 2.3) -------------------------------------------------- */
#define RT_KERNEL_CUBIC_SPLINE 0  /* M4 cubic B-spline, support 2h           */
#define RT_KERNEL_WENDLAND_C4 1   /* the paper's Wendland C4, support h      */

/* ---- flux limiters (Sec. 2.1) ------------------------------------------- */
#define RT_LIMITER_NONE 0         /* lambda = 1/3 (Fick's law)               */
#define RT_LIMITER_LARSEN 1       /* lambda = (3^k + R^k)^(-1/k)             */
#define RT_LIMITER_LEVERMORE 2    /* lambda = (2 + R)/(6 + 3R + R^2)         */

/* ---- solver precision ---------------------------------------------------- */
#define RT_PREC_FP64 0   /* FP64 preconditioned CG                          */
#define RT_PREC_MIXED 1  /* FP32 inner PCG + FP64 iterative refinement       */

typedef struct rt_ctx rt_ctx;
typedef struct rt_neighbors rt_neighbors;
typedef struct rt_matrix rt_matrix;

/* ---- context --------------------------------------------------------------
 * rt_create: bind the calling thread's HIP device `device` and stream
 * `hip_stream` (a hipStream_t; NULL = the null stream).  *ctx receives a new
 * context.  Errors: RT_E_ARG (ctx NULL), RT_E_DEVICE.                        */
int rt_create(rt_ctx** ctx, int device, void* hip_stream);
/* rt_destroy: waits for the context's stream, then frees the context and the
 * device memory the library keeps cached for its device.                    */
void rt_destroy(rt_ctx* ctx);
int rt_set_stream(rt_ctx* ctx, void* hip_stream);
/* Record HIP events around every sparse matrix-vector product launch so that
 * rt_solve_stats.spmv_* report per-launch device time (on = 1).             */
int rt_set_profiling(rt_ctx* ctx, int on);
/* Device memory (a property of this library, not of the paper): buffers of
 * freed handles and of finished calls are kept by the library for reuse, per
 * device, instead of being returned to HIP (up to 96 GiB; an allocation that
 * fails frees them and is retried), so repeated builds of same-sized problems
 * allocate nothing.  rt_cached_bytes reports the bytes kept for ctx's device;
 * rt_release_cached synchronises the device and frees them (*freed_bytes, if
 * not NULL, receives the amount).  rt_destroy frees them too.               */
int rt_cached_bytes(const rt_ctx* ctx, int64_t* bytes);
int rt_release_cached(rt_ctx* ctx, int64_t* freed_bytes);
const char* rt_last_error(void);
const char* rt_version(void);

/* ---- neighbour lists (Sec. 2.3, Sec. 3.1) ----------------------------------
 * Particles i != j are neighbours when r_ij^2 < (kappa * max(h_i, h_j))^2,
 * r_ij^2 accumulated in axis order without fused multiply-add, kappa = 2
 * (cubic spline) or 1 (Wendland C4): every pair on which either term of the
 * symmetrised kernel W_ij = 1/2 [W(x_ij,h_i) + W(x_ij,h_j)] is non-zero.
 *
 * dim in {2, 3}; n_total >= 1; 0 <= n_interior <= n_total;
 * pos: dim x n_total (SoA); h: n_total, h > 0.  The particles are sorted
 * internally by a uniform cell grid; the result *out is library-owned.
 * Errors: RT_E_ARG (bad sizes, non-finite pos/h, h <= 0, grid too large).  */
int rt_build_neighbors(rt_ctx* ctx, int dim, int64_t n_total, int64_t n_interior,
                       const double* pos, const double* h, int kernel,
                       rt_neighbors** out);

/* Neighbour lists in a box with periodic axes (the periodic box of the
 * manufactured problem of Sec. 4.3).  period: host array of dim lengths, or
 * NULL (then this is rt_build_neighbors); period[a] > 0 makes axis a periodic
 * with that length, 0 leaves it open.  On a periodic axis every position must
 * lie in [0, period[a]) and the period must span at least three supports
 * (3 * kappa * max h); each displacement component x_i - x_j is replaced by
 * its nearest image (one period subtracted above period/2, added below
 * -period/2) before it is squared, and the assembly that uses these lists
 * (rt_assemble) takes the same images.
 * Errors: those of rt_build_neighbors; RT_E_ARG for a negative or non-finite
 * period, positions outside [0, period), or a period under three supports. */
int rt_build_neighbors_periodic(rt_ctx* ctx, int dim, int64_t n_total, int64_t n_interior,
                                const double* pos, const double* h, int kernel,
                                const double* period, rt_neighbors** out);

typedef struct {
  int dim;
  int kernel;
  int64_t n_total;
  int64_t n_interior;
  int64_t npairs;        /* directed pairs (each unordered pair counted twice) */
  int64_t ncells;        /* cells of the sorting grid                        */
  double cell_size;
} rt_neighbors_info;

int rt_neighbors_get_info(const rt_neighbors* nb, rt_neighbors_info* info);

/* Neighbour lists in user order, ascending neighbour index per row:
 * nbr_ptr (n_total + 1, int64) and nbr_idx (npairs, int32), device memory
 * provided by the caller.                                                  */
int rt_neighbors_export(rt_ctx* ctx, const rt_neighbors* nb, int64_t* nbr_ptr,
                        int32_t* nbr_idx);

/* perm[s] = user index of the particle at internal (cell-sorted) position s
 * (n_total int32, device).                                                 */
int rt_neighbors_order(rt_ctx* ctx, const rt_neighbors* nb, int32_t* perm);
void rt_neighbors_free(rt_neighbors* nb);

/* ---- per-step assembly (Sec. 2.2, 2.4, 3.2) --------------------------------
 * Material data is frozen at the start of the step (Sec. 3.2):
 *   T = e/c_v, sigma_a = sigma0_a T^opacity_exponent, sigma_t = sigma_a + sigma_s,
 *   f = 1/(1 + c sigma_a dt 4 a T^3/(rho c_v))      (Fleck factor, Sec. 2.2)
 *   V = m/rho                                        (Sec. 2.3)
 *   D = c lambda / sigma_t                           (Sec. 2.4)
 * with lambda = 1/3 or a flux limiter of R = |grad E|/(sigma_t E) using the
 * SPH first derivative of E (Sec. 2.1, 2.3); ghosts always use lambda = 1/3.
 * The diffusion system of Sec. 3.2 (the D^-1 operator), each row multiplied
 * by V_i, is assembled into CSR:
 *   A_ii = V_i (1/dt + c sigma_a,i f_i) + V_i sum_j a_ij,
 *   A_ij = -V_i V_j (D_i + D_j) F_ij                  (interior j),
 *   F_ij = -1/2 [W'(r_ij,h_i) + W'(r_ij,h_j)] / r_ij,  a_ij = V_j (D_i + D_j) F_ij,
 * which is symmetric positive definite; ghost couplings move to the
 * right-hand side.  An aggregation-AMG hierarchy is set up for the
 * preconditioner, once per step (Sec. 3.2 reuses the preconditioner for the
 * whole step).
 *
 * All arrays are n_total long, user order, device.  sigma_s, Q_e and Q_E may
 * be NULL (zero).  e and E hold e^{n-1}, E^{n-1} for interior particles and
 * the boundary values of the step for ghosts.  Q_e/Q_E are the sources Q^n.
 * *A: if non-NULL on entry and built from the same neighbour object, its
 * storage is reused; otherwise a new matrix is created.                      */
typedef struct {
  double dt, c, a;
  double opacity_exponent;
  int limiter;
  double limiter_k;
  const double* m;
  const double* rho;
  const double* cv;
  const double* sigma0_a;
  const double* sigma_s;
  const double* e;
  const double* E;
  const double* Q_e;
  const double* Q_E;
} rt_step_inputs;

typedef struct {
  int max_levels;        /* AMG levels including the fine one; 1 = Jacobi only */
  int coarse_size;       /* stop coarsening at or below this many unknowns     */
  double strength;       /* strength-of-connection threshold theta: a_ij couples
                            i and j strongly when |a_ij| >= theta sqrt(m_i m_j),
                            m_i the largest |a_ik| of row i; rows whose
                            off-diagonal sum is below 5% of a_ii stay out of
                            the coarse space; aggregates grow from one root per
                            neighbour-search cell (Morton block of cells on
                            coarser levels) over strong couplings.  theta <= 0:
                            each cell / Morton block is one aggregate
                            (geometric aggregation).  The hierarchy is rebuilt
                            with every rt_assemble.                           */
  int build_fp32;        /* 1: also build the FP32 copies for RT_PREC_MIXED    */
  int tiled_spmv;        /* 1: also build the tiled product form of each level
                            (16-bit tile-local columns, x staged in LDS)      */
  int smoother;          /* V-cycle smoother on every level above the coarsest:
                            RT_SMOOTHER_L1_JACOBI (one sweep before and one
                            after the coarse correction) or
                            RT_SMOOTHER_CHEBYSHEV (a Chebyshev polynomial of
                            degree smoother_degree in D1^-1 A before and after,
                            D1 the l1 diagonal a_ii + sum_j |a_ij|, on the
                            interval [1/4, 1] that contains the upper part of
                            its spectrum, which lies in (0, 1])               */
  int smoother_degree;   /* 1..8, Chebyshev only                              */
  int cycle;             /* 1: V-cycle; 2: W-cycle (on every level above the
                            coarsest, two coarse corrections, the second from
                            the residual of the first: the same symmetric
                            operator as two steps of the coarse cycle);
                            3: K-cycle (on every coarse level but the
                            coarsest, the two corrections are weighted as two
                            steps of flexible CG, the weights formed from
                            inner products on the device; the preconditioner
                            then varies slightly with its argument)          */
  int prolongation;      /* RT_PROLONG_PIECEWISE: constant over each aggregate;
                            RT_PROLONG_SMOOTHED: smoothed aggregation,
                            P = (I - 4/3 D1^-1 A) P0 with P0 the piecewise
                            constant one and D1 the l1 diagonal (rows left out
                            of the coarse space keep P = 0); the coarse
                            operator is P^T A P either way                    */
} rt_amg_opts;

#define RT_PROLONG_PIECEWISE 0
#define RT_PROLONG_SMOOTHED 1
#define RT_CYCLE_V 1
#define RT_CYCLE_W 2
#define RT_CYCLE_K 3

#define RT_SMOOTHER_L1_JACOBI 0
#define RT_SMOOTHER_CHEBYSHEV 1

int rt_assemble(rt_ctx* ctx, const rt_neighbors* nb, const rt_step_inputs* in,
                const rt_amg_opts* amg /* NULL = defaults */, rt_matrix** A);
/* AMG defaults: max_levels 8, coarse_size 256, strength 0.25, build_fp32 1,
 * tiled_spmv 1, smoother RT_SMOOTHER_L1_JACOBI, smoother_degree 2, cycle 1,
 * prolongation RT_PROLONG_PIECEWISE.
 * Errors: RT_E_ARG for an unknown smoother, a degree outside 1..8, a cycle
 * other than 1, 2 or 3, or an unknown prolongation.                        */

typedef struct {
  int64_t n;             /* unknowns = interior particles                     */
  int64_t nnz;           /* stored entries including the diagonal            */
  int levels;
  int64_t level_n[16];
  int64_t level_nnz[16];
  int64_t level_tile_cols[16]; /* distinct columns summed over the level's
                                  256-row tiles; 0 = level not tiled          */
  int64_t level_p_nnz[16];  /* entries of the smoothed prolongation from this
                               level to the next; 0 = piecewise constant     */
} rt_matrix_info;

int rt_matrix_get_info(const rt_matrix* A, rt_matrix_info* info);

/* The assembled system in user order over interior particles, ascending
 * columns, diagonal included: row_ptr (n+1 int64), col (nnz int32), val (nnz
 * double), ghost_rhs (n double, the ghost coupling g_i added to b).         */
int rt_matrix_export(rt_ctx* ctx, const rt_matrix* A, int64_t* row_ptr, int32_t* col,
                     double* val, double* ghost_rhs);
void rt_matrix_free(rt_matrix* A);

/* ---- SpMV shape tuning (not in the paper; a property of this library) -----
 * Every sparse product y = A x over a level runs with a row-group shape: G
 * lanes per row, each holding E entries, so that one pass covers G*E entries
 * of a row.  Tiled shapes (tiled = 1) use the level's tiled form: each lane
 * loads four consecutive entries as one 16-byte chunk (a pass covers 4*G
 * entries), x is read from LDS, and E is the number of rows a lane group
 * keeps in flight; a level without a tiled form runs its default plain shape
 * instead.
 * rt_spmv_shapes writes the (G, E, tiled) of up to max shapes (any pointer
 * may be NULL) and returns how many exist.  rt_matrix_tune times the Krylov-loop product on every
 * level of A with every shape, in FP64 and, when A holds FP32 copies, FP32,
 * and (with FP32 copies, fine level only) the FP64 residual product b - A x
 * of the mixed-precision refinement loop: one untimed launch, then reps
 * launches between HIP events on the library stream.  It keeps the fastest
 * shape per level and product for all later products of A and writes the
 * timings (microseconds per product; 0 = not timed) and choices (-1 = none)
 * to *rep when rep is not NULL.  It synchronises the stream and allocates
 * temporary vectors.
 * rt_matrix_set_spmv_shape forces a shape (index into the table; -1 restores
 * the default, picked from the level's longest row: tiled shapes with two
 * rows in flight on tiled levels, else the smallest plain shape whose one
 * pass covers the row; the residual product's default is the FP64 product's
 * shape).  Results of a product do not depend on the shape beyond the order
 * of floating-point additions within a row.                                  */
#define RT_MAX_LEVELS 16
#define RT_MAX_SHAPES 24
#define RT_PRODUCT_RESIDUAL 2     /* rt_matrix_set_spmv_shape: the FP64 residual product */
typedef struct {
  int levels;                                 /* levels timed                  */
  int shapes;                                 /* shapes timed per level        */
  double us[RT_MAX_LEVELS][3][RT_MAX_SHAPES]; /* [level][0 FP64, 1 FP32, 2 FP64
                                                 residual][shape]              */
  int chosen[RT_MAX_LEVELS][3];
} rt_tune_report;

int rt_spmv_shapes(int* g, int* ent, int* tiled, int max);
int rt_matrix_tune(rt_ctx* ctx, rt_matrix* A, int reps, rt_tune_report* rep);
/* precision: RT_PREC_FP64 selects the FP64 product, RT_PREC_MIXED the FP32 one,
 * RT_PRODUCT_RESIDUAL the FP64 residual product of the refinement loop      */
int rt_matrix_set_spmv_shape(rt_matrix* A, int level, int precision, int shape);


/* ---- linear solve (Sec. 3.2, the D^-1 operator) ---------------------------
 * Solves A x = b (the V-scaled system above) by preconditioned CG, stopping
 * when ||b - A x||_2 <= tol ||b||_2 evaluated in FP64 and, if cw_tol > 0,
 * also max_i |b - A x|_i / (a_ii |x_i|) <= cw_tol (componentwise test: the
 * largest relative change one Jacobi sweep would make to an unknown; a row
 * with x_i = 0 passes only with a zero residual).  The normwise test alone
 * does not bound the relative error of unknowns far below the largest one
 * (E over several decades); the componentwise test does, up to the factor
 * 1/(1 - rho) of the off-diagonal row sums rho relative to a_ii.
 * b, x: n_interior doubles, user order, device; x is the initial guess on
 * entry (the paper warm-starts with E^l) and the solution on return.
 * precond: 0 = Jacobi, 1 = AMG V-cycle (falls back to Jacobi when the
 * hierarchy has one level).  RT_PREC_MIXED runs FP32 PCG on the correction
 * equation A d = r to inner_tol, adds d in FP64 and recomputes r = b - A x in
 * FP64, until tol (and cw_tol).  Returns RT_NOT_CONVERGED (stats valid) if
 * max_iter (total inner iterations) or max_refine is exhausted.
 * Errors: RT_E_ARG (unknown precision or precond, tol < 0, cw_tol < 0 or NaN,
 * max_iter < 0, MIXED with inner_tol outside (0, 1)).                       */
typedef struct {
  int precision;
  int precond;
  double tol;
  int max_iter;
  double inner_tol;
  int max_refine;
  double cw_tol;         /* componentwise tolerance; 0 = normwise test only   */
} rt_solve_opts;

typedef struct {
  int iterations;          /* Krylov iterations (inner ones in MIXED)        */
  int refinements;         /* FP64 residual recomputations (MIXED)           */
  double rel_residual;     /* final ||b - A x|| / ||b|| in FP64              */
  double seconds;          /* wall time of the solve (device-synchronised)   */
  int spmv_calls;          /* SpMV launches timed (profiling on)             */
  double spmv_seconds;     /* their summed device time                       */
  int spmv32_calls;
  double spmv32_seconds;
  double cw_residual;      /* final max_i |b - A x|_i / (a_ii |x_i|): from an
                              FP64 product (MIXED) or the CG recursion (FP64) */
  int resid_calls;         /* FP64 residual products b - A x timed (profiling on) */
  double resid_seconds;
  double init_rel_residual; /* ||b - A x0|| / ||b|| at the start: from an FP64
                              product, or from the residual rt_newton_step
                              carries over from its last solve              */
  int replacements;        /* FP64: times CG's recursive residual was replaced
                              by a computed b - A x (after more than 32 CG
                              steps since the last computed one, counting
                              steps carried over by rt_newton_step)          */
} rt_solve_stats;

int rt_solve(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
             const rt_solve_opts* opts, rt_solve_stats* stats);

/* V-cycle depth.  rt_matrix_tune_depth solves A x = b from x0 (n_interior
 * doubles each, device, user order; x0 is not changed) with opts (precond
 * must be 1) using the first d levels of the hierarchy, for every d from 1
 * (Jacobi) to the number of levels, reps times each, and keeps the depth with
 * the least mean solve time (rt_solve_stats.seconds) among those that
 * converged; the deepest level used is then smoothed instead of being solved
 * directly unless it is the hierarchy's last.  *rep (may be NULL) receives
 * every depth's mean time, iterations and status and the choice.  The depth
 * holds for later solves and V-cycles of A, also after re-assembly (clamped
 * to the hierarchy's levels).  rt_matrix_set_cycle_depth sets it (0 = all
 * levels).  Errors: RT_E_ARG (NULL arguments, reps < 1, precond not 1, a
 * negative depth); a solve's own errors.                                    */
typedef struct {
  int depths;                      /* depths timed: 1 .. depths              */
  double seconds[RT_MAX_LEVELS];   /* [d - 1]: mean wall time of a solve      */
  int iterations[RT_MAX_LEVELS];   /* Krylov iterations of the last solve     */
  int status[RT_MAX_LEVELS];       /* RT_OK or RT_NOT_CONVERGED               */
  int chosen;                      /* the depth kept                          */
} rt_depth_report;

int rt_matrix_tune_depth(rt_ctx* ctx, rt_matrix* A, const double* b, const double* x0,
                         const rt_solve_opts* opts, int reps, rt_depth_report* rep);
int rt_matrix_set_cycle_depth(rt_matrix* A, int depth);

/* rt_solve_noalloc: rt_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, options, results and errors as rt_solve, but
 * the call makes no device allocation and no hipMalloc/hipFree: the gathered
 * b and x, the Krylov work vectors, block partials and scalars live in one
 * static device array of the library (256 MiB per GPU, set up by rt_create
 * and held until the process ends).  Scratch needed: 256-byte-aligned pieces
 * of 8 bytes x 6n (+ 4 bytes x 6n in RT_PREC_MIXED) plus 3 arrays of block
 * partials of about n/4 + 4096 doubles, about 54 bytes per unknown in FP64
 * and 78 in mixed precision: n up to 4,968,256 unknowns in FP64 and
 * 3,439,552 in mixed precision; a larger matrix is rejected with RT_E_ARG
 * and a message giving the bytes needed.  The matrix (and its
 * AMG hierarchy) must come from rt_assemble, whose buffers the V-cycle uses;
 * the residual rt_newton_step carries between outer iterations is left as
 * it was.  No per-product timings are recorded (stats->spmv_* are 0).
 * Every call on one GPU uses the same array and leaves its contents behind:
 * calls that overlap on one GPU (other streams, other contexts or threads)
 * race, and so do calls on one matrix overlapping with rt_solve or
 * rt_newton_step.                                                           */
int rt_solve_noalloc(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                     const rt_solve_opts* opts, rt_solve_stats* stats);

/* ---- one outer iteration of Algorithm 1 ------------------------------------
 * e, E: n_interior doubles, user order, device, holding the iterate
 * (e^{n,l}, E^{n,l}) on entry and (e^{n,l+1}, E^{n,l+1}) on return.
 * If ell == 0, first solves m(e, E^{n,0}) = 0 for e from e^{n-1} (the
 * initial material solve of Algorithm 1).  Then: right-hand side
 *   b_i = V_i [E_i^{n-1}/dt + c sigma_a a T(e_i^l)^4 - (1 - f_i) c sigma_a E_i^l + Q_E,i] + g_i,
 * linear solve warm-started from E^l, and the per-particle material solve
 *   rho/dt (e - e^{n-1}) + c sigma_a a (e/c_v)^4 = Q_e + c sigma_a E^{l+1}
 * by bracketed Newton from e^l to |de/e| <= material_tol (Sec. 3.2).
 * stats: delta_e = max_i |e^{l+1} - e^l|/|e^{l+1}|, delta_E likewise
 * (Sec. 2.2 convergence test), energy = sum_i (m_i e_i + V_i E_i) (Sec. 2.5).
 * Returns RT_NONPHYSICAL if a material root was negative, RT_NOT_CONVERGED
 * if the linear or a material solve did not converge.
 * state_order 0: e and E are in user order; 1: in the library's cell-sorted
 * order of the neighbour object (rt_to_sorted / rt_to_user convert), which
 * saves two gathers and two scatters per call for callers that keep their
 * state in that order between steps (particles are stationary).             */
typedef struct {
  rt_solve_opts solve;
  double material_tol;
  int material_max_iter;
  int state_order;
  int recompute_residual;  /* 0: an outer iteration after the first starts its
                              solve from the last solve's residual plus the
                              change of b (no product); 1: from b - A x formed
                              by an FP64 product.  rt_batch_newton_step always
                              forms it and ignores this field.                */
} rt_newton_opts;

typedef struct {
  double delta_e;
  double delta_E;
  double energy;
  double energy_prev;      /* sum_i (m_i e_i^{n-1} + V_i E_i^{n-1})           */
  int material_iterations; /* max over particles, last material solve        */
  int64_t nonphysical;     /* particles with a negative root                 */
  rt_solve_stats solve;
  double seconds;
} rt_newton_stats;

int rt_newton_step(rt_ctx* ctx, rt_matrix* A, double* e, double* E, int ell,
                   const rt_newton_opts* opts, rt_newton_stats* stats);

/* ---- residual of the backward-Euler system (Sec. 2.2) ----------------------
 * G = [m, r] at the state (e, E) (n_interior doubles each, device; user
 * order, or the neighbour object's sorted order with state_order 1), with the
 * matrix's frozen data of the step (rt_assemble):
 *   m_i = rho_i/dt (e_i - e_i^{n-1}) + c sigma_a,i (B_i - E_i) - Q_e,i,
 *   r_i = (E_i - E_i^{n-1})/dt - <d(c lambda/sigma_t dE)>_i + c sigma_a,i (E_i - B_i) - Q_E,i,
 * B = a (e/c_v)^4.  Evaluated in FP64 as V r = A E - b(e, E), b the
 * right-hand side of the outer iteration taken at the state itself.  The
 * starting residual of every rt_newton_step solve (rt_solve_stats.
 * init_rel_residual) is rad_rel of the state that call starts from; this call
 * gives it for any state, e.g. the step's last one, at the cost of one FP64
 * product.  It drops the residual rt_newton_step carries over.
 * Errors: RT_E_ARG (NULL argument, state_order not 0 or 1).                */
typedef struct {
  double rad_norm;   /* ||V r||_2 = ||A E - b(e, E)||_2                        */
  double rad_rel;    /* rad_norm / ||b(e, E)||_2                              */
  double mat_rel;    /* max_i |m_i| / (rho_i |e_i| / dt)                      */
} rt_be_residual;

int rt_newton_residual(rt_ctx* ctx, rt_matrix* A, const double* e, const double* E,
                       int state_order, rt_be_residual* out);

/* Interior per-particle vectors between user order and the library's sorted
 * order (n = n_interior doubles, device; in and out must not overlap).      */
int rt_to_sorted(rt_ctx* ctx, const rt_neighbors* nb, const double* user, double* sorted);
int rt_to_user(rt_ctx* ctx, const rt_neighbors* nb, const double* sorted, double* user);

/* ---- GMRES on the unscaled operator (Sec. 3.2, the paper's solver) ---------
 * rt_solve_gmres solves the same system as rt_solve in the paper's own,
 * unscaled form U x = c, U = diag(V)^-1 A, c = diag(V)^-1 b (A, b the
 * V-scaled operator and right-hand side of rt_solve; same solution x), with
 * restarted right-preconditioned GMRES(restart) in FP64.  precond: 0 Jacobi
 * (diag(U)^-1), 1 the matrix's AMG V-cycle applied to V v (Jacobi when the
 * matrix has one level).  Stops when ||c - U x||_2 <= tol ||c||_2 (the final
 * value recomputed from a product, in stats->rel_residual) or after max_iter
 * inner iterations (RT_NOT_CONVERGED, x then holds the last iterate).
 * b, x: n_interior doubles, user order, device; x is the initial guess on
 * entry.  The method keeps restart + 1 basis vectors of n doubles.  Errors:
 * RT_E_ARG (precond not 0/1, tol < 0, max_iter < 0, restart outside 1..64,
 * non-finite b), RT_E_DEVICE (non-finite residual).                         */
typedef struct {
  int precond;
  double tol;
  int max_iter;
  int restart;
} rt_gmres_opts;

int rt_solve_gmres(rt_ctx* ctx, rt_matrix* A, const double* b, double* x,
                   const rt_gmres_opts* opts, rt_solve_stats* stats);

/* ---- time-step control (Sec. 3.3) -----------------------------------------
 * The fractional changes of the material and radiation energies over a step,
 *   eta_e = max_i |e_i^n - e_i^{n-1}| / (e_i^n + eta_target Ebar^n + tiny),
 *   eta_E = max_i |E_i^n - E_i^{n-1}| / (E_i^n + eta_target Ebar^n + tiny),
 * Ebar^n = sum_i E_i^n V_i / sum_i V_i over interior particles (V from A):
 * the floor of both is the mean radiation energy, the reading of Sec. 3.3
 * under which this rule reproduces the step counts of Sec. 4.1 to within one.
 * eta[0] = eta_e, eta[1] = eta_E.  The next step is
 * dt (eta_target / eta)^(1/2), the smaller of the two, within the user's
 * bounds (the host driver applies that rule).  e_*, E_*: n_interior doubles,
 * user order, device; tiny (>= 0) guards an energy that is zero everywhere. */
int rt_fractional_change(rt_ctx* ctx, const rt_matrix* A, const double* e_new,
                         const double* e_old, const double* E_new, const double* E_old,
                         double eta_target, double tiny, double* eta);

/* ---- ensembles of independent problems (Sec. 3.2 per problem, batched) ----
 * Not in the paper: many independent problems advanced together, one launch
 * per kernel for the whole ensemble.  rt_batch_create concatenates the
 * fine-level systems of nprob matrices (each from rt_assemble; FP32 copies
 * in all of them for RT_PREC_MIXED) into one block-diagonal system, each
 * problem padded with identity rows to a multiple of 256 rows, plus the
 * per-particle data of the Newton step; each problem keeps its own dt, c, a.
 * The batch copies what it needs: the matrices may be freed afterwards; after
 * re-assembling them, create a new batch.  Solves use preconditioned CG
 * (cw_tol must be 0) with per-problem Krylov scalars and per-problem
 * convergence: a problem that meets its tolerance stops while the others go
 * on.  precond 0: Jacobi.  precond 1: the V-cycle of the batch's hierarchy,
 * which concatenates the problems' own aggregation hierarchies level by
 * level (built by rt_batch_create when the matrices have more than one level
 * and piecewise-constant prolongations; else precond 1 is Jacobi).  Each
 * problem contributes the levels of its own V-cycle depth at the time of
 * rt_batch_create (all, unless rt_matrix_set_cycle_depth or
 * rt_matrix_tune_depth set it on its matrix).  It is one
 * block-diagonal V-cycle: every problem's own levels, smoother and
 * aggregates; the last level of each problem is smoothed (l1-Jacobi, three
 * sweeps on the batch's last level) rather than solved directly.
 * The V-cycle's products and vector passes skip the rows of problems that
 * have stopped (on coarse levels, 256-row chunks all of whose problems have).
 * graph_iters > 0 replays HIP graphs of that many PCG iterations (Jacobi or
 * V-cycle) between host reads of the convergence flags (extra iterations of
 * finished problems change none of their values); 0 checks after every
 * iteration.
 * Vectors (b, x, e, E) are the problems' interior vectors concatenated in
 * problem order, each in its own user order (problem p at the offset
 * sum_{q<p} n_interior(q)), device memory.  stats arrays hold nprob entries
 * (or are NULL).  Returns the worst status over the problems.               */
typedef struct rt_batch rt_batch;
int rt_batch_create(rt_ctx* ctx, int nprob, rt_matrix* const* mats, rt_batch** out);
void rt_batch_free(rt_batch* B);
/* rows (padded), stored off-diagonal entries, tile columns (0 = untiled) */
int rt_batch_get_info(const rt_batch* B, int64_t* rows, int64_t* nnz, int64_t* tile_cols);
/* rt_matrix_tune / rt_matrix_set_spmv_shape on the batch's hierarchy (level
 * 0 the concatenated fine operator; the shape set applies to level 0)     */
int rt_batch_tune(rt_ctx* ctx, rt_batch* B, int reps, rt_tune_report* rep);
int rt_batch_set_spmv_shape(rt_batch* B, int precision, int shape);
int rt_batch_solve(rt_ctx* ctx, rt_batch* B, const double* b, double* x,
                   const rt_solve_opts* opts, int graph_iters, rt_solve_stats* stats);
/* The depth of the batch's V-cycle: how many levels of its hierarchy the
 * cycle uses (1: Jacobi instead of the V-cycle; 0: all).  A depth shorter
 * than the hierarchy smooths on its last level.  rt_batch_tune_depth runs
 * rt_batch_solve with opts (precond must be 1) and graph_iters at every
 * depth from 1 to the hierarchy's levels, once untimed and then reps times
 * (b, x0: concatenated device vectors as for rt_batch_solve; x0 is not
 * changed), and keeps the depth whose solve took the least wall time among
 * those that converged.  *rep (may be NULL) receives every depth's mean
 * time, the largest per-problem iteration count and the status.  The
 * depth holds for later batched solves and Newton steps of B.  For callers
 * whose ensemble is solved in batches: a depth timed inside the batch, not
 * one tuned per problem on its own solve.  rt_batch_set_cycle_depth sets
 * the depth (negative: RT_E_ARG); both drop the batch's cached graphs.     */
int rt_batch_tune_depth(rt_ctx* ctx, rt_batch* B, const double* b, const double* x0,
                        const rt_solve_opts* opts, int graph_iters, int reps,
                        rt_depth_report* rep);
int rt_batch_set_cycle_depth(rt_batch* B, int depth);
/* One outer iteration of Algorithm 1 for every problem (ell == 0 first does
 * the initial material solve), as rt_newton_step per problem.              */
int rt_batch_newton_step(rt_ctx* ctx, rt_batch* B, double* e, double* E, int ell,
                         const rt_newton_opts* opts, int graph_iters, rt_newton_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */

/*
 * rbf_fmm.h -- C ABI of the MI355X (gfx950) band-limited FMM library.
 *
 * The library computes the RBF sum of Zhao & Stoll, "A Fast Multipole Method based on
 * Band-limited Approximations for Radial Basis Functions" (arXiv 1606.07652),
 *
 *     u_i = sum_{j=1..N} lambda_j Phi(x_i - x_j),   i = 1..N            (section 1, eq. 1)
 *
 * with the near/far split of eq. (38): neighbouring groups are summed directly, all
 * other kept pairs go through the band-limited quadrature kernel of eq. (29)/(35)
 * factorised as in eq. (37) (aggregation, diagonal translation, disaggregation).  It also
 * solves A lambda = f with restarted GMRES (section 1 names GMRES as the Krylov method
 * the fast product serves).
 *
 * Conventions for every entry point:
 *  - Pointers named "device" are HIP device pointers (for example the storage of a torch
 *    tensor on cuda:0).  Pointers named "host" are ordinary host memory.
 *  - Arrays are dense and contiguous; points are row-major (n, d).
 *  - dtype RBF_F32 means float32 arrays, RBF_F64 float64 arrays.  The plan's dtype is the
 *    arithmetic type of the whole path (near field, expansions, output).
 *  - Return value: 0 (RBF_OK) on success, RBF_ENOCONV (+1) for a solve that stopped at
 *    its iteration cap, a negative RBF_E* code on error.  After an error
 *    rbf_last_error() returns a message (thread-local, valid until the next call on the
 *    same thread).  Output arguments are written only on success.
 *  - Work is enqueued on the HIP stream given to rbf_fmm_plan and is asynchronous with
 *    respect to the host unless stated otherwise.  Calls on one plan must not overlap.
 */
#ifndef RBF_FMM_H
#define RBF_FMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RBF_OK = 0, RBF_ENOCONV = 1, RBF_EINVAL = -1, RBF_EUNSUPPORTED = -2, RBF_ENOMEM = -3,
       RBF_EHIP = -4, RBF_ESTATE = -5 };
enum { RBF_F32 = 0, RBF_F64 = 1 };
/* Kernels of the paper's table "Global functions" (section 2.2).  The Gaussian is used in
 * the shape form exp(-r^2 / (2 s^2)) (shape = s > 0); the multiquadric is sqrt(r^2 + c^2)
 * (shape = c > 0). */
enum { RBF_GAUSSIAN = 0, RBF_MULTIQUADRIC = 1 };
enum { RBF_PC_NONE = 0, RBF_PC_BLOCK_JACOBI = 1, RBF_PC_LEARNED = 2 };

/* Optional planning overrides; zero or negative fields mean "choose automatically".
 * Fields override the tolerance rule for tests and tuning. */
typedef struct rbf_opts {
    int    n_max;        /* leaf capacity: boxes with more points are split (default 128) */
    int    max_level;    /* deepest tree level allowed (default: the quantisation depth) */
    int    min_level;    /* levels above this are always split (default: the coarse level) */
    int    coarse_level; /* level l_c of the coarse far-field stencil (-1 = rule) */
    int    coarse_radius;/* stencil radius r in cells at l_c (-1 = rule) */
    int    nodes;        /* quadrature nodes per dimension Mn, even (0 = rule) */
    double band;         /* band limit sigma (0 = rule) */
    int    m2l_schedule; /* leaf-translation block order: 0 or 1 = contiguous leaf ranges per
                            XCD (default), 2 = leaf-major over the whole grid */
    int    reserved[7];
} rbf_opts;

typedef struct rbf_plan rbf_plan;

/* Plan: build the tree, lists and quadrature tables for a fixed point set.
 *   points  device, (n, d) row-major, dtype; copied (sorted) into plan storage, so the
 *           caller may free it after the call returns.
 *   n >= 1, 1 <= d <= 5 (d in {2, 3, 5} are compiled), shape > 0, 0 < tol < 1
 *           (target relative 2-norm error of the product against the exact sum).
 *   opts    host, may be NULL.
 *   stream  a hipStream_t (NULL = default stream); all later work of the plan runs on it.
 *   out     host; receives the plan.  The plan owns its device memory until
 *           rbf_fmm_destroy.
 * Errors: RBF_EINVAL (bad sizes or parameters), RBF_EUNSUPPORTED (kernel, dimension or a
 * quadrature grid too large for the stated tolerance), RBF_ENOMEM, RBF_EHIP.
 * This call synchronises the stream (the tree build reads counts back). */
int rbf_fmm_plan(const void *points, int64_t n, int d, int dtype, int kernel, double shape,
                 double tol, const rbf_opts *opts, void *stream, rbf_plan **out);

/* Matrix-vector product u = A lambda (eq. 1 approximated by eq. 38).
 *   lambda  device, length n, plan dtype, caller's point order.
 *   u       device, length n, plan dtype, caller's order; overwritten.  Must not alias
 *           lambda.  Non-finite inputs propagate and are not checked. */
int rbf_fmm_matvec(rbf_plan *plan, const void *lambda, void *u);

/* Exact O(N^2) product on the device over all pairs (eq. 1), same layout as
 * rbf_fmm_matvec; the reference the fast product is measured against. */
int rbf_direct_matvec(rbf_plan *plan, const void *lambda, void *u);

typedef struct rbf_solve_opts {
    int    restart;      /* Krylov subspace size m of GMRES(m) (default 50) */
    int    max_iters;    /* total inner-iteration cap (default 1000) */
    int    precond;      /* RBF_PC_NONE, RBF_PC_BLOCK_JACOBI or RBF_PC_LEARNED */
    int    zero_init;    /* nonzero: start from lambda = 0, else from the given lambda */
    int    fallback;     /* nonzero: on breakdown, stagnation or non-finite output of the
                            preconditioner, restart without it (default on) */
    double time_limit_s; /* wall-time cap in seconds (0 = none) */
    int    reserved[8];
} rbf_solve_opts;

typedef struct rbf_solve_info {
    int    iters;        /* inner iterations (matrix-vector products inside Arnoldi) */
    int    restarts;
    int    converged;
    int    fallback_used;/* 1 if the preconditioner was switched off during the solve */
    double true_res;     /* ||f - A lambda|| / ||f|| with a fresh product at exit */
    double seconds;      /* wall time of the solve */
    double history[256]; /* true relative residual at each restart (first 256) */
    int    nhistory;
} rbf_solve_info;

/* Solve A lambda = f by restarted GMRES with the fast product (section 1).
 *   f       device, length n, plan dtype, caller order.
 *   lambda  device, length n, plan dtype: initial guess in (unless opts->zero_init), the
 *           solution out (the best iterate when the cap is reached).
 *   rtol    stop when ||f - A lambda|| / ||f|| <= rtol, recomputed with a fresh product.
 * Arnoldi vectors are kept in FP64 on the device (m+1 vectors of n doubles).
 * Returns RBF_OK, RBF_ENOCONV when a cap was reached, or an error.  Synchronous. */
int rbf_interp_solve(rbf_plan *plan, const void *f, void *lambda, double rtol,
                     const rbf_solve_opts *opts, rbf_solve_info *info);

/* Destroy a plan and free its device memory (NULL is accepted). */
int rbf_fmm_destroy(rbf_plan *plan);

/* Message for the last error on this thread ("" if none). */
const char *rbf_last_error(void);

typedef struct rbf_plan_info {
    int64_t n;
    int     d, dtype, kernel;
    int     nleaves, nlevels, coarse_level, coarse_radius, nodes, bits;
    int64_t half_nodes;   /* expansion length per box: nodes^(d-1) * nodes/2 */
    int64_t ncells;       /* cells of the dense coarse grid: 2^(d * coarse_level) */
    int64_t nnear;        /* total length of the near lists */
    int64_t near_pairs;   /* point pairs evaluated directly */
    double  shape, tol, band, period, rcut, rfar, ext;
    double  lo[5];
    int64_t device_bytes;
    int     far_field;    /* 0 when every kept pair is a near pair (no expansions) */
    int     reserved;
} rbf_plan_info;

/* Parameters and sizes chosen by the plan (host struct). */
int rbf_fmm_plan_info(const rbf_plan *plan, rbf_plan_info *info);

/* Copy the tree to host arrays (for comparison with an independent tree):
 *   perm        host int64[n]: input index of the i-th point in Morton order
 *   leaf_begin  host int32[nleaves + 1]
 *   leaf_level  host int32[nleaves]
 *   leaf_prefix host uint64[nleaves]: Morton prefix of each leaf at its level
 *   near_ptr    host int32[nleaves + 1], near_idx host int32[nnear] (sorted per leaf)
 * Any pointer may be NULL to skip that array.  Synchronous. */
int rbf_fmm_tree_export(const rbf_plan *plan, int64_t *perm, int32_t *leaf_begin,
                        int32_t *leaf_level, uint64_t *leaf_prefix, int32_t *near_ptr,
                        int32_t *near_idx);

/* Phase timing with HIP events on the plan's stream.  While enabled, each matvec
 * records an event pair around every phase and waits for them at its end.
 * Phases: 0 permute, 1 near field (P2P), 2 aggregation (P2M), 3 upward sum (M2M),
 * 4 coarse translation (M2L stencil), 5 leaf translation + downward pass (M2L/L2L),
 * 6 disaggregation + combine (L2P). */
enum { RBF_NPHASES = 7 };
int rbf_fmm_set_profiling(rbf_plan *plan, int on);
/* ms: host double[RBF_NPHASES], summed durations since profiling was enabled;
 * calls: host, number of profiled products. */
int rbf_fmm_phase_times(const rbf_plan *plan, double *ms, int64_t *calls);

/* ---- measuring autotuner ------------------------------------------------------------
 * Plans each candidate configuration for the given points (leaf capacity 64, 128, 256,
 * 512 on top of *base, and a near-only tree: uniform at the deepest level whose cells are
 * at least the pruning radius wide, so that every kept pair is a near pair), times `reps`
 * products of each with HIP events on `stream`, and writes the fastest configuration to
 * *best (host) and its time per product to *best_ms (host, may be NULL).  Arguments as in
 * rbf_fmm_plan; base may be NULL.  Synchronous; allocates and frees temporary plans. */
int rbf_fmm_autotune(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                     const rbf_opts *base, int reps, void *stream, rbf_opts *best, double *best_ms);

/* ---- batches of independent problems --------------------------------------------------
 * Many interpolation problems of uneven size, each with its own point set and shape, in
 * one set of launches: every phase of the product runs as one grid over all problems, and
 * the whole batched product is captured once into a HIP graph and replayed.
 *   points   device, concatenated (sum n_p, d) row-major, dtype.
 *   offsets  host int64[nprob + 1]: problem p owns rows offsets[p] .. offsets[p+1]-1
 *            (strictly increasing, offsets[0] = 0).
 *   shapes   host double[nprob]: kernel shape of each problem.
 *   opts     host, may be NULL: applied to every problem (base of the autotuner).
 *   autotune nonzero: choose each problem's configuration with rbf_fmm_autotune (2 reps).
 * The batch owns a private stream ordered after `stream` with events; products are
 * asynchronous with respect to the host and ordered on `stream`. */
typedef struct rbf_batch rbf_batch;
int rbf_fmm_plan_batch(const void *points, const int64_t *offsets, int nprob, int d, int dtype, int kernel,
                       const double *shapes, double tol, const rbf_opts *opts, int autotune, void *stream,
                       rbf_batch **out);
/* u = A_p lambda_p for every problem p; lambda and u are device, concatenated like the
 * points (caller order within each problem), plan dtype, not aliased.  The graph is
 * re-captured when the vector pointers differ from the previous call. */
int rbf_fmm_matvec_batch(rbf_batch *batch, const void *lambda, void *u);
/* on = 0: launch the kernels directly instead of replaying the captured graph. */
int rbf_fmm_batch_set_graph(rbf_batch *batch, int on);
typedef struct rbf_batch_info {
    int     nprob, ngroups, nfar, use_graph;
    int64_t total_n, total_leaves, device_bytes;
    double  plan_seconds;
} rbf_batch_info;
/* Sizes of a batch; n_max and nodes (host int32[nprob], may be NULL) receive each
 * problem's leaf capacity and nodes per dimension (0 for near-only problems). */
int rbf_fmm_batch_info(const rbf_batch *batch, rbf_batch_info *info, int32_t *n_max, int32_t *nodes);
int rbf_fmm_batch_destroy(rbf_batch *batch);

#ifdef __cplusplus
}
#endif
#endif

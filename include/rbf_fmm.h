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
/* Kernels of the paper's table "Global functions" (section 2.2) and of its numerical examples
 * (section 5).  The Gaussian is used in the shape form exp(-r^2 / (2 s^2)) (shape = s > 0);
 * the multiquadric is sqrt(r^2 + c^2) and the inverse multiquadric 1/sqrt(r^2 + c^2)
 * (shape = c > 0); Wendland's compactly supported function is (1 - e r)_+^3 (3 e r + 1)
 * (shape = e > 0, support radius 1/e).  The thin-plate spline r^2 log r (0 at r = 0) and r^5
 * of the paper's Fourier-transform table (section 3) have no shape (any positive value is
 * accepted and ignored); they are conditionally positive definite, so their interpolation
 * needs polynomial terms (rbf_interp_solve_poly); rbf_interp_solve, rbf_interp_solve_batch
 * and block-Jacobi reject them (RBF_EUNSUPPORTED).  Products and evaluation work as for
 * every kernel.
 *   The Gaussian has the band-limited far field of one frequency grid.  The multiquadric and
 *   the inverse multiquadric in 2-D and 3-D have a banded far field: the kernel is split by
 *   Gaussian width into a short-range residual (summed directly over the adjacent cells of a
 *   uniform tree whose level is opts->coarse_level, or about 256 points per cell), bands of
 *   width ratio sqrt 2 (each a decaying Gaussian mixture with its own band limit, coarse
 *   stencil, node count and factor C from the DFT of its samples: section 4.1's per-level
 *   band limits and section 3.2's eq. "M2Loperator") and a windowed top band over the whole
 *   domain; rbf_fmm_band_info reports the bands.  With opts->exact = 1, and in 5-D, their
 *   plans hold a single leaf and the product is the exact O(N^2) sum through the tiled direct
 *   kernel, as for the thin-plate spline and r^5.  A Wendland plan is a uniform tree whose
 *   cells are at least the support radius wide, with the adjacent cells as the near field and
 *   no far field: every pair inside the support is a near pair, so the product is exact (a
 *   single leaf when no such level below the root exists).  For Wendland, thin-plate and r^5
 *   tol and the tree options are ignored.  Any plan of one leaf without a far field computes
 *   its product with the tiled direct kernel.
 *   RBF_GAUSSIAN_BANDLIMITED is the band-limited Gaussian of section 3 (eq. 16, with the
 *   cut-off box [-sigma, sigma]^d of eq. 28): Phi_sigma(x) = prod_k phi_sigma(x_k),
 *   phi_sigma(t) = int_{-sigma}^{sigma} s/sqrt(2 pi) exp(-s^2 xi^2 / 2) cos(xi t) dxi, the
 *   Gaussian of width s (shape) with its transform cut off at the bandwidth sigma, which
 *   opts->band must give (RBF_EINVAL otherwise).  Its matrix is positive definite for
 *   distinct points (section 3.1).  The plan tabulates phi_sigma on the host as piecewise
 *   polynomials over [0, the bounding box's largest side], with a measured error of at most
 *   tol phi_sigma(0) / (4 d) (floor 1e-14 phi_sigma(0)); products, evaluation and solves are
 *   exact sums over all pairs through the tiled direct kernel (one leaf): the box's sharp
 *   cut-off leaves tails decaying like 1/|t|, which a periodic frequency grid would alias.
 *   Batch plans run each problem's exact sum through the near-field kernel (opts->band is the
 *   bandwidth of every problem; autotune is ignored for them).
 *   RBF_EUNSUPPORTED: a table of more than 4096 pieces (min(sigma, 4 / s) times the box side
 *   above about 1600), the autotuner, block-Jacobi and learned preconditioners.
 *   The table costs host time growing with the square of that product: about 30 ms at 250
 *   pieces, about 15 s at the cap. */
enum { RBF_GAUSSIAN = 0, RBF_MULTIQUADRIC = 1, RBF_INVERSE_MULTIQUADRIC = 2, RBF_WENDLAND = 3,
       RBF_THIN_PLATE = 4, RBF_R5 = 5, RBF_GAUSSIAN_BANDLIMITED = 6 };
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
    double band;         /* band limit sigma (0 = rule); the bandwidth of RBF_GAUSSIAN_BANDLIMITED */
    int    m2l_schedule; /* leaf-translation block order: 0 or 1 = contiguous leaf ranges per
                            XCD (default), 2 = leaf-major over the whole grid */
    int    exact;        /* multiquadric and inverse multiquadric: 1 = exact sum (one leaf, the
                            tiled direct kernel) instead of the banded far field */
    int    band_transfer;/* banded far field: the coarsest bands take their expansions from the
                            source band by interpolation (section 4.1): 0 = when it saves work
                            (n >= 64 transfer cells), 1 = always, -1 = never */
    int    reserved[5];
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
 * Errors: RBF_EINVAL (bad sizes or parameters), RBF_EUNSUPPORTED (dimension or a
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

/* Evaluation at separate targets: the sum of eq. 1 taken at points y_t that are not the
 * centres x_j (section 1 names the two roles; evaluating an interpolant is this sum),
 *   u_t = sum_j lambda_j Phi(y_t - x_j),  t = 1..m.
 * rbf_fmm_plan_eval plans for the n sources and the m targets together:
 *   sources  device, (n, d) row-major, dtype, n >= 1;
 *   targets  device, (m, d) row-major, dtype, m >= 0 (may be NULL when m = 0);
 *   the other arguments as for rbf_fmm_plan.  Both sets are copied, so the caller may free
 *   them after the call.  One tree covers both sets (a target outside the sources' bounding
 *   box included); its boxes split on their source counts, and inside each leaf the sources
 *   are aggregated and the targets evaluated, the near field pairing targets with sources.
 *   The tolerance rule is that of rbf_fmm_plan over the n + m points.  An evaluation costs
 *   about one product over the sources plus the targets' near field and disaggregation.
 *   Such a plan is used with rbf_fmm_eval and rbf_direct_eval only; rbf_fmm_matvec,
 *   rbf_direct_matvec, rbf_interp_solve and the preconditioner calls return RBF_EINVAL on
 *   it, and rbf_fmm_eval returns RBF_EINVAL on a plan from rbf_fmm_plan.  Synchronises the
 *   stream.  Errors as rbf_fmm_plan.
 * rbf_fmm_eval: lambda device, length n, plan dtype, the sources' order; u device, length
 *   m, plan dtype, the targets' order, overwritten (nothing is written when m = 0); must not
 *   alias lambda.  Asynchronous on the plan's stream; relative 2-norm error over the
 *   targets within the plan's tolerance.
 * rbf_direct_eval: the same sum over all pairs, exactly (O((n + m) n) on the device). */
int rbf_fmm_plan_eval(const void *sources, int64_t n, const void *targets, int64_t m, int d,
                      int dtype, int kernel, double shape, double tol, const rbf_opts *opts,
                      void *stream, rbf_plan **out);
int rbf_fmm_eval(rbf_plan *plan, const void *lambda, void *u);
int rbf_direct_eval(rbf_plan *plan, const void *lambda, void *u);

typedef struct rbf_solve_opts {
    int    restart;      /* Krylov subspace size m of GMRES(m) (default 50) */
    int    max_iters;    /* total inner-iteration cap (default 1000) */
    int    precond;      /* RBF_PC_NONE, RBF_PC_BLOCK_JACOBI or RBF_PC_LEARNED */
    int    zero_init;    /* nonzero: start from lambda = 0, else from the given lambda */
    int    fallback;     /* nonzero: on a non-finite preconditioner output or a restart cycle
                            that did not reduce the true residual, step down one
                            preconditioner (learned -> block-Jacobi -> none) and restart */
    double time_limit_s; /* wall-time cap in seconds (0 = none) */
    int    reserved[8];
} rbf_solve_opts;

typedef struct rbf_solve_info {
    int    iters;        /* inner iterations (matrix-vector products inside Arnoldi) */
    int    restarts;
    int    converged;
    int    fallback_used;/* number of preconditioner step-downs during the solve */
    double true_res;     /* ||f - A lambda|| / ||f|| of the returned lambda (the best iterate,
                            its residual from a fresh product at the restart that reached it) */
    double seconds;      /* wall time of the solve */
    double history[256]; /* true relative residual at each restart (first 256) */
    int    nhistory;
    double history_s[256];/* wall time from the start of the solve to each history entry */
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

/* Interpolation with the polynomial terms that conditionally positive definite kernels need
 * (the paper's thin-plate spline and r^5 of its Fourier-transform table, section 3, and the
 * multiquadric): u(x) = sum_j lambda_j Phi(x - x_j) + sum_k c_k p_k(t(x)), with
 * sum_j lambda_j p_k(t(x_j)) = 0, solved as the square system [A P; P' 0][lambda; c] = [f; 0]
 * by the same GMRES over vectors of n + q entries.
 *   Degree: 0 for the multiquadric, 1 for the thin-plate spline, 2 for r^5; the positive
 *   definite kernels (Gaussian, inverse multiquadric, Wendland) have q = 0 and this call is
 *   rbf_interp_solve.  Basis: monomials of t = (x - lo) / ext, lo and ext the plan's root
 *   cube (rbf_plan_info.lo and .ext): 1; t_1 .. t_d; t_a t_b for a <= b in row-major order.
 *   coeffs  device, q = rbf_poly_terms(plan) entries, plan dtype: initial guess in (unless
 *           opts->zero_init), coefficients out; may be NULL when q = 0.
 *   rtol    on ||[f; 0] - [A P; P' 0][lambda; c]|| / ||f||.
 * Augmented systems take no preconditioner (RBF_EUNSUPPORTED unless opts->precond is
 * RBF_PC_NONE).  Otherwise as rbf_interp_solve. */
int rbf_interp_solve_poly(rbf_plan *plan, const void *f, void *lambda, void *coeffs, double rtol,
                          const rbf_solve_opts *opts, rbf_solve_info *info);
/* Number q of polynomial terms of rbf_interp_solve_poly for this plan (0, 1, 1 + d or
 * 1 + d + d (d + 1) / 2), or a negative error code. */
int rbf_poly_terms(const rbf_plan *plan);

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
    int     nbands;       /* banded plans (multiquadric kernels): scale bands incl. the top */
    double  residual_width; /* banded plans: Gaussian width s0 below which the kernel is summed
                               directly over the near field */
    int     residual_in_q;  /* banded plans: 1 when the near field's residual table is a piecewise
                               polynomial in q = r^2 + c^2 (no square root per pair), 0 in
                               b = sqrt(q) (where the fit in q misses the accuracy bound) */
    int     reserved_info;
} rbf_plan_info;

/* Parameters and sizes chosen by the plan (host struct). */
int rbf_fmm_plan_info(const rbf_plan *plan, rbf_plan_info *info);

/* One scale band of a banded plan (section 4.1's per-level band limits, section 3.2's factor
 * C from kernel samples): band j in [0, nbands); the last is the windowed top band.  Host
 * struct.  RBF_EINVAL for j out of range. */
typedef struct rbf_band_info {
    int     top;              /* 1: the windowed top band (widths >= width_lo) */
    int     coarse_level, coarse_radius, nodes;
    int64_t half_nodes;       /* stored nodes per expansion */
    int     nunits, nchunks;  /* occupied coarse cells; aggregation chunks */
    double  width_lo, width_hi; /* Gaussian widths of the band (top: width_hi = window width) */
    double  tol;              /* tolerance relative to the band's largest value */
    double  band, period, reach, rfar, scale;
    int     transfer;         /* 1: the band's expansions come from the source band's cells by
                                 Lagrange interpolation, and go back to them by the transposed
                                 map (section 4.1); its own aggregation and disaggregation do
                                 not run.  The source band is the band whose coarse level is
                                 the transfer level with a stencil over the whole grid */
    int     transfer_order;   /* points of the Lagrange stencil per axis (0 without transfer) */
    int     reserved[2];
} rbf_band_info;
int rbf_fmm_band_info(const rbf_plan *plan, int j, rbf_band_info *info);

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
 * 512 on top of *base; a near-only tree: uniform at the deepest level whose cells are at
 * least the pruning radius wide, so that every kept pair is a near pair; and, when the
 * pruning radius is at least half the extent and n <= 2^19, a single leaf holding every
 * point, which is the direct sum), times `reps`
 * products of each with HIP events on `stream`; for a Gaussian with a far field it then times
 * the coarse levels next to the best candidate's (their stencils and so their node counts per
 * dimension differ) and the other leaf-translation block order (m2l_schedule) with the best
 * leaf capacity.  Multiquadric kernels: the near-field tree's level around the default (and
 * the exact sum for n <= 2^17).  It writes the fastest configuration to
 * *best (host) and its time per product to *best_ms (host, may be NULL).  Arguments as in
 * rbf_fmm_plan; base may be NULL.  Synchronous; allocates and frees temporary plans. */
int rbf_fmm_autotune(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                     const rbf_opts *base, int reps, void *stream, rbf_opts *best, double *best_ms);

/* ---- batches of independent problems --------------------------------------------------
 * Many interpolation problems of uneven size, each with its own point set and shape, in
 * one set of launches: problems that share a padded half grid form a group, every phase of
 * the product runs as one grid over a group's problems, the groups run concurrently on up to
 * eight private streams, and the whole batched product is captured once into a HIP graph and
 * replayed.
 *   points   device, concatenated (sum n_p, d) row-major, dtype.
 *   offsets  host int64[nprob + 1]: problem p owns rows offsets[p] .. offsets[p+1]-1
 *            (strictly increasing, offsets[0] = 0).
 *   shapes   host double[nprob]: kernel shape of each problem.
 *   opts     host, may be NULL: applied to every problem (base of the autotuner).
 *   autotune nonzero: choose each problem's configuration with rbf_fmm_autotune (2 reps).
 * The batch owns private streams ordered after `stream` with events (the group streams fork
 * from the first and join it before the product ends); products are asynchronous with
 * respect to the host and ordered on `stream`. */
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

/* Solve A_p lambda_p = f_p for every problem of a batch with restarted GMRES (section 1),
 * all problems together: each Arnoldi step is one batched product, the projections (CGS2,
 * FP64) are segmented per problem, and every problem keeps its own Hessenberg matrix, Givens
 * rotations and stopping test (true residual ||f_p - A_p lambda_p|| / ||f_p|| <= rtol,
 * recomputed at every restart; a problem that stops early takes zero directions).
 *   f, lambda  device, concatenated like the points, batch dtype; lambda is the initial
 *              guess (unless opts->zero_init) and the solution.
 *   opts       as for rbf_interp_solve; precond RBF_PC_NONE or RBF_PC_BLOCK_JACOBI (else
 *              RBF_EUNSUPPORTED).  Block-Jacobi makes the solve flexible GMRES with every
 *              problem's own 64-point blocks (below) as its right preconditioner, applied to
 *              all problems by one launch per direction; blocks missing at the first call are
 *              built with the default regularisation; m more vectors of n doubles are held.
 *   info       host array of nprob rbf_solve_info (may be NULL).
 * Work is ordered on the batch's stream argument.  Returns RBF_OK if every problem
 * converged, RBF_ENOCONV otherwise.  Synchronous. */
int rbf_interp_solve_batch(rbf_batch *batch, const void *f, void *lambda, double rtol,
                           const rbf_solve_opts *opts, rbf_solve_info *info);

/* ---- right preconditioners of the solve ----------------------------------------------
 * Neither preconditioner is part of the paper (which names GMRES and says nothing about
 * preconditioning); rbf_interp_solve applies them as right preconditioners of flexible
 * GMRES, so a nonlinear map is allowed.
 *
 * Blocks: the plan's points in its Morton order are cut into blocks of RBF_PC_BLOCK
 * consecutive points; block b holds sorted points [64 b, min(64 b + 64, n)).
 *
 * Block-Jacobi: y_b = (A_bb + reg I)^{-1} v_b for every block, A_bb the exact kernel
 * matrix of the block's points (built in FP64 by Gauss-Jordan elimination with partial
 * pivoting in LDS, since the multiquadric's blocks are indefinite and Wendland's function
 * is positive definite in one dimension only; stored as one explicit 64 x 64 FP64 inverse
 * per block: 32 KiB per block).
 *
 * Learned: z_b = y_b + s_b g(y_b / s_b), y the block solve of v with the feature
 * regularisation (rbf_pc_learned_features), s_b = ||y_b||_2 (z_b = 0 if s_b = 0), with g the
 * network below evaluated in BF16 with FP32 accumulation.  Trained on pairs (r, e) of a
 * residual and its error e = A^{-1} r to make z close to e.  In rbf_interp_solve a
 * GMRES(m) cycle with the learned preconditioner is block-Jacobi FGMRES for its first
 * m - 1 directions and takes z_{m-1} = learned(v_0) last (v_0 is the normalised residual,
 * the kind of vector the network is trained on): the cycle minimises the residual over
 * the block-Jacobi Krylov directions augmented with the learned error estimate.
 */
#define RBF_PC_BLOCK 64
#define RBF_MLP_IN 64
#define RBF_MLP_HIDDEN 256
#define RBF_MLP_NPARAMS 164672
enum { RBF_MLP_BF16 = 0, RBF_MLP_F32 = 1 };

/* Build (or rebuild) the block-Jacobi inverses with regularisation reg >= 0 (reg < 0: the
 * default, reg = 1e-2 Phi(0)).  Synchronous.  RBF_EINVAL if a block is numerically
 * singular at this reg (a zero pivot after row exchanges).  Kernels: the Gaussian, the
 * multiquadric (Phi(0) = c), the inverse multiquadric (Phi(0) = 1/c) and Wendland's function;
 * RBF_EUNSUPPORTED for the thin-plate spline and r^5.  The learned preconditioner, its
 * features, pairs and harvest take the Gaussian and the multiquadric kernels
 * (RBF_EUNSUPPORTED otherwise); the feature regularisation defaults to 1e-6 Phi(0). */
int rbf_pc_block_jacobi(rbf_plan *plan, double reg);
/* Build the block inverses that form the learned map's features y (and those of
 * rbf_pc_pairs / rbf_pc_harvest) with their own regularisation (reg < 0: the default,
 * 1e-6 Phi(0)).  A network is trained on the features of one reg and should be applied
 * with the same.  Storage is shared with block-Jacobi when the two regs agree. */
int rbf_pc_learned_features(rbf_plan *plan, double reg);

/* z = M^{-1} v for kind RBF_PC_BLOCK_JACOBI or RBF_PC_LEARNED.
 *   v, z  device FP64, length n, caller's point order, not aliased.
 * Builds the block inverses with the default reg if none exist.  RBF_ESTATE for
 * RBF_PC_LEARNED without an attached network.  Enqueued on the plan's stream. */
int rbf_pc_apply(rbf_plan *plan, int kind, const double *v, double *z);

/* Multilayer perceptron g: R^64 -> R^64, hidden layers of 256 units with ReLU, affine
 * output.  Parameters: host or device FP32 vector of RBF_MLP_NPARAMS values in the order
 * W1 (256 x 64, row-major [out][in]), b1 (256), W2 (256 x 256), b2, W3 (256 x 256), b3,
 * W4 (64 x 256), b4 (64).  The handle owns FP32 master weights, a BF16 copy for inference
 * and Adam state on the current device. */
typedef struct rbf_mlp rbf_mlp;
/* params: host, may be NULL: then hidden weights are He-uniform from `seed`, biases and the
 * output layer zero (g = 0).  Synchronous. */
int rbf_mlp_create(const float *params, uint64_t seed, rbf_mlp **out);
int rbf_mlp_destroy(rbf_mlp *mlp);
/* params: host float[RBF_MLP_NPARAMS].  Synchronous. */
int rbf_mlp_get_params(const rbf_mlp *mlp, float *params);
/* Versioned binary weight file: 8-byte magic "RBF-MLP\0", uint32 version (1), uint32 layer
 * count (4), uint32 widths 64 256 256 256 64, uint32 activation (1 = ReLU), uint64 parameter
 * count, then the FP32 parameters, little-endian.  rbf_mlp_load rejects any other layout
 * with RBF_EINVAL. */
int rbf_mlp_save(const rbf_mlp *mlp, const char *path);
int rbf_mlp_load(const char *path, rbf_mlp **out);
/* y = g(x) for `rows` rows: x device float[rows][64], y device float[rows][64].
 * precision RBF_MLP_BF16: the inference kernel (BF16 MFMA, FP32 accumulation);
 * RBF_MLP_F32: the FP32 training kernels.  Enqueued on `stream`. */
int rbf_mlp_forward(rbf_mlp *mlp, const float *x, int64_t rows, float *y, int precision, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the FP32 forward of rbf_mlp_forward
 * (precision RBF_MLP_F32; same kernels, same results bit for bit) with its hidden
 * activations in a fixed static device workspace instead of the network's allocated one.
 * It calls no hipMalloc, hipFree or allocating library routine.
 *   x  device float[rows][64], y device float[rows][64] (may not alias x), stream: HIP stream
 *   0 <= rows <= RBF_MLP_STATIC_MAX_ROWS; more rows -> RBF_EINVAL (split the call).
 * The workspace (2 x 4096 x 256 floats = 8 MiB per device) is one per device, taken on the
 * device current at the call, and shared by every call on that device: calls that overlap
 * in time on one device (different streams, or different host threads without ordering)
 * race and give wrong results.  Calls on one stream are ordered and safe.  The network and
 * the arrays must live on the current device. */
#define RBF_MLP_STATIC_MAX_ROWS 4096
int rbf_mlp_forward_static(rbf_mlp *mlp, const float *x, int64_t rows, float *y, void *stream);
/* Loss L = sum_r w_r ||g(x_r) - t_r||^2 / sum_r w_r of the rows (1 <= rows <= 2^20) in
 * FP32 and its gradient dL/dparams.  x, t device float[rows][64], w device float[rows];
 * loss host (may be NULL), grad host float[RBF_MLP_NPARAMS] (may be NULL).  Synchronous. */
int rbf_mlp_loss_grad(rbf_mlp *mlp, const float *x, const float *t, const float *w, int64_t rows,
                      double *loss, float *grad, void *stream);
typedef struct rbf_train_opts {
    int      epochs;     /* passes over the training rows (default 100) */
    int      batch;      /* rows per Adam step (default 512) */
    int      patience;   /* stop after this many epochs without a better held-out loss (0 = never) */
    int      reserved0;
    double   lr, beta1, beta2, eps;  /* Adam (defaults 1e-3, 0.9, 0.999, 1e-8) */
    double   val_frac;   /* the last floor(val_frac * rows) rows are held out (0 <= val_frac < 1) */
    uint64_t seed;       /* shuffle of the training rows */
    int      reserved[8];
} rbf_train_opts;
typedef struct rbf_train_info {
    int    epochs_run, best_epoch, nhist, reserved0;
    double init_val_loss, best_val_loss, final_train_loss, seconds;
    double train_loss[256], val_loss[256];   /* per epoch (first 256) */
} rbf_train_info;
/* Minibatch Adam on rows (x, t, w) as in rbf_mlp_loss_grad (device arrays).  With held-out
 * rows the parameters with the lowest held-out loss are kept (the initial ones included).
 * opts may be NULL, info may be NULL.  Synchronous. */
int rbf_mlp_train(rbf_mlp *mlp, const float *x, const float *t, const float *w, int64_t rows,
                  const rbf_train_opts *opts, void *stream, rbf_train_info *info);

/* Attach a network for RBF_PC_LEARNED (NULL detaches).  The plan keeps the pointer; the
 * network must outlive its use by the plan. */
int rbf_pc_set_learned(rbf_plan *plan, rbf_mlp *mlp);
/* Training rows of one (residual, error) pair, one row per block:
 *   r, e   device FP64, length n, caller order (e the error of which r is the residual)
 *   x, t   device float[nblk][64]: x_b = y_b / s_b, t_b = (e_b - y_b) / s_b (Morton order
 *          within the block, zero-padded), y = block-Jacobi output of r, s_b = ||y_b||
 *   w      device float[nblk]: s_b^2 / ||e||^2, 0 for a short last block or s_b = 0
 * nblk = ceil(n / 64).  Builds the block inverses with the default reg if none exist. */
int rbf_pc_pairs(rbf_plan *plan, const double *r, const double *e, float *x, float *t, float *w);
/* Training rows from solves of A lambda = f (f device, plan dtype, caller order):
 * lambda* from GMRES(50) to rtol (at most max_iters iterations) with preconditioner
 * `precond` (RBF_PC_NONE or RBF_PC_BLOCK_JACOBI), then for each cap k in caps (host
 * int[ncaps], k >= 0) lambda_k after k iterations from zero with the same solver,
 * e_k = lambda* - lambda_k and r_k = A e_k with the fast product.  Rows of cap c go to
 * x + c nblk 64, t + c nblk 64, w + c nblk (device, sized ncaps nblk rows).  Synchronous. */
int rbf_pc_harvest(rbf_plan *plan, const void *f, double rtol, int max_iters, int precond, const int *caps,
                   int ncaps, float *x, float *t, float *w);
/* The training of the learned preconditioner in one call: rows from solves of
 * A_p lambda = f_p for every plan (rbf_pc_harvest, no preconditioner; caps host int[ncaps],
 * NULL for 0, 1, 2, 5, 10, 20, 50, 100, 200), all rows in plan order and cap order, a network
 * created from `seed` (rbf_mlp_create), minibatch Adam on the rows (rbf_mlp_train with opts,
 * on the first plan's stream; info may be NULL), written to out_path as the versioned weight
 * file (rbf_mlp_save).  plans host array of nplans plans, fs host array of nplans device
 * right-hand sides (each plan's dtype and length).  Device memory for the rows
 * (ncaps * ceil(n_p / 64) * 516 bytes per plan) is allocated for the call.  Synchronous. */
int rbf_pc_train(rbf_plan *const *plans, const void *const *fs, int nplans, double rtol, int max_iters,
                 const int *caps, int ncaps, uint64_t seed, const rbf_train_opts *opts, const char *out_path,
                 rbf_train_info *info);
/* Load a weight file (rbf_mlp_load: RBF_EINVAL for any other layout or version) and attach the
 * network to the plan for RBF_PC_LEARNED (rbf_pc_set_learned).  *out receives the network;
 * the caller destroys it (rbf_mlp_destroy) after the plan's last use of it. */
int rbf_pc_load(rbf_plan *plan, const char *path, rbf_mlp **out);

#ifdef __cplusplus
}
#endif
#endif

// Internal declarations shared by the translation units of librbffmm.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "rbf_fmm.h"

namespace rbf {

void set_error(const char *fmt, ...);

#define RBF_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e__ = (call);                                                        \
        if (e__ != hipSuccess) {                                                        \
            ::rbf::set_error("%s: %s (%s:%d)", #call, hipGetErrorString(e__), __FILE__, \
                             __LINE__);                                                 \
            return RBF_EHIP;                                                            \
        }                                                                               \
    } while (0)

#define RBF_TRY(expr)                  \
    do {                               \
        int rc__ = (expr);             \
        if (rc__ != RBF_OK) return rc__; \
    } while (0)

constexpr int kMaxDim = 5;
constexpr int kWave = 64;

// Device-wide exclusive prefix sum of n int32 values; out may alias in.  If total is
// non-null the sum of all inputs is written to *total (host) -- this synchronises.
int exclusive_scan_i32(const int *in, int *out, int n, int *total, hipStream_t s);

// Ordered set of device allocations owned by a plan.
struct Arena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    int alloc(void **p, size_t nbytes);
    void release();
};

// Spread consecutive workgroups over the 8 XCDs in contiguous chunks: dispatch
// round-robins workgroup ids over XCDs, so id % 8 names the XCD; giving each XCD a
// contiguous range of work keeps neighbouring boxes (which share sources) in one L2.
__device__ __forceinline__ int xcd_swizzle(int bid, int nblocks) {
    const int nx = 8;
    int per = nblocks / nx, rem = nblocks % nx;
    int x = bid % nx, k = bid / nx;
    return x * per + (x < rem ? x : rem) + k;
}

// Near-field work queue: one task counter per XCD, each on its own 128-byte line.
constexpr int kXcds = 8, kCtrStride = 32;
// pair-distance histogram of the band split: bins per factor 2, and their number
constexpr int kPairBins = 8, kPairBinsTotal = 8 * 48;

template <class T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };

// Near-field kernels of a banded plan: the residual of the scale split (widths below s0) of
// the multiquadric (kResTab) and of the inverse multiquadric (kResTabDiv: the table holds b
// times the residual), as a piecewise polynomial in b = sqrt(r^2 + c^2) (kResIntervals pieces
// of degree kResDegree over [c, bmax); zero from r^2 = qmax on), or of either kernel in
// q = r^2 + c^2 (kResTabQ: pieces uniform in q over [c^2, qmax)).  Internal codes, not ABI.
constexpr int kResTab = 16, kResTabDiv = 17, kResTabQ = 18;
constexpr int kResIntervals = 128, kResDegree = 5;
constexpr int kResCoefs = kResIntervals * (kResDegree + 1);
// Band-limited Gaussian (RBF_GAUSSIAN_BANDLIMITED): phi_sigma per axis as pieces in u in
// [-1, 1] over [0, tmax], of degree 7 for FP64 products and 3 for FP32 ones (whose arithmetic
// ends near 1e-7 anyway, and whose LDS reads halve); the table holds the piece count and the
// degree, then degree + 1 monomial coefficients per piece (u^0 first).
constexpr int kBlDegree64 = 7, kBlDegree32 = 3, kBlHead = 2, kBlMaxPieces = 4096;
template <class T> constexpr int kBlDeg = sizeof(T) == 8 ? kBlDegree64 : kBlDegree32;

// One scale band of a banded far field (multiquadric kernels).  A band is a smooth part of
// the kernel with its own quadrature grid (band limit sigma, nodes mn, period L), its own
// dense coarse grid (level lc, stencil radius r), and its own translation table wtab
// (quadrature weight times the factor C from the band's samples).  Its points are
// aggregated in chunks (p2m_*: at most kBandChunk consecutive points of one cell, sorted by
// cell; cell_begin is the chunk range of every dense cell) and disaggregated per occupied
// cell (unit_*: point range and dense cell index of each occupied cell).
struct Band {
    int top = 0;                 // 1: the windowed top band (widths >= s_lo)
    double s_lo = 0, s_hi = 0;   // widths of the band's Gaussians (top: s_hi = window width)
    double tau = 0;              // tolerance of the band relative to its largest value
    double tau_x = 0;            // tolerance of the transfer into this band (the unloosened split)
    double win_k = 4.0;          // top band: its window steps down win_k window widths outside the domain
    double sigma = 0, L = 0, reach = 0, rfar = 0, scale = 0;
    int lc = 0, r = 0, mn = 0, H = 0, HP = 0;
    int64_t R = 0, P = 0, ncells = 0;
    int nunits = 0, nchunks = 0, ntasks = 0, ngroups = 0;
    int *unit_begin = nullptr;   // [nunits + 1]
    int *unit_cell = nullptr;    // [nunits]
    int *chunk_begin = nullptr;  // [nchunks + 1]
    int *cell_begin = nullptr;   // [ncells + 1] chunk ranges
    int2 *tasks = nullptr;       // (unit, first point offset) per 64 points [ntasks]
    int *grp_first = nullptr;    // runs of at most 8 units [ngroups + 1]
    int *uni_ptr = nullptr;      // empty near lists [ngroups + 1]
    int *uni_pad = nullptr;      // zero entries the leaf translation reads ahead [16]
    double *wtab = nullptr;      // [P]
    int xfer = 0;                // 1: expansions transferred from the source band (no aggregation,
                                 //    translation or disaggregation of its own)
    int xk = 0;                  // Lagrange stencil length of the transfer
};
constexpr int kBandChunk = 256;

// Interpolating transfer of one target band's expansions from and to the source band's cell
// expansions (xfer.hip): CSR maps of the 1-D Lagrange stencils (output index -> input index,
// weight), device arrays, and the target grid's phases at the transfer cells.
struct Xfer {
    int band = -1;                                                  // the target band
    int K = 0;
    double err = 0;                                                 // predicted 1-D error
    int *up_ptr = nullptr, *up_idx = nullptr;   double *up_w = nullptr;    // S full -> T full [mnt]
    int *upl_ptr = nullptr, *upl_idx = nullptr; double *upl_w = nullptr;   // S full -> T half [Ht]
    int *dn_ptr = nullptr, *dn_idx = nullptr;   double *dn_w = nullptr;    // T full -> S full [mns]
    int *dnl_ptr = nullptr, *dnl_idx = nullptr; double *dnl_w = nullptr;   // T full -> S half [Hs]
    double2 *phase_t = nullptr;                                     // [cell][d][mnt] e^{i eta_m c_k}
};

}  // namespace rbf

struct rbf_plan {
    int64_t n = 0;
    int d = 0, dtype = 0, kernel = 0;
    double shape = 0, tol = 0;
    hipStream_t stream = nullptr;

    // tree and quadrature parameters
    int n_max = 0, max_level = 0, min_level = 0, lc = 0, r = 0, mn = 0, H = 0, HP = 0, B = 0;
    int64_t R = 0, P = 0;   // rows (nodes^(d-1)) and half-grid length R*H per expansion
    double sigma = 0, L = 0, rcut = 0, rfar = 0, ext = 0;
    double lo[rbf::kMaxDim] = {0, 0, 0, 0, 0};
    int nleaves = 0, nlevels = 0;
    int far = 1;            // 0 when every kept pair is near (all leaves at lc, stencil radius <= 1)
    int nodes_needed = 0;   // nodes per dimension the tolerance rule asked for
    int min_leaf_level = 0, max_leaf_level = 0;
    int64_t ncells = 0, nnear = 0, near_pairs = 0, nranges = 0;

    // device arrays (owned by arena)
    rbf::Arena arena;
    uint64_t *keys = nullptr;        // sorted Morton keys [n]
    int *perm = nullptr;             // input index of sorted point i [n]
    void *xs = nullptr;              // sorted coordinates, SoA [d][n]
    int *leaf_begin = nullptr;       // [nleaves + 1]
    int *leaf_level = nullptr;       // [nleaves]
    uint64_t *leaf_prefix = nullptr; // [nleaves]
    int *leaf_cell = nullptr;        // coarse cell (Morton index at lc) [nleaves]
    int *near_ptr = nullptr;         // [nleaves + 1]
    int *near_idx = nullptr;         // [nnear]
    int *src_ptr = nullptr;          // merged source point ranges of the near field [nleaves + 1]
    int2 *src_rng = nullptr;         // [nranges] (begin, end)
    int *cell_leaf_begin = nullptr;  // [ncells + 1]
    int2 *tasks = nullptr;           // (leaf, first target's offset in the leaf) per 64-target task [ntasks]
    // a plan for separate targets (rbf_fmm_plan_eval): caller points [0, n_src) are the sources,
    // [n_src, n) the targets, which take part with weight 0; 0 for an ordinary plan
    int64_t n_src = 0;
    int *src_end = nullptr;          // such a plan orders each leaf's sources before its targets:
                                     // sources [leaf_begin[a], src_end[a]), targets the rest [nleaves]
    void *ev_lam = nullptr;          // [n] the sources' weights followed by zeros
    void *ev_u = nullptr;            // [n] the product over all n points
    // near-field tasks: (leaf, first target), one per chunk of at most 64 targets of a leaf
    // [nptasks]
    int2 *ptasks = nullptr;
    int nptasks = 0;
    // sibling groups of the leaf translation: runs of at most 8 consecutive leaves with one
    // parent; each group's near lists merged into one ascending list with member masks
    int ngroups = 0;
    int64_t nunion = 0;
    int *grp_first = nullptr;        // first leaf of each group [ngroups + 1]
    int *uni_ptr = nullptr;          // [ngroups + 1]
    int *uni_idx = nullptr;          // near leaf of each entry [nunion + 8]
    int *uni_mask = nullptr;         // bit c set: member c of the group has the leaf as near [nunion + 8]
    double *wtab = nullptr;          // quadrature weight times C(xi) per stored node [P]
    int m2l_sched = 0;               // block order of the leaf translation
    int ntasks = 0;
    void *dl = nullptr;              // lambda-weighted last-dimension phases [n][HP] complex
    double *xi = nullptr;            // quadrature nodes [mn]
    double *wc1 = nullptr;           // w_k C1(xi_k) per dimension (separable kernels) [mn]
    void *lam_s = nullptr;           // sorted coefficients [n]
    void *u_s = nullptr;             // sorted near-field result [n]
    int *p2p_ctr = nullptr;          // near-field work-queue counters [8 * kCtrStride]
    void *W = nullptr;               // leaf expansions [nleaves][P] complex
    void *Lx = nullptr;              // leaf local expansions, rows padded: [nleaves][R][HP] complex
    void *Wc = nullptr;              // coarse expansions [ncells][P]
    void *Lc = nullptr;              // coarse local expansions [ncells][P]
    void *Tmp = nullptr;             // stencil pass buffer [ncells][P]

    // banded far field (multiquadric kernels): the near field (adjacent cells of a uniform
    // tree) sums the residual of the scale split, every band adds its far field; the bands
    // run in order on the plan's stream and share the buffers b* (sized for the largest)
    std::vector<rbf::Band> bands;
    double res_s0 = 0;               // width below which the kernel is summed directly
    double res_qmax = 0;             // r^2 from which the residual is negligible (the cell width^2)
    double res_inv = 0;              // residual pieces per unit of b
    double *res_tab = nullptr;       // residual polynomial pieces [kResCoefs]
    int res_q = 0;                   // 1: the residual table is in q = r^2 + c^2 (kResTabQ)
    // band-limited Gaussian: per-axis table in the layout of kBlHead / kBlDeg (device),
    // pieces per unit t, piece count, measured largest fit error
    double *bl_tab = nullptr;
    double bl_inv = 0, bl_err = 0;
    int bl_pieces = 0;
    double phi_rms = 0;              // rms of the kernel over sampled pairs (tolerance split)
    std::vector<double> pair_cdf;    // sampled pairs closer than each log-spaced distance
    double pair_rlo = 0, pair_min = 0;
    void *bW = nullptr, *bLx = nullptr, *bWc = nullptr, *bLc = nullptr, *bTmp = nullptr, *bdl = nullptr;
    std::vector<hipEvent_t> band_ev; // profiling: event pairs per band and phase
    // interpolating transfers (the coarsest bands take their expansions from the source band's
    // cells at the transfer level, section 4.1): option, source band, cells and buffers
    int band_xfer = 0;               // opts.band_transfer: 0 auto, 1 on, -1 off
    int xfer_src = -1, xfer_level = 0, xfer_ncell = 0;
    std::vector<rbf::Xfer> xfers;
    double2 *xfer_phase_s = nullptr; // [cell][d][mns] e^{i xi_m c_k} of the source grid
    int *xfer_cell_unit = nullptr;   // [cell] the source band's unit of a dense cell, or -1
    void *xfer_keep = nullptr, *xfer_x1 = nullptr, *xfer_x2 = nullptr, *xfer_l = nullptr;

    // the near field of a product runs on a second stream of default priority, forked after the
    // permutation and joined before the disaggregation (it reads nothing the far-field chain
    // writes, and only the disaggregation reads its result)
    // (created at the first single-problem product; a plan used only inside a batch has none)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int side_state = 0;              // 0 not tried, 1 ready, -1 unavailable (one stream)
    // profiling
    int profiling = 0;
    hipEvent_t ev[2 * RBF_NPHASES] = {};
    double phase_ms[RBF_NPHASES] = {0};
    int64_t prof_calls = 0;

    // solver workspace (allocated on first solve)
    rbf::Arena solver_arena;
    int solver_m = 0;
    int64_t solver_na = 0;           // Krylov vector length the solver buffers hold (n + polynomial terms)
    double *V = nullptr;             // Arnoldi basis [(m+1)][n] FP64
    double *Z = nullptr;             // preconditioned basis [m][n] FP64 (flexible GMRES)
    double *sv = nullptr;            // small device vectors (dots, norms)
    void *tvec = nullptr;            // plan-dtype vectors for products [3][n]

    // right preconditioners of the solve (built on first use)
    rbf::Arena pc_arena;
    int64_t nblk = 0;                // 64-point blocks of the Morton order
    double bj_reg = -1.0;            // regularisation of the block-Jacobi inverses (< 0: none built)
    double *bj_inv = nullptr;        // (A_bb + reg I)^{-1}, column-major 64 x 64 per block
    double lp_reg = -1.0;            // regularisation of the learned map's feature inverses
    double *lp_inv = nullptr;        // same layout; aliases bj_inv when the two regs agree
    double *lp_own = nullptr;        // separate storage for lp_inv when they differ
    double *pc_y = nullptr;          // block-Jacobi output, Morton order [n]
    double *pc_s = nullptr;          // block norms [nblk]
    float *pc_x = nullptr;           // network input rows [nblk][64]
    float *pc_g = nullptr;           // network output rows [nblk][64]
    int *pc_flag = nullptr;          // device status word of the block factorisation
    double *pc_scal = nullptr;       // device scalars (||e||^2 of the pair builder)
    rbf_mlp *mlp = nullptr;          // learned correction (not owned)
};

namespace rbf {
int plan_create(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                const rbf_opts *opts, hipStream_t stream, rbf_plan **out);
int build_tree(rbf_plan *p, const void *points);
int build_near_lists(rbf_plan *p);
int launch_matvec(rbf_plan *p, const void *lambda, void *u);
// the product through the per-phase kernels (what a batch runs), never the direct kernel
int launch_matvec_phases(rbf_plan *p, const void *lambda, void *u);
// RBF_EINVAL (with a message naming fn) when p is a plan for separate targets
int reject_eval_plan(const rbf_plan *p, const char *fn);
int launch_direct(rbf_plan *p, const void *lambda, void *u);
int plan_bands(rbf_plan *p);                                         // bands.hip
int bandlimited_table(rbf_plan *p, double sigma);                    // bandlimited.hip
template <class T>
int xfer_band(const rbf_plan *p, const Xfer &x, const Band &S, const Band &Tb, const void *wc_keep, void *lx_s,
              hipStream_t s);                                          // xfer.hip
bool banded_kernel(int kernel, int d);                               // bands.hip
int pc_ready(rbf_plan *p, int kind);                                 // pc.hip
int pc_apply(rbf_plan *p, int kind, const double *v, double *z);     // pc.hip
// Block-Jacobi over the problems of a batch (pc.hip): problem q's vector entries sit at
// [off[q], off[q + 1]) in caller order, its blocks are global blocks [bfirst[q], bfirst[q + 1]).
// All arrays are device arrays of nprob (+ 1) entries.
struct BatchBj {
    const double *const *inv;   // problem q's block inverses (its plan's)
    const int *const *perm;     // problem q's permutation, sorted -> caller order
    const int64_t *off;
    const int64_t *bfirst;
    int nprob;
    int64_t nblk;
};
// builds every plan's block inverses (default regularisation) when missing and fills bj
int batch_bj_prepare(const std::vector<rbf_plan *> &plans, const std::vector<int64_t> &offsets, Arena &ar,
                     hipStream_t s, BatchBj *bj);
int batch_bj_apply(const BatchBj &bj, const double *v, double *z, hipStream_t s);
int mlp_infer_bf16(rbf_mlp *m, const float *x, int64_t rows, float *y, hipStream_t s);   // mlp.hip
}  // namespace rbf

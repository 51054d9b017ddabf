// C ABI entry points: planning (parameter rule, tree, tables), products, info, timing.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace rbf {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int Arena::alloc(void **p, size_t nbytes) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, nbytes ? nbytes : 16);
    if (e != hipSuccess) {
        set_error("hipMalloc(%zu bytes) failed: %s", nbytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? RBF_ENOMEM : RBF_EHIP;
    }
    ptrs.push_back(q);
    bytes += (int64_t)nbytes;
    *p = q;
    return RBF_OK;
}

void Arena::release() {
    for (void *q : ptrs) (void)hipFree(q);
    ptrs.clear();
    bytes = 0;
}

int compute_bbox(rbf_plan *p, const void *points);

// Band limit of the Gaussian: s sigma = t with erfc(t / sqrt 2) = tol / 4 (the largest
// deviation of the band-limited Gaussian from the Gaussian is erfc(s sigma / sqrt 2), at r = 0).
double band_limit_t(double tol) {
    double lo = 0.0, hi = 40.0, target = tol / 4.0;
    for (int i = 0; i < 200; ++i) {
        double mid = 0.5 * (lo + hi);
        if (std::erfc(mid / std::sqrt(2.0)) > target) lo = mid; else hi = mid;
    }
    return hi;
}

namespace {

// Exact-sum plans: the thin-plate spline and r^5 (no far field: their transforms are singular
// at the origin), the multiquadric kernels with opts.exact or outside the dimensions of their
// banded far field, the band-limited Gaussian (its box cut-off leaves tails like 1/|t|, which
// no periodic grid resolves), and the base of the Wendland plan below.  Every pair is a near
// pair of a single leaf: the product is the exact sum, evaluated by the tiled direct kernel.
void multiquadric_params(rbf_plan *p) {
    p->sigma = 1.0;
    p->rcut = p->rfar = p->ext;
    p->lc = 0;
    p->r = 0;
    p->n_max = 1 << 30;
    p->max_level = 0;
    p->min_level = 0;
    p->nodes_needed = 4;
    p->mn = 4;
    p->H = 2;
    p->HP = 4;
    p->R = 1;
    for (int k = 0; k < p->d - 1; ++k) p->R *= p->mn;
    p->P = p->R * p->H;
    p->L = 2.0 * M_PI / (2.0 * p->sigma / (p->mn - 1));
}

// Wendland's function vanishes from r = 1/e on.  In a uniform tree whose cells are at least
// that wide, two points closer than 1/e lie in the same or adjacent cells, so the adjacent
// cells as near field leave an empty far field and the product is exact.  The deepest such
// level does the least work; without one below the root the plan is a single leaf.
void wendland_params(rbf_plan *p) {
    multiquadric_params(p);
    const double rho = 1.0 / p->shape;
    int lstar = 0;
    while (lstar + 1 <= 18 / p->d && p->ext / std::ldexp(1.0, lstar + 1) >= rho) ++lstar;
    p->rcut = rho;
    if (lstar >= 1) {
        p->lc = lstar;
        p->r = 1;
        p->rfar = std::min(2.0 * p->ext / std::ldexp(1.0, lstar), p->ext);
        p->max_level = lstar;
        p->min_level = lstar;
    }
}

// Multiquadric and inverse multiquadric in 2-D and 3-D: banded far field.  The near field is a
// uniform tree (adjacent cells, like the near-only Wendland plan); its level, by default the one
// with about 256 points per cell on average, sets the residual width and so the finest band.
void banded_params(rbf_plan *p, const rbf_opts *o) {
    multiquadric_params(p);
    const int d = p->d;
    int l = (int)std::floor(std::log2(std::max(1.0, (double)p->n / 256.0)) / d + 0.5);
    if (o && o->coarse_level >= 1) l = o->coarse_level;
    l = std::max(1, std::min(l, 18 / d));
    p->lc = l;
    p->r = 1;
    p->rfar = std::min(2.0 * p->ext / std::ldexp(1.0, l), p->ext);
    p->rcut = p->rfar;
    p->max_level = l;
    p->min_level = l;
}

int choose_params(rbf_plan *p, const rbf_opts *o) {
    if (banded_kernel(p->kernel, p->d) && !(o && o->exact)) {
        banded_params(p, o);
        return RBF_OK;
    }
    if (p->kernel == RBF_MULTIQUADRIC || p->kernel == RBF_INVERSE_MULTIQUADRIC || p->kernel == RBF_THIN_PLATE ||
        p->kernel == RBF_R5 || p->kernel == RBF_GAUSSIAN_BANDLIMITED) {
        multiquadric_params(p);
        return RBF_OK;
    }
    if (p->kernel == RBF_WENDLAND) {
        wendland_params(p);
        return RBF_OK;
    }
    const double s = p->shape, tol = p->tol;
    const int d = p->d;
    p->sigma = (o && o->band > 0) ? o->band : band_limit_t(tol) / s;
    p->rcut = s * std::sqrt(2.0 * std::log(4.0 / tol) + 1.0);
    // error budget: tol/4 for the band limit, tol/4 for the pruned pairs, tol/2 (the rest of the
    // tolerance) for the periodic images of the kept pairs
    const double margin = s * std::sqrt(2.0 * std::log(2.0 / tol));
    int lmax = 0;
    if (p->n > p->n_max) lmax = (int)std::floor(std::log((double)p->n / p->n_max) / std::log(std::pow(2.0, d)));
    lmax = std::max(0, std::min(lmax, 18 / d));
    int best_l = 0, best_r = 0;
    double best_far = p->ext;
    for (int l = 1; l <= lmax; ++l) {
        double w = p->ext / std::ldexp(1.0, l);
        int r = 1 + (int)std::floor(p->rcut / w);
        double far = (r + 1) * w;
        if (far >= p->ext) continue;
        if (far < best_far) { best_l = l; best_r = r; best_far = far; }
    }
    if (o && o->coarse_level >= 0) {
        best_l = o->coarse_level;
        if (best_l > 18 / d) { set_error("coarse_level %d too deep for d=%d", best_l, d); return RBF_EINVAL; }
        double w = p->ext / std::ldexp(1.0, best_l);
        best_r = (o->coarse_radius >= 0) ? o->coarse_radius : (best_l == 0 ? 0 : 1 + (int)std::floor(p->rcut / w));
        best_far = (best_l == 0) ? p->ext : std::min((best_r + 1) * w, p->ext);
    }
    if (best_l >= 1 && best_r < 1) {
        // every near leaf must lie inside the coarse stencil for the leaf translation
        // (stencil sum minus near sum) to leave exactly the far field
        set_error("coarse_radius must be >= 1 when coarse_level >= 1 (got %d)", best_r);
        return RBF_EINVAL;
    }
    p->lc = best_l;
    p->r = best_r;
    p->rfar = best_far;
    double L = best_far + margin;
    int mn = (int)std::ceil(p->sigma * L / M_PI) + 1;
    if (mn % 2) ++mn;
    mn = std::max(mn, 4);
    if (o && o->nodes > 0) {
        if (o->nodes % 2 || o->nodes < 4) { set_error("nodes must be even and >= 4 (got %d)", o->nodes); return RBF_EINVAL; }
        mn = o->nodes;
    }
    const int hmax = (d == 5) ? 12 : 32;
    p->nodes_needed = mn;
    if (mn / 2 > hmax) {
        // The grid the kernel's width needs is too large.  If cells at least the pruning
        // radius wide exist, every kept pair can be a near pair instead: a uniform tree at
        // the deepest such level with the adjacent cells as stencil has no far field.
        int lstar = 0;
        while (lstar + 1 <= 18 / d && p->ext / std::ldexp(1.0, lstar + 1) >= p->rcut) ++lstar;
        const bool forced = o && (o->coarse_level >= 0 || o->nodes > 0);
        if (lstar >= 1 && !forced) {
            p->lc = lstar;
            p->r = 1;
            p->rfar = std::min(2.0 * p->ext / std::ldexp(1.0, lstar), p->ext);
            p->max_level = lstar;
            p->n_max = 1 << 30;
            p->nodes_needed = 4;
            mn = 4;
        } else {
            mn = 2 * hmax;   // an error later unless the far field turns out empty
        }
    }
    p->mn = mn;
    p->H = mn / 2;
    {
        static const int hp[] = {4, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32};
        p->HP = 0;
        for (int v : hp) if (v >= p->H) { p->HP = v; break; }
    }
    p->R = 1;
    for (int k = 0; k < d - 1; ++k) p->R *= mn;
    p->P = p->R * p->H;
    p->L = 2.0 * M_PI / (2.0 * p->sigma / (mn - 1));
    p->min_level = std::max(p->lc, (o && o->min_level > 0) ? o->min_level : 0);
    if (p->max_level < p->min_level) p->max_level = p->min_level;
    return RBF_OK;
}

// n_src > 0: a plan for separate targets, points [0, n_src) the sources and the rest targets
int plan_impl(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
              const rbf_opts *opts, void *stream, rbf_plan **out, int64_t n_src = 0) {
    if (!points || !out) { set_error("rbf_fmm_plan: null pointer argument"); return RBF_EINVAL; }
    if (n < 1 || n > (int64_t)0x3fffffff) { set_error("rbf_fmm_plan: n=%lld out of range", (long long)n); return RBF_EINVAL; }
    if (d < 1 || d > kMaxDim) { set_error("rbf_fmm_plan: d=%d out of range [1,5]", d); return RBF_EINVAL; }
    if (d != 2 && d != 3 && d != 5) { set_error("rbf_fmm_plan: d=%d is not compiled (2, 3, 5 are)", d); return RBF_EUNSUPPORTED; }
    if (dtype != RBF_F32 && dtype != RBF_F64) { set_error("rbf_fmm_plan: bad dtype %d", dtype); return RBF_EINVAL; }
    if (kernel < RBF_GAUSSIAN || kernel > RBF_GAUSSIAN_BANDLIMITED) { set_error("rbf_fmm_plan: bad kernel %d", kernel); return RBF_EINVAL; }
    if (kernel == RBF_GAUSSIAN_BANDLIMITED && !(opts && opts->band > 0 && std::isfinite(opts->band))) {
        set_error("rbf_fmm_plan: the band-limited Gaussian needs its bandwidth in opts->band (> 0)");
        return RBF_EINVAL;
    }
    if (!(shape > 0) || !std::isfinite(shape)) { set_error("rbf_fmm_plan: shape must be positive"); return RBF_EINVAL; }
    if (!(tol > 0 && tol < 1)) { set_error("rbf_fmm_plan: tol must lie in (0, 1)"); return RBF_EINVAL; }
    rbf_plan *p = new (std::nothrow) rbf_plan();
    if (!p) { set_error("rbf_fmm_plan: out of host memory"); return RBF_ENOMEM; }
    p->n = n; p->d = d; p->dtype = dtype; p->kernel = kernel; p->shape = shape; p->tol = tol;
    p->n_src = n_src;
    p->stream = (hipStream_t)stream;
    p->n_max = (opts && opts->n_max > 0) ? opts->n_max : 128;
    // leaf translation block order: XCD leaf ranges unless the caller asks for leaf-major
    // (m2l_schedule = 2 selects 0 explicitly, since 0 is the "automatic" value of the field)
    p->m2l_sched = (opts && opts->m2l_schedule == 2) ? 0 : 1;
    p->max_level = (opts && opts->max_level > 0) ? opts->max_level : 64;
    int rc = compute_bbox(p, points);
    if (rc == RBF_OK) rc = choose_params(p, opts);
    if (rc == RBF_OK) rc = build_tree(p, points);
    const size_t tsz = dtype == RBF_F32 ? 4 : 8, csz = 2 * tsz;
    if (rc == RBF_OK) {
        // the far field is empty when every leaf is a coarse cell and the stencil is the
        // adjacent cells (or the root is the only leaf): then every kept pair is near
        const bool uniform_at_lc = p->min_leaf_level == p->lc && p->max_leaf_level == p->lc;
        if (uniform_at_lc && (p->lc == 0 || p->r <= 1)) p->far = 0;
        if (p->far && p->nodes_needed > p->mn) {
            set_error("tolerance %g needs %d quadrature nodes per dimension; at most %d are supported for d=%d "
                      "(a deeper coarse level or a near-only tree, see rbf_fmm_autotune, avoids the far field)",
                      tol, p->nodes_needed, p->mn, d);
            rc = RBF_EUNSUPPORTED;
        }
    }
    p->band_xfer = opts ? opts->band_transfer : 0;
    if (rc == RBF_OK && banded_kernel(kernel, d) && !(opts && opts->exact)) rc = plan_bands(p);
    if (rc == RBF_OK && kernel == RBF_GAUSSIAN_BANDLIMITED) rc = bandlimited_table(p, opts->band);
    const int64_t fboxes = p->far ? 1 : 0;   // expansions are allocated only with a far field
    if (rc == RBF_OK) {
        double need = (double)fboxes * csz * p->P * (2.0 * p->nleaves + 3.0 * p->ncells) +
                      (2.0 * tsz + fboxes * csz * p->HP) * n;
        if (need > 200e9) {
            set_error("rbf_fmm_plan: expansions need %.1f GB (nodes=%d, leaves=%d); raise tol or n_max", need / 1e9,
                      p->mn, p->nleaves);
            rc = RBF_ENOMEM;
        }
    }
    Arena &ar = p->arena;
    if (rc == RBF_OK) rc = ar.alloc(&p->lam_s, tsz * n);
    if (rc == RBF_OK) rc = ar.alloc(&p->u_s, tsz * n);
    if (rc == RBF_OK) rc = ar.alloc((void **)&p->p2p_ctr, sizeof(int) * kXcds * kCtrStride);
    if (rc == RBF_OK) rc = ar.alloc(&p->W, csz * p->P * p->nleaves * fboxes);
    if (rc == RBF_OK) rc = ar.alloc(&p->Lx, csz * p->R * p->HP * p->nleaves * fboxes);
    if (rc == RBF_OK) rc = ar.alloc(&p->dl, csz * p->HP * n * fboxes);
    if (rc == RBF_OK && fboxes) {
        // the padding entries (h >= H) of the local expansions stay zero from here on
        if (hipMemset(p->Lx, 0, csz * p->R * p->HP * p->nleaves) != hipSuccess) {
            set_error("rbf_fmm_plan: clearing the local expansions failed");
            rc = RBF_EHIP;
        }
    }
    if (rc == RBF_OK) rc = ar.alloc(&p->Wc, csz * p->P * p->ncells * fboxes);
    if (rc == RBF_OK) rc = ar.alloc(&p->Lc, csz * p->P * p->ncells * fboxes);
    if (rc == RBF_OK) rc = ar.alloc(&p->Tmp, csz * p->P * p->ncells * fboxes);
    if (rc == RBF_OK) rc = ar.alloc((void **)&p->xi, sizeof(double) * p->mn);
    if (rc == RBF_OK) rc = ar.alloc((void **)&p->wc1, sizeof(double) * p->mn);
    if (rc == RBF_OK) rc = ar.alloc((void **)&p->wtab, sizeof(double) * p->P * fboxes);
    if (rc == RBF_OK) {
        // tensor trapezoid nodes on [-sigma, sigma] and w_k C1(xi_k) for the Gaussian:
        // C(xi) = (2 pi)^-d Phi_hat(xi) = prod_k s/sqrt(2 pi) exp(-s^2 xi_k^2 / 2).
        std::vector<double> xi(p->mn), wc(p->mn);
        const double h = 2.0 * p->sigma / (p->mn - 1);
        for (int m = 0; m < p->mn; ++m) {
            xi[m] = -p->sigma + h * m;
            double w = (m == 0 || m == p->mn - 1) ? 0.5 * h : h;
            wc[m] = w * shape / std::sqrt(2.0 * M_PI) * std::exp(-0.5 * shape * shape * xi[m] * xi[m]);
        }
        hipError_t e1 = hipMemcpy(p->xi, xi.data(), sizeof(double) * p->mn, hipMemcpyHostToDevice);
        hipError_t e2 = hipMemcpy(p->wc1, wc.data(), sizeof(double) * p->mn, hipMemcpyHostToDevice);
        hipError_t e3 = hipSuccess;
        if (fboxes) {
            // w(xi) C(xi) = prod_k wc1[m_k] for every stored node (row digits m_1..m_{d-1}, m_d = H + h)
            std::vector<double> wt(p->P);
            for (int64_t q = 0; q < p->P; ++q) {
                int64_t rest = q / p->H;
                double f = wc[p->H + (int)(q % p->H)];
                for (int k = 0; k < d - 1; ++k) {
                    f *= wc[rest % p->mn];
                    rest /= p->mn;
                }
                wt[q] = f;
            }
            e3 = hipMemcpy(p->wtab, wt.data(), sizeof(double) * p->P, hipMemcpyHostToDevice);
        }
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            set_error("rbf_fmm_plan: table upload failed");
            rc = RBF_EHIP;
        }
    }
    if (rc == RBF_OK) {
        for (int k = 0; k < 2 * RBF_NPHASES && rc == RBF_OK; ++k)
            if (hipEventCreate(&p->ev[k]) != hipSuccess) { set_error("hipEventCreate failed"); rc = RBF_EHIP; }
    }
    if (rc != RBF_OK) {
        for (int k = 0; k < 2 * RBF_NPHASES; ++k) if (p->ev[k]) (void)hipEventDestroy(p->ev[k]);
        p->arena.release();
        delete p;
        return rc;
    }
    *out = p;
    return RBF_OK;
}

}  // namespace

int plan_create(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                const rbf_opts *opts, hipStream_t stream, rbf_plan **out) {
    return plan_impl(points, n, d, dtype, kernel, shape, tol, opts, stream, out);
}

int reject_eval_plan(const rbf_plan *p, const char *fn) {
    if (p && p->n_src > 0) {
        set_error("%s: the plan was made for separate targets (rbf_fmm_plan_eval); use rbf_fmm_eval", fn);
        return RBF_EINVAL;
    }
    return RBF_OK;
}

namespace {

constexpr int kEvalThreads = 256;

// Weights of a plan for separate targets: the sources' weights, then zeros at the targets.
template <class T>
__global__ void __launch_bounds__(kEvalThreads) k_eval_pack(const T *__restrict__ lam, int64_t n_src, int64_t n, T *out) {
    const int64_t i = blockIdx.x * (int64_t)kEvalThreads + threadIdx.x;
    if (i < n) out[i] = i < n_src ? lam[i] : T(0);
}
// The product at the targets: entries [n_src, n) of the product over all points.
template <class T>
__global__ void __launch_bounds__(kEvalThreads) k_eval_unpack(const T *__restrict__ all, int64_t n_src, int64_t m, T *u) {
    const int64_t t = blockIdx.x * (int64_t)kEvalThreads + threadIdx.x;
    if (t < m) u[t] = all[n_src + t];
}

template <class T>
int eval_t(rbf_plan *p, const void *lambda, void *u, bool direct) {
    const int64_t n = p->n, m = n - p->n_src;
    hipStream_t s = p->stream;
    k_eval_pack<T><<<(unsigned)((n + kEvalThreads - 1) / kEvalThreads), kEvalThreads, 0, s>>>((const T *)lambda, p->n_src, n,
                                                                                   (T *)p->ev_lam);
    RBF_HIP(hipGetLastError());
    RBF_TRY(direct ? launch_direct(p, p->ev_lam, p->ev_u) : launch_matvec(p, p->ev_lam, p->ev_u));
    if (m > 0) {
        k_eval_unpack<T><<<(unsigned)((m + kEvalThreads - 1) / kEvalThreads), kEvalThreads, 0, s>>>((const T *)p->ev_u, p->n_src,
                                                                                        m, (T *)u);
        RBF_HIP(hipGetLastError());
    }
    return RBF_OK;
}

int eval_impl(rbf_plan *p, const void *lambda, void *u, bool direct, const char *fn) {
    if (!p || !lambda) { set_error("%s: null argument", fn); return RBF_EINVAL; }
    if (p->n_src > 0 && !u && p->n > p->n_src) { set_error("%s: null u with targets to write", fn); return RBF_EINVAL; }
    if (p->n_src <= 0) { set_error("%s: the plan has no separate targets (make it with rbf_fmm_plan_eval)", fn); return RBF_EINVAL; }
    if (lambda == u) { set_error("%s: lambda and u must not alias", fn); return RBF_EINVAL; }
    return p->dtype == RBF_F32 ? eval_t<float>(p, lambda, u, direct) : eval_t<double>(p, lambda, u, direct);
}

}  // namespace

}  // namespace rbf

using namespace rbf;

extern "C" {

const char *rbf_last_error(void) { return g_err; }

int rbf_fmm_plan(const void *points, int64_t n, int d, int dtype, int kernel, double shape, double tol,
                 const rbf_opts *opts, void *stream, rbf_plan **out) {
    g_err[0] = 0;
    return plan_impl(points, n, d, dtype, kernel, shape, tol, opts, stream, out);
}

int rbf_fmm_matvec(rbf_plan *plan, const void *lambda, void *u) {
    if (!plan || !lambda || !u) { set_error("rbf_fmm_matvec: null argument"); return RBF_EINVAL; }
    if (lambda == u) { set_error("rbf_fmm_matvec: lambda and u must not alias"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_fmm_matvec"));
    return launch_matvec(plan, lambda, u);
}

int rbf_direct_matvec(rbf_plan *plan, const void *lambda, void *u) {
    if (!plan || !lambda || !u) { set_error("rbf_direct_matvec: null argument"); return RBF_EINVAL; }
    if (lambda == u) { set_error("rbf_direct_matvec: lambda and u must not alias"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_direct_matvec"));
    return launch_direct(plan, lambda, u);
}

int rbf_fmm_plan_eval(const void *sources, int64_t n, const void *targets, int64_t m, int d, int dtype, int kernel,
                      double shape, double tol, const rbf_opts *opts, void *stream, rbf_plan **out) {
    g_err[0] = 0;
    if (!sources || !out || (m > 0 && !targets)) { set_error("rbf_fmm_plan_eval: null pointer argument"); return RBF_EINVAL; }
    if (n < 1 || m < 0 || n + m > (int64_t)0x3fffffff) {
        set_error("rbf_fmm_plan_eval: n=%lld, m=%lld out of range", (long long)n, (long long)m);
        return RBF_EINVAL;
    }
    if (d < 1 || d > kMaxDim || (dtype != RBF_F32 && dtype != RBF_F64)) {
        set_error("rbf_fmm_plan_eval: bad d=%d or dtype=%d", d, dtype);
        return RBF_EINVAL;
    }
    // one point set: the sources, then the targets (the plan copies it and sorts its copy)
    const size_t tsz = dtype == RBF_F32 ? 4 : 8;
    hipStream_t s = (hipStream_t)stream;
    void *all = nullptr;
    if (hipMalloc(&all, tsz * (size_t)d * (size_t)(n + m)) != hipSuccess) {
        set_error("rbf_fmm_plan_eval: hipMalloc of the joined point set failed");
        return RBF_ENOMEM;
    }
    int rc = RBF_OK;
    if (hipMemcpyAsync(all, sources, tsz * d * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        (m > 0 && hipMemcpyAsync((char *)all + tsz * d * n, targets, tsz * d * m, hipMemcpyDeviceToDevice, s) !=
                      hipSuccess)) {
        set_error("rbf_fmm_plan_eval: copying the points failed");
        rc = RBF_EHIP;
    }
    rbf_plan *p = nullptr;
    if (rc == RBF_OK) rc = plan_impl(all, n + m, d, dtype, kernel, shape, tol, opts, stream, &p, n);
    (void)hipStreamSynchronize(s);
    (void)hipFree(all);
    if (rc != RBF_OK) return rc;
    rc = p->arena.alloc(&p->ev_lam, tsz * (size_t)(n + m));
    if (rc == RBF_OK) rc = p->arena.alloc(&p->ev_u, tsz * (size_t)(n + m));
    if (rc != RBF_OK) {
        rbf_fmm_destroy(p);
        return rc;
    }
    *out = p;
    return RBF_OK;
}

int rbf_fmm_eval(rbf_plan *plan, const void *lambda, void *u) {
    return eval_impl(plan, lambda, u, false, "rbf_fmm_eval");
}

int rbf_direct_eval(rbf_plan *plan, const void *lambda, void *u) {
    return eval_impl(plan, lambda, u, true, "rbf_direct_eval");
}

int rbf_fmm_destroy(rbf_plan *plan) {
    if (!plan) return RBF_OK;
    (void)hipStreamSynchronize(plan->stream);
    for (int k = 0; k < 2 * RBF_NPHASES; ++k) if (plan->ev[k]) (void)hipEventDestroy(plan->ev[k]);
    for (hipEvent_t e : plan->band_ev) if (e) (void)hipEventDestroy(e);
    if (plan->side) (void)hipStreamSynchronize(plan->side);
    if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
    if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
    if (plan->side) (void)hipStreamDestroy(plan->side);
    plan->solver_arena.release();
    plan->pc_arena.release();
    plan->arena.release();
    delete plan;
    return RBF_OK;
}

int rbf_fmm_plan_info(const rbf_plan *p, rbf_plan_info *info) {
    if (!p || !info) { set_error("rbf_fmm_plan_info: null argument"); return RBF_EINVAL; }
    std::memset(info, 0, sizeof(*info));
    info->n = p->n; info->d = p->d; info->dtype = p->dtype; info->kernel = p->kernel;
    info->nleaves = p->nleaves; info->nlevels = p->nlevels; info->coarse_level = p->lc;
    info->coarse_radius = p->r; info->nodes = p->mn; info->bits = p->B;
    info->half_nodes = p->P; info->ncells = p->ncells; info->nnear = p->nnear;
    info->near_pairs = p->near_pairs;
    info->shape = p->shape; info->tol = p->tol; info->band = p->sigma; info->period = p->L;
    info->rcut = p->rcut; info->rfar = p->rfar; info->ext = p->ext;
    for (int k = 0; k < kMaxDim; ++k) info->lo[k] = p->lo[k];
    info->device_bytes = p->arena.bytes + p->solver_arena.bytes + p->pc_arena.bytes;
    info->far_field = (p->far || !p->bands.empty()) ? 1 : 0;
    info->nbands = (int)p->bands.size();
    info->residual_width = p->res_s0;
    info->residual_in_q = p->res_q;
    return RBF_OK;
}

int rbf_fmm_band_info(const rbf_plan *p, int j, rbf_band_info *info) {
    if (!p || !info) { set_error("rbf_fmm_band_info: null argument"); return RBF_EINVAL; }
    if (j < 0 || j >= (int)p->bands.size()) {
        set_error("rbf_fmm_band_info: band %d out of range (the plan has %d)", j, (int)p->bands.size());
        return RBF_EINVAL;
    }
    const Band &b = p->bands[j];
    std::memset(info, 0, sizeof(*info));
    info->top = b.top;
    info->coarse_level = b.lc;
    info->coarse_radius = b.r;
    info->nodes = b.mn;
    info->half_nodes = b.P;
    info->nunits = b.nunits;
    info->nchunks = b.nchunks;
    info->width_lo = b.s_lo;
    info->width_hi = b.s_hi;
    info->tol = b.tau;
    info->band = b.sigma;
    info->period = b.L;
    info->reach = b.reach;
    info->rfar = b.rfar;
    info->scale = b.scale;
    info->transfer = b.xfer;
    info->transfer_order = b.xk;
    return RBF_OK;
}

int rbf_fmm_tree_export(const rbf_plan *p, int64_t *perm, int32_t *leaf_begin, int32_t *leaf_level,
                        uint64_t *leaf_prefix, int32_t *near_ptr, int32_t *near_idx) {
    if (!p) { set_error("rbf_fmm_tree_export: null plan"); return RBF_EINVAL; }
    RBF_HIP(hipStreamSynchronize(p->stream));
    if (perm) {
        std::vector<int> tmp(p->n);
        RBF_HIP(hipMemcpy(tmp.data(), p->perm, sizeof(int) * p->n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < p->n; ++i) perm[i] = tmp[i];
    }
    if (leaf_begin) RBF_HIP(hipMemcpy(leaf_begin, p->leaf_begin, sizeof(int) * (p->nleaves + 1), hipMemcpyDeviceToHost));
    if (leaf_level) RBF_HIP(hipMemcpy(leaf_level, p->leaf_level, sizeof(int) * p->nleaves, hipMemcpyDeviceToHost));
    if (leaf_prefix) RBF_HIP(hipMemcpy(leaf_prefix, p->leaf_prefix, sizeof(uint64_t) * p->nleaves, hipMemcpyDeviceToHost));
    if (near_ptr) RBF_HIP(hipMemcpy(near_ptr, p->near_ptr, sizeof(int) * (p->nleaves + 1), hipMemcpyDeviceToHost));
    if (near_idx && p->nnear) RBF_HIP(hipMemcpy(near_idx, p->near_idx, sizeof(int) * p->nnear, hipMemcpyDeviceToHost));
    return RBF_OK;
}

int rbf_fmm_set_profiling(rbf_plan *p, int on) {
    if (!p) { set_error("rbf_fmm_set_profiling: null plan"); return RBF_EINVAL; }
    p->profiling = on ? 1 : 0;
    for (int k = 0; k < RBF_NPHASES; ++k) p->phase_ms[k] = 0;
    p->prof_calls = 0;
    return RBF_OK;
}

int rbf_fmm_phase_times(const rbf_plan *p, double *ms, int64_t *calls) {
    if (!p || !ms) { set_error("rbf_fmm_phase_times: null argument"); return RBF_EINVAL; }
    for (int k = 0; k < RBF_NPHASES; ++k) ms[k] = p->phase_ms[k];
    if (calls) *calls = p->prof_calls;
    return RBF_OK;
}

}  // extern "C"

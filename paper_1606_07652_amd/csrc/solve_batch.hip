// Restarted GMRES for every problem of a batch at once (section 1 names GMRES as the Krylov
// method the fast product serves).  All problems advance together: each Arnoldi step is one
// batched product (one graph launch for all problems); the Gram-Schmidt projections (CGS2,
// FP64) are segmented per problem with a fixed blocking, so every problem's arithmetic is
// deterministic.  Each problem keeps its own Hessenberg matrix, Givens rotations and stopping
// test on the host; a problem that has converged (or reached its cap) in a cycle takes zero
// directions for the rest of it, which the batched product maps to zero.  Convergence is
// judged on the true residual ||f_p - A_p lambda_p|| / ||f_p||, recomputed at every restart.
// With block-Jacobi the solve is flexible GMRES with every problem's own blocks as the right
// preconditioner (one launch for all problems): direction z_j = M^{-1} v_j is kept beside v_j
// and the cycle's update is x += Z y.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.h"

namespace rbf {
namespace {

constexpr int kT = 256;
constexpr int kSeg = 4096;   // elements of one problem per workgroup of the segmented kernels

struct Seg {
    const int64_t *off;   // problem offsets [nprob + 1]
    const int *bstart;    // first workgroup of each problem [nprob + 1]
    int nprob;
};

__device__ __forceinline__ int seg_problem(const Seg &s, int g) {
    int lo = 0, hi = s.nprob;   // largest q with bstart[q] <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s.bstart[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// part[g * k + v] = sum over workgroup g's slice of V_v . w
__global__ void __launch_bounds__(kT) k_seg_dots(Seg s, const double *__restrict__ V, int64_t n, int k,
                                                 const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double sh[kT];
    const int g = blockIdx.x, q = seg_problem(s, g);
    const int64_t e0 = s.off[q] + (int64_t)(g - s.bstart[q]) * kSeg;
    const int64_t e1 = min(s.off[q + 1], e0 + kSeg);
    for (int v = 0; v < k; ++v) {
        const double *vv = V + (int64_t)v * n;
        double a = 0.0;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) a += vv[e] * w[e];
        a = block_sum(a, sh);
        if (threadIdx.x == 0) part[(int64_t)g * k + v] = a;
    }
}

// out[q * k + v] = sum of problem q's workgroup partials, in order
__global__ void __launch_bounds__(kT) k_seg_reduce(Seg s, const double *__restrict__ part, int k,
                                                   double *__restrict__ out) {
    __shared__ double sh[kT];
    const int q = blockIdx.x;
    const int b0 = s.bstart[q], b1 = s.bstart[q + 1];
    for (int v = 0; v < k; ++v) {
        double a = 0.0;
        for (int b = b0 + threadIdx.x; b < b1; b += kT) a += part[(int64_t)b * k + v];
        a = block_sum(a, sh);
        if (threadIdx.x == 0) out[(int64_t)q * k + v] = a;
    }
}

// w += sign * sum_v h[q * k + v] V_v on every problem's segment
__global__ void __launch_bounds__(kT) k_seg_axpy(Seg s, double *__restrict__ w, const double *__restrict__ V,
                                                 int64_t n, int k, const double *__restrict__ h, double sign) {
    const int g = blockIdx.x, q = seg_problem(s, g);
    const int64_t e0 = s.off[q] + (int64_t)(g - s.bstart[q]) * kSeg;
    const int64_t e1 = min(s.off[q + 1], e0 + kSeg);
    const double *hq = h + (int64_t)q * k;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) {
        double a = 0.0;
        for (int v = 0; v < k; ++v) a += hq[v] * V[(int64_t)v * n + e];
        w[e] += sign * a;
    }
}

// dst = src * scale[q] on every problem's segment
__global__ void __launch_bounds__(kT) k_seg_scale(Seg s, const double *__restrict__ src, const double *__restrict__ sc,
                                                  double *__restrict__ dst) {
    const int g = blockIdx.x, q = seg_problem(s, g);
    const int64_t e0 = s.off[q] + (int64_t)(g - s.bstart[q]) * kSeg;
    const int64_t e1 = min(s.off[q + 1], e0 + kSeg);
    const double f = sc[q];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kT) dst[e] = f * src[e];
}

template <class A, class B>
__global__ void k_cvt(const A *__restrict__ in, B *__restrict__ out, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) out[i] = (B)in[i];
}

__global__ void k_sub(const double *__restrict__ f, const double *__restrict__ ax, double *__restrict__ r, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) r[i] = f[i] - ax[i];
}

struct BatchSolver {
    rbf_batch *b;
    hipStream_t s;
    int64_t n;
    int nprob, nblk;
    Seg seg;
    unsigned gn;
    double *part = nullptr, *hdev = nullptr;
    void *tin = nullptr, *tout = nullptr;   // fixed product buffers (plan dtype)

    // y = A x in FP64 through fixed buffers (the batch's graph is captured once for them)
    int product(const double *x, double *y) {
        if (b->dtype == RBF_F64) {
            RBF_HIP(hipMemcpyAsync(tin, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            RBF_TRY(batch_product(b, tin, tout));
            RBF_HIP(hipMemcpyAsync(y, tout, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        } else {
            k_cvt<double, float><<<gn, kT, 0, s>>>(x, (float *)tin, n);
            RBF_HIP(hipGetLastError());
            RBF_TRY(batch_product(b, tin, tout));
            k_cvt<float, double><<<gn, kT, 0, s>>>((const float *)tout, y, n);
            RBF_HIP(hipGetLastError());
        }
        return RBF_OK;
    }

    // out (host) [nprob][k] = per-problem dots of V_0..V_{k-1} with w
    int dots(const double *V, int k, const double *w, double *host_out) {
        RBF_TRY(dots_dev(V, k, w, hdev));
        if (host_out) {
            RBF_HIP(hipMemcpyAsync(host_out, hdev, sizeof(double) * nprob * k, hipMemcpyDeviceToHost, s));
            RBF_HIP(hipStreamSynchronize(s));
        }
        return RBF_OK;
    }

    // the same dots into device memory out [nprob][k], no host read
    int dots_dev(const double *V, int k, const double *w, double *out) {
        k_seg_dots<<<nblk, kT, 0, s>>>(seg, V, n, k, w, part);
        RBF_HIP(hipGetLastError());
        k_seg_reduce<<<nprob, kT, 0, s>>>(seg, part, k, out);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }

    // w += sign * V h with h already on the device
    int axpy_dev(double *w, const double *V, int k, const double *h, double sign) {
        k_seg_axpy<<<nblk, kT, 0, s>>>(seg, w, V, n, k, h, sign);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }

    int axpy(double *w, const double *V, int k, const std::vector<double> &h, double sign) {
        RBF_HIP(hipMemcpyAsync(hdev, h.data(), sizeof(double) * nprob * k, hipMemcpyHostToDevice, s));
        k_seg_axpy<<<nblk, kT, 0, s>>>(seg, w, V, n, k, hdev, sign);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }

    int scale(const double *src, const std::vector<double> &sc, double *dst) {
        RBF_HIP(hipMemcpyAsync(hdev, sc.data(), sizeof(double) * nprob, hipMemcpyHostToDevice, s));
        k_seg_scale<<<nblk, kT, 0, s>>>(seg, src, hdev, dst);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }
};

int solve_batch_impl(rbf_batch *b, const void *f, void *lambda, double rtol, const rbf_solve_opts *o,
                     rbf_solve_info *infos) {
    auto t_start = std::chrono::steady_clock::now();
    const int m = (o && o->restart > 0) ? o->restart : 50;
    const int maxit = (o && o->max_iters > 0) ? o->max_iters : 1000;
    const double tlim = (o && o->time_limit_s > 0) ? o->time_limit_s : 0.0;
    const int P = b->nprob;
    const int64_t n = b->offsets[P];
    BatchSolver S;
    S.b = b;
    S.s = b->user_stream;
    S.n = n;
    S.nprob = P;
    S.gn = (unsigned)((n + kT - 1) / kT);
    // workgroup layout of the segmented kernels
    std::vector<int> bst(P + 1, 0);
    for (int q = 0; q < P; ++q) bst[q + 1] = bst[q] + (int)((b->offsets[q + 1] - b->offsets[q] + kSeg - 1) / kSeg);
    S.nblk = bst[P];
    Arena ar;
    const size_t tsz = b->dtype == RBF_F32 ? 4 : 8;
    double *V = nullptr, *Z = nullptr, *x = nullptr, *fd = nullptr, *r = nullptr, *w = nullptr;
    const bool pc = o && o->precond == RBF_PC_BLOCK_JACOBI;
    int64_t *offd = nullptr;
    int *bstd = nullptr;
    auto fail = [&](int rc) {
        ar.release();
        return rc;
    };
    int rc;
    if ((rc = ar.alloc((void **)&V, sizeof(double) * (size_t)(m + 1) * n)) != RBF_OK ||
        (rc = ar.alloc((void **)&x, sizeof(double) * n)) != RBF_OK ||
        (rc = ar.alloc((void **)&fd, sizeof(double) * n)) != RBF_OK ||
        (rc = ar.alloc((void **)&r, sizeof(double) * n)) != RBF_OK ||
        (rc = ar.alloc((void **)&w, sizeof(double) * n)) != RBF_OK ||
        (rc = ar.alloc(&S.tin, tsz * n)) != RBF_OK || (rc = ar.alloc(&S.tout, tsz * n)) != RBF_OK ||
        (rc = ar.alloc((void **)&S.part, sizeof(double) * (size_t)S.nblk * (m + 1))) != RBF_OK ||
        (rc = ar.alloc((void **)&S.hdev, sizeof(double) * (size_t)P * (2 * (m + 1) + 1))) != RBF_OK ||
        (rc = ar.alloc((void **)&offd, sizeof(int64_t) * (P + 1))) != RBF_OK ||
        (rc = ar.alloc((void **)&bstd, sizeof(int) * (P + 1))) != RBF_OK)
        return fail(rc);
    hipStream_t s = S.s;
    BatchBj bj{};
    if (pc) {
        if ((rc = ar.alloc((void **)&Z, sizeof(double) * (size_t)m * n)) != RBF_OK) return fail(rc);
        if ((rc = batch_bj_prepare(b->plans, b->offsets, ar, s, &bj)) != RBF_OK) return fail(rc);
    }
    if (hipMemcpyAsync(offd, b->offsets.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(bstd, bst.data(), sizeof(int) * (P + 1), hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("rbf_interp_solve_batch: upload failed");
        return fail(RBF_EHIP);
    }
    S.seg = Seg{offd, bstd, P};
    const bool zero = o && o->zero_init;
    if (b->dtype == RBF_F64) {
        if (hipMemcpyAsync(fd, f, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(RBF_EHIP);
        if (zero) { if (hipMemsetAsync(x, 0, sizeof(double) * n, s) != hipSuccess) return fail(RBF_EHIP); }
        else if (hipMemcpyAsync(x, lambda, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(RBF_EHIP);
    } else {
        k_cvt<float, double><<<S.gn, kT, 0, s>>>((const float *)f, fd, n);
        if (zero) { if (hipMemsetAsync(x, 0, sizeof(double) * n, s) != hipSuccess) return fail(RBF_EHIP); }
        else k_cvt<float, double><<<S.gn, kT, 0, s>>>((const float *)lambda, x, n);
    }
    std::vector<double> fn(P), tmp((size_t)P * (m + 1));
    if ((rc = S.dots(fd, 1, fd, tmp.data())) != RBF_OK) return fail(rc);
    for (int q = 0; q < P; ++q) fn[q] = std::sqrt(tmp[q]);
    std::vector<rbf_solve_info> inf(P);
    std::memset(inf.data(), 0, sizeof(rbf_solve_info) * P);
    std::vector<double> H((size_t)P * (m + 1) * m), cs((size_t)P * m), sn((size_t)P * m), g((size_t)P * (m + 1));
    std::vector<double> h1((size_t)P * (m + 1)), h2((size_t)P * (m + 1)), hn(P), sc(P), coef;
    std::vector<double> hstep((size_t)P * (2 * (m + 1) + 1));
    std::vector<int> its(P, 0), kq(P, 0), done(P, 0);
    std::vector<double> rel(P, 0.0);
    auto Hq = [&](int q, int i, int j) -> double & { return H[((size_t)q * (m + 1) + i) * m + j]; };
    while (true) {
        // true residuals
        if ((rc = S.product(x, w)) != RBF_OK) return fail(rc);
        k_sub<<<S.gn, kT, 0, s>>>(fd, w, r, n);
        if ((rc = S.dots(r, 1, r, tmp.data())) != RBF_OK) return fail(rc);
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        int nactive = 0;
        for (int q = 0; q < P; ++q) {
            const double beta = std::sqrt(tmp[q]);
            rel[q] = fn[q] > 0 ? beta / fn[q] : 0.0;
            if (inf[q].nhistory < 256) {
                inf[q].history_s[inf[q].nhistory] = el;
                inf[q].history[inf[q].nhistory++] = rel[q];
            }
            const bool act = fn[q] > 0 && rel[q] > rtol && its[q] < maxit && std::isfinite(rel[q]);
            done[q] = act ? 0 : 1;
            sc[q] = act ? 1.0 / beta : 0.0;
            nactive += act;
            std::fill(&g[(size_t)q * (m + 1)], &g[(size_t)q * (m + 1)] + m + 1, 0.0);
            g[(size_t)q * (m + 1)] = act ? beta : 0.0;
            kq[q] = 0;
        }
        if (nactive == 0 || (tlim > 0 && el >= tlim)) break;
        std::fill(H.begin(), H.end(), 0.0);
        if ((rc = S.scale(r, sc, V)) != RBF_OK) return fail(rc);
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n;
            if (pc) {
                double *zj = Z + (size_t)j * n;
                if ((rc = batch_bj_apply(bj, vj, zj, s)) != RBF_OK) return fail(rc);
                vj = zj;
            }
            if ((rc = S.product(vj, w)) != RBF_OK) return fail(rc);
            const int k = j + 1;
            // CGS2 per problem, projections and norms on the device; one read of the step's
            // scalars: h1 [P][k], h2 [P][k], ||w_q||^2 [P]
            double *d1 = S.hdev, *d2 = S.hdev + (size_t)P * k, *dn = S.hdev + 2 * (size_t)P * k;
            if ((rc = S.dots_dev(V, k, w, d1)) != RBF_OK) return fail(rc);
            if ((rc = S.axpy_dev(w, V, k, d1, -1.0)) != RBF_OK) return fail(rc);
            if ((rc = S.dots_dev(V, k, w, d2)) != RBF_OK) return fail(rc);
            if ((rc = S.axpy_dev(w, V, k, d2, -1.0)) != RBF_OK) return fail(rc);
            if ((rc = S.dots_dev(w, 1, w, dn)) != RBF_OK) return fail(rc);
            if (hipMemcpyAsync(hstep.data(), S.hdev, sizeof(double) * (size_t)P * (2 * k + 1), hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("rbf_interp_solve_batch: device error");
                return fail(RBF_EHIP);
            }
            for (size_t e = 0; e < (size_t)P * k; ++e) {
                h1[e] = hstep[e];
                h2[e] = hstep[(size_t)P * k + e];
            }
            for (int q = 0; q < P; ++q) tmp[q] = hstep[2 * (size_t)P * k + q];
            int nlive = 0;
            for (int q = 0; q < P; ++q) {
                hn[q] = std::sqrt(tmp[q]);
                sc[q] = 0.0;
                if (done[q]) continue;
                for (int i = 0; i <= j; ++i) Hq(q, i, j) = h1[(size_t)q * k + i] + h2[(size_t)q * k + i];
                Hq(q, j + 1, j) = hn[q];
                double *csq = &cs[(size_t)q * m], *snq = &sn[(size_t)q * m], *gq = &g[(size_t)q * (m + 1)];
                for (int i = 0; i < j; ++i) {
                    const double a = Hq(q, i, j), bb = Hq(q, i + 1, j);
                    Hq(q, i, j) = csq[i] * a + snq[i] * bb;
                    Hq(q, i + 1, j) = -snq[i] * a + csq[i] * bb;
                }
                const double a = Hq(q, j, j), den = std::hypot(a, hn[q]);
                if (den == 0.0) { csq[j] = 1.0; snq[j] = 0.0; } else { csq[j] = a / den; snq[j] = hn[q] / den; }
                Hq(q, j, j) = den;
                Hq(q, j + 1, j) = 0.0;
                gq[j + 1] = -snq[j] * gq[j];
                gq[j] = csq[j] * gq[j];
                ++its[q];
                kq[q] = j + 1;
                const bool stop = !(hn[q] > 0.0) || !std::isfinite(hn[q]) || std::fabs(gq[j + 1]) / fn[q] <= rtol ||
                                  its[q] >= maxit;
                if (stop) done[q] = 1;
                else { sc[q] = 1.0 / hn[q]; ++nlive; }
            }
            if (nlive == 0 || j + 1 == m) break;
            if ((rc = S.scale(w, sc, V + (size_t)(j + 1) * n)) != RBF_OK) return fail(rc);
        }
        // x += V y per problem (coefficients beyond a problem's k_q are zero)
        int kmax = 0;
        for (int q = 0; q < P; ++q) kmax = std::max(kmax, kq[q]);
        if (kmax > 0) {
            coef.assign((size_t)P * kmax, 0.0);
            for (int q = 0; q < P; ++q) {
                const int k = kq[q];
                const double *gq = &g[(size_t)q * (m + 1)];
                for (int i = k - 1; i >= 0; --i) {
                    double t = gq[i];
                    for (int l = i + 1; l < k; ++l) t -= Hq(q, i, l) * coef[(size_t)q * kmax + l];
                    coef[(size_t)q * kmax + i] = t / Hq(q, i, i);
                }
                if (k > 0) ++inf[q].restarts;
            }
            if ((rc = S.axpy(x, pc ? Z : V, kmax, coef, 1.0)) != RBF_OK) return fail(rc);
        }
    }
    // solution in the batch's dtype
    if (b->dtype == RBF_F64) {
        if (hipMemcpyAsync(lambda, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s) != hipSuccess) return fail(RBF_EHIP);
    } else {
        k_cvt<double, float><<<S.gn, kT, 0, s>>>(x, (float *)lambda, n);
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("rbf_interp_solve_batch: device error");
        return fail(RBF_EHIP);
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    int nconv = 0;
    for (int q = 0; q < P; ++q) {
        inf[q].iters = its[q];
        inf[q].true_res = fn[q] > 0 ? rel[q] : 0.0;
        inf[q].converged = inf[q].true_res <= rtol;
        inf[q].seconds = secs;
        nconv += inf[q].converged;
        if (infos) infos[q] = inf[q];
    }
    ar.release();
    return nconv == P ? RBF_OK : RBF_ENOCONV;
}

}  // namespace
}  // namespace rbf

using namespace rbf;

extern "C" int rbf_interp_solve_batch(rbf_batch *batch, const void *f, void *lambda, double rtol,
                                      const rbf_solve_opts *opts, rbf_solve_info *info) {
    if (!batch || !f || !lambda) { set_error("rbf_interp_solve_batch: null argument"); return RBF_EINVAL; }
    if (batch->kernel == RBF_THIN_PLATE || batch->kernel == RBF_R5) {
        set_error("rbf_interp_solve_batch: the thin-plate spline and r^5 need polynomial terms, which only the "
                  "single-problem rbf_interp_solve_poly provides");
        return RBF_EUNSUPPORTED;
    }
    if (!(rtol > 0 && rtol < 1)) { set_error("rbf_interp_solve_batch: rtol must lie in (0, 1)"); return RBF_EINVAL; }
    if (opts && (opts->restart < 0 || opts->restart > 1000)) {
        set_error("rbf_interp_solve_batch: restart out of range");
        return RBF_EINVAL;
    }
    if (opts && opts->precond != RBF_PC_NONE && opts->precond != RBF_PC_BLOCK_JACOBI) {
        set_error("rbf_interp_solve_batch: batched solves take no preconditioner or block-Jacobi");
        return RBF_EUNSUPPORTED;
    }
    return solve_batch_impl(batch, f, lambda, rtol, opts, info);
}

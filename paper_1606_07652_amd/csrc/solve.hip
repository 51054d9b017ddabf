// Restarted (flexible) GMRES for A lambda = f with the fast product (section 1 names
// GMRES as the Krylov method the fast product serves; the paper gives no details).
//
// Arnoldi vectors live on the device in FP64.  Orthogonalisation is classical
// Gram-Schmidt applied twice (CGS2: two block projections, each a multi-dot and a
// multi-axpy), which is mathematically the modified Gram-Schmidt of the CPU reference
// and differs from it only in rounding.  Reductions use a fixed blocking, so a solve is
// deterministic.  The (m+1) x m Hessenberg system, its Givens rotations and the
// restart logic run on the host; each inner step moves j+2 doubles to the host.
// Convergence is judged on the true residual ||f - A lambda|| / ||f||, recomputed with
// a fresh product at every restart.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace rbf {
namespace {

constexpr int kThreads = 256;
constexpr int kDotBlocks = 512;

template <class A, class B>
__global__ void k_cvt(const A *__restrict__ in, B *__restrict__ out, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) out[i] = (B)in[i];
}

__global__ void k_sub(const double *__restrict__ f, const double *__restrict__ ax, double *__restrict__ r, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) r[i] = f[i] - ax[i];
}

__global__ void k_scale(const double *__restrict__ src, double a, double *__restrict__ dst, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) dst[i] = a * src[i];
}

// dst = src / sqrt(*nrm2): the next Arnoldi vector, normalised on the device so that the host
// reads the step's scalars once
__global__ void k_scale_rsqrt(const double *__restrict__ src, const double *__restrict__ nrm2,
                              double *__restrict__ dst, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) dst[i] = (1.0 / sqrt(*nrm2)) * src[i];
}

__device__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// part[b * k + v] = sum over block b's slice of V[v] . w
__global__ void __launch_bounds__(kThreads) k_multidot(const double *__restrict__ V, int64_t n, int k,
                                                       const double *__restrict__ w, double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    for (int v = 0; v < k; ++v) {
        const double *vv = V + (int64_t)v * n;
        double s = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) s += vv[i] * w[i];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) part[blockIdx.x * k + v] = s;
    }
}

__global__ void __launch_bounds__(kThreads) k_reduce_parts(const double *__restrict__ part, int nb, int k,
                                                           double *__restrict__ out) {
    __shared__ double sh[kThreads];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) s += part[b * k + v];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[v] = s;
}

// w -= sum_v h[v] V[v]   (sign = -1)   or   x += sum_v h[v] V[v]   (sign = +1)
__global__ void k_multiaxpy(double *__restrict__ w, const double *__restrict__ V, int64_t n, int k,
                            const double *__restrict__ h, double sign) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int v = 0; v < k; ++v) s += h[v] * V[(int64_t)v * n + i];
    w[i] += sign * s;
}

// Polynomial part of an augmented product (conditionally positive definite kernels): the
// monomials of t = (x - lo) / ext up to degree 2 (1; t_1 .. t_d; t_a t_b for a <= b).
struct Poly {
    int q = 0, deg = -1, d = 0;
    double lo[kMaxDim] = {0, 0, 0, 0, 0};
    double inv_ext = 1.0;
};
constexpr int kMaxPolyTerms = 1 + kMaxDim + kMaxDim * (kMaxDim + 1) / 2;

int poly_degree(int kernel) {
    switch (kernel) {
        case RBF_MULTIQUADRIC: return 0;
        case RBF_THIN_PLATE: return 1;
        case RBF_R5: return 2;
        default: return -1;
    }
}

int poly_terms(int d, int deg) {
    if (deg < 0) return 0;
    return 1 + (deg >= 1 ? d : 0) + (deg >= 2 ? d * (d + 1) / 2 : 0);
}

template <class T>
__device__ __forceinline__ void monomials(const T *__restrict__ xs, int64_t n, int64_t s, const Poly &P,
                                          double (&m)[kMaxPolyTerms]) {
    double t[kMaxDim];
    for (int a = 0; a < P.d; ++a) t[a] = ((double)xs[(int64_t)a * n + s] - P.lo[a]) * P.inv_ext;
    int k = 0;
    m[k++] = 1.0;
    if (P.deg >= 1)
        for (int a = 0; a < P.d; ++a) m[k++] = t[a];
    if (P.deg >= 2)
        for (int a = 0; a < P.d; ++a)
            for (int b = a; b < P.d; ++b) m[k++] = t[a] * t[b];
}

// y[perm[s]] += sum_k c_k p_k(t_s)
template <class T>
__global__ void k_poly_add(const T *__restrict__ xs, const int *__restrict__ perm, int64_t n, Poly P,
                           const double *__restrict__ c, double *__restrict__ y) {
    const int64_t s = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (s >= n) return;
    double m[kMaxPolyTerms];
    monomials(xs, n, s, P, m);
    double v = 0.0;
    for (int k = 0; k < P.q; ++k) v = fma(c[k], m[k], v);
    y[perm[s]] += v;
}

// part[b * q + k] = sum over block b's slice of x[perm[s]] p_k(t_s)
template <class T>
__global__ void __launch_bounds__(kThreads) k_poly_dots(const T *__restrict__ xs, const int *__restrict__ perm,
                                                        int64_t n, Poly P, const double *__restrict__ x,
                                                        double *__restrict__ part) {
    __shared__ double sh[kThreads];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    double acc[kMaxPolyTerms];
    for (int k = 0; k < kMaxPolyTerms; ++k) acc[k] = 0.0;
    for (int64_t s = i0 + threadIdx.x; s < i1; s += kThreads) {
        double m[kMaxPolyTerms];
        monomials(xs, n, s, P, m);
        const double v = x[perm[s]];
        for (int k = 0; k < P.q; ++k) acc[k] = fma(v, m[k], acc[k]);
    }
    for (int k = 0; k < P.q; ++k) {
        const double t = block_sum(acc[k], sh);
        if (threadIdx.x == 0) part[blockIdx.x * P.q + k] = t;
    }
}

__global__ void k_isfinite(const double *__restrict__ v, int64_t n, int *flag) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n && !isfinite(v[i])) *flag = 1;
}

// Krylov vectors have na = n + q entries: the weights in caller order, then the q polynomial
// coefficients of an augmented system (q = 0 otherwise).
struct Solver {
    rbf_plan *p;
    int64_t n, na;
    unsigned nb;
    Poly poly;
    double *part = nullptr, *hdev = nullptr, *xd = nullptr, *fd = nullptr, *rd = nullptr, *wd = nullptr;
    int *flag = nullptr;

    int product(const double *x64, double *y64) {
        // y = A x through the plan's dtype, then the polynomial blocks [P c; P' lambda]
        hipStream_t s = p->stream;
        if (p->dtype == RBF_F64) {
            RBF_TRY(launch_matvec(p, x64, y64));
        } else {
            float *tin = (float *)p->tvec, *tout = tin + n;
            k_cvt<double, float><<<nb, kThreads, 0, s>>>(x64, tin, n);
            RBF_HIP(hipGetLastError());
            RBF_TRY(launch_matvec(p, tin, tout));
            k_cvt<float, double><<<nb, kThreads, 0, s>>>(tout, y64, n);
            RBF_HIP(hipGetLastError());
        }
        if (poly.q > 0) {
            if (p->dtype == RBF_F64) {
                k_poly_add<double><<<nb, kThreads, 0, s>>>((const double *)p->xs, p->perm, n, poly, x64 + n, y64);
                k_poly_dots<double><<<kDotBlocks, kThreads, 0, s>>>((const double *)p->xs, p->perm, n, poly, x64,
                                                                    part);
            } else {
                k_poly_add<float><<<nb, kThreads, 0, s>>>((const float *)p->xs, p->perm, n, poly, x64 + n, y64);
                k_poly_dots<float><<<kDotBlocks, kThreads, 0, s>>>((const float *)p->xs, p->perm, n, poly, x64,
                                                                   part);
            }
            RBF_HIP(hipGetLastError());
            k_reduce_parts<<<poly.q, kThreads, 0, s>>>(part, kDotBlocks, poly.q, y64 + n);
            RBF_HIP(hipGetLastError());
        }
        return RBF_OK;
    }

    int dots(const double *V, int k, const double *w, double *host_out) {
        hipStream_t s = p->stream;
        k_multidot<<<kDotBlocks, kThreads, 0, s>>>(V, na, k, w, part);
        RBF_HIP(hipGetLastError());
        k_reduce_parts<<<k, kThreads, 0, s>>>(part, kDotBlocks, k, hdev);
        RBF_HIP(hipGetLastError());
        if (host_out) {
            RBF_HIP(hipMemcpyAsync(host_out, hdev, sizeof(double) * k, hipMemcpyDeviceToHost, s));
            RBF_HIP(hipStreamSynchronize(s));
        }
        return RBF_OK;
    }

    // the k dots into device memory, no host read
    int dots_dev(const double *V, int k, const double *w, double *out) {
        hipStream_t s = p->stream;
        k_multidot<<<kDotBlocks, kThreads, 0, s>>>(V, na, k, w, part);
        RBF_HIP(hipGetLastError());
        k_reduce_parts<<<k, kThreads, 0, s>>>(part, kDotBlocks, k, out);
        RBF_HIP(hipGetLastError());
        return RBF_OK;
    }

    int norm(const double *w, double *out) {
        double v = 0;
        RBF_TRY(dots(w, 1, w, &v));
        *out = std::sqrt(v);
        return RBF_OK;
    }
};

// coeffs: the q polynomial coefficients of an augmented solve (plan dtype, device; q = 0: unused)
int solve_impl(rbf_plan *p, const void *f, void *lambda, double rtol, const rbf_solve_opts *o,
               rbf_solve_info *info, int q = 0, void *coeffs = nullptr) {
    auto t_start = std::chrono::steady_clock::now();
    const int64_t n = p->n, na = n + q;
    const int m = (o && o->restart > 0) ? o->restart : 50;
    const int maxit = (o && o->max_iters > 0) ? o->max_iters : 1000;
    int pck = o ? o->precond : RBF_PC_NONE;
    const bool fallback = o ? (o->fallback != 0) : true;
    const double tlim = (o && o->time_limit_s > 0) ? o->time_limit_s : 0.0;
    if (pck != RBF_PC_NONE) {
        int rc = pc_ready(p, pck);
        if (rc != RBF_OK) return rc;
    }
    hipStream_t s = p->stream;
    if (p->solver_m < m || p->solver_na < na) {
        p->solver_arena.release();
        p->solver_m = 0;
        p->solver_na = 0;
        Arena &ar = p->solver_arena;
        const int kp = std::max(m + 2, kMaxPolyTerms);   // partial sums of the dots and of P' x
        RBF_TRY(ar.alloc((void **)&p->V, sizeof(double) * (size_t)(m + 1) * na));
        RBF_TRY(ar.alloc((void **)&p->Z, sizeof(double) * (size_t)m * na));
        RBF_TRY(ar.alloc((void **)&p->sv, sizeof(double) * ((size_t)kDotBlocks * kp + 4 * (m + 2) + 8)));
        RBF_TRY(ar.alloc(&p->tvec, sizeof(double) * (size_t)7 * na));
        p->solver_m = m;
        p->solver_na = na;
    }
    Solver S;
    S.p = p;
    S.n = n;
    S.na = na;
    S.nb = (unsigned)((n + kThreads - 1) / kThreads);
    S.poly.q = q;
    S.poly.deg = poly_degree(p->kernel);
    S.poly.d = p->d;
    for (int a = 0; a < p->d; ++a) S.poly.lo[a] = p->lo[a];
    S.poly.inv_ext = 1.0 / p->ext;
    const int kp = std::max(m + 2, kMaxPolyTerms);
    S.part = p->sv;
    S.hdev = p->sv + (size_t)kDotBlocks * kp;
    // hdev: h1 [m + 2], h2 [m + 2], ||w||^2, the preconditioner's status word (one double slot)
    S.flag = (int *)(S.hdev + 2 * (m + 2) + 1);
    double *base = (double *)p->tvec;
    S.xd = base + 2 * na;  // tvec[0..2n) holds the float in/out pair for F32 plans
    S.fd = base + 3 * na;
    S.rd = base + 4 * na;
    S.wd = base + 5 * na;
    double *const xbest = base + 6 * na;   // the iterate with the lowest true residual so far
    const unsigned nb = (unsigned)((na + kThreads - 1) / kThreads);   // grid over the Krylov length
    const size_t tsz = p->dtype == RBF_F64 ? 8 : 4;
    // x0 and f in FP64: [lambda; c] and [f; 0]
    if (q > 0) RBF_HIP(hipMemsetAsync(S.fd + n, 0, sizeof(double) * q, s));
    if (o && o->zero_init) RBF_HIP(hipMemsetAsync(S.xd, 0, sizeof(double) * na, s));
    if (p->dtype == RBF_F64) {
        RBF_HIP(hipMemcpyAsync(S.fd, f, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (!(o && o->zero_init)) {
            RBF_HIP(hipMemcpyAsync(S.xd, lambda, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            if (q > 0) RBF_HIP(hipMemcpyAsync(S.xd + n, coeffs, tsz * q, hipMemcpyDeviceToDevice, s));
        }
    } else {
        k_cvt<float, double><<<S.nb, kThreads, 0, s>>>((const float *)f, S.fd, n);
        if (!(o && o->zero_init)) {
            k_cvt<float, double><<<S.nb, kThreads, 0, s>>>((const float *)lambda, S.xd, n);
            if (q > 0) k_cvt<float, double><<<1, kThreads, 0, s>>>((const float *)coeffs, S.xd + n, q);
        }
        RBF_HIP(hipGetLastError());
    }
    double bnorm = 0;
    RBF_TRY(S.norm(S.fd, &bnorm));
    rbf_solve_info inf;
    std::memset(&inf, 0, sizeof(inf));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hstep(2 * (m + 2) + 1);
    int its = 0, restarts = 0;
    int cur = pck;   // active preconditioner: steps down learned -> block-Jacobi -> none
    auto step_down = [&]() {
        cur = cur == RBF_PC_LEARNED ? RBF_PC_BLOCK_JACOBI : RBF_PC_NONE;
        ++inf.fallback_used;
    };
    double best = INFINITY;
    double last_cycle_res = INFINITY;
    if (bnorm == 0.0) {
        RBF_HIP(hipMemsetAsync(S.xd, 0, sizeof(double) * na, s));
    }
    while (bnorm > 0.0) {
        RBF_TRY(S.product(S.xd, S.wd));
        k_sub<<<nb, kThreads, 0, s>>>(S.fd, S.wd, S.rd, na);
        RBF_HIP(hipGetLastError());
        double beta = 0;
        RBF_TRY(S.norm(S.rd, &beta));
        double rel = beta / bnorm;
        if (inf.nhistory < 256) {
            inf.history_s[inf.nhistory] =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            inf.history[inf.nhistory++] = rel;
        }
        if (rel < best) {
            best = rel;
            RBF_HIP(hipMemcpyAsync(xbest, S.xd, sizeof(double) * na, hipMemcpyDeviceToDevice, s));
        }
        double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (!(rel > rtol) || its >= maxit || (tlim > 0 && el >= tlim) || !std::isfinite(rel)) break;
        if (cur != RBF_PC_NONE && fallback && restarts > 0 && rel > 0.999 * last_cycle_res)
            step_down();   // the preconditioned cycle did not reduce the true residual
        last_cycle_res = rel;
        k_scale<<<nb, kThreads, 0, s>>>(S.rd, 1.0 / beta, p->V, na);
        RBF_HIP(hipGetLastError());
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        bool pc_failed = false;
        const bool use_pc = cur != RBF_PC_NONE;
        for (int j = 0; j < m; ++j) {
            double *vj = p->V + (size_t)j * na;
            double *zj = use_pc ? p->Z + (size_t)j * na : vj;
            if (use_pc) {
                // Flexible GMRES accepts any direction z_j.  With the learned map the cycle
                // is block-Jacobi FGMRES except for its last direction, z_{m-1} =
                // learned(v_0): the network is trained on residuals and v_0 is the
                // normalised residual (the cycle's space is augmented with the learned
                // error estimate, the block-Jacobi directions before it are unchanged).
                int kind = cur;
                const double *src = vj;
                if (cur == RBF_PC_LEARNED) {
                    const bool last = j == m - 1 && m > 1;
                    kind = last ? RBF_PC_LEARNED : RBF_PC_BLOCK_JACOBI;
                    if (last) src = p->V;
                }
                RBF_TRY(pc_apply(p, kind, src, zj));
                int hf = 0;
                RBF_HIP(hipMemsetAsync(S.flag, 0, sizeof(int), s));
                k_isfinite<<<nb, kThreads, 0, s>>>(zj, na, S.flag);
                RBF_HIP(hipMemcpyAsync(&hf, S.flag, sizeof(int), hipMemcpyDeviceToHost, s));
                RBF_HIP(hipStreamSynchronize(s));
                if (hf) { pc_failed = true; break; }
            }
            RBF_TRY(S.product(zj, S.wd));
            // CGS2 with the projections and the norm on the device, and the next vector
            // normalised there; one read of the step's scalars
            double *h1 = S.hdev, *h2 = S.hdev + (m + 2), *nrm2 = S.hdev + 2 * (m + 2);
            RBF_TRY(S.dots_dev(p->V, j + 1, S.wd, h1));
            k_multiaxpy<<<nb, kThreads, 0, s>>>(S.wd, p->V, na, j + 1, h1, -1.0);
            RBF_HIP(hipGetLastError());
            RBF_TRY(S.dots_dev(p->V, j + 1, S.wd, h2));
            k_multiaxpy<<<nb, kThreads, 0, s>>>(S.wd, p->V, na, j + 1, h2, -1.0);
            RBF_HIP(hipGetLastError());
            RBF_TRY(S.dots_dev(S.wd, 1, S.wd, nrm2));
            k_scale_rsqrt<<<nb, kThreads, 0, s>>>(S.wd, nrm2, p->V + (size_t)(j + 1) * na, na);
            RBF_HIP(hipGetLastError());
            RBF_HIP(hipMemcpyAsync(hstep.data(), S.hdev, sizeof(double) * (2 * (m + 2) + 1), hipMemcpyDeviceToHost, s));
            RBF_HIP(hipStreamSynchronize(s));
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hstep[i] + hstep[(size_t)(m + 2) + i];
            const double hn = std::sqrt(hstep[2 * (size_t)(m + 2)]);
            H[(size_t)(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[(size_t)j * m + j], den = std::hypot(a, hn);
            if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; } else { cs[j] = a / den; sn[j] = hn / den; }
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++its;
            k = j + 1;
            if (!std::isfinite(hn)) { pc_failed = use_pc; k = j; break; }
            if (hn == 0.0 || std::fabs(g[j + 1]) / bnorm <= rtol || its >= maxit) break;
        }
        if (pc_failed) {
            if (!fallback) { set_error("rbf_interp_solve: preconditioner produced non-finite values"); return RBF_EINVAL; }
            step_down();
            ++restarts;
            continue;
        }
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int l = i + 1; l < k; ++l) t -= H[(size_t)i * m + l] * y[l];
            y[i] = t / H[(size_t)i * m + i];
        }
        if (k > 0) {
            RBF_HIP(hipMemcpyAsync(S.hdev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
            k_multiaxpy<<<nb, kThreads, 0, s>>>(S.xd, use_pc ? p->Z : p->V, na, k, S.hdev, 1.0);
            RBF_HIP(hipGetLastError());
            RBF_HIP(hipStreamSynchronize(s));
        }
        ++restarts;
    }
    // the best iterate (a cycle after a preconditioner fallback can raise the true residual)
    if (bnorm > 0.0 && std::isfinite(best))
        RBF_HIP(hipMemcpyAsync(S.xd, xbest, sizeof(double) * na, hipMemcpyDeviceToDevice, s));
    // write the solution (and the polynomial coefficients) in the plan's dtype
    if (p->dtype == RBF_F64) {
        RBF_HIP(hipMemcpyAsync(lambda, S.xd, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (q > 0) RBF_HIP(hipMemcpyAsync(coeffs, S.xd + n, sizeof(double) * q, hipMemcpyDeviceToDevice, s));
    } else {
        k_cvt<double, float><<<S.nb, kThreads, 0, s>>>(S.xd, (float *)lambda, n);
        if (q > 0) k_cvt<double, float><<<1, kThreads, 0, s>>>(S.xd + n, (float *)coeffs, q);
        RBF_HIP(hipGetLastError());
    }
    RBF_HIP(hipStreamSynchronize(s));
    inf.iters = its;
    inf.restarts = restarts;
    inf.true_res = (bnorm > 0.0 && std::isfinite(best)) ? best : 0.0;
    if (bnorm == 0.0) inf.true_res = 0.0;
    inf.converged = inf.true_res <= rtol;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (info) *info = inf;
    return inf.converged ? RBF_OK : RBF_ENOCONV;
}

}  // namespace
}  // namespace rbf

extern "C" int rbf_interp_solve(rbf_plan *plan, const void *f, void *lambda, double rtol, const rbf_solve_opts *opts,
                                rbf_solve_info *info) {
    using namespace rbf;
    if (!plan || !f || !lambda) { set_error("rbf_interp_solve: null argument"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_interp_solve"));
    if (plan->kernel == RBF_THIN_PLATE || plan->kernel == RBF_R5) {
        set_error("rbf_interp_solve: the thin-plate spline and r^5 are conditionally positive definite; their "
                  "interpolation needs the polynomial terms of rbf_interp_solve_poly");
        return RBF_EUNSUPPORTED;
    }
    if (!(rtol > 0 && rtol < 1)) { set_error("rbf_interp_solve: rtol must lie in (0, 1)"); return RBF_EINVAL; }
    if (opts && (opts->restart < 0 || opts->restart > 1000)) { set_error("rbf_interp_solve: restart out of range"); return RBF_EINVAL; }
    if (opts && (opts->precond < RBF_PC_NONE || opts->precond > RBF_PC_LEARNED)) {
        set_error("rbf_interp_solve: unknown preconditioner %d", opts->precond);
        return RBF_EINVAL;
    }
    return solve_impl(plan, f, lambda, rtol, opts, info);
}

extern "C" int rbf_poly_terms(const rbf_plan *plan) {
    using namespace rbf;
    if (!plan) { set_error("rbf_poly_terms: null plan"); return RBF_EINVAL; }
    return poly_terms(plan->d, poly_degree(plan->kernel));
}

extern "C" int rbf_interp_solve_poly(rbf_plan *plan, const void *f, void *lambda, void *coeffs, double rtol,
                                     const rbf_solve_opts *opts, rbf_solve_info *info) {
    using namespace rbf;
    if (!plan || !f || !lambda) { set_error("rbf_interp_solve_poly: null argument"); return RBF_EINVAL; }
    RBF_TRY(reject_eval_plan(plan, "rbf_interp_solve_poly"));
    const int q = poly_terms(plan->d, poly_degree(plan->kernel));
    if (q > 0 && !coeffs) { set_error("rbf_interp_solve_poly: %d polynomial coefficients need a buffer", q); return RBF_EINVAL; }
    if (!(rtol > 0 && rtol < 1)) { set_error("rbf_interp_solve_poly: rtol must lie in (0, 1)"); return RBF_EINVAL; }
    if (opts && (opts->restart < 0 || opts->restart > 1000)) { set_error("rbf_interp_solve_poly: restart out of range"); return RBF_EINVAL; }
    if (opts && (opts->precond < RBF_PC_NONE || opts->precond > RBF_PC_LEARNED)) {
        set_error("rbf_interp_solve_poly: unknown preconditioner %d", opts->precond);
        return RBF_EINVAL;
    }
    if (q > 0 && opts && opts->precond != RBF_PC_NONE) {
        set_error("rbf_interp_solve_poly: augmented systems run without a preconditioner");
        return RBF_EUNSUPPORTED;
    }
    return solve_impl(plan, f, lambda, rtol, opts, info, q, coeffs);
}

// The fast product u = A lambda on the device (Zhao & Stoll, section 4, eq. 35-38, 54).
//
// eq. (37) factorises the quadrature kernel of a far pair through box centres,
//   Phi^Q(x_i - x_j) = sum_m w_m e^{i xi_m r_ia} C(xi_m) e^{i xi_m r_ab} e^{i xi_m r_bj}.
// All boxes here share one frequency grid, so the centre phases telescope and every
// expansion can be referred to the origin:
//   W_b(xi)  = sum_{j in b} lam_j e^{-i xi . x_j}                     (aggregation, P2M)
//   W_c(xi)  = sum_{leaves b in cell c} W_b(xi)                          (upward pass, M2M)
//   Lc_A(xi) = sum_{cells B within r of A} W_B(xi)                       (coarse translation)
//   L_a(xi)  = w(xi) C(xi) [Lc_{A(a)}(xi) - sum_{b in U(a)} W_b(xi)]    (leaf translation, L2L)
//   u_i     += sum_xi e^{i xi . x_i} L_a(xi)                            (disaggregation, L2P)
// which is eq. (38)'s far field over every kept pair outside the near list U(a); the
// near field (eq. 38 first term, eq. 54 sparse part including the diagonal) is summed
// directly.  lambda is real, so W(-xi) = conj W(xi): only nodes with xi_d > 0 are stored
// and the far field is 2 Re of the half sum.
//
// Expansion layout: [box][row][h], row = (m_1 .. m_{d-1}) with m_{d-1} fastest, h = m_d - Mn/2.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace rbf {
namespace {

constexpr int kThreads = 256;

template <class C> __device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc += a * b as four fused multiply-adds
template <class C> __device__ __forceinline__ void cmac(C &acc, const C a, const C b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

template <class T> struct KFun;

// Gaussian exp(-r^2/(2 s^2)): coef = -log2(e)/(2 s^2) for float (hardware exp2),
// -1/(2 s^2) for double.
template <> struct KFun<float> {
    static __device__ __forceinline__ float gauss(float r2, float coef) { return __builtin_amdgcn_exp2f(r2 * coef); }
    static __device__ __forceinline__ float mq(float r2, float c2) { return __builtin_amdgcn_sqrtf(r2 + c2); }
};
template <> struct KFun<double> {
    static __device__ __forceinline__ double gauss(double r2, double coef) { return exp(r2 * coef); }
    static __device__ __forceinline__ double mq(double r2, double c2) { return sqrt(r2 + c2); }
};

// ---- permutation --------------------------------------------------------------------
template <class T>
__global__ void k_gather(const T *__restrict__ lam, const int *__restrict__ perm, int64_t n, T *__restrict__ out) {
    int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) out[i] = lam[perm[i]];
}

// ---- near field (P2P) ---------------------------------------------------------------
constexpr int kTile = 256;

template <int D> struct Pad { static constexpr int v = (D + 2) & ~1; };

// One wave per task (up to 64 targets of one leaf); sources are the merged point ranges
// of the leaf's near list, staged through LDS in tiles of kTile points (x_1..x_d, lam).
template <class T, int D, int KER>
__global__ void __launch_bounds__(kWave) k_p2p(const T *__restrict__ xs, int64_t n, const T *__restrict__ lam_s,
                                               const int2 *__restrict__ tasks, const int *__restrict__ leaf_begin,
                                               const int *__restrict__ src_ptr, const int2 *__restrict__ src_rng,
                                               T coef, T *__restrict__ u_s) {
    constexpr int DP = Pad<D>::v;
    __shared__ T sdat[kTile * DP];
    __shared__ int rb[kTile], roff[kTile + 1];
    const int2 tk = tasks[xcd_swizzle(blockIdx.x, gridDim.x)];
    const int a = tk.x;
    const int t1 = leaf_begin[a + 1];
    const int ti = leaf_begin[a] + tk.y + threadIdx.x;
    const bool act = ti < t1;
    const int r0 = src_ptr[a], r1 = src_ptr[a + 1];
    T y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = act ? xs[k * n + ti] : T(0);
    T acc = 0;
    for (int rbase = r0; rbase < r1; rbase += kTile) {
        const int nr = min(kTile, r1 - rbase);
        __syncthreads();
        if (threadIdx.x == 0) {
            int o = 0;
            for (int q = 0; q < nr; ++q) {
                int2 g = src_rng[rbase + q];
                rb[q] = g.x;
                roff[q] = o;
                o += g.y - g.x;
            }
            roff[nr] = o;
        }
        __syncthreads();
        const int tot = roff[nr];
        for (int base = 0; base < tot; base += kTile) {
            const int cnt = min(kTile, tot - base);
            __syncthreads();
            for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
                int g = base + e;
                int q = 0;
                while (roff[q + 1] <= g) ++q;
                int j = rb[q] + (g - roff[q]);
#pragma unroll
                for (int k = 0; k < D; ++k) sdat[e * DP + k] = xs[k * n + j];
                sdat[e * DP + D] = lam_s[j];
            }
            __syncthreads();
            for (int e = 0; e < cnt; ++e) {
                T r2 = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    T t = y[k] - sdat[e * DP + k];
                    r2 += t * t;
                }
                T ph = (KER == RBF_GAUSSIAN) ? KFun<T>::gauss(r2, coef) : KFun<T>::mq(r2, coef);
                acc += sdat[e * DP + D] * ph;
            }
        }
    }
    if (act) u_s[ti] = acc;
}

// Exact product over all pairs (rows of targets per workgroup, all sources tiled).
template <class T, int D, int KER>
__global__ void __launch_bounds__(kThreads) k_direct(const T *__restrict__ xs, int64_t n, const T *__restrict__ lam_s,
                                                     T coef, const int *__restrict__ perm, T *__restrict__ u) {
    constexpr int DP = Pad<D>::v;
    __shared__ T sdat[kTile * DP];
    const int64_t ti = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    const bool act = ti < n;
    T y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = act ? xs[k * n + ti] : T(0);
    T acc = 0;
    for (int64_t base = 0; base < n; base += kTile) {
        const int cnt = (int)min((int64_t)kTile, n - base);
        __syncthreads();
        if (threadIdx.x < cnt) {
#pragma unroll
            for (int k = 0; k < D; ++k) sdat[threadIdx.x * DP + k] = xs[k * n + base + threadIdx.x];
            sdat[threadIdx.x * DP + D] = lam_s[base + threadIdx.x];
        }
        __syncthreads();
        for (int e = 0; e < cnt; ++e) {
            T r2 = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                T t = y[k] - sdat[e * DP + k];
                r2 += t * t;
            }
            T ph = (KER == RBF_GAUSSIAN) ? KFun<T>::gauss(r2, coef) : KFun<T>::mq(r2, coef);
            acc += sdat[e * DP + D] * ph;
        }
    }
    if (act) u[perm[ti]] = acc;
}

// ---- aggregation (P2M) -------------------------------------------------------------
// Last-dimension phases, weighted by lambda: dl[i][h] = lam_i e^{-i xi_{H+h} x_{i,d}} for
// h < H, zero up to HMAX (FP64 rotation recurrence from an FP64 phase, stored in T).
template <class T, int HMAX>
__global__ void k_phase_dl(const T *__restrict__ xlast, const T *__restrict__ lam_s, int64_t n, int H, double xiH,
                           double dxi, typename cplx<T>::type *__restrict__ dl) {
    using C = typename cplx<T>::type;
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i >= n) return;
    const double x = (double)xlast[i], l = (double)lam_s[i];
    double sb, cb, ss, cs;
    sincos(-xiH * x, &sb, &cb);
    sincos(-dxi * x, &ss, &cs);
    double er = l * cb, ei = l * sb;
    C *o = dl + i * HMAX;
#pragma unroll
    for (int h = 0; h < HMAX; ++h) {
        o[h] = (h < H) ? C{(T)er, (T)ei} : C{0, 0};
        double nr = er * cs - ei * ss;
        ei = er * ss + ei * cs;
        er = nr;
    }
}

// Workgroups (leaf, part): thread = one row (m_1..m_{d-1}) of the half grid, all HMAX
// last-dimension nodes in registers.  Per chunk of CH points the workgroup builds the
// per-thread factors e^{-i xi_m x_k} (k < d-1) in LDS; the lambda-weighted last-dimension
// phases of a point are uniform across the workgroup and come through scalar loads.
template <class T, int D, int HMAX>
__global__ void __launch_bounds__(kThreads) k_p2m(const T *__restrict__ xs, int64_t n,
                                                  const typename cplx<T>::type *__restrict__ dl,
                                                  const int *__restrict__ leaf_begin, int wpl, int mn, int H, int R,
                                                  int CH, double xi0, double dxi,
                                                  typename cplx<T>::type *__restrict__ W) {
    using C = typename cplx<T>::type;
    extern __shared__ char smem_raw[];
    C *tab = reinterpret_cast<C *>(smem_raw);
    constexpr int DM = D > 1 ? D - 1 : 1;
    const int ST = DM * mn;
    const int bid = xcd_swizzle(blockIdx.x, gridDim.x);
    const int a = bid / wpl, part = bid % wpl;
    const int t0 = leaf_begin[a], t1 = leaf_begin[a + 1];
    const int row = part * blockDim.x + threadIdx.x;
    const bool act = row < R;
    int md[DM];
    {
        int rr = act ? row : 0;
        for (int k = D - 2; k >= 0; --k) { md[k] = rr % mn; rr /= mn; }
    }
    C acc[HMAX];
#pragma unroll
    for (int h = 0; h < HMAX; ++h) acc[h] = C{0, 0};
    for (int c0 = t0; c0 < t1; c0 += CH) {
        const int cn = min(CH, t1 - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn * DM; t += blockDim.x) {
            const int j = t / DM, k = t % DM;
            C *dst = tab + j * ST + k * mn;
            const double x = (double)xs[k * n + c0 + j];
            double sb, cb, ss, cs;
            sincos(-dxi * x, &ss, &cs);
            sincos(-xi0 * x, &sb, &cb);
            double er = cb, ei = sb;
            for (int m = 0; m < mn; ++m) {
                dst[m] = C{(T)er, (T)ei};
                double nr = er * cs - ei * ss;
                ei = er * ss + ei * cs;
                er = nr;
            }
        }
        __syncthreads();
        if constexpr (sizeof(T) == 4) {
            // prefetch the next point's uniform operands while the current one is used
            C cur[HMAX], nxt[HMAX];
            const C *d0 = dl + (int64_t)c0 * HMAX;
#pragma unroll
            for (int h = 0; h < HMAX; ++h) cur[h] = d0[h];
            for (int j = 0; j < cn; ++j) {
                const C *dn = dl + (int64_t)(c0 + min(j + 1, cn - 1)) * HMAX;
#pragma unroll
                for (int h = 0; h < HMAX; ++h) nxt[h] = dn[h];
                const C *pt = tab + j * ST;
                C kv = pt[md[0]];
#pragma unroll
                for (int k = 1; k < D - 1; ++k) kv = cmul(kv, pt[k * mn + md[k]]);
#pragma unroll
                for (int h = 0; h < HMAX; ++h) cmac(acc[h], kv, cur[h]);
#pragma unroll
                for (int h = 0; h < HMAX; ++h) cur[h] = nxt[h];
            }
        } else {
            for (int j = 0; j < cn; ++j) {
                const C *pt = tab + j * ST;
                C kv = pt[md[0]];
#pragma unroll
                for (int k = 1; k < D - 1; ++k) kv = cmul(kv, pt[k * mn + md[k]]);
                const C *dj = dl + (int64_t)(c0 + j) * HMAX;
#pragma unroll
                for (int h = 0; h < HMAX; ++h) cmac(acc[h], kv, dj[h]);
            }
        }
    }
    if (act) {
        C *out = W + (int64_t)a * R * H + (int64_t)row * H;
#pragma unroll
        for (int h = 0; h < HMAX; ++h)
            if (h < H) out[h] = acc[h];
    }
}

// ---- upward pass: coarse cell = sum of its leaves ------------------------------------
template <class C>
__global__ void k_m2m(const C *__restrict__ W, const int *__restrict__ cell_begin, int64_t P, C *__restrict__ Wc) {
    const int64_t c = blockIdx.x;
    const int64_t p = blockIdx.y * (int64_t)kThreads + threadIdx.x;
    if (p >= P) return;
    const int a0 = cell_begin[c], a1 = cell_begin[c + 1];
    C s{0, 0};
    for (int a = a0; a < a1; ++a) {
        C v = W[(int64_t)a * P + p];
        s.x += v.x;
        s.y += v.y;
    }
    Wc[c * P + p] = s;
}

// ---- coarse translation: box sum of radius r along one axis of the dense grid ---------
template <class C, int D>
__global__ void k_m2l_axis(const C *__restrict__ in, int64_t P, int lc, int r, int axis, C *__restrict__ out) {
    const int64_t c = blockIdx.x;
    const int64_t p = blockIdx.y * (int64_t)kThreads + threadIdx.x;
    if (p >= P) return;
    int64_t cc[D];
#pragma unroll
    for (int k = 0; k < D; ++k) cc[k] = 0;
    for (int b = 0; b < lc; ++b)
#pragma unroll
        for (int k = 0; k < D; ++k) cc[k] |= (int64_t)((c >> (b * D + k)) & 1) << b;
    const int64_t side = (int64_t)1 << lc;
    const int64_t lo = max((int64_t)0, cc[axis] - r), hi = min(side - 1, cc[axis] + r);
    const int64_t base = c & ~(int64_t)0;
    // Morton index with the axis coordinate replaced: clear that axis' bits, then insert.
    int64_t mask = 0;
    for (int b = 0; b < lc; ++b) mask |= (int64_t)1 << (b * D + axis);
    const int64_t rest = base & ~mask;
    C s{0, 0};
    for (int64_t v = lo; v <= hi; ++v) {
        int64_t ins = 0;
        for (int b = 0; b < lc; ++b) ins |= ((v >> b) & 1) << (b * D + axis);
        C x = in[(rest | ins) * P + p];
        s.x += x.x;
        s.y += x.y;
    }
    out[c * P + p] = s;
}

// ---- leaf translation + downward pass --------------------------------------------------
// Output rows are padded to HMAX entries (zeros beyond H) so that the disaggregation
// can load a whole row unconditionally.
template <class T, int D>
__global__ void k_m2l_leaf(const typename cplx<T>::type *__restrict__ W, const typename cplx<T>::type *__restrict__ Lc,
                           const int *__restrict__ leaf_cell, const int *__restrict__ near_ptr,
                           const int *__restrict__ near_idx, const double *__restrict__ wc1, int mn, int H,
                           int HP, int64_t P, typename cplx<T>::type *__restrict__ L) {
    using C = typename cplx<T>::type;
    const int a = blockIdx.x;
    const int64_t q = blockIdx.y * (int64_t)kThreads + threadIdx.x;   // padded index
    const int64_t RP = P / H * HP;
    if (q >= RP) return;
    const int64_t rowq = q / HP;
    const int h = (int)(q % HP);
    if (h >= H) {
        L[(int64_t)a * RP + q] = C{0, 0};
        return;
    }
    const int64_t p = rowq * H + h;
    // separable weight w C(xi) = prod_k wc1[m_k]
    int64_t rest = rowq;
    double f = wc1[H + h];
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
        f *= wc1[rest % mn];
        rest /= mn;
    }
    C s = Lc[(int64_t)leaf_cell[a] * P + p];
    const int e0 = near_ptr[a], e1 = near_ptr[a + 1];
    for (int e = e0; e < e1; ++e) {
        C v = W[(int64_t)near_idx[e] * P + p];
        s.x -= v.x;
        s.y -= v.y;
    }
    L[(int64_t)a * RP + q] = C{(T)(f * s.x), (T)(f * s.y)};
}

// ---- disaggregation (L2P) + combine ---------------------------------------------------
// One wave per task (up to 64 target points of one leaf), one lane per target.  The lane
// keeps e^{+i xi_{H+h} x_d} for all h in registers and walks the rows with an FP64
// odometer recurrence for the other factors; the leaf's L rows (padded to HMAX) are
// uniform across the wave and come through scalar loads.
template <class T, int D, int HMAX>
__global__ void __launch_bounds__(kWave) k_l2p(const T *__restrict__ xs, int64_t n, const int2 *__restrict__ tasks,
                                               const int *__restrict__ leaf_begin,
                                               const typename cplx<T>::type *__restrict__ L, int mn, int H, int R,
                                               double xi0, double xiH, double dxi, const T *__restrict__ u_near,
                                               const int *__restrict__ perm, T *__restrict__ u) {
    using C = typename cplx<T>::type;
    constexpr int DM = D > 1 ? D - 1 : 1;
    const int2 tk = tasks[xcd_swizzle(blockIdx.x, gridDim.x)];
    const int a = tk.x;
    const int t1 = leaf_begin[a + 1];
    const int ti = leaf_begin[a] + tk.y + threadIdx.x;
    const bool act = ti < t1;
    const int tj = act ? ti : t1 - 1;
    const C *La = L + (int64_t)a * R * HMAX;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = (double)xs[k * n + tj];
    C e[HMAX];
    {
        double sb, cb, ss, cs;
        sincos(xiH * x[D - 1], &sb, &cb);
        sincos(dxi * x[D - 1], &ss, &cs);
        double er = cb, ei = sb;
#pragma unroll
        for (int h = 0; h < HMAX; ++h) {
            e[h] = C{(T)er, (T)ei};
            double nr = er * cs - ei * ss;
            ei = er * ss + ei * cs;
            er = nr;
        }
    }
    double br[DM], bi[DM], sr[DM], si[DM], cr[DM], ci[DM];
    int dig[DM];
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
        sincos(xi0 * x[k], &bi[k], &br[k]);
        sincos(dxi * x[k], &si[k], &sr[k]);
        cr[k] = br[k];
        ci[k] = bi[k];
        dig[k] = 0;
    }
    T acc = 0;
    for (int row = 0; row < R; ++row) {
        const C *lr = La + (int64_t)row * HMAX;
        C g{0, 0};
#pragma unroll
        for (int h = 0; h < HMAX; ++h) cmac(g, lr[h], e[h]);
        const T gr = g.x, gi = g.y;
        double kr = cr[0], ki = ci[0];
#pragma unroll
        for (int k = 1; k < D - 1; ++k) {
            double t = kr * cr[k] - ki * ci[k];
            ki = kr * ci[k] + ki * cr[k];
            kr = t;
        }
        acc = fma((T)kr, gr, acc);
        acc = fma(-(T)ki, gi, acc);
        // odometer: advance the fastest digit (k = d-2), carry towards k = 0
        for (int k = D - 2; k >= 0; --k) {
            if (++dig[k] < mn) {
                double t = cr[k] * sr[k] - ci[k] * si[k];
                ci[k] = cr[k] * si[k] + ci[k] * sr[k];
                cr[k] = t;
                break;
            }
            dig[k] = 0;
            cr[k] = br[k];
            ci[k] = bi[k];
        }
    }
    if (act) u[perm[ti]] = u_near[ti] + T(2) * acc;
}

template <class T> T kernel_coef(int kernel, double shape) {
    if (kernel == RBF_GAUSSIAN) {
        if (sizeof(T) == 4) return (T)(-1.4426950408889634 / (2.0 * shape * shape));
        return (T)(-1.0 / (2.0 * shape * shape));
    }
    return (T)(shape * shape);
}

struct PhaseTimer {
    rbf_plan *p;
    int ph = -1;
    explicit PhaseTimer(rbf_plan *pp) : p(pp) {}
    hipError_t begin(int k) {
        ph = k;
        return p->profiling ? hipEventRecord(p->ev[2 * k], p->stream) : hipSuccess;
    }
    hipError_t end() { return p->profiling ? hipEventRecord(p->ev[2 * ph + 1], p->stream) : hipSuccess; }
};

template <class T, int D, int HMAX>
int far_field(rbf_plan *p, PhaseTimer &pt) {
    using C = typename cplx<T>::type;
    hipStream_t s = p->stream;
    const int mn = p->mn, H = p->H, R = (int)p->R;
    const int64_t P = p->P;
    const double dxi = 2.0 * p->sigma / (mn - 1);
    const double xi0 = -p->sigma, xiH = -p->sigma + H * dxi;
    // P2M
    RBF_HIP(pt.begin(2));
    {
        const T *xlast = (const T *)p->xs + (int64_t)(p->d - 1) * p->n;
        k_phase_dl<T, HMAX><<<(unsigned)((p->n + kThreads - 1) / kThreads), kThreads, 0, s>>>(
            xlast, (const T *)p->lam_s, p->n, H, xiH, dxi, (C *)p->dl);
        RBF_HIP(hipGetLastError());
        int wpl = (R + kThreads - 1) / kThreads;
        int rows = (R + wpl - 1) / wpl;
        int bd = std::min(kThreads, ((rows + kWave - 1) / kWave) * kWave);
        // point chunk sized so the LDS tables stay within 32 KB
        const size_t per_point = sizeof(C) * (size_t)((D > 1 ? D - 1 : 1) * mn);
        int CH = (int)std::max<size_t>(4, std::min<size_t>(64, (32 * 1024) / per_point));
        size_t sh = per_point * CH;
        k_p2m<T, D, HMAX><<<p->nleaves * wpl, bd, sh, s>>>((const T *)p->xs, p->n, (const C *)p->dl, p->leaf_begin,
                                                           wpl, mn, H, R, CH, xi0, dxi, (C *)p->W);
        RBF_HIP(hipGetLastError());
    }
    RBF_HIP(pt.end());
    // M2M
    RBF_HIP(pt.begin(3));
    dim3 gp((unsigned)p->ncells, (unsigned)((P + kThreads - 1) / kThreads));
    k_m2m<C><<<gp, kThreads, 0, s>>>((const C *)p->W, p->cell_leaf_begin, P, (C *)p->Wc);
    RBF_HIP(hipGetLastError());
    RBF_HIP(pt.end());
    // coarse stencil, one axis at a time: Wc -> Tmp -> Wc -> ... -> Lc
    RBF_HIP(pt.begin(4));
    if (p->lc == 0 || p->r == 0) {
        RBF_HIP(hipMemcpyAsync(p->Lc, p->Wc, sizeof(C) * P * p->ncells, hipMemcpyDeviceToDevice, s));
    } else {
        C *src = (C *)p->Wc;
        for (int ax = 0; ax < D; ++ax) {
            C *dst = (ax == D - 1) ? (C *)p->Lc : ((ax % 2 == 0) ? (C *)p->Tmp : (C *)p->Wc);
            k_m2l_axis<C, D><<<gp, kThreads, 0, s>>>(src, P, p->lc, p->r, ax, dst);
            RBF_HIP(hipGetLastError());
            src = dst;
        }
    }
    RBF_HIP(pt.end());
    // leaf translation (output rows padded to HMAX)
    RBF_HIP(pt.begin(5));
    {
        const int64_t RP = (int64_t)R * HMAX;
        dim3 gl((unsigned)p->nleaves, (unsigned)((RP + kThreads - 1) / kThreads));
        k_m2l_leaf<T, D><<<gl, kThreads, 0, s>>>((const C *)p->W, (const C *)p->Lc, p->leaf_cell, p->near_ptr,
                                                 p->near_idx, p->wc1, mn, H, HMAX, P, (C *)p->Lx);
        RBF_HIP(hipGetLastError());
    }
    RBF_HIP(pt.end());
    return RBF_OK;
}

template <class T, int D, int HMAX>
int l2p(rbf_plan *p, T *u, PhaseTimer &pt) {
    using C = typename cplx<T>::type;
    const int mn = p->mn, H = p->H, R = (int)p->R;
    const double dxi = 2.0 * p->sigma / (mn - 1);
    const double xi0 = -p->sigma, xiH = -p->sigma + H * dxi;
    RBF_HIP(pt.begin(6));
    k_l2p<T, D, HMAX><<<p->ntasks, kWave, 0, p->stream>>>((const T *)p->xs, p->n, p->tasks, p->leaf_begin,
                                                          (const C *)p->Lx, mn, H, R, xi0, xiH, dxi,
                                                          (const T *)p->u_s, p->perm, u);
    RBF_HIP(hipGetLastError());
    RBF_HIP(pt.end());
    return RBF_OK;
}

template <class T, int D>
int matvec_d(rbf_plan *p, const T *lam, T *u, PhaseTimer &pt) {
    hipStream_t s = p->stream;
    const int64_t n = p->n;
    RBF_HIP(pt.begin(0));
    k_gather<T><<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(lam, p->perm, n, (T *)p->lam_s);
    RBF_HIP(hipGetLastError());
    RBF_HIP(pt.end());
    RBF_HIP(pt.begin(1));
    const T coef = kernel_coef<T>(p->kernel, p->shape);
    if (p->kernel == RBF_GAUSSIAN)
        k_p2p<T, D, RBF_GAUSSIAN><<<p->ntasks, kWave, 0, s>>>((const T *)p->xs, n, (const T *)p->lam_s, p->tasks,
                                                              p->leaf_begin, p->src_ptr, p->src_rng, coef,
                                                              (T *)p->u_s);
    else
        k_p2p<T, D, RBF_MULTIQUADRIC><<<p->ntasks, kWave, 0, s>>>((const T *)p->xs, n, (const T *)p->lam_s,
                                                                  p->tasks, p->leaf_begin, p->src_ptr, p->src_rng,
                                                                  coef, (T *)p->u_s);
    RBF_HIP(hipGetLastError());
    RBF_HIP(pt.end());
#define FAR(HM)                                         \
    do {                                                \
        RBF_TRY((far_field<T, D, HM>(p, pt)));          \
        RBF_TRY((l2p<T, D, HM>(p, u, pt)));             \
    } while (0)
    switch (p->HP) {
        case 4: FAR(4); break;
        case 6: FAR(6); break;
        case 8: FAR(8); break;
        case 10: FAR(10); break;
        case 12: FAR(12); break;
#define BIGH(V) case V: if constexpr (D < 5) { FAR(V); break; } else { set_error("half grid %d not compiled for d=5", V); return RBF_EUNSUPPORTED; }
        BIGH(14)
        BIGH(16)
        BIGH(20)
        BIGH(24)
        BIGH(28)
        BIGH(32)
#undef BIGH
        default: set_error("padded half grid %d not compiled", p->HP); return RBF_EUNSUPPORTED;
    }
#undef FAR
    return RBF_OK;
}

template <class T>
int matvec_t(rbf_plan *p, const void *lam, void *u) {
    PhaseTimer pt(p);
    int rc;
    switch (p->d) {
        case 2: rc = matvec_d<T, 2>(p, (const T *)lam, (T *)u, pt); break;
        case 3: rc = matvec_d<T, 3>(p, (const T *)lam, (T *)u, pt); break;
        case 5: rc = matvec_d<T, 5>(p, (const T *)lam, (T *)u, pt); break;
        default: set_error("dimension %d not compiled", p->d); return RBF_EUNSUPPORTED;
    }
    if (rc != RBF_OK) return rc;
    if (p->profiling) {
        RBF_HIP(hipEventSynchronize(p->ev[2 * RBF_NPHASES - 1]));
        for (int k = 0; k < RBF_NPHASES; ++k) {
            float ms = 0.f;
            RBF_HIP(hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]));
            p->phase_ms[k] += ms;
        }
        p->prof_calls += 1;
    }
    return RBF_OK;
}

template <class T, int D>
int direct_d(rbf_plan *p, const T *lam, T *u) {
    hipStream_t s = p->stream;
    const int64_t n = p->n;
    unsigned nb = (unsigned)((n + kThreads - 1) / kThreads);
    k_gather<T><<<nb, kThreads, 0, s>>>(lam, p->perm, n, (T *)p->lam_s);
    RBF_HIP(hipGetLastError());
    const T coef = kernel_coef<T>(p->kernel, p->shape);
    if (p->kernel == RBF_GAUSSIAN)
        k_direct<T, D, RBF_GAUSSIAN><<<nb, kThreads, 0, s>>>((const T *)p->xs, n, (const T *)p->lam_s, coef, p->perm, u);
    else
        k_direct<T, D, RBF_MULTIQUADRIC><<<nb, kThreads, 0, s>>>((const T *)p->xs, n, (const T *)p->lam_s, coef,
                                                                 p->perm, u);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

template <class T>
int direct_t(rbf_plan *p, const void *lam, void *u) {
    switch (p->d) {
        case 2: return direct_d<T, 2>(p, (const T *)lam, (T *)u);
        case 3: return direct_d<T, 3>(p, (const T *)lam, (T *)u);
        case 5: return direct_d<T, 5>(p, (const T *)lam, (T *)u);
    }
    set_error("dimension %d not compiled", p->d);
    return RBF_EUNSUPPORTED;
}

}  // namespace

int launch_matvec(rbf_plan *p, const void *lambda, void *u) {
    return p->dtype == RBF_F32 ? matvec_t<float>(p, lambda, u) : matvec_t<double>(p, lambda, u);
}

int launch_direct(rbf_plan *p, const void *lambda, void *u) {
    return p->dtype == RBF_F32 ? direct_t<float>(p, lambda, u) : direct_t<double>(p, lambda, u);
}

}  // namespace rbf

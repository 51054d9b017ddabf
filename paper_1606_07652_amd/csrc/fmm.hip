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
//
// Every kernel body is a device function over a per-problem descriptor (Desc) and a
// problem-local block id.  A single plan launches one grid per phase; a batch of plans
// launches one grid per phase for all its problems, each block finding its problem by a
// binary search over the per-problem block counts.
#include <algorithm>
#include <cmath>
#include <functional>

#include "fmm_desc.h"
#include "internal.h"

namespace rbf {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 256;

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

// ---- matrix cores ---------------------------------------------------------------------
// 16x16x4 MFMA with one K element per lane: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and accumulates four C values whose rows depend on the instruction.
typedef double mfd4 __attribute__((ext_vector_type(4)));
typedef float mff4 __attribute__((ext_vector_type(4)));
template <class T> struct Mfma;
template <> struct Mfma<double> {
    using V = mfd4;
    static __device__ __forceinline__ V mac(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lane) { return 4 * q + (lane >> 4); }   // C[row][lane % 16]
};
template <> struct Mfma<float> {
    using V = mff4;
    static __device__ __forceinline__ V mac(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lane) { return 4 * (lane >> 4) + q; }
};

// Row digits (m_0 .. m_{d-2}, fastest last) of an expansion row r < 2^22, dividing by mn
// with a multiply-high (exact in that range for every mn up to 128).
template <int DM>
__device__ __forceinline__ void row_digits(unsigned r, int mn, unsigned magic, int (&md)[DM]) {
#pragma unroll
    for (int k = DM - 1; k >= 0; --k) {
        const unsigned q = __umulhi(r, magic);
        md[k] = (int)(r - q * (unsigned)mn);
        r = q;
    }
}

// Aggregation geometry: row tiles of 16 per wave and rows per workgroup of four waves.
__host__ __device__ constexpr int p2m_rtiles(int dim) { return dim > 2 ? 4 : 1; }
__host__ __device__ constexpr int p2m_rows(int dim) { return 4 * 16 * p2m_rtiles(dim); }
// Disaggregation: targets per workgroup; a 64-target task is split over 64 / NT workgroups.
// FP32 takes whole tasks (64) where their phase tables fit in 96 KiB of LDS: each loaded row
// tile then feeds four target tiles.  FP64 takes 32 (its A fragments for 64 targets would
// leave two waves per SIMD), or 16 where the tables of 32 targets exceed 64 KiB.
__host__ __device__ constexpr size_t l2p_lds(int csize, int dim, int hmax, int nt) {
    return (size_t)csize * nt * (hmax + (dim - 1) * 2 * hmax) + (size_t)(csize / 2) * 4 * nt;
}
__host__ __device__ constexpr int l2p_targets(int csize, int dim, int hmax) {
    return (csize == 8 && l2p_lds(csize, dim, hmax, 64) <= 98304) ? 64
           : l2p_lds(csize, dim, hmax, 32) <= 65536               ? 32
                                                                   : 16;
}

template <class T> struct KFun;

// 2^t in FP64 by the table-driven reduction of P. T. P. Tang (ACM TOMS 15(2), 1989), for the
// near field and the direct sum: with s = 256 t rounded to the integer q = 256 k + j
// (0 <= j < 256) and u = s - q (exact, |u| <= 1/2), 2^t = 2^k 2^(j/256) 2^(u/256); tab holds
// 2^(j/256) and 2^(u/256) comes from its degree-4 Taylor polynomial, coefficients
// (ln 2 / 256)^n / n! (truncation below 4e-17 relative).  The argument is s = 256 t; very
// negative s underflows to 0 in the scaling.
constexpr int kExpBits = 8, kExpTab = 1 << kExpBits;
constexpr double exp2_tab_taylor(int n) {
    double c = 1.0;
    for (int k = 1; k <= n; ++k) c *= 0.693147180559945309417232121458176568 / kExpTab / k;
    return c;
}
__device__ __forceinline__ double exp2_tab(double s, const double *tab) {
    const double qd = rint(s);
    const double u = s - qd;
    const int q = (int)qd;   // saturates; a saturated q gives 2^(huge negative) = 0
    double p = exp2_tab_taylor(4);
    p = fma(p, u, exp2_tab_taylor(3));
    p = fma(p, u, exp2_tab_taylor(2));
    p = fma(p, u, exp2_tab_taylor(1));
    p = fma(p, u, 1.0);
    return ldexp(p * tab[q & (kExpTab - 1)], q >> kExpBits);   // q >> 8 = floor(q / 256)
}

// Natural logarithm of a positive normal a by the table-driven method of P. T. P. Tang (ACM TOMS
// 16(4), 1990): a = 2^e m with m in [1, 2); c = 1 + j/256 the table point at or below m (j the top
// eight fraction bits); r = (m - c) / c through the tabulated 1/c (m - c is exact), |r| < 2^-8;
// log a = e ln 2 + log c + log1p(r) with log1p(r) from its Taylor polynomial of degree 6
// (truncation below 2^-56 / 7).  tab holds log(1 + j/256) then 1 / (1 + j/256).
constexpr int kLogBits = 8, kLogTab = 1 << kLogBits;
__device__ __forceinline__ double log_tab(double a, const double *tab) {
    int e;
    const double m = 2.0 * frexp(a, &e);   // a = m 2^(e - 1), m in [1, 2)
    const int j = (int)((m - 1.0) * kLogTab);
    const double c = 1.0 + j * (1.0 / kLogTab);
    const double r = (m - c) * tab[kLogTab + j];
    double p = fma(r, -1.0 / 6.0, 1.0 / 5.0);
    p = fma(p, r, -0.25);
    p = fma(p, r, 1.0 / 3.0);
    p = fma(p, r, -0.5);
    p = fma(p, r, 1.0);
    return fma((double)(e - 1), 0.693147180559945309417232121458176568, fma(p, r, tab[j]));
}

// Gaussian exp(-r^2/(2 s^2)) = 2^(r^2 coef), coef = -log2(e)/(2 s^2): hardware exp2 in FP32 (in
// FP64 the kernels call exp2_tab with its LDS table).  Multiquadric sqrt(r^2 + c^2) and inverse
// multiquadric 1/sqrt(r^2 + c^2): coef = c^2.  Wendland's (1 - e r)_+^3 (3 e r + 1) (section 5):
// coef = e, zero from r = 1/e on.  The thin-plate spline r^2 log r = r^2 log(r^2) / 2 (0 at
// r = 0) and r^5 have no shape.
template <> struct KFun<float> {
    static __device__ __forceinline__ float gauss(float r2, float coef) { return __builtin_amdgcn_exp2f(r2 * coef); }
    static __device__ __forceinline__ float mq(float r2, float c2) { return __builtin_amdgcn_sqrtf(r2 + c2); }
    static __device__ __forceinline__ float imq(float r2, float c2) { return __builtin_amdgcn_rsqf(r2 + c2); }
    static __device__ __forceinline__ float wendland(float r2, float e) {
        const float er = e * __builtin_amdgcn_sqrtf(r2);
        const float t = fmaxf(1.0f - er, 0.0f);
        return t * t * t * fmaf(3.0f, er, 1.0f);
    }
    static __device__ __forceinline__ float thin_plate(float r2) { return r2 > 0.0f ? 0.5f * r2 * logf(r2) : 0.0f; }
    static __device__ __forceinline__ float r5(float r2) { return r2 * r2 * __builtin_amdgcn_sqrtf(r2); }
};
// Square root of a squared distance (0 <= a, far above the subnormal range) without the
// library's range scaling: Goldschmidt's iteration from the hardware reciprocal square root,
// y ~ 1/sqrt(a), g = a y, h = y/2, one multiplicative step and two additive corrections
// g += (a - g^2) h; a = 0 gives 0.
__device__ __forceinline__ double sqrt_dist2(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double e = fma(-g, g, a);
    g = fma(e, h, g);
    e = fma(-g, g, a);
    g = fma(e, h, g);
    return a > 0.0 ? g : 0.0;
}

// 1/sqrt(a) for a positive normal a: two Newton steps y += y (1 - a y^2) / 2 from the hardware
// reciprocal square root (each step squares the relative error).
__device__ __forceinline__ double rsqrt_pos(double a) {
    double y = __builtin_amdgcn_rsq(a);
    double e = fma(-a * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-a * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

template <> struct KFun<double> {
    static __device__ __forceinline__ double mq(double r2, double c2) {
        const double a = r2 + c2;
        return a * rsqrt_pos(a);
    }
    static __device__ __forceinline__ double imq(double r2, double c2) { return rsqrt_pos(r2 + c2); }
    static __device__ __forceinline__ double wendland(double r2, double e) {
        const double er = e * sqrt_dist2(r2);
        const double t = fmax(1.0 - er, 0.0);
        return t * t * t * fma(3.0, er, 1.0);
    }
    static __device__ __forceinline__ double thin_plate(double r2) { return r2 > 0.0 ? 0.5 * r2 * log(r2) : 0.0; }
    static __device__ __forceinline__ double r5(double r2) { return r2 * r2 * sqrt_dist2(r2); }
};

template <int D> struct Pad { static constexpr int v = (D + 2) & ~1; };

// Read-only view for operands that are uniform across a wave and not written by the
// kernel: the constant address space lets the compiler fetch them with scalar loads.
template <class T> using cptr = const __attribute__((address_space(4))) T *;
// complex element i of a read-only array of (re, im) pairs
template <class T> struct CView {
    cptr<T> p;
    __device__ __forceinline__ typename cplx<T>::type operator[](int64_t i) const {
        return typename cplx<T>::type{p[2 * i], p[2 * i + 1]};
    }
    __device__ __forceinline__ CView operator+(int64_t o) const { return CView{p + 2 * o}; }
};
// The base address is made explicitly wave-uniform (readfirstlane), so that element
// addresses built from it and from uniform loop counters stay in scalar registers.
template <class T> __device__ __forceinline__ CView<T> as_const(const typename cplx<T>::type *q) {
    const uint64_t a = (uint64_t)q;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return CView<T>{(cptr<T>)(const T *)(((uint64_t)hi << 32) | lo)};
}

// A wave-uniform read-only int array, read with scalar loads.
__device__ __forceinline__ cptr<int> uconst(const int *q) {
    const uint64_t a = (uint64_t)q;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return (cptr<int>)(const int *)(((uint64_t)hi << 32) | lo);
}

// A per-problem descriptor read through the constant address space (see resolve()).
template <class T> using DescC = const __attribute__((address_space(4))) Desc<T>;

// ---- bodies --------------------------------------------------------------------------

// permutation of the coefficients into Morton order
template <class T>
__device__ __forceinline__ void gather_body(DescC<T> &d, const T *__restrict__ lam, int bid) {
    int64_t i = bid * (int64_t)kThreads + threadIdx.x;
    if (i < d.n) d.lam_s[i] = lam[d.off + d.perm[i]];
    if (bid == 0 && threadIdx.x < kXcds && d.p2p_ctr) d.p2p_ctr[threadIdx.x * kCtrStride] = 0;   // queue reset
}

// Near field (P2P): one wave per task, a chunk of up to 64 targets of one leaf.  The
// sources are the merged point ranges of the leaf's near list.
//  * G = 1 (one target per lane): the wave walks the ranges in order in steps of kP2pStep
//    points read with scalar loads, so every source coordinate and weight is an SGPR operand
//    shared by the 64 lanes (no LDS staging, no barrier); a range's last partial step
//    repeats its last point with weight 0.
//  * G = 2, 4, 8 (a leaf's last chunk of at most 64 / G targets): the lanes form G groups of
//    64 / G, one target per lane of a group; group g takes the sources j with j - j0 = g mod G
//    of each range [j0, j1), read with per-lane vector loads, and the G partial sums of a
//    target are added over the groups at the end.  A leaf of 80 points then costs one full
//    wave and a quarter wave of source steps instead of two full waves.
template <class T> constexpr int kP2pStep = sizeof(T) == 8 ? 4 : 8;

// The FP64 Gaussian of the near field goes through exp2_tab (coef then carries the factor 256
// and tab the 256 table entries in LDS); other kernels and FP32 through KFun.
template <class T, int KER> constexpr bool kTabExp = KER == RBF_GAUSSIAN && sizeof(T) == 8;
// The FP64 thin-plate spline goes through log_tab (tab: its two tables of 256 entries).
template <class T, int KER> constexpr bool kTabLog = KER == RBF_THIN_PLATE && sizeof(T) == 8;
// The residual kernel of a banded plan reads its polynomial pieces from tab.
template <int KER> constexpr bool kRes = KER == kResTab || KER == kResTabDiv || KER == kResTabQ;
// residual pieces in LDS: kResStride entries per piece (its coefficients, unpadded), a piece of
// zeros after the last (b >= bmax, where the residual is negligible, lands on it), then 3
// parameters; FP32 products hold them as floats.  Unpadded FP64 pieces are 48 bytes apart, so
// the pieces of 8 consecutive indices start on 8 different groups of 4 banks; 64-byte pieces
// start on only 2, and the random per-lane piece reads measured six times the bank conflicts
constexpr int kResStride = kResDegree + 1;
constexpr int kResLds = (kResIntervals + 1) * kResStride + 4;
template <class T, int KER>
constexpr int kTabLen = KER == RBF_GAUSSIAN_BANDLIMITED ? 1   // its table stays in global memory
                        : kTabLog<T, KER> ? 2 * kLogTab
                        : kRes<KER>     ? (sizeof(T) == 8 ? kResLds : (kResLds + 1) / 2)
                                        : kExpTab;
// fills the LDS table of the kernel (stride: the workgroup size); a barrier must follow
template <class T, int KER> __device__ __forceinline__ void fill_tab(double *tab, int stride) {
    if constexpr (kTabExp<T, KER>) {
        for (int j = threadIdx.x; j < kExpTab; j += stride) tab[j] = exp2((double)j / kExpTab);
    } else if constexpr (kTabLog<T, KER>) {
        for (int j = threadIdx.x; j < kLogTab; j += stride) {
            tab[j] = log1p((double)j / kLogTab);
            tab[kLogTab + j] = 1.0 / (1.0 + (double)j / kLogTab);
        }
    }
}

// Residual of the scale split of the multiquadric kernels (every Gaussian width below s0) at
// squared distance r2.  Tables in b (kResTab, kResTabDiv): with b = sqrt(r2 + c^2), piece
// i = floor((b - c) inv) (the zero piece from b = bmax on, i.e. from r2 = qmax on), a polynomial
// of degree kResDegree in v = (b - c) inv - i; the inverse multiquadric's table holds b times the
// residual.  Table in q = r2 + c^2 (kResTabQ), where the plan's fit meets its accuracy: pieces
// uniform in q, which are coarse in b near b = c when the near zone is wide.
template <class T, int KER> __device__ __forceinline__ T kres(T r2, T c2, const double *tab_raw) {
    const T *tab = reinterpret_cast<const T *>(tab_raw);        // entries in the product's precision
    constexpr int kP = (kResIntervals + 1) * kResStride;         // parameters after the pieces
    if constexpr (KER == kResTabQ) {
        // pieces uniform in q = r2 + c^2 from c^2: piece floor(r2 inv), no square root and no
        // division (the table holds the residual of either kernel itself)
        const T s = min(r2 * tab[kP], (T)kResIntervals);          // r2 >= 0; NaN: the zero piece
        const int i = (int)s;
        const T v = s - (T)i;
        const T *c = tab + i * kResStride;
        T y = c[kResDegree];
#pragma unroll
        for (int k = kResDegree - 1; k >= 0; --k) y = fma(y, v, c[k]);
        return y;
    }
    // 1/b from the hardware reciprocal square root (relative error 5e-8 in FP64, measured; one
    // Newton step: 4e-15), b = q / sqrt q; the inverse multiquadric's division is a product
    const T q = r2 + c2;
    T rb;
    if constexpr (sizeof(T) == 8) {
        rb = __builtin_amdgcn_rsq(q);
        rb = rb * fma(T(-0.5) * q * rb, rb, T(1.5));
    } else {
        rb = __builtin_amdgcn_rsqf(q);
    }
    const T b = q * rb;
    const T s = (b - tab[kP + 2]) * tab[kP];
    const int i = max(0, min((int)s, kResIntervals));
    const T v = s - (T)i;
    const T *c = tab + i * kResStride;
    T y = c[kResDegree];
#pragma unroll
    for (int k = kResDegree - 1; k >= 0; --k) y = fma(y, v, c[k]);
    if constexpr (KER == kResTabDiv) y = y * rb;
    return y;
}

// Phi at squared distance r2 for every kernel of the near field and the direct sum.
template <class T, int KER> __device__ __forceinline__ T kphi(T r2, T coef, const double *tab) {
    if constexpr (kRes<KER>) return kres<T, KER>(r2, coef, tab);
    else if constexpr (kTabExp<T, KER>) return exp2_tab(r2 * coef, tab);
    else if constexpr (KER == RBF_GAUSSIAN) return KFun<T>::gauss(r2, coef);
    else if constexpr (KER == RBF_MULTIQUADRIC) return KFun<T>::mq(r2, coef);
    else if constexpr (KER == RBF_INVERSE_MULTIQUADRIC) return KFun<T>::imq(r2, coef);
    else if constexpr (KER == RBF_WENDLAND) return KFun<T>::wendland(r2, coef);
    else if constexpr (kTabLog<T, KER>) return r2 > 0.0 ? 0.5 * r2 * log_tab(r2, tab) : 0.0;
    else if constexpr (KER == RBF_THIN_PLATE) return KFun<T>::thin_plate(r2);
    else return KFun<T>::r5(r2);
}

// Band-limited Gaussian (section 3, eq. 16 with the box of eq. 28): Phi_sigma(x) = prod_k
// phi(x_k), phi from the plan's table in global memory (kBlHead, then kBlDeg<T> + 1 monomial
// coefficients in u = 2 v - 1 per piece, v the position in the piece); inv = pieces per unit t,
// last = the last piece, which also takes |t| rounded past the box side.  The piece position is
// clamped before its conversion to an integer, so the index stays in the table for any input;
// a NaN difference takes the last piece and yields NaN through u.
// pieces: the first piece's coefficients, ST apart (the table in global memory past its head,
// as doubles, or the direct kernel's LDS copy in T)
template <class T, class P, int ST = kBlDeg<T> + 1>
__device__ __forceinline__ T bl_axis(T t, T inv, int last, const P *__restrict__ pieces) {
    constexpr int DEG = kBlDeg<T>;
    const T s = fabs(t) * inv;
    const int i = min((int)min(s, (T)last), last);
    const T u = T(2) * (s - (T)i) - T(1);
    const P *c = pieces + i * ST;
    T y = (T)c[DEG];
#pragma unroll
    for (int k = DEG - 1; k >= 0; --k) y = fma(y, u, (T)c[k]);
    return y;
}

template <class T, int D, class P, int ST = kBlDeg<T> + 1>
__device__ __forceinline__ T bl_pair(const T (&y)[D], const T (&x)[D], T inv, int last, const P *pieces) {
    T f = bl_axis<T, P, ST>(y[0] - x[0], inv, last, pieces);
#pragma unroll
    for (int k = 1; k < D; ++k) f *= bl_axis<T, P, ST>(y[k] - x[k], inv, last, pieces);
    return f;
}
// Tables up to this size are staged in the direct kernel's LDS (in T), the pieces kBlLds<T>
// entries apart: unpadded pieces (a power of two bytes) start on only a few bank groups, so
// that the lanes' different pieces collide; one entry of padding spreads them (FP64, 2^16
// points: 77 ms unpadded, 25 ms padded, 54 ms reading the table from global memory).
constexpr int kBlLdsBytes = 48 * 1024;
template <class T> constexpr int kBlLds = kBlDeg<T> + 2;

template <class T, int D, int KER>
__device__ __forceinline__ T p2p_pair(const T (&y)[D], const T (&x)[D], T coef, const double *tab) {
    T r2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T t = y[k] - x[k];
        r2 = fma(t, t, r2);
    }
    return kphi<T, KER>(r2, coef, tab);
}

template <class T, int D>
__device__ __forceinline__ T dist2(const T (&y)[D], const T (&x)[D]) {
    T r2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const T t = y[k] - x[k];
        r2 = fma(t, t, r2);
    }
    return r2;
}

// One step of S sources for the wave's targets.  Wendland's function vanishes from r = 1/e on
// (cut2 = 1/e^2), and the residual kernels of banded plans are negligible from r^2 = cut2 on:
// when no source of the step lies inside that radius of any target of the wave, the step
// adds only zeros and is skipped (a wave-uniform branch).
template <class T, int D, int KER, int S>
__device__ __forceinline__ T p2p_step(const T (&y)[D], const T (&x)[S][D], const T (&w)[S], T coef, T cut2,
                                      const double *tab, T acc) {
    if constexpr (kRes<KER>) {
        T r2[S];
#pragma unroll
        for (int v = 0; v < S; ++v) r2[v] = dist2<T, D>(y, x[v]);
        T mn = r2[0];
#pragma unroll
        for (int v = 1; v < S; ++v) mn = min(mn, r2[v]);
        if (__any(mn < cut2)) {
#pragma unroll
            for (int v = 0; v < S; ++v) acc = fma(w[v], kres<T, KER>(r2[v], coef, tab), acc);
        }
    } else if constexpr (KER == RBF_WENDLAND) {
        T r2[S];
#pragma unroll
        for (int v = 0; v < S; ++v) r2[v] = dist2<T, D>(y, x[v]);
        T mn = r2[0];
#pragma unroll
        for (int v = 1; v < S; ++v) mn = min(mn, r2[v]);
        if (__any(mn < cut2)) {
#pragma unroll
            for (int v = 0; v < S; ++v) acc = fma(w[v], KFun<T>::wendland(r2[v], coef), acc);
        }
    } else if constexpr (KER == RBF_GAUSSIAN_BANDLIMITED) {
        // coef: pieces per unit t; cut2: the last piece; tab: the table in global memory
#pragma unroll
        for (int v = 0; v < S; ++v) acc = fma(w[v], bl_pair<T, D>(y, x[v], coef, (int)cut2, tab + kBlHead), acc);
    } else {
#pragma unroll
        for (int v = 0; v < S; ++v) acc = fma(w[v], p2p_pair<T, D, KER>(y, x[v], coef, tab), acc);
    }
    return acc;
}

template <class T, int D, int KER>
__device__ __forceinline__ T p2p_whole(DescC<T> &d, const T (&y)[D], int r0, int r1, T coef, T cut2,
                                       const double *tab) {
    constexpr int S = kP2pStep<T>;
    const int64_t n = d.n;
    const cptr<int> rng = uconst((const int *)d.src_rng);
    const cptr<T> X = (cptr<T>)d.xs, L = (cptr<T>)d.lam_s;
    T acc = 0;
    for (int q = r0; q < r1; ++q) {
        const int j0 = rng[2 * q], j1 = rng[2 * q + 1];
        int j = j0;
        for (; j + S <= j1; j += S) {
            T x[S][D], w[S];
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
                for (int v = 0; v < S; ++v) x[v][k] = X[k * n + j + v];
#pragma unroll
            for (int v = 0; v < S; ++v) w[v] = L[j + v];
            acc = p2p_step<T, D, KER, S>(y, x, w, coef, cut2, tab, acc);
        }
        if (j < j1) {
            T x[S][D], w[S];
#pragma unroll
            for (int v = 0; v < S; ++v) {
                const int jj = min(j + v, j1 - 1);
#pragma unroll
                for (int k = 0; k < D; ++k) x[v][k] = X[k * n + jj];
                w[v] = j + v < j1 ? L[jj] : T(0);
            }
            acc = p2p_step<T, D, KER, S>(y, x, w, coef, cut2, tab, acc);
        }
    }
    return acc;
}

// Lane group g = lane / (64 / G) sums the sources j0 + g + G m of every range; two sources
// per lane per step, a source past the range end repeats the last one with weight 0.  The
// result is the group sums added over the groups (in every lane of the target).
template <class T, int D, int KER, int G>
__device__ __forceinline__ T p2p_split(DescC<T> &d, const T (&y)[D], int r0, int r1, T coef, T cut2,
                                       const double *tab) {
    constexpr int TP = kWave / G, U = 2;
    const int64_t n = d.n;
    const cptr<int> rng = uconst((const int *)d.src_rng);
    const T *__restrict__ X = d.xs;
    const T *__restrict__ L = d.lam_s;
    const int g = ((int)threadIdx.x % kWave) / TP;
    T acc = 0;
    for (int q = r0; q < r1; ++q) {
        const int j0 = rng[2 * q], j1 = rng[2 * q + 1];
        for (int jb = j0; jb < j1; jb += G * U) {
            T x[U][D], w[U];
#pragma unroll
            for (int v = 0; v < U; ++v) {
                const int j = jb + g + G * v;
                const int jj = min(j, j1 - 1);
#pragma unroll
                for (int k = 0; k < D; ++k) x[v][k] = X[k * n + jj];
                w[v] = j < j1 ? L[jj] : T(0);
            }
            acc = p2p_step<T, D, KER, U>(y, x, w, coef, cut2, tab, acc);
        }
    }
#pragma unroll
    for (int o = TP; o < kWave; o *= 2) acc += __shfl_xor(acc, o, kWave);
    return acc;
}

// The near-field kernel's LDS table (FP64 Gaussian: 2^(j/256); FP64 thin-plate: log tables;
// banded plans: residual pieces), filled by the NT threads of the workgroup; a barrier must
// follow.
template <class T, int KER>
__device__ __forceinline__ void p2p_fill(DescC<T> &d, double *tab, int nt) {
    if constexpr (kTabExp<T, KER> || kTabLog<T, KER>) fill_tab<T, KER>(tab, nt);
    if constexpr (kRes<KER>) {
        T *rt = reinterpret_cast<T *>(tab);
        constexpr int kP = (kResIntervals + 1) * kResStride;
        for (int j = threadIdx.x; j < kP; j += nt) rt[j] = j < kResCoefs ? (T)d.res_tab[j] : T(0);
        if (threadIdx.x == 0) {
            rt[kP] = (T)d.res_inv;
            rt[kP + 1] = (T)d.res_cut2;
            rt[kP + 2] = (T)sqrt((double)d.coef);   // c (coef = c^2)
        }
    }
}
template <class T, int KER> constexpr bool kP2pTab = kTabExp<T, KER> || kTabLog<T, KER> || kRes<KER>;

// One task of the near field by the calling wave (lanes = threadIdx.x mod 64), its table filled.
template <class T, int D, int KER>
__device__ __forceinline__ void p2p_task(DescC<T> &d, T *__restrict__ u, int bid, const double *tab) {
    const int64_t n = d.n;
    const cptr<int> tasks = uconst((const int *)d.ptasks), lb = uconst(d.leaf_begin);
    const cptr<int> sp = uconst(d.src_ptr);
    const int a = tasks[2 * bid], t0 = tasks[2 * bid + 1];   // leaf, first target
    const int t1 = min(t0 + kWave, lb[a + 1]);
    // lane groups: the largest G <= 8 with the chunk's m targets fitting 64 / G lanes
    const int m = t1 - t0;
    const int gl = m <= kWave / 8 ? 3 : m <= kWave / 4 ? 2 : m <= kWave / 2 ? 1 : 0;
    const int TP = kWave >> gl;
    const int lane = (int)threadIdx.x % kWave;
    const int ti = t0 + lane % TP;
    const bool act = ti < t1;
    // a lane without a target takes the chunk's first one (its sum is not written)
    T y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = d.xs[k * n + (act ? ti : t0)];
    const int r0 = sp[a], r1 = sp[a + 1];
    T coef = d.coef;
    if constexpr (kTabExp<T, KER>) coef *= kExpTab;   // exact
    const T cut2 = KER == RBF_WENDLAND ? T(1) / (coef * coef) : (kRes<KER> || KER == RBF_GAUSSIAN_BANDLIMITED) ? (T)d.res_cut2 : T(0);
    if constexpr (KER == RBF_GAUSSIAN_BANDLIMITED) tab = d.res_tab;
    T acc;
    switch (gl) {
        case 0: acc = p2p_whole<T, D, KER>(d, y, r0, r1, coef, cut2, tab); break;
        case 1: acc = p2p_split<T, D, KER, 2>(d, y, r0, r1, coef, cut2, tab); break;
        case 2: acc = p2p_split<T, D, KER, 4>(d, y, r0, r1, coef, cut2, tab); break;
        default: acc = p2p_split<T, D, KER, 8>(d, y, r0, r1, coef, cut2, tab); break;
    }
    if (act && lane < TP) {
        if (d.far) d.u_s[ti] = acc;
        else u[d.off + d.perm[ti]] = acc;   // near-only plan: this is the result
    }
}

template <class T, int D, int KER>
__device__ __forceinline__ void p2p_body(DescC<T> &d, T *__restrict__ u, int bid) {
    __shared__ __align__(32) double tab[kTabLen<T, KER>];
    if constexpr (kP2pTab<T, KER>) {
        p2p_fill<T, KER>(d, tab, kWave);
        __syncthreads();
    }
    p2p_task<T, D, KER>(d, u, bid, tab);
}

// Exact product over all pairs (rows of targets per workgroup, all sources tiled): targets
// [dir_t0, n), sources [0, dir_ns) of the sorted points.
template <class T, int D, int KER>
__device__ __forceinline__ void direct_body(DescC<T> &d, T *__restrict__ u, int bid, char *smem_raw) {
    constexpr int DP = Pad<D>::v;
    __shared__ T sdat[kTile * DP];
    const T *__restrict__ xs = d.xs;
    const int64_t n = d.n, ns = d.dir_ns;
    const int64_t ti = d.dir_t0 + bid * (int64_t)kThreads + threadIdx.x;
    const bool act = ti < n;
    T y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = act ? xs[k * n + ti] : T(0);
    __shared__ double tab[kTabLen<T, KER>];   // the kernel's table (filled before the first barrier)
    T coef = d.coef;
    fill_tab<T, KER>(tab, kThreads);
    if constexpr (kTabExp<T, KER>) coef *= kExpTab;   // exact
    T *const bt = reinterpret_cast<T *>(smem_raw);     // band-limited table in LDS (bl_lds)
    if constexpr (KER == RBF_GAUSSIAN_BANDLIMITED) {
        // ordered before its first use by the barriers of the first tile
        if (d.bl_lds)
            for (int j = threadIdx.x; j < ((int)d.res_cut2 + 1) * (kBlDeg<T> + 1); j += kThreads)
                bt[(j / (kBlDeg<T> + 1)) * kBlLds<T> + j % (kBlDeg<T> + 1)] = (T)d.res_tab[kBlHead + j];
    }
    T acc = 0;
    for (int64_t base = 0; base < ns; base += kTile) {
        const int cnt = (int)min((int64_t)kTile, ns - base);
        __syncthreads();
        if (threadIdx.x < cnt) {
#pragma unroll
            for (int k = 0; k < D; ++k) sdat[threadIdx.x * DP + k] = xs[k * n + base + threadIdx.x];
            sdat[threadIdx.x * DP + D] = d.lam_s[base + threadIdx.x];
        }
        __syncthreads();
        if constexpr (KER == RBF_GAUSSIAN_BANDLIMITED) {
            // coef: pieces per unit t; the last piece from the descriptor; the pieces from LDS
            // when the launch staged them there, else from global memory
            const int last = (int)d.res_cut2;
            if (d.bl_lds) {
                for (int e = 0; e < cnt; ++e) {
                    T x[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) x[k] = sdat[e * DP + k];
                    acc += sdat[e * DP + D] * bl_pair<T, D, T, kBlLds<T>>(y, x, coef, last, (const T *)bt);
                }
            } else {
                const double *gt = d.res_tab + kBlHead;
                for (int e = 0; e < cnt; ++e) {
                    T x[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) x[k] = sdat[e * DP + k];
                    acc += sdat[e * DP + D] * bl_pair<T, D>(y, x, coef, last, gt);
                }
            }
        } else {
            for (int e = 0; e < cnt; ++e) {
                T r2 = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    T t = y[k] - sdat[e * DP + k];
                    r2 += t * t;
                }
                acc += sdat[e * DP + D] * kphi<T, KER>(r2, coef, tab);
            }
        }
    }
    if (act) u[d.off + d.perm[ti]] = acc;
}

// Last-dimension phases, weighted by lambda: dl[i][h] = lam_i e^{-i xi_{H+h} x_{i,d}} for
// h < H, zero up to HMAX (FP64 rotation recurrence from an FP64 phase, stored in T).  A
// one-wave block builds the rows of its 64 points in LDS (rows padded by one entry against
// bank conflicts) and copies them out as one contiguous span: written straight from the
// recurrence, each store instruction strides by a row and the kernel ran at half the rate.
// (One wave keeps the block's LDS at 17 KB for FP64 rows of 16, so that it finds room beside
// the near field's workgroups.)
constexpr int kPhaseThreads = kWave;
template <class T, int D, int HMAX>
__device__ __forceinline__ void phase_dl_body(DescC<T> &d, int bid) {
    using C = typename cplx<T>::type;
    constexpr int ROW = HMAX + 1;
    __shared__ C st[kPhaseThreads * ROW];
    const int64_t i0 = bid * (int64_t)kPhaseThreads, i = i0 + threadIdx.x;
    if (i < d.n) {
        const double x = (double)d.xs[(int64_t)(D - 1) * d.n + i], l = (double)d.lam_s[i];
        double sb, cb, ss, cs;
        sincos(-d.xiH * x, &sb, &cb);
        sincos(-d.dxi * x, &ss, &cs);
        double er = l * cb, ei = l * sb;
        C *o = st + threadIdx.x * ROW;
#pragma unroll
        for (int h = 0; h < HMAX; ++h) {
            o[h] = (h < d.H) ? C{(T)er, (T)ei} : C{0, 0};
            const double nr = er * cs - ei * ss;
            ei = er * ss + ei * cs;
            er = nr;
        }
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kPhaseThreads, d.n - i0);
    C *out = d.dl + i0 * HMAX;
    for (int e = threadIdx.x; e < cnt * HMAX; e += kPhaseThreads) {
        const int q = e / HMAX;
        out[e] = st[q * ROW + (e - q * HMAX)];
    }
}

// Aggregation (P2M) on the vector ALUs (the FP64 path).  Blocks (leaf, part): thread = one row (m_1..m_{d-1}) of the half
// grid, all HMAX last-dimension nodes in registers.  Per chunk of CH points the block
// builds the per-thread factors e^{-i xi_m x_k} (k < d-1) in LDS; the lambda-weighted
// last-dimension phases of a point are uniform across the block and come through scalar
// loads.
template <class T, int D, int HMAX>
__device__ __forceinline__ void p2m_valu_body(DescC<T> &d, int bid, char *smem_raw) {
    using C = typename cplx<T>::type;
    C *tab = reinterpret_cast<C *>(smem_raw);
    constexpr int DM = D > 1 ? D - 1 : 1;
    const int mn = d.mn, R = d.R, CH = d.p2m_ch;
    const int ST = DM * mn;
    const int a = bid / d.wpl, part = bid % d.wpl;
    const int t0 = d.p2m_begin[a], t1 = d.p2m_end[a];   // the unit's sources
    const int row = part * blockDim.x + threadIdx.x;
    const bool act = row < R;
    // a wave past the last row (the last part of a unit) builds tables and meets the barriers
    // but skips the sums: 676 rows in 768 threads would otherwise run 12 waves of sums for 11
    const bool wlive = __builtin_amdgcn_readfirstlane(part * (int)blockDim.x + ((int)threadIdx.x & ~(kWave - 1))) < R;
    const int64_t n = d.n;
    int md[DM];
    {
        int rr = act ? row : 0;
        for (int k = D - 2; k >= 0; --k) { md[k] = rr % mn; rr /= mn; }
    }
    C acc[HMAX];
#pragma unroll
    for (int h = 0; h < HMAX; ++h) acc[h] = C{0, 0};
    // The chunk's point phases d.dl are read below with scalar loads, one point per step, and
    // every such load that goes to HBM stalls the whole workgroup.  Coalesced vector loads of
    // the chunk's rows, issued before its tables are built, bring them into L2 first.  Their
    // bits feed a value tested once at the end (never true), which keeps the loads alive.
    constexpr int kPre = 4;
    uint32_t sink = 0;
    for (int c0 = t0; c0 < t1; c0 += CH) {
        const int cn = min(CH, t1 - c0);
        uint32_t pre[kPre];
#pragma unroll
        for (int v = 0; v < kPre; ++v) {
            const int e = (int)threadIdx.x + v * (int)blockDim.x;
            pre[v] = e < cn * HMAX ? (uint32_t)__double_as_longlong((double)d.dl[(int64_t)c0 * HMAX + e].x) : 0u;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < cn * DM; t += blockDim.x) {
            const int j = t / DM, k = t % DM;
            C *dst = tab + j * ST + k * mn;
            const double x = (double)d.xs[k * n + c0 + j];
            double sb, cb, ss, cs;
            sincos(-d.dxi * x, &ss, &cs);
            sincos(-d.xi0 * x, &sb, &cb);
            double er = cb, ei = sb;
            for (int m = 0; m < mn; ++m) {
                dst[m] = C{(T)er, (T)ei};
                double nr = er * cs - ei * ss;
                ei = er * ss + ei * cs;
                er = nr;
            }
        }
#pragma unroll
        for (int v = 0; v < kPre; ++v) sink |= pre[v];
        __syncthreads();
        if (!wlive) continue;
        if constexpr (sizeof(T) == 4) {
            // prefetch the next point's uniform operands while the current one is used
            C cur[HMAX], nxt[HMAX];
            const CView<T> d0 = as_const<T>(d.dl + (int64_t)c0 * HMAX);
#pragma unroll
            for (int h = 0; h < HMAX; ++h) cur[h] = d0[h];
            for (int j = 0; j < cn; ++j) {
                const CView<T> dn = as_const<T>(d.dl + (int64_t)(c0 + min(j + 1, cn - 1)) * HMAX);
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
                const CView<T> dj = as_const<T>(d.dl + (int64_t)(c0 + j) * HMAX);
#pragma unroll
                for (int h = 0; h < HMAX; ++h) cmac(acc[h], kv, dj[h]);
            }
        }
    }
    if (act) {
        const int H = d.H;
        C *out = d.W + (int64_t)a * R * H + (int64_t)row * H;
#pragma unroll
        for (int h = 0; h < HMAX; ++h)
            if (h < H) out[h] = acc[h];
    }
    if (sink == 1u && n < 0) d.W[0] = C{0, 0};   // n >= 0: never taken
}

// Aggregation (P2M) on the matrix cores (the FP32 path): per leaf, W[r][h] = sum_j KV_j[r] DL_j[h] with
// KV_j[r] = prod_{k<d-1} e^{-i xi_{m_k(r)} x_jk} and DL_j[h] = lambda_j e^{-i xi_{H+h} x_jd}.
// The complex product is two real products over K' = 2 x points (k' = 2 j + c):
// A'[r][2j] = Re KV, A'[r][2j+1] = Im KV; B_re = [Re DL; -Im DL], B_im = [Im DL; Re DL].
// Workgroup (leaf, part) of four waves; each wave owns p2m_rtiles row tiles of 16 and all
// h tiles.  Per chunk of CH points the factors e^{-i xi_m x_jk} (k < d-1) are built in LDS
// (FP64 recurrences stored in T); the A fragment of a lane is one complex product of
// those, the B fragment one entry of the point's lambda-weighted phases.
template <class T, int D, int HMAX>
__device__ __forceinline__ void p2m_body(DescC<T> &d, int bid, char *smem_raw) {
    using C = typename cplx<T>::type;
    using M = Mfma<T>;
    using V = typename M::V;
    constexpr int DM = D - 1;
    constexpr int NRT = p2m_rtiles(D);
    constexpr int HT = (HMAX + 15) / 16;
    C *tab = reinterpret_cast<C *>(smem_raw);       // [CH][DM][mn]
    C *dls = tab + d.p2m_ch * DM * d.mn;            // [CH][HMAX] phases of the chunk's points
    const int mn = d.mn, R = d.R, CH = d.p2m_ch, H = d.H;
    const int ST = DM * mn;
    const int a = bid / d.wpl, part = bid % d.wpl;
    const int t0 = d.p2m_begin[a], t1 = d.p2m_end[a];   // the unit's sources
    const int64_t n = d.n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, jsel = lane >> 5, csel = (lane >> 4) & 1;
    const int rbase = part * p2m_rows(D) + wave * 16 * NRT;
    // row digits of this lane's A rows (fastest digit k = d-2)
    int md[NRT][DM];
#pragma unroll
    for (int t = 0; t < NRT; ++t) row_digits<DM>((unsigned)min(rbase + 16 * t + lr, R - 1), mn, d.mn_magic, md[t]);
    V wr[NRT][HT], wi[NRT][HT];
#pragma unroll
    for (int t = 0; t < NRT; ++t)
#pragma unroll
        for (int u = 0; u < HT; ++u) { wr[t][u] = V{0, 0, 0, 0}; wi[t][u] = V{0, 0, 0, 0}; }
    for (int c0 = t0; c0 < t1; c0 += CH) {
        const int cn = min(CH, t1 - c0);
        __syncthreads();
        for (int e = tid; e < cn * HMAX; e += blockDim.x) dls[e] = d.dl[(int64_t)c0 * HMAX + e];
        for (int job = tid; job < cn * DM; job += blockDim.x) {
            const int j = job / DM, k = job % DM;
            C *dst = tab + j * ST + k * mn;
            const double x = (double)d.xs[k * n + c0 + j];
            double sb, cb, ss, cs;
            sincos(-d.dxi * x, &ss, &cs);
            sincos(-d.xi0 * x, &sb, &cb);
            double er = cb, ei = sb;
            for (int m = 0; m < mn; ++m) {
                dst[m] = C{(T)er, (T)ei};
                double nr = er * cs - ei * ss;
                ei = er * ss + ei * cs;
                er = nr;
            }
        }
        __syncthreads();
        // K step j0 covers points j0 and j0 + 1; a point past the end of the chunk is clamped
        // and its B entries are zero
        for (int j0 = 0; j0 < cn; j0 += 2) {
            const int jl = j0 + jsel;
            const int jc = min(jl, cn - 1);
            T bre[HT], bim[HT];
#pragma unroll
            for (int u = 0; u < HT; ++u) {
                const int h = 16 * u + lr;
                const C v = (jl < cn && h < HMAX) ? dls[jc * HMAX + h] : C{0, 0};
                bre[u] = csel ? -v.y : v.x;
                bim[u] = csel ? v.x : v.y;
            }
            const C *pt = tab + jc * ST;
#pragma unroll
            for (int t = 0; t < NRT; ++t) {
                C kv = pt[md[t][0]];
#pragma unroll
                for (int k = 1; k < DM; ++k) kv = cmul(kv, pt[k * mn + md[t][k]]);
                const T av = csel ? kv.y : kv.x;
#pragma unroll
                for (int u = 0; u < HT; ++u) {
                    wr[t][u] = M::mac(av, bre[u], wr[t][u]);
                    wi[t][u] = M::mac(av, bim[u], wi[t][u]);
                }
            }
        }
    }
    C *out = d.W + (int64_t)a * R * H;
#pragma unroll
    for (int t = 0; t < NRT; ++t)
#pragma unroll
        for (int u = 0; u < HT; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rbase + 16 * t + M::row(q, lane), h = 16 * u + lr;
                if (r < R && h < H) out[(int64_t)r * H + h] = C{wr[t][u][q], wi[t][u][q]};
            }
}

// Upward pass: coarse cell = sum of its leaves.  Blocks (cell, 256-node chunk).
template <class T>
__device__ __forceinline__ void m2m_body(DescC<T> &d, int bid) {
    using C = typename cplx<T>::type;
    const int64_t P = d.P;
    const int nch = (int)((P + kThreads - 1) / kThreads);
    const int64_t c = bid / nch;
    const int64_t p = (int64_t)(bid % nch) * kThreads + threadIdx.x;
    if (p >= P) return;
    const int a0 = d.cell_begin[c], a1 = d.cell_begin[c + 1];
    C s{0, 0};
    // eight leaf rows in flight per step, added in leaf order
    for (int a = a0; a < a1; a += 8) {
        C v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = d.W[(int64_t)min(a + u, a1 - 1) * P + p];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (a + u < a1) {
                s.x += v[u].x;
                s.y += v[u].y;
            }
    }
    d.Wc[c * P + p] = s;
}

// Coarse translation: box sum of radius r along one axis of the dense coarse grid.
// Pass k reads the output of pass k-1 (the first reads Wc) and the last writes Lc.
// Every grid runs one workgroup per (line along the axis, 256-entry chunk).  Grids with at
// most kLineMax cells per side hold the line's values in registers, so every cell is read
// once per pass and each output adds its inputs in increasing order along the axis; larger
// grids walk the line with a running window sum (add the cell entering the window, subtract
// the one leaving it: two reads per output whatever the radius, in a fixed order).
constexpr int kLineMax = 16;

__host__ __device__ constexpr bool axis_by_lines(int lc) { return lc >= 1; }

template <int D> __device__ __forceinline__ int64_t axis_bits(int64_t v, int lc, int axis) {
    int64_t ins = 0;
    for (int b = 0; b < lc; ++b) ins |= ((v >> b) & 1) << (b * D + axis);
    return ins;
}

template <class T, int D>
__device__ __forceinline__ void m2l_axis_body(DescC<T> &d, int axis, int bid) {
    using C = typename cplx<T>::type;
    const int64_t P = d.P;
    const int nch = (int)((P + kThreads - 1) / kThreads);
    const int64_t c = bid / nch;
    const int64_t p = (int64_t)(bid % nch) * kThreads + threadIdx.x;
    if (p >= P) return;
    const int lc = d.lc;
    if (lc == 0 || d.r == 0) {   // single cell: the stencil sum is the cell itself
        if (axis == 0) d.Lc[c * P + p] = d.Wc[c * P + p];
        return;
    }
    C *const Wc = d.Wc, *const Tmp = d.Tmp, *const Lc = d.Lc;   // values, not field addresses
    const C *in = (axis == 0) ? Wc : ((axis % 2 == 1) ? Tmp : Wc);
    C *out = (axis == D - 1) ? Lc : ((axis % 2 == 0) ? Tmp : Wc);
    int64_t mask = 0;
    for (int b = 0; b < lc; ++b) mask |= (int64_t)1 << (b * D + axis);
    const int64_t side = (int64_t)1 << lc;
    if (axis_by_lines(lc)) {
        // c numbers the line: the other axes' bits of its cells, packed (the axis bits removed)
        int64_t rest = 0;
        {
            int k = 0;
            for (int b = 0; b < lc * D; ++b)
                if (!((mask >> b) & 1)) rest |= ((c >> k++) & 1) << b;
        }
        if (side > kLineMax) {
            const int64_t r = d.r;
            C acc{0, 0};
            for (int64_t j = 0; j <= min(r, side - 1); ++j) {
                const C v = in[(rest | axis_bits<D>(j, lc, axis)) * P + p];
                acc.x += v.x;
                acc.y += v.y;
            }
            out[(rest | axis_bits<D>(0, lc, axis)) * P + p] = acc;
            for (int64_t k = 1; k < side; ++k) {
                if (k + r < side) {
                    const C v = in[(rest | axis_bits<D>(k + r, lc, axis)) * P + p];
                    acc.x += v.x;
                    acc.y += v.y;
                }
                if (k - r - 1 >= 0) {
                    const C v = in[(rest | axis_bits<D>(k - r - 1, lc, axis)) * P + p];
                    acc.x -= v.x;
                    acc.y -= v.y;
                }
                out[(rest | axis_bits<D>(k, lc, axis)) * P + p] = acc;
            }
            return;
        }
        C v[kLineMax];
#pragma unroll
        for (int k = 0; k < kLineMax; ++k)
            if (k < side) v[k] = in[(rest | axis_bits<D>(k, lc, axis)) * P + p];
        const int r = d.r;
#pragma unroll
        for (int k = 0; k < kLineMax; ++k) {
            if (k >= side) break;
            C acc{0, 0};
#pragma unroll
            for (int j = 0; j < kLineMax; ++j)
                if (j < side && j >= k - r && j <= k + r) {
                    acc.x += v[j].x;
                    acc.y += v[j].y;
                }
            out[(rest | axis_bits<D>(k, lc, axis)) * P + p] = acc;
        }
        return;
    }
}

// Leaf translation + downward pass.  Blocks (sibling group, kLeafThreads-entry chunk of the
// expansion): the group's members (at most 8 consecutive leaves with one parent) share one
// ascending list of the leaves near any of them, with a mask of the members each entry is
// near to (padded to whole steps of 8 with entries of no member); every near row is loaded
// once for the whole group and subtracted from the members' copies of their coarse cell's
// local expansion (the same sequence of operations
// per member as a per-leaf walk of its own near list).  The quadrature weight w(xi) C(xi)
// is applied on output.  Output rows are padded to HP entries; the padding was zeroed at
// plan time and is not written.
// Block order (d.m2l_sched): 0 = group fastest, chunk slowest; 1 = the same order split
// into 8 contiguous group ranges, one per XCD (dispatch puts block g on XCD g % 8), so that
// the near rows a range re-reads stay in one XCD's L2.  In a batch every problem then has a
// multiple of 8 blocks, so its problem-local block ids keep their XCD.
constexpr int kLeafThreads = 256;   // expansion entries per leaf-translation workgroup

template <class T, int D>
__device__ __forceinline__ void m2l_leaf_body(DescC<T> &d, int g) {
    using C = typename cplx<T>::type;
    const int ng = d.ngroups, H = d.H, HP = d.HP;
    const int P = (int)d.P;
    int grp, chunk;
    if (d.m2l_sched == 1) {
        const int x = g & 7, k = g >> 3;
        const int per = (ng + 7) >> 3;                 // groups per XCD range (last may be short)
        const int lo = min(x * per, ng), hi = min(lo + per, ng);
        const int len = max(hi - lo, 1);
        grp = lo + k % len;
        chunk = k / len;
        if (hi - lo == 0 || grp >= hi) return;
    } else {
        grp = g % ng;
        chunk = g / ng;
    }
    // lanes past the end of the expansion read its last entry and store nothing, so that the
    // loop below stays in wave-uniform control flow (its indices and masks are scalar loads)
    const int pl = chunk * kLeafThreads + (int)threadIdx.x;
    const bool live = pl < P;
    const int p = live ? pl : P - 1;
    const cptr<int> gfirst = uconst(d.grp_first), uptr = uconst(d.uni_ptr);
    const cptr<int> uidx = uconst(d.uni_idx), umask = uconst(d.uni_mask), lcell = uconst(d.leaf_cell);
    const C *const W = d.W, *const Lc = d.Lc;
    const int a0 = gfirst[grp], na = gfirst[grp + 1] - a0;
    C s[8];
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (c < na) s[c] = Lc[(int64_t)lcell[a0 + c] * P + p];
    // The list holds whole steps of 8 (padding entries have no members) and one readable
    // step past its end: the next step's indices and masks are fetched while this step's
    // near rows load.
    const int e0 = uptr[grp], e1 = uptr[grp + 1];
    int bn[8], mn[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        bn[u] = uidx[e0 + u];
        mn[u] = umask[e0 + u];
    }
    for (int e = e0; e < e1; e += 8) {
        int b[8], m[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            b[u] = bn[u];
            m[u] = mn[u];
        }
        C v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = W[(int64_t)b[u] * P + p];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            bn[u] = uidx[e + 8 + u];
            mn[u] = umask[e + 8 + u];
        }
        // keep all eight row loads ahead of the sums (the scheduler would otherwise interleave
        // them with the arithmetic to save registers, leaving one or two loads in flight)
        __builtin_amdgcn_sched_barrier(0);
        // member c takes s - v (an fma with the scalar 1), a non-member s + 0 (fma with 0):
        // two FMAs per pair instead of a subtract and a select of each half
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < na)
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T k = ((m[u] >> c) & 1) ? T(-1) : T(0);
                    s[c].x = fma(k, v[u].x, s[c].x);
                    s[c].y = fma(k, v[u].y, s[c].y);
                }
    }
    if (!live) return;
    const double f = d.wtab[p];
    const int row = p / H, h = p - row * H;
    C *const Lx = d.Lx;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        if (c < na) Lx[((int64_t)(a0 + c) * d.R + row) * HP + h] = C{(T)(f * s[c].x), (T)(f * s[c].y)};
}

// Disaggregation (L2P) + combine on the matrix cores.  For the targets i of a workgroup
// (NT of one 64-target task) and the leaf's local rows r:
//   G[i][r] = sum_h E_i[h] L[r][h]   (E_i[h] = e^{+i xi_{H+h} x_id}),   a real product over
//   K' = 2 HMAX with A'[i][2h] = Re E, A'[i][2h+1] = Im E, B_re = [Re L; -Im L], B_im = [Im L; Re L];
//   u_i = u_near_i + 2 Re sum_r KV_i[r] G[i][r],  KV_i[r] = prod_{k<d-1} e^{+i xi_{m_k(r)} x_ik}.
// The four waves split the row tiles; the phase tables of the NT targets are built once in
// LDS (FP64 recurrences stored in T); per-target sums are reduced over the 16 lanes of a row
// group and then over the waves in a fixed order.
template <class T, int D, int HMAX>
__device__ __forceinline__ void l2p_body(DescC<T> &d, T *__restrict__ u, int bid, char *smem_raw) {
    using C = typename cplx<T>::type;
    using M = Mfma<T>;
    using V = typename M::V;
    constexpr int DM = D - 1;
    constexpr int KS = HMAX / 2;                       // K steps of 4 over k' = 2 h + c
    constexpr int NT = l2p_targets((int)sizeof(C), D, HMAX);
    constexpr int IT = NT / 16, SPLIT = 64 / NT;
    const int2 tk = d.tasks[bid / SPLIT];
    const int a = tk.x;
    const int tb = d.leaf_begin[a] + tk.y + (bid % SPLIT) * NT;
    const int t1 = d.leaf_begin[a + 1];
    const int nt = min(NT, t1 - tb);
    if (nt <= 0) return;                               // the same for the whole workgroup
    const int R = d.R, mn = d.mn;
    const int64_t n = d.n;
    C *E = reinterpret_cast<C *>(smem_raw);            // [NT][HMAX]
    C *Tt = E + NT * HMAX;                             // [DM][NT][mn]
    T *red = reinterpret_cast<T *>(Tt + DM * NT * mn); // [4][NT]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, hsel = lane >> 5, csel = (lane >> 4) & 1;
    for (int job = tid; job < NT * (1 + DM); job += blockDim.x) {
        const int i = job % NT, k = job / NT;
        const int64_t ti = tb + min(i, nt - 1);
        double sb, cb, ss, cs;
        if (k == 0) {
            const double x = (double)d.xs[(int64_t)(D - 1) * n + ti];
            sincos(d.xiH * x, &sb, &cb);
            sincos(d.dxi * x, &ss, &cs);
        } else {
            const double x = (double)d.xs[(int64_t)(k - 1) * n + ti];
            sincos(d.xi0 * x, &sb, &cb);
            sincos(d.dxi * x, &ss, &cs);
        }
        C *dst = k == 0 ? E + i * HMAX : Tt + ((k - 1) * NT + i) * mn;
        const int len = k == 0 ? HMAX : mn;
        double er = cb, ei = sb;
        for (int m = 0; m < len; ++m) {
            dst[m] = C{(T)er, (T)ei};
            double nr = er * cs - ei * ss;
            ei = er * ss + ei * cs;
            er = nr;
        }
    }
    __syncthreads();
    T afr[IT][KS];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const C e = E[(16 * it + lr) * HMAX + 2 * s + hsel];
            afr[it][s] = csel ? e.y : e.x;
        }
    T acc[IT][4];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[it][q] = 0;
    const C *La = d.Lx + (int64_t)a * R * HMAX;
    const int NR = (R + 15) / 16;
    for (int rt = wave; rt < NR; rt += 4) {
        const int r = rt * 16 + lr;
        const bool rv = r < R;
        // B fragments of the row tile (a row past the end reads as zero), then per target tile
        // the MFMA chain and the stage-2 sums of its rows
        T br[KS], bi[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const C l = rv ? La[(int64_t)r * HMAX + 2 * s + hsel] : C{0, 0};
            br[s] = csel ? -l.y : l.x;
            bi[s] = csel ? l.x : l.y;
        }
        int md[DM];
        {
            int rr = rv ? r : 0;
#pragma unroll
            for (int k = DM - 1; k >= 0; --k) { md[k] = rr % mn; rr /= mn; }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            V gr = V{0, 0, 0, 0}, gi = V{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                gr = M::mac(afr[it][s], br[s], gr);
                gi = M::mac(afr[it][s], bi[s], gi);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * it + M::row(q, lane);
                C kv = Tt[i * mn + md[0]];
#pragma unroll
                for (int k = 1; k < DM; ++k) kv = cmul(kv, Tt[(k * NT + i) * mn + md[k]]);
                acc[it][q] = fma(kv.x, gr[q], acc[it][q]);
                acc[it][q] = fma(-kv.y, gi[q], acc[it][q]);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T v = acc[it][q];
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            v += __shfl_xor(v, 8, 64);
            if (lr == 0) red[wave * NT + 16 * it + M::row(q, lane)] = v;
        }
    __syncthreads();
    if (tid < nt) {
        const T sum = ((red[tid] + red[NT + tid]) + red[2 * NT + tid]) + red[3 * NT + tid];
        const int ti = tb + tid;
        if (d.l2p_acc) d.u_s[ti] = d.u_s[ti] + T(2) * sum;   // a band before the last
        else u[d.off + d.perm[ti]] = d.u_s[ti] + T(2) * sum;
    }
}

// ---- kernels: single problem (descriptor by value) or batch (descriptor array) --------
__device__ __forceinline__ int find_prob(const int *__restrict__ bstart, int nprob, int g) {
    int lo = 0, hi = nprob;   // largest q with bstart[q] <= g
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (bstart[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Launch argument: either one descriptor (nprob == 0) or a descriptor array with the
// exclusive prefix of per-problem block counts.
template <class T> struct Work {
    Desc<T> one;
    const Desc<T> *many;
    const int *bstart;
    int nprob;
    const T *lam;
    T *u;
};

// Resolves the calling block to (descriptor, problem-local block id).  The descriptor is
// returned as a constant-address-space pointer: its fields are then read with scalar loads
// and stay wave-uniform (a read through a generic pointer would be a flat load, whose result
// the compiler must treat as per-lane), and the device pointers read from it are known to
// be global.
template <class T, bool SWIZZLE = true>
__device__ __forceinline__ cptr<Desc<T>> resolve(const Work<T> &w, int &lb) {
    const int g = SWIZZLE ? xcd_swizzle(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    if (w.nprob == 0) {
        lb = g;
        return (cptr<Desc<T>>)&w.one;
    }
    const int q = find_prob(w.bstart, w.nprob, g);
    lb = g - w.bstart[q];
    return (cptr<Desc<T>>)(w.many + q);
}

template <class T> __global__ void __launch_bounds__(kThreads) k_gather(Work<T> w) {
    int lb;
    DescC<T> &d = *resolve(w, lb);
    gather_body<T>(d, w.lam, lb);
}
template <class T, int D, int KER> __global__ void __launch_bounds__(kWave) k_p2p(Work<T> w) {
    int lb;
    DescC<T> &d = *resolve(w, lb);
    p2p_body<T, D, KER>(d, w.u, lb);
}
// The near field as a work queue (a single problem whose near field runs beside its far
// field on another stream): a fixed grid of one-wave blocks takes tasks from per-XCD counters
// over the task ranges that xcd_swizzle gives each XCD, then from the other XCDs' ranges once
// its own is done.  The grid holds fewer waves than the chip has slots, which leaves the rest
// to the far-field kernels: a grid of one block per task fills every slot with near-field
// waves that live long, and the memory-bound kernels beside it wait for them to drain.
// Its workgroups are kQueueWaves waves that share one copy of the kernel's LDS table (one copy
// per one-wave workgroup would hold, at the residual kernel's 6 KB, most of a CU's LDS for the
// whole run and keep the far-field kernels that need LDS off the CU); after the fill every wave
// runs its own loop, with no further barrier.
constexpr int kQueueWaves = 4;
template <class T, int D, int KER>
__global__ void __launch_bounds__(kQueueWaves * kWave) k_p2p_queue(Work<T> w) {
    DescC<T> &d = *(cptr<Desc<T>>)&w.one;
    __shared__ __align__(32) double tab[kTabLen<T, KER>];
    if constexpr (kP2pTab<T, KER>) {
        p2p_fill<T, KER>(d, tab, kQueueWaves * kWave);
        __syncthreads();
    }
    const int nv = d.nptasks, per = nv / kXcds, rem = nv % kXcds;
    const int x0 = (int)blockIdx.x % kXcds;
    for (int k = 0; k < kXcds; ++k) {
        const int x = (x0 + k) % kXcds;
        const int lo = x * per + min(x, rem), cnt = per + (x < rem ? 1 : 0);
        for (;;) {
            int v = 0;
            if (threadIdx.x % kWave == 0) v = atomicAdd(d.p2p_ctr + x * kCtrStride, 1);
            v = __builtin_amdgcn_readfirstlane(__shfl(v, 0, kWave));
            if (v >= cnt) break;
            p2p_task<T, D, KER>(d, w.u, lo + v, tab);
        }
    }
}
template <class T, int D, int KER> __global__ void __launch_bounds__(kThreads) k_direct(Work<T> w) {
    extern __shared__ char smem_raw[];
    int lb;
    DescC<T> &d = *resolve(w, lb);
    direct_body<T, D, KER>(d, w.u, lb, smem_raw);
}
template <class T, int D, int HMAX> __global__ void __launch_bounds__(kPhaseThreads) k_phase_dl(Work<T> w) {
    int lb;
    DescC<T> &d = *resolve(w, lb);
    phase_dl_body<T, D, HMAX>(d, lb);
}
// The FP64 aggregation runs on the vector ALUs: on this chip the FP64 matrix rate equals the
// FP64 vector rate, and its VALU kernel measured faster than the MFMA one.  FP32 aggregation
// and the disaggregation in both precisions use the matrix cores.
template <class T> constexpr bool kExpMfma = sizeof(T) == 4;

template <class T, int D, int HMAX> __global__ void __launch_bounds__(kThreads) k_p2m(Work<T> w) {
    extern __shared__ char smem_raw[];
    int lb;
    DescC<T> &d = *resolve(w, lb);
    if constexpr (kExpMfma<T>) p2m_body<T, D, HMAX>(d, lb, smem_raw);
    else p2m_valu_body<T, D, HMAX>(d, lb, smem_raw);
}
// The upward pass runs beside the near field (on the plan's second stream); its memory-bound
// waves take instruction-issue priority over the near field's arithmetic waves on shared CUs.
template <class T> __global__ void __launch_bounds__(kThreads) k_m2m(Work<T> w) {
    __builtin_amdgcn_s_setprio(2);
    int lb;
    DescC<T> &d = *resolve(w, lb);
    m2m_body<T>(d, lb);
}
template <class T, int D> __global__ void __launch_bounds__(kThreads) k_m2l_axis(Work<T> w, int axis) {
    int lb;
    DescC<T> &d = *resolve(w, lb);
    m2l_axis_body<T, D>(d, axis, lb);
}
template <class T, int D> __global__ void __launch_bounds__(kLeafThreads) k_m2l_leaf(Work<T> w) {
    int lb;
    DescC<T> &d = *resolve<T, false>(w, lb);
    m2l_leaf_body<T, D>(d, lb);
}
template <class T, int D, int HMAX> __global__ void __launch_bounds__(kThreads) k_l2p(Work<T> w) {
    extern __shared__ char smem_raw[];
    int lb;
    DescC<T> &d = *resolve(w, lb);
    l2p_body<T, D, HMAX>(d, w.u, lb, smem_raw);
}

// ---- host side -----------------------------------------------------------------------
// Per-product launch context: phase timing (HIP events, when the plan profiles) and the
// optional side stream of the near field with its fork and join events (single problems).
struct ProductRun {
    rbf_plan *p;   // null: no timing
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int ph = -1;
    hipStream_t st = nullptr;
    ProductRun(rbf_plan *pp, bool overlap)
        : p(pp && pp->profiling ? pp : nullptr), side(overlap && pp ? pp->side : nullptr),
          fork(overlap && pp ? pp->ev_fork : nullptr), join(overlap && pp ? pp->ev_join : nullptr) {}
    // timing events go on stream s (the stream the phase runs on)
    hipError_t begin(int k, hipStream_t s) {
        ph = k;
        st = s;
        return p ? hipEventRecord(p->ev[2 * k], s) : hipSuccess;
    }
    hipError_t end() { return p ? hipEventRecord(p->ev[2 * ph + 1], st) : hipSuccess; }
};

// Per-phase block counts of one problem (the grid of a single-problem launch).
template <class T> int64_t phase_blocks(const Desc<T> &d, int phase) {
    const int64_t nb_pts = (d.n + kThreads - 1) / kThreads;
    const int64_t nch = (d.P + kThreads - 1) / kThreads;
    if (!d.far && phase != PH_GATHER && phase != PH_P2P && phase != PH_DIRECT) return 0;
    switch (phase) {
        case PH_GATHER: case PH_DIRECT: return nb_pts;
        case PH_PHASE_DL: return (d.n + kPhaseThreads - 1) / kPhaseThreads;
        case PH_P2P: return d.nptasks;
        case PH_L2P:
            return (int64_t)d.ntasks * (64 / l2p_targets((int)sizeof(typename cplx<T>::type), d.dim, d.HP));
        case PH_P2M: return (int64_t)d.p2m_n * d.wpl;
        case PH_M2M: return d.ncells * nch;
        case PH_M2L_AXIS: return (axis_by_lines(d.lc) ? d.ncells >> d.lc : d.ncells) * nch;
        case PH_M2L_LEAF: {
            const int64_t nch_l = (d.P + kLeafThreads - 1) / kLeafThreads;
            if (d.m2l_sched == 1) return 8 * nch_l * ((d.ngroups + 7) / 8);
            return nch_l * d.ngroups;
        }
    }
    return 0;
}

template <class T> size_t p2m_shmem(const Desc<T> &d, int) { return (size_t)d.p2m_lds; }

// Launch one phase for a single problem or a batch (see Work).
template <class T, int D, int HMAX>
int launch_phase(const Work<T> &w, int phase, int64_t nblocks, hipStream_t s, int axis, size_t shmem, int kernel) {
    if (nblocks <= 0) return RBF_OK;
    const unsigned g = (unsigned)nblocks;
    switch (phase) {
        case PH_GATHER: k_gather<T><<<g, kThreads, 0, s>>>(w); break;
        case PH_P2P:
            switch (kernel) {
                case RBF_GAUSSIAN: k_p2p<T, D, RBF_GAUSSIAN><<<g, kWave, 0, s>>>(w); break;
                case RBF_MULTIQUADRIC: k_p2p<T, D, RBF_MULTIQUADRIC><<<g, kWave, 0, s>>>(w); break;
                case RBF_INVERSE_MULTIQUADRIC: k_p2p<T, D, RBF_INVERSE_MULTIQUADRIC><<<g, kWave, 0, s>>>(w); break;
                case RBF_WENDLAND: k_p2p<T, D, RBF_WENDLAND><<<g, kWave, 0, s>>>(w); break;
                case RBF_THIN_PLATE: k_p2p<T, D, RBF_THIN_PLATE><<<g, kWave, 0, s>>>(w); break;
                case kResTab: k_p2p<T, D, kResTab><<<g, kWave, 0, s>>>(w); break;
                case kResTabDiv: k_p2p<T, D, kResTabDiv><<<g, kWave, 0, s>>>(w); break;
                case kResTabQ: k_p2p<T, D, kResTabQ><<<g, kWave, 0, s>>>(w); break;
                case RBF_GAUSSIAN_BANDLIMITED: k_p2p<T, D, RBF_GAUSSIAN_BANDLIMITED><<<g, kWave, 0, s>>>(w); break;
                case RBF_R5: k_p2p<T, D, RBF_R5><<<g, kWave, 0, s>>>(w); break;
                default:
                    set_error("near-field kernel: unknown kernel %d", kernel);
                    return RBF_EUNSUPPORTED;
            }
            break;
        case PH_DIRECT:
            switch (kernel) {
                case RBF_GAUSSIAN: k_direct<T, D, RBF_GAUSSIAN><<<g, kThreads, 0, s>>>(w); break;
                case RBF_MULTIQUADRIC: k_direct<T, D, RBF_MULTIQUADRIC><<<g, kThreads, 0, s>>>(w); break;
                case RBF_INVERSE_MULTIQUADRIC: k_direct<T, D, RBF_INVERSE_MULTIQUADRIC><<<g, kThreads, 0, s>>>(w); break;
                case RBF_WENDLAND: k_direct<T, D, RBF_WENDLAND><<<g, kThreads, 0, s>>>(w); break;
                case RBF_THIN_PLATE: k_direct<T, D, RBF_THIN_PLATE><<<g, kThreads, 0, s>>>(w); break;
                case RBF_GAUSSIAN_BANDLIMITED:
                    k_direct<T, D, RBF_GAUSSIAN_BANDLIMITED><<<g, kThreads, shmem, s>>>(w);
                    break;
                case RBF_R5: k_direct<T, D, RBF_R5><<<g, kThreads, 0, s>>>(w); break;
                default:
                    set_error("direct kernel: unknown kernel %d", kernel);
                    return RBF_EUNSUPPORTED;
            }
            break;
        case PH_PHASE_DL: k_phase_dl<T, D, HMAX><<<g, kPhaseThreads, 0, s>>>(w); break;
        case PH_P2M: k_p2m<T, D, HMAX><<<g, (kExpMfma<T> || D > 2) ? kThreads : kWave, shmem, s>>>(w); break;
        case PH_M2M: k_m2m<T><<<g, kThreads, 0, s>>>(w); break;
        case PH_M2L_AXIS: k_m2l_axis<T, D><<<g, kThreads, 0, s>>>(w, axis); break;
        case PH_M2L_LEAF: k_m2l_leaf<T, D><<<g, kLeafThreads, 0, s>>>(w); break;
        case PH_L2P: {
            constexpr int csz = (int)sizeof(typename cplx<T>::type);
            constexpr size_t lds = l2p_lds(csz, D, HMAX, l2p_targets(csz, D, HMAX));
            k_l2p<T, D, HMAX><<<g, kThreads, lds, s>>>(w);
            break;
        }
    }
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

// Near-field work queue of a single problem: its grid holds this many waves per SIMD (of the
// 8 a SIMD can hold at the kernel's register count).  Measured on the 2^20-point 3-D
// workloads (banded multiquadric beside its bands, Gaussian beside its far field): against one
// workgroup per task, the queue at 8, 4 and 2 waves took the multiquadric product to 93%, 93%
// and 98% of its time, the Gaussian to 100%, 99% and 98%.
constexpr int kP2pQueueWaves = 4;
template <class T, int D>
int launch_p2p_queue(const Work<T> &w, hipStream_t s, int kernel) {
    const int64_t ntask = w.one.nptasks;
    if (ntask <= 0) return RBF_OK;
    // 256 CUs x 4 SIMDs x kP2pQueueWaves waves, kQueueWaves to a workgroup
    const int64_t waves = std::min<int64_t>(ntask, (int64_t)256 * 4 * kP2pQueueWaves);
    const unsigned g = (unsigned)((waves + kQueueWaves - 1) / kQueueWaves);
    constexpr int bt = kQueueWaves * kWave;
    switch (kernel) {
        case RBF_GAUSSIAN: k_p2p_queue<T, D, RBF_GAUSSIAN><<<g, bt, 0, s>>>(w); break;
        case RBF_MULTIQUADRIC: k_p2p_queue<T, D, RBF_MULTIQUADRIC><<<g, bt, 0, s>>>(w); break;
        case RBF_INVERSE_MULTIQUADRIC: k_p2p_queue<T, D, RBF_INVERSE_MULTIQUADRIC><<<g, bt, 0, s>>>(w); break;
        case kResTab: k_p2p_queue<T, D, kResTab><<<g, bt, 0, s>>>(w); break;
        case kResTabDiv: k_p2p_queue<T, D, kResTabDiv><<<g, bt, 0, s>>>(w); break;
        case kResTabQ: k_p2p_queue<T, D, kResTabQ><<<g, bt, 0, s>>>(w); break;
        default:
            set_error("near-field work queue: kernel %d has no far field", kernel);
            return RBF_EUNSUPPORTED;
    }
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

// The whole product for one problem or one batch group (all problems with the same HP).
// bstarts[phase] holds the per-problem block prefix of each phase (batch only).
template <class T, int D, int HMAX>
int product_d(const Work<T> &w0, int64_t const *nblocks, const int *const *bstarts, size_t p2m_sh, int kernel,
              hipStream_t s, ProductRun &pt) {
    Work<T> w = w0;
    auto bs = [&](int ph) {
        if (w0.nprob) w.bstart = bstarts[ph];
    };
    RBF_HIP(pt.begin(0, s));
    bs(PH_GATHER);
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_GATHER, nblocks[PH_GATHER], s, 0, 0, kernel)));
    RBF_HIP(pt.end());
    RBF_HIP(pt.begin(2, s));
    bs(PH_PHASE_DL);
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_PHASE_DL, nblocks[PH_PHASE_DL], s, 0, 0, kernel)));
    bs(PH_P2M);
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_P2M, nblocks[PH_P2M], s, 0, p2m_sh, kernel)));
    RBF_HIP(pt.end());
    // near field: on the side stream when there is one, forked after the aggregation so that it
    // runs beside the memory-bound upward pass and translations rather than beside the
    // aggregation's arithmetic
    hipStream_t sn = s;
    if (pt.side) {
        RBF_HIP(hipEventRecord(pt.fork, s));
        RBF_HIP(hipStreamWaitEvent(pt.side, pt.fork, 0));
        sn = pt.side;
    }
    RBF_HIP(pt.begin(1, sn));
    bs(PH_P2P);
    if (pt.side && w.nprob == 0 && w.one.far)
        RBF_TRY((launch_p2p_queue<T, D>(w, sn, kernel)));
    else
        RBF_TRY((launch_phase<T, D, HMAX>(w, PH_P2P, nblocks[PH_P2P], sn, 0, 0, kernel)));
    RBF_HIP(pt.end());
    if (pt.side) RBF_HIP(hipEventRecord(pt.join, sn));
    RBF_HIP(pt.begin(3, s));
    bs(PH_M2M);
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_M2M, nblocks[PH_M2M], s, 0, 0, kernel)));
    RBF_HIP(pt.end());
    RBF_HIP(pt.begin(4, s));
    bs(PH_M2L_AXIS);
    for (int ax = 0; ax < D; ++ax)
        RBF_TRY((launch_phase<T, D, HMAX>(w, PH_M2L_AXIS, nblocks[PH_M2L_AXIS], s, ax, 0, kernel)));
    RBF_HIP(pt.end());
    RBF_HIP(pt.begin(5, s));
    bs(PH_M2L_LEAF);
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_M2L_LEAF, nblocks[PH_M2L_LEAF], s, 0, 0, kernel)));
    RBF_HIP(pt.end());
    if (pt.side) RBF_HIP(hipStreamWaitEvent(s, pt.join, 0));   // the disaggregation reads u_s
    RBF_HIP(pt.begin(6, s));
    bs(PH_L2P);
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_L2P, nblocks[PH_L2P], s, 0, 0, kernel)));
    RBF_HIP(pt.end());
    return RBF_OK;
}

template <class T, int D>
int product_dispatch(int HP, const Work<T> &w, int64_t const *nblocks, const int *const *bstarts, size_t p2m_sh,
                     int kernel, hipStream_t s, ProductRun &pt) {
#define CASE_H(V) \
    case V: return product_d<T, D, V>(w, nblocks, bstarts, p2m_sh, kernel, s, pt);
    switch (HP) {
        CASE_H(4)
        CASE_H(6)
        CASE_H(8)
        CASE_H(10)
        CASE_H(12)
        default: break;
    }
    if constexpr (D < 5) {
        switch (HP) {
            CASE_H(14)
            CASE_H(16)
            CASE_H(20)
            CASE_H(24)
            CASE_H(28)
            CASE_H(32)
            default: break;
        }
    }
#undef CASE_H
    set_error("padded half grid %d not compiled for d=%d", HP, D);
    return RBF_EUNSUPPORTED;
}

template <class T>
int product_t(int d, int HP, const Work<T> &w, int64_t const *nblocks, const int *const *bstarts, size_t p2m_sh,
              int kernel, hipStream_t s, ProductRun &pt) {
    switch (d) {
        case 2: return product_dispatch<T, 2>(HP, w, nblocks, bstarts, p2m_sh, kernel, s, pt);
        case 3: return product_dispatch<T, 3>(HP, w, nblocks, bstarts, p2m_sh, kernel, s, pt);
        case 5: return product_dispatch<T, 5>(HP, w, nblocks, bstarts, p2m_sh, kernel, s, pt);
    }
    set_error("dimension %d not compiled", d);
    return RBF_EUNSUPPORTED;
}

// Creates the plan's near-field stream and its fork/join events on first use; without them
// the product runs on one stream.
void ensure_side_stream(rbf_plan *p) {
    if (p->side_state != 0) return;
    if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess &&
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) == hipSuccess) {
        p->side_state = 1;
        return;
    }
    (void)hipGetLastError();   // clear the failure: the product falls back to one stream
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->side) (void)hipStreamDestroy(p->side);
    p->side = nullptr;
    p->ev_fork = p->ev_join = nullptr;
    p->side_state = -1;
}

// Adds the phase durations of the product just launched (events ev[2k], ev[2k + 1]).
int add_phase_times(rbf_plan *p) {
    RBF_HIP(hipEventSynchronize(p->ev[2 * RBF_NPHASES - 1]));
    for (int k = 0; k < RBF_NPHASES; ++k) {
        float ms = 0.f;
        RBF_HIP(hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]));
        p->phase_ms[k] += ms;
    }
    p->prof_calls += 1;
    return RBF_OK;
}

template <class T>
int matvec_t(rbf_plan *p, const void *lam, void *u) {
    Work<T> w{};
    fill_desc<T>(p, &w.one);
    w.nprob = 0;
    w.lam = (const T *)lam;
    w.u = (T *)u;
    int64_t nb[PH_COUNT];
    for (int k = 0; k < PH_COUNT; ++k) nb[k] = phase_blocks<T>(w.one, k);
    ensure_side_stream(p);
    ProductRun pt(p, p->side_state == 1);
    RBF_TRY(product_t<T>(p->d, p->HP, w, nb, nullptr, p2m_shmem<T>(w.one, p->d), p->kernel, p->stream, pt));
    if (p->profiling) RBF_TRY(add_phase_times(p));
    return RBF_OK;
}

template <class T, int D>
int direct_d(rbf_plan *p, const T *lam, T *u) {
    Work<T> w{};
    fill_desc<T>(p, &w.one);
    w.lam = lam;
    w.u = u;
    const int64_t nb = phase_blocks<T>(w.one, PH_DIRECT);   // every point (the gather)
    // A plan of one leaf for separate targets holds its sources first: the direct kernel then
    // pairs the targets [n_src, n) with the sources [0, n_src) only.  Otherwise every point is a
    // target and a source (an evaluation plan of several leaves interleaves them; its packed
    // weights are zero at the targets).
    if (p->n_src > 0 && p->nleaves == 1) {
        w.one.dir_t0 = p->n_src;
        w.one.dir_ns = p->n_src;
    }
    const int64_t nbd = (p->n - w.one.dir_t0 + kThreads - 1) / kThreads;
    // the band-limited Gaussian's table in the direct kernel's LDS (fill_desc sets bl_lds when
    // it fits in kBlLdsBytes)
    const size_t sh = w.one.bl_lds ? sizeof(T) * (size_t)p->bl_pieces * kBlLds<T> : 0;
    RBF_TRY((launch_phase<T, D, 4>(w, PH_GATHER, nb, p->stream, 0, 0, p->kernel)));
    RBF_TRY((launch_phase<T, D, 4>(w, PH_DIRECT, nbd, p->stream, 0, sh, p->kernel)));
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

// ---- banded far field (multiquadric kernels) -------------------------------------------
// The product of a banded plan: the near field sums the residual kernel over the adjacent
// cells of the uniform tree into u_s (on the side stream when there is one), then every band
// runs aggregation, upward sum, coarse stencil, translation (empty near lists: the band
// covers near and far pairs alike) and disaggregation, each adding its far field to u_s; the
// last band writes u = u_s + its far field in caller order.

template <class T> void fill_band_desc(const rbf_plan *p, const Band &b, bool acc, Desc<T> *d) {
    using C = typename cplx<T>::type;
    fill_desc<T>(p, d);
    d->leaf_begin = b.unit_begin;
    d->src_end = b.unit_begin + 1;
    d->leaf_cell = b.unit_cell;
    d->cell_begin = b.cell_begin;
    d->tasks = b.tasks;
    d->ntasks = b.ntasks;
    d->nptasks = 0;
    d->nleaves = b.nunits;
    d->ncells = b.ncells;
    d->lc = b.lc;
    d->r = b.r;
    d->mn = b.mn;
    d->H = b.H;
    d->HP = b.HP;
    d->R = (int)b.R;
    d->P = b.P;
    const double dxi = 2.0 * b.sigma / (b.mn - 1);
    d->dxi = dxi;
    d->xi0 = -b.sigma;
    d->xiH = -b.sigma + b.H * dxi;
    d->W = (C *)p->bW;
    d->Lx = (C *)p->bLx;
    d->Wc = (C *)p->bWc;
    d->Lc = (C *)p->bLc;
    d->Tmp = (C *)p->bTmp;
    d->dl = (C *)p->bdl;
    d->wtab = b.wtab;
    set_p2m_shape<T>(d, p->d, b.R, b.mn, b.HP);
    d->far = 1;
    d->ngroups = b.ngroups;
    d->grp_first = b.grp_first;
    d->uni_ptr = b.uni_ptr;
    d->uni_idx = b.uni_pad;
    d->uni_mask = b.uni_pad;
    d->mn_magic = (unsigned)((1ull << 32) / (unsigned)b.mn + 1);
    d->p2m_begin = b.chunk_begin;
    d->p2m_end = b.chunk_begin + 1;
    d->p2m_n = b.nchunks;
    d->l2p_acc = acc ? 1 : 0;
}

// Phase timing of a banded product: event pair k of band j at band_ev[(j * NPHASES + k) * 2].
struct BandTimer {
    rbf_plan *p;
    int j = 0, k = 0;
    hipStream_t st = nullptr;
    explicit BandTimer(rbf_plan *pp) : p(pp && pp->profiling ? pp : nullptr) {}
    hipError_t begin(int kk, hipStream_t s) {
        k = kk;
        st = s;
        return p ? hipEventRecord(p->band_ev[(size_t)(j * RBF_NPHASES + k) * 2], s) : hipSuccess;
    }
    hipError_t end() { return p ? hipEventRecord(p->band_ev[(size_t)(j * RBF_NPHASES + k) * 2 + 1], st) : hipSuccess; }
};

// Hooks of the source band of the interpolating transfers: after its upward pass (its cell
// expansions are complete) and after its leaf translation (before its disaggregation).
struct BandHooks {
    std::function<int()> after_m2m, after_leaf;
};

template <class T, int D, int HMAX>
int run_band(const Work<T> &w, hipStream_t s, hipEvent_t join, BandTimer &bt, const BandHooks *hk) {
    int64_t nb[PH_COUNT];
    for (int k = 0; k < PH_COUNT; ++k) nb[k] = phase_blocks<T>(w.one, k);
    const size_t sh = p2m_shmem<T>(w.one, D);
    const int kernel = RBF_GAUSSIAN;   // unused by the far-field phases
    RBF_HIP(bt.begin(2, s));
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_PHASE_DL, nb[PH_PHASE_DL], s, 0, 0, kernel)));
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_P2M, nb[PH_P2M], s, 0, sh, kernel)));
    RBF_HIP(bt.end());
    RBF_HIP(bt.begin(3, s));
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_M2M, nb[PH_M2M], s, 0, 0, kernel)));
    if (hk) RBF_TRY(hk->after_m2m());
    RBF_HIP(bt.end());
    RBF_HIP(bt.begin(4, s));
    for (int ax = 0; ax < D; ++ax)
        RBF_TRY((launch_phase<T, D, HMAX>(w, PH_M2L_AXIS, nb[PH_M2L_AXIS], s, ax, 0, kernel)));
    RBF_HIP(bt.end());
    RBF_HIP(bt.begin(5, s));
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_M2L_LEAF, nb[PH_M2L_LEAF], s, 0, 0, kernel)));
    if (hk) RBF_TRY(hk->after_leaf());
    RBF_HIP(bt.end());
    if (join) RBF_HIP(hipStreamWaitEvent(s, join, 0));   // u_s holds the near field from here on
    RBF_HIP(bt.begin(6, s));
    RBF_TRY((launch_phase<T, D, HMAX>(w, PH_L2P, nb[PH_L2P], s, 0, 0, kernel)));
    RBF_HIP(bt.end());
    return RBF_OK;
}

template <class T, int D>
int run_band_hp(int HP, const Work<T> &w, hipStream_t s, hipEvent_t join, BandTimer &bt, const BandHooks *hk) {
    switch (HP) {
        case 4: return run_band<T, D, 4>(w, s, join, bt, hk);
        case 6: return run_band<T, D, 6>(w, s, join, bt, hk);
        case 8: return run_band<T, D, 8>(w, s, join, bt, hk);
        case 10: return run_band<T, D, 10>(w, s, join, bt, hk);
        case 12: return run_band<T, D, 12>(w, s, join, bt, hk);
        case 14: return run_band<T, D, 14>(w, s, join, bt, hk);
        case 16: return run_band<T, D, 16>(w, s, join, bt, hk);
        case 20: return run_band<T, D, 20>(w, s, join, bt, hk);
        case 24: return run_band<T, D, 24>(w, s, join, bt, hk);
        case 28: return run_band<T, D, 28>(w, s, join, bt, hk);
        case 32: return run_band<T, D, 32>(w, s, join, bt, hk);
    }
    set_error("padded half grid %d not compiled for banded products", HP);
    return RBF_EUNSUPPORTED;
}

template <class T, int D>
int banded_matvec_d(rbf_plan *p, const T *lam, T *u) {
    Work<T> w{};
    fill_desc<T>(p, &w.one);
    w.one.far = 1;   // the near field writes u_s, which the bands complete
    w.one.res_tab = p->res_tab;
    w.one.res_inv = p->res_inv;
    w.one.res_cut2 = p->res_qmax;
    w.lam = lam;
    w.u = u;
    const hipStream_t s = p->stream;
    ensure_side_stream(p);
    ProductRun pt(p, p->side_state == 1);
    BandTimer bt(p);
    RBF_HIP(pt.begin(0, s));
    RBF_TRY((launch_phase<T, D, 4>(w, PH_GATHER, phase_blocks<T>(w.one, PH_GATHER), s, 0, 0, p->kernel)));
    RBF_HIP(pt.end());
    hipStream_t sn = s;
    if (pt.side) {
        RBF_HIP(hipEventRecord(pt.fork, s));
        RBF_HIP(hipStreamWaitEvent(pt.side, pt.fork, 0));
        sn = pt.side;
    }
    const int rk = p->res_q ? kResTabQ : p->kernel == RBF_INVERSE_MULTIQUADRIC ? kResTabDiv : kResTab;
    RBF_HIP(pt.begin(1, sn));
    if (pt.side)
        RBF_TRY((launch_p2p_queue<T, D>(w, sn, rk)));
    else
        RBF_TRY((launch_phase<T, D, 4>(w, PH_P2P, phase_blocks<T>(w.one, PH_P2P), sn, 0, 0, rk)));
    RBF_HIP(pt.end());
    if (pt.side) RBF_HIP(hipEventRecord(pt.join, sn));
    const int nbands = (int)p->bands.size();
    int last = -1;   // the last band with a run of its own writes u through the permutation
    for (int j = 0; j < nbands; ++j)
        if (!p->bands[j].xfer) last = j;
    BandHooks hooks;
    if (p->xfer_src >= 0) {
        const Band &S = p->bands[p->xfer_src];
        const size_t csz = sizeof(typename cplx<T>::type);
        hooks.after_m2m = [p, &S, s, csz]() -> int {
            // the source's cell expansions, before the stencil passes reuse the buffer
            RBF_HIP(hipMemcpyAsync(p->xfer_keep, p->bWc, csz * (size_t)S.ncells * S.P, hipMemcpyDeviceToDevice, s));
            return RBF_OK;
        };
        hooks.after_leaf = [p, &S, s]() -> int {
            for (const Xfer &x : p->xfers)
                RBF_TRY(xfer_band<T>(p, x, S, p->bands[x.band], p->xfer_keep, p->bLx, s));
            return RBF_OK;
        };
    }
    bool first = true;
    for (int j = 0; j < nbands; ++j) {
        if (p->bands[j].xfer) continue;
        Work<T> wb{};
        fill_band_desc<T>(p, p->bands[j], j != last, &wb.one);
        wb.lam = lam;
        wb.u = u;
        bt.j = j;
        RBF_TRY((run_band_hp<T, D>(p->bands[j].HP, wb, s, (first && pt.side) ? pt.join : nullptr, bt,
                                   j == p->xfer_src ? &hooks : nullptr)));
        first = false;
    }
    if (p->profiling) {
        // phases 0 and 1 from the plan's events, 2..6 summed over the bands
        RBF_HIP(hipStreamSynchronize(s));   // every recorded event (transferred bands record none)
        RBF_HIP(hipEventSynchronize(p->ev[3]));
        for (int k = 0; k < 2; ++k) {
            float ms = 0.f;
            RBF_HIP(hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]));
            p->phase_ms[k] += ms;
        }
        for (int j = 0; j < nbands; ++j)
            for (int k = 2; k < RBF_NPHASES && !p->bands[j].xfer; ++k) {
                float ms = 0.f;
                RBF_HIP(hipEventElapsedTime(&ms, p->band_ev[(size_t)(j * RBF_NPHASES + k) * 2],
                                            p->band_ev[(size_t)(j * RBF_NPHASES + k) * 2 + 1]));
                p->phase_ms[k] += ms;
            }
        p->prof_calls += 1;
    }
    return RBF_OK;
}

template <class T>
int banded_matvec_t(rbf_plan *p, const void *lam, void *u) {
    if (p->profiling && p->band_ev.size() != p->bands.size() * 2 * RBF_NPHASES) {
        for (hipEvent_t e : p->band_ev) (void)hipEventDestroy(e);
        p->band_ev.assign(p->bands.size() * 2 * RBF_NPHASES, nullptr);
        for (hipEvent_t &e : p->band_ev) RBF_HIP(hipEventCreate(&e));
    }
    switch (p->d) {
        case 2: return banded_matvec_d<T, 2>(p, (const T *)lam, (T *)u);
        case 3: return banded_matvec_d<T, 3>(p, (const T *)lam, (T *)u);
    }
    set_error("banded products are compiled for d = 2 and 3, not %d", p->d);
    return RBF_EUNSUPPORTED;
}

}  // namespace

// Aggregation launch shape: rows per workgroup, and per point of a chunk the factors of the
// d-1 leading dimensions (plus, on the matrix cores, the point's HP phases) in LDS.
template <class T> void set_p2m_shape(Desc<T> *d, int dim, int64_t R, int mn, int HP) {
    using C = typename cplx<T>::type;
    const int rows = kExpMfma<T> ? p2m_rows(dim) : (dim > 2 ? kThreads : kWave);
    d->wpl = (int)((R + rows - 1) / rows);
    const size_t per_point = sizeof(C) * (size_t)((dim > 1 ? dim - 1 : 1) * mn + (kExpMfma<T> ? HP : 0));
    d->p2m_ch = (int)std::max<size_t>(4, std::min<size_t>(64, (32 * 1024) / per_point)) & ~1;
    d->p2m_lds = (int)(per_point * d->p2m_ch);
}

template <class T> void fill_desc(const rbf_plan *p, Desc<T> *d) {
    using C = typename cplx<T>::type;
    d->xs = (const T *)p->xs;
    d->n = p->n;
    d->off = 0;
    d->perm = p->perm;
    d->leaf_begin = p->leaf_begin;
    d->src_end = p->src_end ? p->src_end : p->leaf_begin + 1;
    d->leaf_cell = p->leaf_cell;
    d->near_ptr = p->near_ptr;
    d->near_idx = p->near_idx;
    d->src_ptr = p->src_ptr;
    d->cell_begin = p->cell_leaf_begin;
    d->src_rng = p->src_rng;
    d->tasks = p->tasks;
    d->ptasks = p->ptasks;
    d->nptasks = p->nptasks;
    d->nleaves = p->nleaves;
    d->ntasks = p->ntasks;
    d->ncells = p->ncells;
    d->lc = p->lc;
    d->r = p->r;
    d->mn = p->mn;
    d->H = p->H;
    d->HP = p->HP;
    d->R = (int)p->R;
    d->P = p->P;
    const double dxi = 2.0 * p->sigma / (p->mn - 1);
    d->dxi = dxi;
    d->xi0 = -p->sigma;
    d->xiH = -p->sigma + p->H * dxi;
    d->wc1 = p->wc1;
    if (p->kernel == RBF_GAUSSIAN)
        d->coef = (T)(-1.4426950408889634 / (2.0 * p->shape * p->shape));
    else if (p->kernel == RBF_WENDLAND)
        d->coef = (T)p->shape;
    else
        d->coef = (T)(p->shape * p->shape);
    d->lam_s = (T *)p->lam_s;
    d->u_s = (T *)p->u_s;
    d->W = (C *)p->W;
    d->Lx = (C *)p->Lx;
    d->Wc = (C *)p->Wc;
    d->Lc = (C *)p->Lc;
    d->Tmp = (C *)p->Tmp;
    d->dl = (C *)p->dl;
    d->wtab = p->wtab;
    d->m2l_sched = p->m2l_sched;
    set_p2m_shape<T>(d, p->d, p->R, p->mn, p->HP);
    d->far = p->far;
    d->dim = p->d;
    d->ngroups = p->ngroups;
    d->grp_first = p->grp_first;
    d->uni_ptr = p->uni_ptr;
    d->uni_idx = p->uni_idx;
    d->uni_mask = p->uni_mask;
    d->mn_magic = (unsigned)((1ull << 32) / (unsigned)p->mn + 1);
    d->p2m_begin = d->leaf_begin;
    d->p2m_end = d->src_end;
    d->p2m_n = p->nleaves;
    d->l2p_acc = 0;
    d->p2p_ctr = p->p2p_ctr;
    d->res_tab = nullptr;
    d->res_inv = d->res_cut2 = 0.0;
    d->dir_t0 = 0;
    d->dir_ns = p->n;
    d->bl_lds = 0;
    if (p->kernel == RBF_GAUSSIAN_BANDLIMITED) {
        // the per-axis table: pieces per unit t as coef, the last piece in res_cut2
        d->coef = (T)p->bl_inv;
        d->res_tab = p->bl_tab;
        d->res_cut2 = p->bl_pieces - 1;
        d->bl_lds = sizeof(T) * (size_t)p->bl_pieces * kBlLds<T> <= (size_t)kBlLdsBytes ? 1 : 0;
    }
}
template void fill_desc<float>(const rbf_plan *, Desc<float> *);
template void fill_desc<double>(const rbf_plan *, Desc<double> *);

template <class T> int64_t desc_blocks(const Desc<T> &d, int phase) { return phase_blocks<T>(d, phase); }
template int64_t desc_blocks<float>(const Desc<float> &, int);
template int64_t desc_blocks<double>(const Desc<double> &, int);

// Batched product for one group of problems sharing (d, HP, kernel): descriptors and
// per-phase block prefixes are device arrays prepared by the batch planner.
template <class T>
int launch_batch_group(int d, int HP, int kernel, const Desc<T> *descs, int nprob, const int *const *bstarts,
                       const int64_t *nblocks, size_t p2m_sh, const T *lam, T *u, hipStream_t s) {
    Work<T> w{};
    w.many = descs;
    w.nprob = nprob;
    w.lam = lam;
    w.u = u;
    ProductRun pt(nullptr, false);
    return product_t<T>(d, HP, w, nblocks, bstarts, p2m_sh, kernel, s, pt);
}
template int launch_batch_group<float>(int, int, int, const Desc<float> *, int, const int *const *, const int64_t *,
                                       size_t, const float *, float *, hipStream_t);
template int launch_batch_group<double>(int, int, int, const Desc<double> *, int, const int *const *,
                                        const int64_t *, size_t, const double *, double *, hipStream_t);

// A plan of one leaf without a far field (the autotuner's direct choice, the multiquadric) is the
// exact sum over all pairs; the tiled direct kernel computes it faster than the near-field
// kernel, whose waves would each stream the whole point set through scalar loads.  With
// profiling the whole sum counts as the near field.  A one-leaf plan for separate targets
// takes it too, pairing its targets with its sources only (direct_d).
int direct_product(rbf_plan *p, const void *lambda, void *u) {
    hipStream_t s = p->stream;
    if (p->profiling)
        for (int k = 0; k < 3; ++k) RBF_HIP(hipEventRecord(p->ev[k], s));
    RBF_TRY(p->dtype == RBF_F32 ? direct_t<float>(p, lambda, u) : direct_t<double>(p, lambda, u));
    if (p->profiling) {
        for (int k = 3; k < 2 * RBF_NPHASES; ++k) RBF_HIP(hipEventRecord(p->ev[k], s));
        RBF_TRY(add_phase_times(p));
    }
    return RBF_OK;
}

int launch_matvec_phases(rbf_plan *p, const void *lambda, void *u) {
    return p->dtype == RBF_F32 ? matvec_t<float>(p, lambda, u) : matvec_t<double>(p, lambda, u);
}

int launch_matvec(rbf_plan *p, const void *lambda, void *u) {
    if (!p->bands.empty())
        return p->dtype == RBF_F32 ? banded_matvec_t<float>(p, lambda, u) : banded_matvec_t<double>(p, lambda, u);
    if (p->nleaves == 1 && !p->far) return direct_product(p, lambda, u);
    return launch_matvec_phases(p, lambda, u);
}

int launch_direct(rbf_plan *p, const void *lambda, void *u) {
    return p->dtype == RBF_F32 ? direct_t<float>(p, lambda, u) : direct_t<double>(p, lambda, u);
}

}  // namespace rbf

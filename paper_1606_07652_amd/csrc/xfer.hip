// Transfer of expansions between the frequency grids of two bands (section 4.1: the
// interpolating multilevel scheme moves a box's expansion to another level's nodes by local
// Lagrange interpolation of e^{i xi (x - c)} in xi, and back by the transposed map,
// eq. 43-48 and 53).
//
// Setting (banded far field): a source band S whose aggregation runs over the cells of a
// transfer level l_I, and target bands T whose own grids have smaller band limits.  For a cell
// c (centre c_c) the centred expansion V_c(xi) = e^{i xi.c_c} W_c(xi) is a smooth function of
// xi (its points lie within half a cell of c_c), so its values at T's nodes follow from S's
// nodes by a K-point Lagrange stencil along each axis:
//   up:    W_T(eta) = sum_c e^{-i eta.c_c} sum_xi prod_k l_{xi_k}(eta_k) e^{i xi.c_c} W_S,c(xi)
//          (summed over the cells: the target bands are level-0 bands, one expansion for all);
//   down:  the local expansion L_T(eta) acts on a point x of cell c through e^{i eta.x}; with
//          e^{i eta (x - c)} ~ sum_xi l_xi(eta) e^{i xi (x - c)} it becomes S's local expansion
//          A_c(xi) = e^{-i xi.c_c} sum_eta prod_k l_{xi_k}(eta_k) e^{i eta.c_c} L_T(eta),
//          added to the cell's own local expansion before S's disaggregation.
// Expansions hold the half grid: every axis but the last in full, the last from its positive
// nodes (index H..Mn-1), the rest by W(-xi) = conj W(xi) (real weights).  Per-cell tensors are
// laid out [cell][m_0]..[m_{d-2}][h] (m_{d-2} fastest among the rows, h fastest overall).  The
// 1-D maps are CSR tables (output index -> (input index, weight)); every output sums its
// entries in table order, so the transfer is deterministic.
#include "internal.h"

namespace rbf {
namespace {

constexpr int kT = 256;

template <class T> struct cx { using type = float2; };
template <> struct cx<double> { using type = double2; };

template <class C> __device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class C> __device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }

// phase of the row `row` (indices over the first d-1 axes, grid of mn nodes) and last-axis
// node j (full index): prod_k E[k][m_k], E = the cell's per-axis table [d][mn]
__device__ __forceinline__ double2 row_phase(const double2 *E, int d, int mn, int64_t row, int j) {
    double2 ph = E[(int64_t)(d - 1) * mn + j];
    int64_t rr = row;
    for (int k = d - 2; k >= 0; --k) {
        const int m = (int)(rr % mn);
        rr /= mn;
        ph = cmul(ph, E[(int64_t)k * mn + m]);
    }
    return ph;
}

// mirror of a row (every index m_k -> n - 1 - m_k) on a grid with n nodes per axis
__device__ __forceinline__ int64_t mirror_row(int64_t row, int d, int n) {
    int64_t out = 0, rr = row, scale = 1;
    for (int k = d - 2; k >= 0; --k) {
        const int m = (int)(rr % n);
        rr /= n;
        out += (int64_t)(n - 1 - m) * scale;
        scale *= n;
    }
    return out;
}

// out[c][row][h] = phase(c, row, H + h) * in[c or 0][row][h]; conj_phase: use e^{-i...};
// in_stride 0: the same input for every cell
template <class T>
__global__ void __launch_bounds__(kT) k_xphase(const typename cx<T>::type *__restrict__ in, int64_t in_stride,
                                               typename cx<T>::type *__restrict__ out, const double2 *__restrict__ E,
                                               int ncell, int d, int mn, int H, int conj_phase) {
    using C = typename cx<T>::type;
    int64_t R = 1;
    for (int k = 0; k < d - 1; ++k) R *= mn;
    const int64_t P = R * H;
    const int64_t g = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (g >= P * ncell) return;
    const int64_t c = g / P, p = g - c * P;
    const int64_t row = p / H;
    const int h = (int)(p - row * H);
    double2 ph = row_phase(E + (int64_t)c * d * mn, d, mn, row, H + h);
    if (conj_phase) ph.y = -ph.y;
    const C v = in[c * in_stride + p];
    const double re = ph.x * (double)v.x - ph.y * (double)v.y, im = ph.x * (double)v.y + ph.y * (double)v.x;
    out[g] = C{(T)re, (T)im};
}

// Last axis, up: in [c][rows (n per axis)][Hs] (source stored half) -> out [c][rows][Ht],
// out[.][h'] = sum_e w_e Vfull[.][idx_e], Vfull[row][j] = V[row][j - Hs] (j >= Hs), else
// conj V[mirror row][mns - 1 - j - Hs]
template <class T>
__global__ void __launch_bounds__(kT) k_xup_last(const typename cx<T>::type *__restrict__ in,
                                                 typename cx<T>::type *__restrict__ out, int ncell, int d, int n,
                                                 int mns, int Hs, int Ht, const int *__restrict__ ptr,
                                                 const int *__restrict__ idx, const double *__restrict__ w) {
    using C = typename cx<T>::type;
    int64_t R = 1;
    for (int k = 0; k < d - 1; ++k) R *= n;
    const int64_t Po = R * Ht, Pi = R * Hs;
    const int64_t g = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (g >= Po * ncell) return;
    const int64_t c = g / Po, p = g - c * Po;
    const int64_t row = p / Ht;
    const int h = (int)(p - row * Ht);
    const int64_t mrow = mirror_row(row, d, n);
    const C *src = in + c * Pi;
    double re = 0, im = 0;
    for (int e = ptr[h]; e < ptr[h + 1]; ++e) {
        const int j = idx[e];
        C v;
        if (j >= Hs) v = src[row * Hs + (j - Hs)];
        else v = cconj(src[mrow * Hs + (mns - 1 - j - Hs)]);
        re += w[e] * (double)v.x;
        im += w[e] * (double)v.y;
    }
    out[g] = C{(T)re, (T)im};
}

// One axis k < d - 1 of a per-cell tensor with dims (n_0 .. n_{d-2}, NH): the axis goes from
// nin to nout nodes through the CSR map.  dims_in[k'] for every k' (the mapped axis holds nin).
template <class T>
__global__ void __launch_bounds__(kT) k_xaxis(const typename cx<T>::type *__restrict__ in,
                                              typename cx<T>::type *__restrict__ out, int ncell, int d, int4 dims_lo,
                                              int NH, int axis, int nout, const int *__restrict__ ptr,
                                              const int *__restrict__ idx, const double *__restrict__ w) {
    using C = typename cx<T>::type;
    int din[4] = {dims_lo.x, dims_lo.y, dims_lo.z, dims_lo.w};   // the first d - 1 dims (input)
    int64_t Pi = NH, Po = NH;
    for (int k = 0; k < d - 1; ++k) {
        Pi *= din[k];
        Po *= (k == axis ? nout : din[k]);
    }
    const int64_t g = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (g >= Po * ncell) return;
    const int64_t c = g / Po;
    int64_t p = g - c * Po;
    // strides of the input along the mapped axis, and the output index split at it
    int64_t inner = NH;   // product of the dims after `axis` (input = output there)
    for (int k = axis + 1; k < d - 1; ++k) inner *= din[k];
    const int64_t lo = p % inner;
    p /= inner;
    const int o = (int)(p % nout);
    const int64_t hi = p / nout;
    const int64_t base = (hi * din[axis]) * inner + lo;
    const C *src = in + c * Pi;
    double re = 0, im = 0;
    for (int e = ptr[o]; e < ptr[o + 1]; ++e) {
        const C v = src[base + (int64_t)idx[e] * inner];
        re += w[e] * (double)v.x;
        im += w[e] * (double)v.y;
    }
    out[g] = C{(T)re, (T)im};
}

// L[p] = wtab[p] * sum_c conj(phase(c, p)) U[c][p] over the target's stored half, cells in order
template <class T>
__global__ void __launch_bounds__(kT) k_xroot(const typename cx<T>::type *__restrict__ U, const double2 *__restrict__ E,
                                              int ncell, int d, int mn, int H, const double *__restrict__ wtab,
                                              typename cx<T>::type *__restrict__ L) {
    using C = typename cx<T>::type;
    int64_t R = 1;
    for (int k = 0; k < d - 1; ++k) R *= mn;
    const int64_t P = R * H;
    const int64_t p = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (p >= P) return;
    const int64_t row = p / H;
    const int h = (int)(p - row * H);
    double re = 0, im = 0;
    for (int c = 0; c < ncell; ++c) {
        const double2 ph = row_phase(E + (int64_t)c * d * mn, d, mn, row, H + h);
        const C v = U[(int64_t)c * P + p];
        // conj(ph) * v
        re += ph.x * (double)v.x + ph.y * (double)v.y;
        im += ph.x * (double)v.y - ph.y * (double)v.x;
    }
    const double f = wtab[p];
    L[p] = C{(T)(f * re), (T)(f * im)};
}

// Last axis, down: in [c][rows (n per axis)][Ht] -> the source's stored half,
// A[h] = sum_e w_e Xfull[idx_e], Xfull[row][i] = X[row][i - Ht] (i >= Ht), else
// conj X[mirror row][mnt - 1 - i - Ht]; times conj(phase_S(c, row, Hs + h)), added to
// Lx[unit(c)][row][HP] (cells without a unit are skipped)
template <class T>
__global__ void __launch_bounds__(kT) k_xdown_last(const typename cx<T>::type *__restrict__ in, int ncell, int d,
                                                   int n, int mnt, int Ht, int Hs, int HP, const int *__restrict__ ptr,
                                                   const int *__restrict__ idx, const double *__restrict__ w,
                                                   const double2 *__restrict__ Es, const int *__restrict__ cell_unit,
                                                   typename cx<T>::type *__restrict__ Lx) {
    using C = typename cx<T>::type;
    int64_t R = 1;
    for (int k = 0; k < d - 1; ++k) R *= n;
    const int64_t Po = R * Hs, Pi = R * Ht;
    const int64_t g = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (g >= Po * ncell) return;
    const int64_t c = g / Po, p = g - c * Po;
    const int unit = cell_unit[c];
    if (unit < 0) return;
    const int64_t row = p / Hs;
    const int h = (int)(p - row * Hs);
    const int64_t mrow = mirror_row(row, d, n);
    const C *src = in + c * Pi;
    double re = 0, im = 0;
    for (int e = ptr[h]; e < ptr[h + 1]; ++e) {
        const int i = idx[e];
        C v;
        if (i >= Ht) v = src[row * Ht + (i - Ht)];
        else v = cconj(src[mrow * Ht + (mnt - 1 - i - Ht)]);
        re += w[e] * (double)v.x;
        im += w[e] * (double)v.y;
    }
    const double2 ph = row_phase(Es + (int64_t)c * d * n, d, n, row, Hs + h);
    const double ar = ph.x * re + ph.y * im, ai = ph.x * im - ph.y * re;   // conj(ph) * (re, im)
    C *dst = Lx + ((int64_t)unit * R + row) * HP + h;
    const C old = *dst;
    *dst = C{(T)((double)old.x + ar), (T)((double)old.y + ai)};
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

template <class T>
int xfer_band(const rbf_plan *p, const Xfer &x, const Band &S, const Band &Tb, const void *wc_keep, void *lx_s,
              hipStream_t s) {
    using C = typename cx<T>::type;
    const int d = p->d, nc = p->xfer_ncell;
    const int mns = S.mn, Hs = S.H, mnt = Tb.mn, Ht = Tb.H;
    C *X1 = (C *)p->xfer_x1, *X2 = (C *)p->xfer_x2, *L = (C *)p->xfer_l;
    int64_t rs = 1, rt = 1;
    for (int k = 0; k < d - 1; ++k) {
        rs *= mns;
        rt *= mnt;
    }
    // up: centred source expansions, last axis to the target's stored half, then the others
    k_xphase<T><<<blocks_of(rs * Hs * nc), kT, 0, s>>>((const C *)wc_keep, rs * Hs, X1, p->xfer_phase_s, nc, d, mns,
                                                       Hs, 0);
    RBF_HIP(hipGetLastError());
    k_xup_last<T><<<blocks_of(rs * Ht * nc), kT, 0, s>>>(X1, X2, nc, d, mns, mns, Hs, Ht, x.upl_ptr, x.upl_idx,
                                                         x.upl_w);
    RBF_HIP(hipGetLastError());
    int dims[4] = {mns, mns, mns, mns};
    C *a = X2, *b = X1;
    for (int k = 0; k < d - 1; ++k) {
        int64_t po = Ht;
        for (int q = 0; q < d - 1; ++q) po *= (q == k ? mnt : dims[q]);
        k_xaxis<T><<<blocks_of(po * nc), kT, 0, s>>>(a, b, nc, d, int4{dims[0], dims[1], dims[2], dims[3]}, Ht, k,
                                                     mnt, x.up_ptr, x.up_idx, x.up_w);
        RBF_HIP(hipGetLastError());
        dims[k] = mnt;
        std::swap(a, b);
    }
    k_xroot<T><<<blocks_of(rt * Ht), kT, 0, s>>>(a, x.phase_t, nc, d, mnt, Ht, Tb.wtab, L);
    RBF_HIP(hipGetLastError());
    // down: the target's local expansion at every cell centre, the axes back to the source's
    // grid, the last axis to the source's stored half, added to the cells' local expansions
    k_xphase<T><<<blocks_of(rt * Ht * nc), kT, 0, s>>>(L, 0, X1, x.phase_t, nc, d, mnt, Ht, 0);
    RBF_HIP(hipGetLastError());
    for (int k = 0; k < 4; ++k) dims[k] = mnt;
    a = X1;
    b = X2;
    for (int k = 0; k < d - 1; ++k) {
        int64_t po = Ht;
        for (int q = 0; q < d - 1; ++q) po *= (q == k ? mns : dims[q]);
        k_xaxis<T><<<blocks_of(po * nc), kT, 0, s>>>(a, b, nc, d, int4{dims[0], dims[1], dims[2], dims[3]}, Ht, k,
                                                     mns, x.dn_ptr, x.dn_idx, x.dn_w);
        RBF_HIP(hipGetLastError());
        dims[k] = mns;
        std::swap(a, b);
    }
    k_xdown_last<T><<<blocks_of(rs * Hs * nc), kT, 0, s>>>(a, nc, d, mns, mnt, Ht, Hs, S.HP, x.dnl_ptr, x.dnl_idx,
                                                           x.dnl_w, p->xfer_phase_s, p->xfer_cell_unit, (C *)lx_s);
    RBF_HIP(hipGetLastError());
    return RBF_OK;
}

template int xfer_band<float>(const rbf_plan *, const Xfer &, const Band &, const Band &, const void *, void *,
                              hipStream_t);
template int xfer_band<double>(const rbf_plan *, const Xfer &, const Band &, const Band &, const void *, void *,
                               hipStream_t);

}  // namespace rbf

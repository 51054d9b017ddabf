// Banded far field of the multiquadric kernels: planning (host).
//
// The multiquadric sqrt(r^2 + c^2) and the inverse multiquadric 1/sqrt(r^2 + c^2) (the
// paper's table of global functions) do not decay, or decay like a power, so no single band
// limit serves every separation.  The paper's multilevel method gives every level its own
// band limit, scaled with the level's box size (section 4.1, the scaling lemma), and builds
// the translation factor C from samples of the kernel (section 3.2, eq. "M2Loperator").
// Here the scales are separated in the kernel itself: both kernels are superpositions of
// Gaussians exp(-b^2 / (2 s^2)), b = sqrt(r^2 + c^2), over the width s,
//     sqrt(b^2) = c + sqrt(2/pi) int_0^inf [exp(-c^2/(2 s^2)) - exp(-b^2/(2 s^2))] ds,
//     1 / b     = sqrt(2/pi) int_0^inf s^-2 exp(-b^2/(2 s^2)) ds,
// and cutting the width axis at s_0 < s_1 < ... < s_J gives
//   * the residual (widths below s_0): short-range, summed directly over the adjacent cells
//     of a uniform tree whose cells are wide enough for it to vanish beyond them;
//   * bands j (widths in [s_j, s_{j+1}), ratio sqrt 2): Gaussian mixtures, smooth on the
//     scale s_j and decaying like a Gaussian of width s_{j+1}; each gets the band limit,
//     period, coarse stencil and node count that the Gaussian far field would get for those
//     widths, and its C from the DFT of its samples;
//   * the top band (widths from s_J = 2 ext on): smooth on the scale of the domain, not
//     decaying; windowed by erfc steps per axis (1 inside the bounding cube, negligible at
//     the half period) and expanded on one grid over the whole domain.
// The quadrature kernel of a grid with an even node count is anti-periodic (period L per axis);
// a band's samples are those of its anti-periodisation (the sum over its images one period
// apart with alternating signs), so that the DFT gives exactly the coefficients of the
// function the quadrature kernel reproduces.
// The sum of the pieces is the kernel exactly; each piece is approximated to a tolerance
// that splits the requested relative error over the pieces by their size.
// Interpolating transfers (section 4.1): the coarsest bands (the whole domain as one cell)
// would each aggregate and disaggregate every point on their own grid.  Instead the first of
// them (the source) aggregates over the cells of a transfer level, and the others take their
// expansions from its cell expansions by K-point Lagrange interpolation in the frequency
// variable and return their local expansions by the transposed map (xfer.hip); K per band is
// the smallest whose interpolation error, evaluated here on the host over the cells' extent,
// is below the band's tolerance / (20 d).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace rbf {

double band_limit_t(double tol);   // api.hip: s sigma with erfc(s sigma / sqrt 2) = tol / 4

bool banded_kernel(int kernel, int d) {
    return (kernel == RBF_MULTIQUADRIC || kernel == RBF_INVERSE_MULTIQUADRIC) && (d == 2 || d == 3);
}

namespace {

constexpr double kSq2pi = 0.79788456080286535588;   // sqrt(2 / pi)
constexpr double kRatio = 1.41421356237309504880;   // width ratio of consecutive band edges
// node counts with a compiled half grid (HP = mn / 2, no padding of the local expansions)
constexpr int kBandNodes[] = {8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64};

int round_nodes(int mn) {
    for (int v : kBandNodes)
        if (v >= mn) return v;
    return 0;
}

// antiderivative in s of exp(-b^2 / (2 s^2))
double G(double s, double b) {
    return s * std::exp(-b * b / (2.0 * s * s)) - b * std::sqrt(M_PI / 2.0) * std::erfc(b / (std::sqrt(2.0) * s));
}

double band_value(int kernel, double b, double lo, double hi) {
    if (kernel == RBF_MULTIQUADRIC) return -kSq2pi * (G(hi, b) - G(lo, b));
    const double r2 = std::sqrt(2.0);
    return (std::erf(b / (r2 * lo)) - std::erf(b / (r2 * hi))) / b;
}

double top_value(int kernel, double b, double st) {
    const double x = b / (std::sqrt(2.0) * st);
    if (kernel == RBF_MULTIQUADRIC) return b * std::erf(x) + kSq2pi * st * std::exp(-x * x);
    return std::erf(x) / b;
}

double kernel_value(int kernel, double r2, double c) {
    return kernel == RBF_MULTIQUADRIC ? std::sqrt(r2 + c * c) : 1.0 / std::sqrt(r2 + c * c);
}

// window of the top band along one axis: 1 to within erfc(k)/2 on |t| <= ext (7.7e-9 at the
// k = 4 of tolerances from 1e-6 up; the plan raises k for tighter ones), below 1e-12 from
// |t| = ext + (k + 5) tau on (the half period)
double window(double t, double ext, double tau, double k) {
    return 0.5 * std::erfc((std::fabs(t) - (ext + k * tau)) / tau);
}

// Root-mean-square of the kernel over all pairs of an evenly spaced sample of the points
// (at most 2048 of them, in Morton order): the scale against which the tolerance is split.
// The same pairs give the distribution of pair distances (p->pair_cdf, log-spaced bins).
int kernel_rms(rbf_plan *p, double *rms) {
    const int64_t n = p->n;
    const int d = p->d;
    const int m = (int)std::min<int64_t>(n, 2048);
    const size_t tsz = p->dtype == RBF_F32 ? 4 : 8;
    std::vector<char> buf((size_t)n * tsz);
    std::vector<double> x((size_t)m * d);
    for (int k = 0; k < d; ++k) {
        RBF_HIP(hipMemcpy(buf.data(), (const char *)p->xs + (size_t)k * n * tsz, (size_t)n * tsz, hipMemcpyDeviceToHost));
        for (int i = 0; i < m; ++i) {
            const int64_t j = (int64_t)((double)i * n / m);
            x[(size_t)i * d + k] = p->dtype == RBF_F32 ? (double)((const float *)buf.data())[j]
                                                       : ((const double *)buf.data())[j];
        }
    }
    double acc = 0;
    // pair distances in log-spaced bins (kPairBins per factor 2, from ext / 2^40 up)
    std::vector<double> hist(kPairBinsTotal + 1, 0.0);
    const double rlo = p->ext * std::ldexp(1.0, -40);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double r2 = 0;
            for (int k = 0; k < d; ++k) {
                const double t = x[(size_t)i * d + k] - x[(size_t)j * d + k];
                r2 += t * t;
            }
            const double v = kernel_value(p->kernel, r2, p->shape);
            acc += v * v;
            const double r = std::sqrt(r2);
            const double t = r <= rlo ? -1.0 : std::log2(r / rlo) * kPairBins;
            const int b = !(t >= 0.0) ? 0 : t >= kPairBinsTotal - 1 ? kPairBinsTotal : 1 + (int)t;   // NaN: bin 0
            hist[b] += 1.0;
        }
    *rms = std::sqrt(acc / ((double)m * m));
    p->pair_cdf.assign(kPairBinsTotal + 1, 0.0);
    double c = 0;
    for (int b = 0; b <= kPairBinsTotal; ++b) { c += hist[b]; p->pair_cdf[b] = c / ((double)m * m); }
    p->pair_rlo = rlo;
    p->pair_min = 1.0 / m;
    return RBF_OK;
}

// Fraction of the sampled pairs (self pairs included) closer than R, from the histogram: the
// upper edge of R's bin, so never below the true fraction.
double pair_fraction(const rbf_plan *p, double R) {
    if (p->pair_cdf.empty() || !(p->pair_rlo > 0.0)) return 1.0;   // no sample, or all points equal
    if (R <= p->pair_rlo) return std::max(p->pair_cdf[0], p->pair_min);
    const double t = std::log2(R / p->pair_rlo) * kPairBins;
    const int b = !(t < kPairBinsTotal - 1) ? kPairBinsTotal : 1 + (int)t;   // NaN: the last bin
    return std::max(p->pair_cdf[b], p->pair_min);
}

// w(xi) C(xi) for the stored nodes of a band: C from the DFT of the band's samples over one
// period (eq. "M2Loperator" in physical units: C(xi) = (h / 2 pi)^d sum_q K(q h) e^{-i h q.xi},
// h = pi / sigma, the mn - 1 offsets q = -(mn-2)/2 .. (mn-2)/2 per axis), with K even in every
// coordinate so that the DFT is a cosine transform along each axis; times the tensor
// trapezoid weights.  Stored nodes: row digits m_1..m_{d-1} (any order: K is symmetric under
// permutations of the axes, so C is too) and m_d = H + h.
std::vector<double> band_table(const rbf_plan *p, const Band &b) {
    const int d = p->d, mn = b.mn, Q = mn - 1;
    const double dxi = 2.0 * b.sigma / (mn - 1);
    const double h = M_PI / b.sigma;
    std::vector<double> qx(Q), xi(mn), w(mn);
    for (int i = 0; i < Q; ++i) qx[i] = (i - (mn - 2) / 2) * h;
    for (int m = 0; m < mn; ++m) {
        xi[m] = -b.sigma + m * dxi;
        w[m] = (m == 0 || m == mn - 1) ? 0.5 * dxi : dxi;
    }
    // samples of the piece the quadrature kernel reproduces.  With an even node count the
    // nodes are odd multiples of dxi / 2, so e^{i xi (r + L)} = -e^{i xi r}: the kernel is
    // anti-periodic with period L along every axis (the (-1)^n of the Poisson sum).  A band
    // is therefore summed over its images r + n L with the sign prod_k (-1)^{n_k}, within its
    // reach (a coarse band's period can be shorter than its decay); the windowed top band
    // vanishes beyond the half period and is sampled as it is.
    int64_t nq = 1;
    for (int k = 0; k < d; ++k) nq *= Q;
    std::vector<double> K(nq);
    const double c = p->shape, L = b.L;
    const int nimg = b.top ? 0 : (int)std::ceil((b.reach + 0.5 * L) / L);
    int64_t nimages = 1;
    for (int k = 0; k < d; ++k) nimages *= 2 * nimg + 1;
    for (int64_t s = 0; s < nq; ++s) {
        double t[kMaxDim];
        int64_t rest = s;
        for (int k = 0; k < d; ++k) {
            t[k] = qx[rest % Q];
            rest /= Q;
        }
        if (b.top) {
            double r2 = 0, win = 1.0;
            for (int k = 0; k < d; ++k) {
                r2 += t[k] * t[k];
                win *= window(t[k], p->ext, b.s_hi, b.win_k);
            }
            K[s] = top_value(p->kernel, std::sqrt(r2 + c * c), b.s_lo) * win;
            continue;
        }
        double acc = 0;
        for (int64_t im = 0; im < nimages; ++im) {
            int64_t ir = im;
            double r2 = 0;
            int odd = 0;
            for (int k = 0; k < d; ++k) {
                const int nk = (int)(ir % (2 * nimg + 1)) - nimg;
                ir /= 2 * nimg + 1;
                const double v = t[k] + L * (double)nk;
                r2 += v * v;
                odd ^= nk & 1;
            }
            if (r2 > b.reach * b.reach) continue;   // below the band's tolerance
            const double v = band_value(p->kernel, std::sqrt(r2 + c * c), b.s_lo, b.s_hi);
            acc += odd ? -v : v;
        }
        K[s] = acc;
    }
    // cosine transform along each axis: axis 0 is the fastest index of K; each pass maps the
    // fastest axis from Q samples to mn nodes and rotates it to the slowest position
    std::vector<double> A((size_t)Q * mn);
    for (int i = 0; i < Q; ++i)
        for (int m = 0; m < mn; ++m) A[(size_t)i * mn + m] = std::cos(qx[i] * xi[m]);
    std::vector<double> cur = K, nxt;
    int64_t rest_len = nq / Q;   // product of the other axes' current lengths
    int fast = Q;
    for (int k = 0; k < d; ++k) {
        nxt.assign((size_t)rest_len * mn, 0.0);
        // cur[rest][fast] (fast index i), out[m][rest]: the transformed axis becomes the slowest
        for (int64_t rr = 0; rr < rest_len; ++rr) {
            const double *src = cur.data() + rr * fast;
            for (int m = 0; m < mn; ++m) {
                double acc = 0;
                for (int i = 0; i < fast; ++i) acc += src[i] * A[(size_t)i * mn + m];
                nxt[(size_t)m * rest_len + rr] = acc;
            }
        }
        cur.swap(nxt);
        // the new fastest axis is the next untransformed one (length Q) unless all are done
        if (k + 1 < d) {
            rest_len = (int64_t)cur.size() / Q;
            fast = Q;
        }
    }
    // cur is now indexed [m_{d-1}]...[m_0] with m_0 slowest: index = sum m_k mn^(d-1-k)... every
    // axis has length mn and C is symmetric in the axes, so the order of the digits is immaterial
    const double scale = std::pow(h / (2.0 * M_PI), d);
    std::vector<double> wt(b.P);
    for (int64_t q = 0; q < b.P; ++q) {
        const int hh = (int)(q % b.H);
        int64_t rest = q / b.H;
        int64_t idx = b.H + hh;
        double wgt = w[b.H + hh];
        int64_t stride = mn;
        for (int k = 0; k < d - 1; ++k) {
            const int m = (int)(rest % mn);
            rest /= mn;
            idx += m * stride;
            stride *= mn;
            wgt *= w[m];
        }
        wt[q] = scale * cur[idx] * wgt;
    }
    return wt;
}

double residual_value(int kernel, double b, double s0) {
    const double x = b / (std::sqrt(2.0) * s0);
    if (kernel == RBF_MULTIQUADRIC) return b * std::erfc(x) - kSq2pi * s0 * std::exp(-x * x);
    return std::erfc(x) / b;
}

// Polynomial pieces over [c, bmax) of g(b) = residual (multiquadric) or b * residual (inverse
// multiquadric: erfc(x), smooth where the residual itself has the 1/b of the kernel): on each
// of kResIntervals equal pieces the interpolant of degree kResDegree at Chebyshev points, as
// monomial coefficients in the piece's local variable v in [0, 1).  Returns the largest
// deviation of the residual it gives from the closed form on a finer sample of every piece.
double residual_table(int kernel, double c, double bmax, double s0, std::vector<double> &tab, double *inv) {
    const bool times_b = kernel == RBF_INVERSE_MULTIQUADRIC;
    constexpr int n = kResDegree + 1;
    const double db = (bmax - c) / kResIntervals;
    *inv = 1.0 / db;
    tab.assign(kResCoefs, 0.0);
    double vmax = 0, emax = 0;
    for (int k = 0; k < kResIntervals; ++k) {
        double A[n][n + 1];
        for (int i = 0; i < n; ++i) {
            const double v = 0.5 - 0.5 * std::cos(M_PI * (2 * i + 1) / (2.0 * n));
            double pw = 1.0;
            for (int j = 0; j < n; ++j) { A[i][j] = pw; pw *= v; }
            const double b = c + (k + v) * db;
            A[i][n] = residual_value(kernel, b, s0) * (times_b ? b : 1.0);
        }
        // Gaussian elimination with partial pivoting on the n x n Vandermonde system
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int r = col + 1; r < n; ++r) if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
            for (int j = 0; j <= n; ++j) std::swap(A[col][j], A[piv][j]);
            for (int r = 0; r < n; ++r) {
                if (r == col) continue;
                const double f = A[r][col] / A[col][col];
                for (int j = col; j <= n; ++j) A[r][j] -= f * A[col][j];
            }
        }
        for (int j = 0; j < n; ++j) tab[k * n + j] = A[j][n] / A[j][j];
        for (int t = 0; t <= 16; ++t) {
            const double v = t / 16.0, b = c + (k + v) * db;
            double y = tab[k * n + n - 1];
            for (int j = n - 2; j >= 0; --j) y = y * v + tab[k * n + j];
            if (times_b) y /= b;
            emax = std::max(emax, std::fabs(y - residual_value(kernel, b, s0)));
        }
    }
    return emax;
}

// Polynomial pieces over q = r^2 + c^2 in [c^2, qmax) of the residual at b = sqrt q (smooth in
// q there, since b >= c > 0): on each of kResIntervals equal pieces the interpolant of degree
// kResDegree at Chebyshev points, as monomial coefficients in the piece's local variable v in
// [0, 1); *inv = pieces per unit of r^2.  Returns the largest deviation of the residual it gives
// from the closed form on a finer sample of every piece.
double residual_table_q(int kernel, double c, double qmax, double s0, std::vector<double> &tab, double *inv) {
    constexpr int n = kResDegree + 1;
    const double q0 = c * c, dq = (qmax - q0) / kResIntervals;
    *inv = 1.0 / dq;
    tab.assign(kResCoefs, 0.0);
    double emax = 0;
    for (int k = 0; k < kResIntervals; ++k) {
        double A[n][n + 1];
        for (int i = 0; i < n; ++i) {
            const double v = 0.5 - 0.5 * std::cos(M_PI * (2 * i + 1) / (2.0 * n));
            double pw = 1.0;
            for (int j = 0; j < n; ++j) { A[i][j] = pw; pw *= v; }
            A[i][n] = residual_value(kernel, std::sqrt(q0 + (k + v) * dq), s0);
        }
        // Gaussian elimination with partial pivoting on the n x n Vandermonde system
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int r = col + 1; r < n; ++r) if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
            for (int j = 0; j <= n; ++j) std::swap(A[col][j], A[piv][j]);
            for (int r = 0; r < n; ++r) {
                if (r == col) continue;
                const double f = A[r][col] / A[col][col];
                for (int j = col; j <= n; ++j) A[r][j] -= f * A[col][j];
            }
        }
        for (int j = 0; j < n; ++j) tab[k * n + j] = A[j][n] / A[j][j];
        for (int t = 0; t <= 16; ++t) {
            const double v = t / 16.0;
            double y = tab[k * n + n - 1];
            for (int j = n - 2; j >= 0; --j) y = y * v + tab[k * n + j];
            emax = std::max(emax, std::fabs(y - residual_value(kernel, std::sqrt(q0 + (k + v) * dq), s0)));
        }
    }
    return emax;
}

int upload(Arena &ar, void **dst, const void *src, size_t bytes) {
    RBF_TRY(ar.alloc(dst, bytes));
    RBF_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return RBF_OK;
}

// Grid of a band: the cheapest (coarse level, radius, nodes) whose stencil holds every pair
// closer than the band's reach and whose period exceeds the stencil by the band's margin.
bool choose_grid(const rbf_plan *p, Band &b, double margin) {
    const int d = p->d;
    double best = INFINITY;
    for (int l = 0; l <= p->lc; ++l) {
        int r = 0;
        double rfar = p->ext;
        if (l >= 1) {
            const double w = p->ext / std::ldexp(1.0, l);
            r = 1 + (int)std::floor(b.reach / w);
            rfar = (r + 1) * w;
            if (rfar >= p->ext) continue;   // the whole domain: level 0 does it with one cell
        }
        const double L = rfar + margin;
        const int mn = round_nodes((int)std::ceil(b.sigma * L / M_PI) + 1);
        if (mn == 0) continue;
        int64_t P = mn / 2;
        for (int k = 0; k < d - 1; ++k) P *= mn;
        // per point: aggregation and disaggregation; per cell: upward pass and translation,
        // the stencil passes reading each cell once per axis on grids of at most 16 cells a
        // side and twice (running window) on larger ones
        const double cells = std::ldexp(1.0, d * l);
        const double reads = (l >= 1 && (1 << l) > 16) ? 2.0 * d : (double)d;
        const double cost = (double)P * ((double)p->n + (8.0 + reads) * cells);
        if (cost < best) {
            best = cost;
            b.lc = l;
            b.r = r;
            b.rfar = rfar;
            b.mn = mn;
        }
    }
    return best < INFINITY;
}

// Lagrange stencil of node t on the grid xs (spacing dx, n nodes): K consecutive nodes around
// t, clamped to the grid, and their weights
void lagrange_stencil(double x0, double dx, int n, int K, double t, int *first, double *w) {
    int j = (int)std::floor((t - x0) / dx) - K / 2 + 1;
    j = std::max(0, std::min(n - K, j));
    *first = j;
    for (int k = 0; k < K; ++k) {
        double v = 1.0;
        const double xk = x0 + (j + k) * dx;
        for (int l = 0; l < K; ++l)
            if (l != k) v *= (t - (x0 + (j + l) * dx)) / (xk - (x0 + (j + l) * dx));
        w[k] = v;
    }
}

// largest |sum_k w_k e^{i xi_k y} - e^{i eta y}| over the target nodes eta and |y| <= a
double transfer_error(const Band &S, const Band &Tb, double a, int K) {
    const double dxs = 2.0 * S.sigma / (S.mn - 1), dxt = 2.0 * Tb.sigma / (Tb.mn - 1);
    double worst = 0.0, w[32];
    for (int i = 0; i < Tb.mn; ++i) {
        const double eta = -Tb.sigma + i * dxt;
        int j0;
        lagrange_stencil(-S.sigma, dxs, S.mn, K, eta, &j0, w);
        for (int q = 0; q <= 128; ++q) {
            const double y = a * (2.0 * q / 128.0 - 1.0);
            double re = -std::cos(eta * y), im = -std::sin(eta * y);
            for (int k = 0; k < K; ++k) {
                const double xi = -S.sigma + (j0 + k) * dxs;
                re += w[k] * std::cos(xi * y);
                im += w[k] * std::sin(xi * y);
            }
            worst = std::max(worst, std::hypot(re, im));
        }
    }
    return worst;
}

// Choose the source band and the transferred bands (flags, stencil lengths; the source moves
// to the transfer level with a stencil over the whole grid, which is its level-0 far field).
// The transfer level trades cells for stencil length: a level finer by one has 2^d times the
// cells but half their width, so shorter stencils reach the same error.  Each level from 1 to
// min(l_n, 3) is costed as cells x sum over the moved bands of K x (the largest per-cell
// tensor of the band's passes), bands that no stencil of at most 16 points serves staying on
// their own, and the cheapest level is taken.
void plan_transfers(rbf_plan *p, std::vector<Band> &bands) {
    p->xfer_src = -1;
    if (p->band_xfer < 0) return;
    const int d = p->d;
    int src = -1;
    for (int j = 0; j < (int)bands.size(); ++j)
        if (bands[j].lc == 0 && !bands[j].top) { src = j; break; }
    if (src < 0) return;
    Band &S = bands[src];
    const int nb = (int)bands.size();
    int best_l = 0;
    double best_cost = INFINITY;
    std::vector<int> best_k(nb, 0);
    for (int li = 1; li <= std::min(p->lc, 3); ++li) {
        const int64_t ncell = (int64_t)1 << (d * li);
        if (p->band_xfer == 0 && p->n < 64 * ncell) break;
        const double a = 0.5 * p->ext / std::ldexp(1.0, li) * (1.0 + 1e-6);
        std::vector<int> ks(nb, 0);
        double cost = 0.0, saved = 0.0;
        for (int j = src + 1; j < nb; ++j) {
            const Band &b = bands[j];
            if (b.lc != 0 || b.sigma > S.sigma) continue;
            for (int K = 4; K <= std::min(16, S.mn); K += 2)
                if (transfer_error(S, b, a, K) <= b.tau_x / (20.0 * d)) {
                    ks[j] = K;
                    double big = b.mn / 2;
                    for (int k = 0; k < d - 1; ++k) big *= std::max(S.mn, b.mn);
                    cost += (double)ncell * K * big * 2.0 * d;                  // up and down passes
                    saved += (double)p->n * (b.mn / 2) * std::pow((double)b.mn, d - 1) * 2.0;   // P2M + L2P
                    break;
                }
        }
        if (saved > 0 && (p->band_xfer == 1 || cost < saved) && cost < best_cost) {
            best_cost = cost;
            best_l = li;
            best_k = ks;
        }
    }
    if (best_l == 0) return;
    for (int j = 0; j < nb; ++j)
        if (best_k[j]) {
            bands[j].xfer = 1;
            bands[j].xk = best_k[j];
        }
    p->xfer_src = src;
    p->xfer_level = best_l;
    p->xfer_ncell = 1 << (d * best_l);
    S.lc = best_l;
    S.r = (1 << best_l) - 1;   // every cell: the whole domain, as at level 0
}

// CSR tables of one 1-D map (outputs [nout], entries (input, weight))
struct Csr {
    std::vector<int> ptr, idx;
    std::vector<double> w;
};

int upload_csr(Arena &ar, const Csr &c, int **ptr, int **idx, double **w) {
    RBF_TRY(upload(ar, (void **)ptr, c.ptr.data(), sizeof(int) * c.ptr.size()));
    RBF_TRY(upload(ar, (void **)idx, c.idx.data(), sizeof(int) * std::max<size_t>(c.idx.size(), 1)));
    RBF_TRY(upload(ar, (void **)w, c.w.data(), sizeof(double) * std::max<size_t>(c.w.size(), 1)));
    return RBF_OK;
}

// per-axis phase tables e^{i xi_m c_k} at the centres of the dense transfer cells (Morton order)
std::vector<double2> cell_phases(const rbf_plan *p, const Band &b) {
    const int d = p->d, li = p->xfer_level, nc = p->xfer_ncell;
    const double w = p->ext / std::ldexp(1.0, li), dxi = 2.0 * b.sigma / (b.mn - 1);
    std::vector<double2> E((size_t)nc * d * b.mn);
    for (int c = 0; c < nc; ++c)
        for (int k = 0; k < d; ++k) {
            int ik = 0;
            for (int bit = 0; bit < li; ++bit) ik |= ((c >> (bit * d + k)) & 1) << bit;
            const double ck = p->lo[k] + (ik + 0.5) * w;
            for (int m = 0; m < b.mn; ++m) {
                const double ph = (-b.sigma + m * dxi) * ck;
                E[((size_t)c * d + k) * b.mn + m] = double2{std::cos(ph), std::sin(ph)};
            }
        }
    return E;
}

// the tables of every transferred band, the source's cell phases and unit map, and buffers
int build_transfers(rbf_plan *p, const std::vector<int> &src_ucell, size_t csz) {
    if (p->xfer_src < 0) return RBF_OK;
    Arena &ar = p->arena;
    const int d = p->d, nc = p->xfer_ncell;
    const Band &S = p->bands[p->xfer_src];
    const double dxs = 2.0 * S.sigma / (S.mn - 1);
    int64_t rs = 1;
    for (int k = 0; k < d - 1; ++k) rs *= S.mn;
    int64_t xmax = rs * S.H, lmax = 0;
    const double a = 0.5 * p->ext / std::ldexp(1.0, p->xfer_level) * (1.0 + 1e-6);
    for (int j = 0; j < (int)p->bands.size(); ++j) {
        Band &b = p->bands[j];
        if (!b.xfer) continue;
        Xfer x;
        x.band = j;
        x.K = b.xk;
        x.err = transfer_error(S, b, a, b.xk);
        const int K = b.xk, mnt = b.mn, Ht = b.H;
        const double dxt = 2.0 * b.sigma / (mnt - 1);
        // stencils of every target node (full grid)
        std::vector<int> first(mnt);
        std::vector<double> wts((size_t)mnt * K);
        for (int i = 0; i < mnt; ++i)
            lagrange_stencil(-S.sigma, dxs, S.mn, K, -b.sigma + i * dxt, &first[i], &wts[(size_t)i * K]);
        Csr up, upl, dn, dnl;
        up.ptr.push_back(0);
        for (int i = 0; i < mnt; ++i) {
            for (int k = 0; k < K; ++k) {
                up.idx.push_back(first[i] + k);
                up.w.push_back(wts[(size_t)i * K + k]);
            }
            up.ptr.push_back((int)up.idx.size());
        }
        upl.ptr.push_back(0);
        for (int h = 0; h < Ht; ++h) {
            const int i = Ht + h;
            for (int k = 0; k < K; ++k) {
                upl.idx.push_back(first[i] + k);
                upl.w.push_back(wts[(size_t)i * K + k]);
            }
            upl.ptr.push_back((int)upl.idx.size());
        }
        // transposes: source node j collects (target node i, weight of j in i's stencil)
        for (Csr *t : {&dn, &dnl}) t->ptr.push_back(0);
        for (int j2 = 0; j2 < S.mn; ++j2) {
            for (int i = 0; i < mnt; ++i)
                if (j2 >= first[i] && j2 < first[i] + K) {
                    dn.idx.push_back(i);
                    dn.w.push_back(wts[(size_t)i * K + (j2 - first[i])]);
                }
            dn.ptr.push_back((int)dn.idx.size());
        }
        for (int h = 0; h < S.H; ++h) {
            const int j2 = S.H + h;
            for (int i = 0; i < mnt; ++i)
                if (j2 >= first[i] && j2 < first[i] + K) {
                    dnl.idx.push_back(i);
                    dnl.w.push_back(wts[(size_t)i * K + (j2 - first[i])]);
                }
            dnl.ptr.push_back((int)dnl.idx.size());
        }
        RBF_TRY(upload_csr(ar, up, &x.up_ptr, &x.up_idx, &x.up_w));
        RBF_TRY(upload_csr(ar, upl, &x.upl_ptr, &x.upl_idx, &x.upl_w));
        RBF_TRY(upload_csr(ar, dn, &x.dn_ptr, &x.dn_idx, &x.dn_w));
        RBF_TRY(upload_csr(ar, dnl, &x.dnl_ptr, &x.dnl_idx, &x.dnl_w));
        const std::vector<double2> Et = cell_phases(p, b);
        RBF_TRY(upload(ar, (void **)&x.phase_t, Et.data(), sizeof(double2) * Et.size()));
        p->xfers.push_back(x);
        int64_t big = Ht;
        for (int k = 0; k < d - 1; ++k) big *= std::max(S.mn, mnt);
        xmax = std::max(xmax, big);
        lmax = std::max(lmax, b.P);
    }
    const std::vector<double2> Es = cell_phases(p, S);
    RBF_TRY(upload(ar, (void **)&p->xfer_phase_s, Es.data(), sizeof(double2) * Es.size()));
    std::vector<int> cu(nc, -1);
    for (int u = 0; u < (int)src_ucell.size(); ++u) cu[src_ucell[u]] = u;
    RBF_TRY(upload(ar, (void **)&p->xfer_cell_unit, cu.data(), sizeof(int) * cu.size()));
    RBF_TRY(ar.alloc(&p->xfer_keep, csz * (size_t)nc * S.P));
    RBF_TRY(ar.alloc(&p->xfer_x1, csz * (size_t)nc * xmax));
    RBF_TRY(ar.alloc(&p->xfer_x2, csz * (size_t)nc * xmax));
    RBF_TRY(ar.alloc(&p->xfer_l, csz * (size_t)lmax));
    return RBF_OK;
}

}  // namespace

int plan_bands(rbf_plan *p) {
    const int d = p->d, kernel = p->kernel;
    const double ext = p->ext, c = p->shape, tol = p->tol;
    const double wn = ext / std::ldexp(1.0, p->lc);
    // residual: negligible (x = b / (sqrt 2 s0) >= xcut) beyond the adjacent cells
    const double xcut = std::sqrt(std::log(1.0 / tol) + 4.0);
    p->res_s0 = wn / (std::sqrt(2.0) * xcut);
    RBF_TRY(kernel_rms(p, &p->phi_rms));
    {
        // the residual over the near zone: pairs closer than one cell width (farther ones are
        // beyond x = xcut, where it is below the tolerance) as polynomial pieces in b
        p->res_qmax = wn * wn;
        std::vector<double> tab;
        // the table in q (no square root per pair) where its fit meets the bound, else in b
        const double bound = 1e-3 * tol * p->phi_rms;
        double err = residual_table_q(kernel, c, wn * wn + c * c, p->res_s0, tab, &p->res_inv);
        p->res_q = err <= bound ? 1 : 0;
        if (!p->res_q) err = residual_table(kernel, c, std::sqrt(wn * wn + c * c), p->res_s0, tab, &p->res_inv);
        if (!(err <= bound)) {
            set_error("rbf_fmm_plan: the near-field residual table deviates by %.2e (kernel rms %.2e, tol %g)",
                      err, p->phi_rms, tol);
            return RBF_EUNSUPPORTED;
        }
        RBF_TRY(upload(p->arena, (void **)&p->res_tab, tab.data(), sizeof(double) * tab.size()));
    }
    const double s_top = 2.0 * ext;
    std::vector<double> edges{p->res_s0};
    while (edges.back() * kRatio * 1.1 < s_top) edges.push_back(edges.back() * kRatio);
    edges.push_back(s_top);
    const int J = (int)edges.size() - 1;
    // Tolerance of a piece relative to its largest value: the requested relative error times
    // the kernel's rms over pairs, split over the pieces (bands, top, residual) as independent
    // errors.  The band-limit rule bounds a piece's error by its value at r = 0; that error (the
    // band-limit, aliasing and pruning terms) lives within about 6 widths s_hi of r = 0, so
    // only the pairs that close carry it: a band's tolerance is divided by the square root of
    // the fraction of sampled pairs closer than 6 s_hi (1 for the wide bands, much less for the
    // narrow ones).  On top of that the bound still overstates the error, and FP64 plans take
    // bands 16 times looser.  Measured over the test sets (3-D and 2-D, 1 to 2^20 points) at tol
    // 1e-6: at most 5.4e-7 in FP64 (2.8e-7 / 2.0e-7 for the 2^20-point multiquadric / inverse
    // multiquadric), at most 4.8e-6 in FP32 at 1e-4.  (FP32 bands 16 times looser measured 2.6e-4.)
    // The transfers' stencils keep the plain split's tolerance.
    const double split = 0.25 * std::sqrt((double)(J + 2));
    const double loose = p->dtype == RBF_F64 ? 16.0 : 1.0;
    constexpr double kErrWidths = 6.0;
    auto tau_at = [&](double mag, double f) { return std::min(1e-2, std::max(1e-3 * tol, f * tol * p->phi_rms / (mag * split))); };
    std::vector<Band> bands;
    for (int j = 0; j < J; ++j) {
        Band b;
        b.s_lo = edges[j];
        b.s_hi = edges[j + 1];
        const double mag = std::fabs(band_value(kernel, c, b.s_lo, b.s_hi));
        b.scale = mag;
        b.tau = tau_at(mag, loose / std::sqrt(pair_fraction(p, kErrWidths * b.s_hi)));
        b.tau_x = tau_at(mag, 1.0);
        b.sigma = band_limit_t(b.tau) / b.s_lo;
        b.reach = b.s_hi * std::sqrt(2.0 * std::log(4.0 / b.tau) + 1.0);
        const double margin = b.s_hi * std::sqrt(2.0 * std::log(4.0 / b.tau));
        if (!choose_grid(p, b, margin)) {
            set_error("rbf_fmm_plan: band %d (widths %g..%g) needs more than 64 nodes per dimension at tol %g", j,
                      b.s_lo, b.s_hi, tol);
            return RBF_EUNSUPPORTED;
        }
        b.L = M_PI * (b.mn - 1) / b.sigma;
        bands.push_back(b);
    }
    {
        Band b;
        b.top = 1;
        b.s_lo = s_top;
        b.s_hi = 1.4 * s_top;   // window width
        const double bmax = std::sqrt((double)d) * ext + c;
        const double mag = kernel == RBF_MULTIQUADRIC ? top_value(kernel, bmax, s_top) : top_value(kernel, c, s_top);
        b.scale = mag;
        b.tau = tau_at(mag, loose);   // every pair sees the top band (pair fraction 1)
        b.tau_x = tau_at(mag, 1.0);
        // the window's deviation from 1 inside the domain, times the top band's size (a few
        // times the kernel's rms), stays two orders below the tolerance: at k = 4 it set a floor
        // of 1.4e-8 under the multiquadric product whatever the tolerance
        while (0.5 * std::erfc(b.win_k) > 1e-2 * tol && b.win_k < 8.0) b.win_k += 0.1;
        b.L = 2.0 * (ext + (b.win_k + 5.0) * b.s_hi);
        // the band limit of the top band's narrowest width, s_top, as for every other band (a
        // limit at 1.2 s_top, enough at 1e-6, left 2e-7 of the multiquadric product's error)
        const double sig = band_limit_t(b.tau) / s_top;
        b.mn = round_nodes((int)std::ceil(sig * b.L / M_PI) + 1);
        if (b.mn == 0) {
            set_error("rbf_fmm_plan: the top band needs more than 64 nodes per dimension at tol %g", tol);
            return RBF_EUNSUPPORTED;
        }
        b.sigma = M_PI * (b.mn - 1) / b.L;   // the window fixes the period
        b.reach = INFINITY;
        b.lc = 0;
        b.r = 0;
        b.rfar = ext;
        bands.push_back(b);
    }
    plan_transfers(p, bands);
    // units, chunks and tasks per band from the uniform leaves (all at level p->lc)
    const int nl = p->nleaves;
    std::vector<int> lb(nl + 1);
    std::vector<uint64_t> pre(nl);
    RBF_HIP(hipMemcpy(lb.data(), p->leaf_begin, sizeof(int) * (nl + 1), hipMemcpyDeviceToHost));
    RBF_HIP(hipMemcpy(pre.data(), p->leaf_prefix, sizeof(uint64_t) * nl, hipMemcpyDeviceToHost));
    Arena &ar = p->arena;
    int64_t maxW = 0, maxLx = 0, maxC = 0, maxHP = 0;
    std::vector<int> src_ucell;
    for (int jb = 0; jb < (int)bands.size(); ++jb) {
        Band &b = bands[jb];
        b.H = b.mn / 2;
        b.HP = b.H;
        b.R = 1;
        for (int k = 0; k < d - 1; ++k) b.R *= b.mn;
        b.P = b.R * b.H;
        if (b.xfer) {   // no units of its own: its expansions come from the source band
            const std::vector<double> wt = band_table(p, b);
            RBF_TRY(upload(ar, (void **)&b.wtab, wt.data(), sizeof(double) * wt.size()));
            continue;
        }
        b.ncells = (int64_t)1 << (d * b.lc);
        const int sh = d * (p->lc - b.lc);
        std::vector<int> ub, ucell, cb, ccell, cellb(b.ncells + 1, 0);
        std::vector<int> task;
        for (int a = 0; a < nl;) {
            const uint64_t cell = pre[a] >> sh;
            int e = a;
            while (e < nl && (pre[e] >> sh) == cell) ++e;
            const int u = (int)ucell.size();
            ub.push_back(lb[a]);
            ucell.push_back((int)cell);
            for (int t = lb[a]; t < lb[e]; t += kBandChunk) {
                cb.push_back(t);
                ccell.push_back((int)cell);
            }
            for (int t = 0; t < lb[e] - lb[a]; t += kWave) {
                task.push_back(u);
                task.push_back(t);
            }
            a = e;
        }
        ub.push_back(lb[nl]);
        b.nunits = (int)ucell.size();
        b.nchunks = (int)cb.size();
        if (jb == p->xfer_src) src_ucell = ucell;
        cb.push_back(lb[nl]);
        b.ntasks = (int)(task.size() / 2);
        // chunk range of every dense cell (chunks are in cell order)
        for (int64_t cc = 0; cc <= b.ncells; ++cc)
            cellb[cc] = (int)(std::lower_bound(ccell.begin(), ccell.end(), (int)std::min<int64_t>(cc, INT32_MAX)) -
                              ccell.begin());
        cellb[b.ncells] = b.nchunks;
        b.ngroups = (b.nunits + 7) / 8;
        std::vector<int> gf(b.ngroups + 1), up(b.ngroups + 1, 0), pad(16, 0);
        for (int g = 0; g <= b.ngroups; ++g) gf[g] = std::min(8 * g, b.nunits);
        const std::vector<double> wt = band_table(p, b);
        RBF_TRY(upload(ar, (void **)&b.unit_begin, ub.data(), sizeof(int) * ub.size()));
        RBF_TRY(upload(ar, (void **)&b.unit_cell, ucell.data(), sizeof(int) * ucell.size()));
        RBF_TRY(upload(ar, (void **)&b.chunk_begin, cb.data(), sizeof(int) * cb.size()));
        RBF_TRY(upload(ar, (void **)&b.cell_begin, cellb.data(), sizeof(int) * cellb.size()));
        RBF_TRY(upload(ar, (void **)&b.tasks, task.data(), sizeof(int) * task.size()));
        RBF_TRY(upload(ar, (void **)&b.grp_first, gf.data(), sizeof(int) * gf.size()));
        RBF_TRY(upload(ar, (void **)&b.uni_ptr, up.data(), sizeof(int) * up.size()));
        RBF_TRY(upload(ar, (void **)&b.uni_pad, pad.data(), sizeof(int) * pad.size()));
        RBF_TRY(upload(ar, (void **)&b.wtab, wt.data(), sizeof(double) * wt.size()));
        maxW = std::max<int64_t>(maxW, (int64_t)b.nchunks * b.P);
        maxLx = std::max<int64_t>(maxLx, (int64_t)b.nunits * b.R * b.HP);
        maxC = std::max<int64_t>(maxC, b.ncells * b.P);
        maxHP = std::max<int64_t>(maxHP, b.HP);
    }
    const size_t csz = p->dtype == RBF_F32 ? 8 : 16;
    const double need = (double)csz * (maxW + maxLx + 3.0 * maxC + (double)maxHP * p->n);
    if (need > 200e9) {
        set_error("rbf_fmm_plan: band expansions need %.1f GB; raise tol", need / 1e9);
        return RBF_ENOMEM;
    }
    RBF_TRY(ar.alloc(&p->bW, csz * maxW));
    RBF_TRY(ar.alloc(&p->bLx, csz * maxLx));
    RBF_TRY(ar.alloc(&p->bWc, csz * maxC));
    RBF_TRY(ar.alloc(&p->bLc, csz * maxC));
    RBF_TRY(ar.alloc(&p->bTmp, csz * maxC));
    RBF_TRY(ar.alloc(&p->bdl, csz * maxHP * p->n));
    p->bands = std::move(bands);
    RBF_TRY(build_transfers(p, src_ucell, csz));
    return RBF_OK;
}

}  // namespace rbf

// Band-limited Gaussian (section 3, eq. 16, with the box cut-off of eq. 28): host tabulation.
//
// The Gaussian exp(-|x|^2 / (2 s^2)) has the transform (2 pi)^d prod_k c1(xi_k),
// c1(xi) = s / sqrt(2 pi) exp(-s^2 xi^2 / 2), so cutting it off at the box [-sigma, sigma]^d
// leaves a product over the axes,
//     Phi_sigma(x) = prod_k phi(x_k),   phi(t) = int_{-sigma}^{sigma} c1(xi) cos(xi t) dxi.
// phi is even, band-limited with bandwidth sigma (so its k-th derivative is at most
// sigma^k phi(0)) and, with the sharp cut-off, decays only like 1/|t|.  The plan tabulates it
// over [0, tmax], tmax the largest side of the points' bounding box (every coordinate
// difference lies in [-tmax, tmax]), as pieces of degree kBlDegree64 (FP64 plans) or
// kBlDegree32 (FP32 plans): each piece interpolates
// phi at the Chebyshev points of the first kind of its interval, converted to monomials in
// the piece's variable u in [-1, 1].  phi itself comes from composite Gauss-Legendre
// quadrature of its defining integral, with panels short enough (at most one radian of the
// cosine and half a width 1/s of the Gaussian) that the 16-point rule is exact to rounding.
// The fit error is measured at points between the nodes of every piece; the piece count
// grows until it is below the plan's bound.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace rbf {

namespace {

constexpr int kGl = 16;   // Gauss-Legendre points per panel

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on the Legendre polynomial
// P_kGl (three-term recurrence), from the usual cosine start.
struct GaussLegendre {
    double x[kGl], w[kGl];
    GaussLegendre() {
        for (int i = 0; i < kGl; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (kGl + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= kGl; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = kGl * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

// phi(t) = 2 int_0^sigma c1(xi) cos(xi t) dxi; beyond xi = 12 / s the integrand is below
// exp(-72) times its peak, so the integral stops at min(sigma, 12 / s)
double phi_axis(double t, double s, double sigma, const GaussLegendre &g) {
    const double top = std::min(sigma, 12.0 / s);
    const int m = 1 + (int)std::ceil(top * std::fabs(t) + 2.0 * top * s);
    const double h = top / m, a = s / std::sqrt(2.0 * M_PI);
    double sum = 0.0;
    for (int q = 0; q < m; ++q) {
        const double c = (q + 0.5) * h;
        double part = 0.0;
        for (int i = 0; i < kGl; ++i) {
            const double xi = c + 0.5 * h * g.x[i];
            part += g.w[i] * std::exp(-0.5 * s * s * xi * xi) * std::cos(xi * t);
        }
        sum += 0.5 * h * part;
    }
    return 2.0 * a * sum;
}

// Monomial coefficients (u^0 first) of the Chebyshev polynomials T_0..T_kMaxK-1.
constexpr int kMaxK = kBlDegree64 + 1;
struct ChebMonomials {
    double c[kMaxK][kMaxK] = {};
    ChebMonomials() {
        c[0][0] = 1.0;
        c[1][1] = 1.0;
        for (int k = 2; k < kMaxK; ++k)
            for (int j = 0; j < kMaxK; ++j)
                c[k][j] = (j > 0 ? 2.0 * c[k - 1][j - 1] : 0.0) - c[k - 2][j];
    }
};

// Tabulate with np pieces of degree deg (at most kBlDegree64); returns the largest error found
// at the check points.
double fit_pieces(double s, double sigma, double tmax, int np, int deg, const GaussLegendre &g,
                  std::vector<double> &tab) {
    static const ChebMonomials cm;
    const int K = deg + 1;
    tab.assign(kBlHead + (size_t)np * K, 0.0);
    tab[0] = np;
    tab[1] = deg;
    const double h = tmax / np;
    double un[kMaxK];
    for (int j = 0; j < K; ++j) un[j] = std::cos(M_PI * (j + 0.5) / K);
    // check points: the piece's ends and two points between nodes
    const double uc[4] = {-1.0, -0.37, 0.61, 1.0};
    double emax = 0.0;
    for (int i = 0; i < np; ++i) {
        const double a0 = i * h;
        double f[kMaxK], a[kMaxK];
        for (int j = 0; j < K; ++j) f[j] = phi_axis(a0 + 0.5 * h * (un[j] + 1.0), s, sigma, g);
        // Chebyshev coefficients a_k = (2 / K) sum_j f_j T_k(u_j), a_0 halved
        for (int k = 0; k < K; ++k) {
            double v = 0.0;
            for (int j = 0; j < K; ++j) v += f[j] * std::cos(k * M_PI * (j + 0.5) / K);
            a[k] = (k == 0 ? 1.0 : 2.0) * v / K;
        }
        double *b = tab.data() + kBlHead + (size_t)i * K;
        for (int k = 0; k < K; ++k)
            for (int j = 0; j < K; ++j) b[j] += a[k] * cm.c[k][j];
        for (double u : uc) {
            double y = b[deg];
            for (int k = deg - 1; k >= 0; --k) y = y * u + b[k];
            emax = std::max(emax, std::fabs(y - phi_axis(a0 + 0.5 * h * (u + 1.0), s, sigma, g)));
        }
    }
    return emax;
}

}  // namespace

// Build and upload the per-axis table of the plan's band-limited Gaussian.
int bandlimited_table(rbf_plan *p, double sigma) {
    static const GaussLegendre g;
    const double s = p->shape;
    const double tmax = p->ext * (1.0 + 1e-9);
    const double phi0 = std::erf(s * sigma / std::sqrt(2.0));   // phi(0)
    const bool f64 = p->dtype == RBF_F64;
    const int deg = f64 ? kBlDegree64 : kBlDegree32;
    // floors: what the product's own arithmetic resolves
    const double bound = std::max(p->tol / (4.0 * p->d), f64 ? 1e-14 : 3e-8) * phi0;
    // start from pieces of 0.4 rad of the bandwidth for degree 7 (fit error about 5e-15 of
    // phi(0)), 0.3 rad for degree 3 (about 1e-7), or of 0.1 s, 0.075 s where the Gaussian's own
    // scale is the finer one; the fit costs pieces x panels, so a first estimate above the cap
    // is refused before any fitting
    const double want = std::ceil(tmax * std::min(sigma, 4.0 / s) / (f64 ? 0.4 : 0.3));
    if (!(want <= kBlMaxPieces)) {
        set_error("band-limited Gaussian: sigma %g over the box side %g needs about %.0f table pieces, more than %d",
                  sigma, tmax, want, kBlMaxPieces);
        return RBF_EUNSUPPORTED;
    }
    int np = (int)std::max(4.0, want);
    std::vector<double> tab;
    double err = INFINITY;
    for (;;) {
        err = fit_pieces(s, sigma, tmax, np, deg, g, tab);
        if (err <= bound || np >= kBlMaxPieces) break;
        np = std::min(kBlMaxPieces, (int)std::ceil(np * 1.5));
    }
    if (!(err <= bound)) {
        set_error("band-limited Gaussian: %d pieces fit phi_sigma to %.3g, above %.3g (sigma %g times the box "
                  "side %g is too large; raise tol or lower sigma)", np, err, bound, sigma, tmax);
        return RBF_EUNSUPPORTED;
    }
    RBF_TRY(p->arena.alloc((void **)&p->bl_tab, sizeof(double) * tab.size()));
    RBF_HIP(hipMemcpy(p->bl_tab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
    p->bl_inv = np / tmax;
    p->bl_pieces = np;
    p->bl_err = err;
    p->sigma = sigma;
    return RBF_OK;
}

}  // namespace rbf

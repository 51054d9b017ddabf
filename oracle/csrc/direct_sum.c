/*
 * Oracle A: the plain O(N^2) RBF sum u(y_i) = sum_j lambda_j Phi(y_i - x_j)
 * (Zhao & Stoll, section 1, eq. 1; all pairs, including j = i).
 *
 * TEST INFRASTRUCTURE ONLY: built and called by the oracle package, never by the
 * product library.  Plain double-precision loops, IEEE arithmetic (no fast-math),
 * one OpenMP thread per block of targets.  Kernels: 0 = Gaussian exp(-r^2/(2 s^2)),
 * 1 = multiquadric sqrt(r^2 + c^2), 2 = inverse multiquadric 1/sqrt(r^2 + c^2),
 * 3 = Wendland (1 - e r)_+^3 (3 e r + 1) (section 5), 4 = thin-plate spline r^2 log r
 * (0 at r = 0), 5 = r^5 (the Fourier-transform table; shape ignored).  Points are row-major
 * (n, d).
 */
#include <math.h>
#include <stdint.h>

int oracle_threads(void);

void oracle_direct_sum(const double *src, int64_t n, int d, const double *lam,
                       const double *tgt, int64_t nt, int kernel, double shape,
                       double *out)
{
    const double inv2s2 = 1.0 / (2.0 * shape * shape);
    const double c2 = shape * shape;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        const double *y = tgt + i * d;
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double *x = src + j * d;
            double r2 = 0.0;
            for (int k = 0; k < d; ++k) {
                double t = y[k] - x[k];
                r2 += t * t;
            }
            double phi;
            if (kernel == 0) {
                phi = exp(-r2 * inv2s2);
            } else if (kernel == 1) {
                phi = sqrt(r2 + c2);
            } else if (kernel == 2) {
                phi = 1.0 / sqrt(r2 + c2);
            } else if (kernel == 3) {
                double er = shape * sqrt(r2);
                double t = er < 1.0 ? 1.0 - er : 0.0;
                phi = t * t * t * (3.0 * er + 1.0);
            } else if (kernel == 4) {
                phi = r2 > 0.0 ? 0.5 * r2 * log(r2) : 0.0;
            } else {
                phi = r2 * r2 * sqrt(r2);
            }
            acc += lam[j] * phi;
        }
        out[i] = acc;
    }
}

#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
#else
int oracle_threads(void) { return 1; }
#endif

/*
 * ORACLE -- test infrastructure only.  Plain FP64 direct N-body sum on the
 * unit sphere.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library; the GPU library never does.
 *
 * Computes the midpoint-rule sum of paper eq. (nbodysum),
 *
 *     phi_i = sum_j K(x_i, y_j) w_j ,
 *
 * over every source j, with the singular self term left out (paper §1 leaves
 * the term of a particle with itself out of the sum).  A source is left out of target i exactly
 * when its three coordinates equal those of x_i bit for bit; for a point set
 * without duplicates used as both targets and sources this is the i=j rule,
 * and for distinct sets it drops exact coincidences only.
 *
 * Kernels (x, y on the unit sphere, so 1 - x.y = |x-y|^2 / 2):
 *   1  Poisson log (paper eq. G_L):      -(1/4pi) ln(1 - x.y)
 *   2  Biot-Savart (paper eq. K_BS):     -(1/4pi) (x cross y) / (1 - x.y)   (3 outputs)
 *   3  inverse distance (the 1/gamma term of paper eq. G_SAL_approx): 1/|x-y|
 *   4  biharmonic (paper eq. G_B):       (1/4pi) dilog((1 + x.y)/2)
 *   5  SAL closed form (paper eq. G_SAL_approx):
 *        (3 rw/(4 pi re)) ((1 - b0)/gamma - (a1 - b1) ln(gamma/2 + gamma^2/4)),
 *        gamma = |x-y|, a1 = -2.7, b0 = -6.21196, b1 = 6.1 (§2.4), and the
 *        density ratio rw/re = 1025/5514 (seawater over mean Earth density;
 *        the paper names the ratio without a number).
 * 1 - x.y is evaluated as |x-y|^2/2, which is the same number on the sphere
 * and keeps its relative accuracy for close pairs; likewise the dilogarithm's
 * argument u = (1 + x.y)/2 is carried as 1 - u = |x-y|^2/4.
 *
 * dilog(u) = -int_0^u ln(1-t)/t dt (§2.2) is summed from its power series
 * sum_k u^k/k^2 (integrate the series of -ln(1-t)/t term by term) when
 * u <= 1/2, and through Euler's reflection formula
 * dilog(u) = pi^2/6 - ln(u) ln(1-u) - dilog(1-u) when u > 1/2, so the series
 * argument never exceeds 1/2.
 *
 * Loop: OpenMP over targets, sources in ascending order, one plain FP64 sum
 * per target.  No blocking, no reordering, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846
#define SAL_A1 (-2.7)
#define SAL_B0 (-6.21196)
#define SAL_B1 6.1
#define SAL_RHO_RATIO (1025.0 / 5514.0)

/* sum_{k>=1} x^k / k^2 for 0 <= x <= 1/2, summed until the terms stop
 * changing the sum. */
static double dilog_series(double x)
{
    double sum = 0.0, xk = 1.0;
    for (int k = 1; k < 200; ++k) {
        xk *= x;
        double term = xk / ((double)k * (double)k);
        double next = sum + term;
        if (next == sum) break;
        sum = next;
    }
    return sum;
}

/* dilog(u) for u = 1 - v, 0 <= v <= 1. */
static double dilog_one_minus(double v)
{
    double u = 1.0 - v;
    if (u <= 0.5) return dilog_series(u);
    if (v == 0.0) return ORACLE_PI * ORACLE_PI / 6.0;
    return ORACLE_PI * ORACLE_PI / 6.0 - log1p(-v) * log(v) - dilog_series(v);
}

static double half_dist2(const double* x, const double* y)
{
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    return 0.5 * (dx * dx + dy * dy + dz * dz);
}

static int same_point(const double* x, const double* y)
{
    return x[0] == y[0] && x[1] == y[1] && x[2] == y[2];
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Returns 0 on success, -1 on a bad kernel id or size. out is [nt] or, for
 * Biot-Savart, [nt][3]. nthreads <= 0 means the OpenMP default. */
int oracle_direct(int kernel, const double* tgt, int64_t nt, const double* src,
                  int64_t ns, const double* w, double* out, int nthreads)
{
    if (nt < 0 || ns < 0 || kernel < 1 || kernel > 5) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const double c = 1.0 / (4.0 * ORACLE_PI);
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < nt; ++i) {
        const double* x = tgt + 3 * i;
        if (kernel == 2) {
            double u0 = 0.0, u1 = 0.0, u2 = 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                const double* y = src + 3 * j;
                if (same_point(x, y)) continue;
                double d = half_dist2(x, y);
                /* x cross y */
                double cx = x[1] * y[2] - x[2] * y[1];
                double cy = x[2] * y[0] - x[0] * y[2];
                double cz = x[0] * y[1] - x[1] * y[0];
                double s = -c * w[j] / d;
                u0 += s * cx;
                u1 += s * cy;
                u2 += s * cz;
            }
            out[3 * i + 0] = u0;
            out[3 * i + 1] = u1;
            out[3 * i + 2] = u2;
        } else {
            double acc = 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                const double* y = src + 3 * j;
                if (same_point(x, y)) continue;
                double d = half_dist2(x, y);
                double k;
                if (kernel == 1) {
                    k = -c * log(d);
                } else if (kernel == 3) {
                    k = 1.0 / sqrt(2.0 * d);
                } else if (kernel == 4) {
                    double v = 0.5 * d; /* 1 - (1 + x.y)/2 */
                    if (v > 1.0) v = 1.0;
                    k = c * dilog_one_minus(v);
                } else {
                    double g = sqrt(2.0 * d); /* gamma = |x - y| */
                    k = 3.0 * SAL_RHO_RATIO * c *
                        ((1.0 - SAL_B0) / g - (SAL_A1 - SAL_B1) * log(0.5 * g + 0.25 * g * g));
                }
                acc += k * w[j];
            }
            out[i] = acc;
        }
    }
    return 0;
}

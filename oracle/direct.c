/*
 * ORACLE -- test infrastructure only.  Plain FP64 direct N-body sum on the
 * unit sphere.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library; the GPU library never does.
 *
 * Computes the midpoint-rule sum of paper eq. (nbodysum),
 *
 *     phi_i = sum_j K(x_i, y_j) w_j ,
 *
 * over every source j, with the singular self term left out (paper §1: "the
 * i=j term in the sum is omitted").  A source is left out of target i exactly
 * when its three coordinates equal those of x_i bit for bit; for a point set
 * without duplicates used as both targets and sources this is the i=j rule,
 * and for distinct sets it drops exact coincidences only.
 *
 * Kernels (x, y on the unit sphere, so 1 - x.y = |x-y|^2 / 2):
 *   1  Poisson log (paper eq. G_L):      -(1/4pi) ln(1 - x.y)
 *   2  Biot-Savart (paper eq. K_BS):     -(1/4pi) (x cross y) / (1 - x.y)   (3 outputs)
 *   3  inverse distance (the 1/gamma term of paper eq. G_SAL_approx): 1/|x-y|
 * 1 - x.y is evaluated as |x-y|^2/2, which is the same number on the sphere
 * and keeps its relative accuracy for close pairs.
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
    if (nt < 0 || ns < 0 || kernel < 1 || kernel > 3) return -1;
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
                if (kernel == 1)
                    k = -c * log(d);
                else
                    k = 1.0 / sqrt(2.0 * d);
                acc += k * w[j];
            }
            out[i] = acc;
        }
    }
    return 0;
}

// Barotropic vorticity equation on the rotating sphere (paper §2.3, eqs. BVE
// and BVE_ODEs; §12): Lagrangian particles x_i with vorticity zeta_i and
// fixed areas A_i,
//     dx_i/dt = sum_j K_BS(x_i, x_j) zeta_j A_j,   dzeta_i/dt = -2 Omega dz_i/dt,
// one classical 4th order Runge-Kutta step per call.  Every stage builds a
// plan on the stage positions (the particles move) and evaluates the
// Biot-Savart sum with it (or with the direct sum); stage positions and the
// final positions are projected back onto the sphere.
#include <cmath>

#include "common.h"

namespace csfmm {
namespace {

// Stage input: xs = x + c kx projected onto the sphere, ws = (zeta + c kz) A.
// With c = 0 this is x itself (already on the sphere) and zeta A.
__global__ void k_bve_stage(const double* __restrict__ x, const double* __restrict__ zeta,
                            const double* __restrict__ area, const double* __restrict__ u,
                            double c, double omega, int64_t n, double* __restrict__ xs,
                            double* __restrict__ ws) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p0 = x[3 * i], p1 = x[3 * i + 1], p2 = x[3 * i + 2];
    double z = zeta[i];
    if (c != 0.0) {
        p0 += c * u[3 * i];
        p1 += c * u[3 * i + 1];
        p2 += c * u[3 * i + 2];
        z += c * (-2.0 * omega * u[3 * i + 2]);
        const double r = 1.0 / sqrt(p0 * p0 + p1 * p1 + p2 * p2);
        p0 *= r;
        p1 *= r;
        p2 *= r;
    }
    xs[3 * i] = p0;
    xs[3 * i + 1] = p1;
    xs[3 * i + 2] = p2;
    ws[i] = z * area[i];
}

// x += dt/6 (u1 + 2 u2 + 2 u3 + u4), projected; zeta += dt/6 (-2 Omega) (same sum of z parts).
__global__ void k_bve_final(double* __restrict__ x, double* __restrict__ zeta,
                            const double* __restrict__ u1, const double* __restrict__ u2,
                            const double* __restrict__ u3, const double* __restrict__ u4,
                            double dt, double omega, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s[3];
    for (int d = 0; d < 3; ++d) {
        const int64_t k = 3 * i + d;
        s[d] = u1[k] + 2.0 * u2[k] + 2.0 * u3[k] + u4[k];
    }
    double p0 = x[3 * i] + (dt / 6.0) * s[0];
    double p1 = x[3 * i + 1] + (dt / 6.0) * s[1];
    double p2 = x[3 * i + 2] + (dt / 6.0) * s[2];
    const double r = 1.0 / sqrt(p0 * p0 + p1 * p1 + p2 * p2);
    x[3 * i] = p0 * r;
    x[3 * i + 1] = p1 * r;
    x[3 * i + 2] = p2 * r;
    zeta[i] += (dt / 6.0) * (-2.0 * omega * s[2]);
}

}  // namespace
}  // namespace csfmm

using namespace csfmm;

extern "C" int csfmm_bve_rk4_step(double* x, double* zeta, const double* area, int64_t n,
                                  double dt, double omega, int p, double theta, int leaf_size,
                                  unsigned flags, int use_direct, void* stream) {
    clear_error();
    if (!x || !zeta || !area || n < 1 || !(dt > 0.0) || !std::isfinite(omega)) {
        set_error("bve: non-NULL arrays, n >= 1, dt > 0 and a finite omega required");
        return CSFMM_E_INVALID;
    }
    if (flags & ~unsigned(CSFMM_FP32_FORM)) {
        set_error("unknown flags 0x%x", flags);
        return CSFMM_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* buf = nullptr;
    // four stage velocities [n][3], stage positions [n][3], stage weights [n]
    CSFMM_HIP_TRY(hipMallocAsync((void**)&buf, sizeof(double) * size_t(n) * (4 * 3 + 3 + 1), s));
    double* u[4];
    for (int k = 0; k < 4; ++k) u[k] = buf + size_t(k) * 3 * n;
    double* xs = buf + size_t(12) * n;
    double* ws = buf + size_t(15) * n;
    const unsigned grid = unsigned((n + 255) / 256);
    const double cstage[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
    int rc = CSFMM_OK;
    for (int k = 0; k < 4 && rc == CSFMM_OK; ++k) {
        k_bve_stage<<<grid, 256, 0, s>>>(x, zeta, area, k ? u[k - 1] : nullptr, cstage[k], omega,
                                         n, xs, ws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("bve stage launch failed: %s", hipGetErrorString(e));
            rc = CSFMM_E_HIP;
            break;
        }
        if (use_direct) {
            rc = launch_direct(xs, n, xs, n, ws, CSFMM_K_BIOT_SAVART, (flags & CSFMM_FP32_FORM) != 0,
                               u[k], s);
        } else {
            csfmm_plan_t plan = nullptr;
            rc = csfmm_plan(xs, n, nullptr, 0, CSFMM_K_BIOT_SAVART, p, theta, leaf_size, flags, s,
                            &plan);
            if (rc == CSFMM_OK) rc = csfmm_eval(plan, ws, u[k], s);
            if (plan) {
                // the plan's buffers are in use by the eval until the stream gets there
                hipError_t e = hipStreamSynchronize(s);
                if (e != hipSuccess && rc == CSFMM_OK) {
                    set_error("bve: %s", hipGetErrorString(e));
                    rc = CSFMM_E_HIP;
                }
                csfmm_plan_destroy(plan);
            }
        }
    }
    if (rc == CSFMM_OK) {
        k_bve_final<<<grid, 256, 0, s>>>(x, zeta, u[0], u[1], u[2], u[3], dt, omega, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("bve final launch failed: %s", hipGetErrorString(e));
            rc = CSFMM_E_HIP;
        }
    }
    (void)hipFreeAsync(buf, s);
    return rc;
}

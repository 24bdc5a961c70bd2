// Barotropic vorticity equation on the rotating sphere (paper §2.3, eqs. BVE
// and BVE_ODEs; §12): Lagrangian particles x_i with vorticity zeta_i and
// fixed areas A_i,
//     dx_i/dt = sum_j K_BS(x_i, x_j) zeta_j A_j,   dzeta_i/dt = -2 Omega dz_i/dt,
// one classical 4th order Runge-Kutta step per call.  Every stage builds a
// plan on the stage positions (the particles move) and evaluates the
// Biot-Savart sum with it (or with the direct sum); stage positions and the
// final positions are projected back onto the sphere.  csfmm_bve_remesh maps
// the particles back onto the cubed-sphere grid after a step.
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

// ---- remeshing (paper §12: every step, by local biquadratic interpolation),
// read as a backward remap onto the equiangular cubed-sphere grid the step
// started from.  Particle g started at cell centre y_g and ended at x_g.  The
// flow map is the biquadratic interpolant of the displacement D = x - y over
// the grid; the departure point a of each cell centre solves
// normalize(a + D(a)) = y by kRemeshIters fixed-point steps
// a <- normalize(y - D(a)) from a = y; the particles carry the absolute
// vorticity q = zeta + 2 Omega z, so the new vorticity at y is
// q(a) - 2 Omega z(y).

constexpr int kRemeshIters = 8;

// Face frames of the grid (outward normal, first tangent, second tangent):
// point f E^2 + i E + j is the centre of cell (i, j) of face f.
__constant__ double kFace[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},  {{-1, 0, 0}, {0, 0, 1}, {0, 1, 0}},
    {{0, 1, 0}, {0, 0, 1}, {1, 0, 0}},  {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{0, 0, 1}, {1, 0, 0}, {0, 1, 0}},  {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

__device__ __forceinline__ double dot3(const double* u, double a0, double a1, double a2) {
    return u[0] * a0 + u[1] * a1 + u[2] * a2;
}

// The face whose normal is closest to a (the first of equals), or `face` if
// it is not negative, and a's angles on it: (atan(a.e1 / a.n), atan(a.e2 / a.n)).
__device__ __forceinline__ int face_angles(double a0, double a1, double a2, int face, double& xi,
                                           double& eta) {
    int f = face;
    if (f < 0) {
        f = 0;
        double best = dot3(kFace[0][0], a0, a1, a2);
        for (int k = 1; k < 6; ++k) {
            const double v = dot3(kFace[k][0], a0, a1, a2);
            if (v > best) {
                best = v;
                f = k;
            }
        }
    }
    const double an = dot3(kFace[f][0], a0, a1, a2);
    xi = atan(dot3(kFace[f][1], a0, a1, a2) / an);
    eta = atan(dot3(kFace[f][2], a0, a1, a2) / an);
    return f;
}

// Nearest node of an angle (clamped to [lo, hi]) and its three Lagrange
// weights at the uniform angle spacing d.
__device__ __forceinline__ int stencil3(double ang, double d, int lo, int hi, double* w) {
    const double q = 0.25 * M_PI;
    const int c = int(fmin(fmax(rint((ang + q) / d - 0.5), double(lo)), double(hi)));
    const double s = (ang - (-q + (c + 0.5) * d)) / d;
    w[0] = 0.5 * s * (s - 1.0);
    w[1] = (1.0 - s) * (1.0 + s);
    w[2] = 0.5 * s * (s + 1.0);
    return c;
}

__device__ __forceinline__ void axpy4(double w, const double4& v, double4& acc) {
    acc.x += w * v.x;
    acc.y += w * v.y;
    acc.z += w * v.z;
    acc.w += w * v.w;
}

// Biquadratic interpolation of V at unit vector a on face `face`, the stencil
// clamped to that face (one-sided within a cell of its edges).
__device__ double4 interp_clamped(const double4* __restrict__ V, int64_t E, double a0, double a1,
                                  double a2, int face) {
    const double d = (0.5 * M_PI) / double(E);
    double xi, eta, wi[3], wj[3];
    const int f = face_angles(a0, a1, a2, face, xi, eta);
    const int ci = stencil3(xi, d, 1, int(E) - 2, wi);
    const int cj = stencil3(eta, d, 1, int(E) - 2, wj);
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int di = 0; di < 3; ++di)
        for (int dj = 0; dj < 3; ++dj)
            axpy4(wi[di] * wj[dj], V[(f * E + ci + di - 1) * E + cj + dj - 1], acc);
    return acc;
}

// Biquadratic interpolation of V at unit vector a: the 3 x 3 stencil centred
// on the nearest node of a's face; a node beyond the face edge (angle index -1
// or E) lies on a node line of the face across that edge (gnomonic
// projection) and takes the value interpolated there by interp_clamped.  A
// corner node (both indices beyond) is as far from the faces across either
// edge; it takes the one across its first angle's edge, so that no rounding
// decides.
__device__ double4 interp_ghost(const double4* __restrict__ V, int64_t E, double a0, double a1,
                                double a2) {
    const double d = (0.5 * M_PI) / double(E), q = 0.25 * M_PI;
    double xi, eta, wi[3], wj[3];
    const int f = face_angles(a0, a1, a2, -1, xi, eta);
    const int ci = stencil3(xi, d, 0, int(E) - 1, wi);
    const int cj = stencil3(eta, d, 0, int(E) - 1, wj);
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int di = 0; di < 3; ++di) {
        for (int dj = 0; dj < 3; ++dj) {
            const int i = ci + di - 1, j = cj + dj - 1;
            double4 v;
            if (i >= 0 && i < E && j >= 0 && j < E) {
                v = V[(f * E + i) * E + j];
            } else {
                const double ta = tan(-q + (i + 0.5) * d), tb = tan(-q + (j + 0.5) * d);
                double p[3];
                for (int k = 0; k < 3; ++k)
                    p[k] = kFace[f][0][k] + ta * kFace[f][1][k] + tb * kFace[f][2][k];
                const double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
                // the face across the edge: normal -e1 / +e1 if i is beyond,
                // else -e2 / +e2
                const int t = (i < 0 || i >= E) ? 1 : 2;
                const double sg = (i < 0 || (i < E && j < 0)) ? -1.0 : 1.0;
                int across = 0;
                for (int k = 1; k < 6; ++k)
                    if (dot3(kFace[k][0], sg * kFace[f][t][0], sg * kFace[f][t][1],
                             sg * kFace[f][t][2]) > 0.5)
                        across = k;
                v = interp_clamped(V, E, p[0] / r, p[1] / r, p[2] / r, across);
            }
            axpy4(wi[di] * wj[dj], v, acc);
        }
    }
    return acc;
}

// (D, q) of every particle: the displacement from its cell centre and its
// absolute vorticity.
__global__ void k_remesh_prep(const double* __restrict__ grid, const double* __restrict__ x,
                              const double* __restrict__ zeta, double omega, int64_t n,
                              double4* __restrict__ dq) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    dq[g] = make_double4(x[3 * g] - grid[3 * g], x[3 * g + 1] - grid[3 * g + 1],
                         x[3 * g + 2] - grid[3 * g + 2], zeta[g] + 2.0 * omega * x[3 * g + 2]);
}

// One thread per cell centre: departure point, new vorticity, particle back
// at the centre.
__global__ void k_remesh(const double* __restrict__ grid, int64_t E,
                         const double4* __restrict__ dq, double omega, int64_t n,
                         double* __restrict__ x, double* __restrict__ zeta) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const double y0 = grid[3 * g], y1 = grid[3 * g + 1], y2 = grid[3 * g + 2];
    double a0 = y0, a1 = y1, a2 = y2;
    for (int it = 0; it < kRemeshIters; ++it) {
        const double4 v = interp_ghost(dq, E, a0, a1, a2);
        const double p0 = y0 - v.x, p1 = y1 - v.y, p2 = y2 - v.z;
        const double r = sqrt(p0 * p0 + p1 * p1 + p2 * p2);
        a0 = p0 / r;
        a1 = p1 / r;
        a2 = p2 / r;
    }
    zeta[g] = interp_ghost(dq, E, a0, a1, a2).w - 2.0 * omega * y2;
    x[3 * g] = y0;
    x[3 * g + 1] = y1;
    x[3 * g + 2] = y2;
}

}  // namespace
}  // namespace csfmm

using namespace csfmm;

extern "C" int csfmm_bve_remesh(const double* grid, int64_t E, double* x, double* zeta,
                                double omega, void* stream) {
    clear_error();
    if (!grid || !x || !zeta || E < 3 || E > (int64_t(1) << 14) || !std::isfinite(omega)) {
        set_error("bve remesh: non-NULL arrays, 3 <= E <= 16384 and a finite omega required");
        return CSFMM_E_INVALID;
    }
    const int64_t n = 6 * E * E;
    if ((grid < x + 3 * n && x < grid + 3 * n) || (zeta < grid + 3 * n && grid < zeta + n) ||
        (zeta < x + 3 * n && x < zeta + n)) {
        set_error("bve remesh: grid, x and zeta must not overlap");
        return CSFMM_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double4* dq = nullptr;
    CSFMM_HIP_TRY(hipMallocAsync((void**)&dq, sizeof(double4) * size_t(n), s));
    const unsigned grd = unsigned((n + 255) / 256);
    k_remesh_prep<<<grd, 256, 0, s>>>(grid, x, zeta, omega, n, dq);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        k_remesh<<<grd, 256, 0, s>>>(grid, E, dq, omega, n, x, zeta);
        e = hipGetLastError();
    }
    (void)hipFreeAsync(dq, s);
    if (e != hipSuccess) {
        set_error("bve remesh launch failed: %s", hipGetErrorString(e));
        return CSFMM_E_HIP;
    }
    return CSFMM_OK;
}

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

"""Pins of the inputs and of the FP64 direct-sum oracle against what the paper
and the mathematics fix (no GPU).

* grid: paper Table 1 (N, delta_phi), total area 4 pi, the ~0.7 area ratio
  of the equiangular cubed sphere (§3);
* spherical harmonics: orthonormality by an independent quadrature;
* Poisson eigenrelation (§2.1, eq. G_L with -Laplace(phi) = f, read with the
  sign that agrees with eq. G_L_2) and its second order convergence (§10.2);
* eq. G_L_2 for the constant harmonic;
* the 1/|x-y| eigenvalue 4 pi/(2n+1) from eq. (Legendre) and eq.
  (kernel_Legendre) (Funk-Hecke), first order because of the omitted
  singular cell;
* Biot-Savart: K_BS = grad G_L x x (§2.3) gives u = grad(psi) x x;
* symmetry of the kernels; 50-digit brute force with the literal formulas;
* biharmonic (eq. G_B): Legendre coefficients 1/(n^2 (n+1)^2) (the
  eigenvalues of the biharmonic operator, §2.2) and pi^2/6 - 1 for n = 0,
  by Funk-Hecke quadrature of the oracle's kernel; closed-form dilogarithm
  values; second order convergence of the eigenrelation on the grid;
* SAL (eq. G_SAL_approx): Legendre coefficients (1 - b0) + (a1 - b1)/n of
  the series eq. (G_SAL) with the Love number fit, i.e. the multipliers of
  eq. (salsh), by the same quadrature.
"""

import math
import os

import mpmath
import numpy as np
import pytest

from workloads import cubed_sphere_grid, random_sphere_points, real_sph_harm_all, real_y43, real_y41
from oracle import direct

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel_err(a, b, area, ref):
    d = np.asarray(a) - np.asarray(b)
    if d.ndim == 2:
        num = np.sum(np.sum(d * d, axis=1) * area)
        den = np.sum(np.sum(ref * ref, axis=1) * area)
    else:
        num = np.sum(d * d * area)
        den = np.sum(ref * ref * area)
    return math.sqrt(num / den)


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------------ inputs

def test_grid_matches_table1():
    for L, N, dphi in _read_golden("table1_cubed_sphere.txt"):
        L, N, dphi = int(L), int(N), float(dphi)
        E = 2 ** L  # paper level L: N = 6 * 4^L cells, E = 2^L per face edge
        assert 6 * E * E == N
        got = math.sqrt(4.0 * math.pi / N) * 180.0 / math.pi
        assert abs(got - dphi) <= 0.5 * 10 ** (math.floor(math.log10(dphi)) - 2) + 1e-12
        if N <= 98304:
            P, A = cubed_sphere_grid(E)
            assert P.shape == (N, 3)


@pytest.mark.parametrize("E", [2, 8, 32, 128])
def test_grid_areas_and_norms(E):
    P, A = cubed_sphere_grid(E)
    assert abs(A.sum() - 4.0 * math.pi) < 1e-12
    assert np.max(np.abs(np.sqrt((P * P).sum(1)) - 1.0)) < 4e-16
    # distinct points
    assert np.unique(P, axis=0).shape[0] == P.shape[0]
    if E >= 32:
        r = A.min() / A.max()
        assert 0.70 < r < 0.73  # §3: ratio approximately 0.7


def test_grid_area_by_monte_carlo():
    """Independent check of the exact areas: uniform random points counted per cell."""
    E = 4
    P, A = cubed_sphere_grid(E)
    X = random_sphere_points(400000, 11)
    ax = np.argmax(np.abs(X), axis=1)
    d = (math.pi / 2) / E
    # points of the +z face, binned by their equiangular cell
    sel = (ax == 2) & (X[:, 2] > 0)
    a = np.arctan(X[sel, 0] / X[sel, 2])
    b = np.arctan(X[sel, 1] / X[sel, 2])
    ia = np.floor((a + math.pi / 4) / d).astype(int)
    ib = np.floor((b + math.pi / 4) / d).astype(int)
    frac = np.bincount(ia * E + ib, minlength=E * E) / X.shape[0]
    # the +z face areas are the first-face block pattern (all faces identical)
    exact = A[: E * E].reshape(E, E).reshape(-1) / (4 * math.pi)
    assert np.allclose(np.sort(frac), np.sort(exact), atol=5e-4)


def test_sph_orthonormal_by_quadrature():
    nmax = 8
    zq, wq = np.polynomial.legendre.leggauss(24)
    nl = 40
    lam = 2 * np.pi * np.arange(nl) / nl
    Z, LAM = np.meshgrid(zq, lam, indexing="ij")
    s = np.sqrt(1 - Z * Z)
    pts = np.stack([s * np.cos(LAM), s * np.sin(LAM), Z], axis=-1).reshape(-1, 3)
    wts = (wq[:, None] * np.full(nl, 2 * np.pi / nl)[None, :]).reshape(-1)
    Y = real_sph_harm_all(pts, nmax)
    G = (Y * wts[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(G.shape[1]))) < 1e-12


def test_closed_form_harmonics_match_recurrence():
    pts = random_sphere_points(500, 3)
    Y = real_sph_harm_all(pts, 4)
    y43 = Y[:, 16 + 4 + 3] / math.sqrt(2.0)
    y41 = Y[:, 16 + 4 + 1] / math.sqrt(2.0)
    for got, ref in ((real_y43(pts), y43), (real_y41(pts), y41)):
        sgn = np.sign(np.dot(got, ref))
        assert np.max(np.abs(got - sgn * ref)) < 1e-13


# --------------------------------------------------------- direct oracle

def _poisson_err(E, f_fn, exact_scale):
    P, A = cubed_sphere_grid(E)
    f = f_fn(P)
    phi = direct(1, P, P, f * A)
    return _rel_err(phi, exact_scale * f, A, exact_scale * f)


def test_P1_poisson_eigenrelation_sign_and_order():
    """-Lap(phi) = f and Lap Y = -n(n+1) Y give phi = +Y/(n(n+1)) = f/20 for n = 4."""
    errs = [_poisson_err(E, real_y43, 1.0 / 20.0) for E in (16, 32, 64)]
    assert errs[1] < 4e-2
    for a, b in zip(errs, errs[1:]):
        assert 3.0 <= a / b <= 4.5, errs
    # the sign printed in eq. (G_L_1) fails outright
    assert _poisson_err(32, real_y43, -1.0 / 20.0) > 1.5


def test_P2_constant_harmonic():
    """eq. (G_L_2): constant Y00 maps to (1 - ln 2)/(2 sqrt(pi))."""
    rows = dict((r[0], float(r[1])) for r in _read_golden("eq_G_L_2.txt"))
    assert abs(rows["Y00"] - 1 / (2 * math.sqrt(math.pi))) < 1e-16
    errs = []
    for E in (8, 16, 32):
        P, A = cubed_sphere_grid(E)
        phi = direct(1, P, P, np.full(P.shape[0], rows["Y00"]) * A)
        errs.append(np.max(np.abs(phi - rows["result"])) / rows["result"])
    assert errs[-1] < 2e-2
    assert errs[0] > errs[1] > errs[2]


def test_P3_inverse_distance_eigenvalue():
    """1/|x-y| = sum_n P_n(x.y) (eq. Legendre) -> eigenvalue 4 pi/(2n+1)."""
    errs = []
    for E in (16, 32, 64):
        P, A = cubed_sphere_grid(E)
        f = real_y43(P)
        phi = direct(3, P, P, f * A)
        ref = 4 * math.pi / 9 * f
        errs.append(_rel_err(phi, ref, A, ref))
    for a, b in zip(errs, errs[1:]):
        assert 1.8 <= a / b <= 2.2, errs
    assert errs[-1] < 0.1


def _bs_exact(P):
    """u = grad(psi) x x with psi = zeta/20, zeta = Re Y_4^1 = c x z (4z^2-3x^2-3y^2)."""
    c = -(3.0 / 8.0) * math.sqrt(5.0 / math.pi)
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    gx = c * (4 * z ** 3 - 9 * x * x * z - 3 * y * y * z)
    gy = c * (-6 * x * y * z)
    gz = c * (12 * x * z * z - 3 * x ** 3 - 3 * x * y * y)
    g = np.stack([gx, gy, gz], axis=1) / 20.0
    return np.cross(g, P)


def test_P4_biot_savart_closed_form():
    errs = []
    for E in (16, 32, 64):
        P, A = cubed_sphere_grid(E)
        u = direct(2, P, P, real_y41(P) * A)
        ref = _bs_exact(P)
        errs.append(_rel_err(u, ref, A, ref))
    for a, b in zip(errs, errs[1:]):
        assert 3.5 <= a / b <= 4.5, errs
    assert errs[1] < 1e-2


def test_P5_symmetry():
    P, A = cubed_sphere_grid(8)
    rng = np.random.default_rng(5)
    v, w = rng.standard_normal(P.shape[0]), rng.standard_normal(P.shape[0])
    for k in (1, 3):
        a = np.dot(v, direct(k, P, P, w))
        b = np.dot(w, direct(k, P, P, v))
        assert abs(a - b) <= 1e-13 * (abs(a) + abs(b))
    # K_BS(x, y) = -K_BS(y, x): with unit weights on single points
    X = random_sphere_points(2, 9)
    uxy = direct(2, X[:1], X[1:], np.ones(1))
    uyx = direct(2, X[1:], X[:1], np.ones(1))
    assert np.allclose(uxy, -uyx, rtol=1e-14, atol=0)


def _mp_direct(kernel, X, Y, w):
    mpmath.mp.dps = 50
    out = []
    for x in X:
        xs = [mpmath.mpf(float(v)) for v in x]
        acc = [mpmath.mpf(0)] * 3
        for y, wj in zip(Y, w):
            if x[0] == y[0] and x[1] == y[1] and x[2] == y[2]:
                continue
            ys = [mpmath.mpf(float(v)) for v in y]
            dot = xs[0] * ys[0] + xs[1] * ys[1] + xs[2] * ys[2]
            om = 1 - dot
            wm = mpmath.mpf(float(wj))
            if kernel == 1:
                acc[0] += -mpmath.log(om) / (4 * mpmath.pi) * wm
            elif kernel == 3:
                acc[0] += wm / mpmath.sqrt(2 * om)
            elif kernel == 4:
                acc[0] += mpmath.polylog(2, (1 + dot) / 2) / (4 * mpmath.pi) * wm
            elif kernel == 5:
                g = mpmath.sqrt(2 * om)
                a1, b0, b1 = mpmath.mpf("-2.7"), mpmath.mpf("-6.21196"), mpmath.mpf("6.1")
                c = 3 * mpmath.mpf(1025) / mpmath.mpf(5514) / (4 * mpmath.pi)
                acc[0] += c * ((1 - b0) / g - (a1 - b1) * mpmath.log(g / 2 + g * g / 4)) * wm
            else:
                cr = [xs[1] * ys[2] - xs[2] * ys[1], xs[2] * ys[0] - xs[0] * ys[2],
                      xs[0] * ys[1] - xs[1] * ys[0]]
                for k in range(3):
                    acc[k] += -cr[k] / (4 * mpmath.pi * om) * wm
        out.append([float(a) for a in acc])
    out = np.array(out)
    return out if kernel == 2 else out[:, 0]


@pytest.mark.parametrize("kernel", [1, 2, 3, 4, 5])
def test_P6_mpmath_brute_force(kernel):
    P, A = cubed_sphere_grid(2)
    X = random_sphere_points(40, 21)
    rng = np.random.default_rng(22)
    for T, S in ((P, P), (X, P), (X, X)):
        w = rng.standard_normal(S.shape[0])
        ref = _mp_direct(kernel, T, S, w)
        got = direct(kernel, T, S, w)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale


def test_oracle_rejects_bad_kernel():
    P, A = cubed_sphere_grid(1)
    with pytest.raises(ValueError):
        direct(9, P, P, A)


# ------------------------------------------- biharmonic and SAL kernels

SAL_A1, SAL_B0, SAL_B1 = -2.7, -6.21196, 6.1
SAL_RHO = 1025.0 / 5514.0


def _kernel_profile(kernel, s):
    """G(t) at t = 1 - 2 s^2 (|x - y| = 2 s) from the oracle, one pair per target."""
    X = np.stack([2 * s * np.sqrt(1 - s * s), np.zeros_like(s), 1 - 2 * s * s], axis=1)
    return direct(kernel, X, np.array([[0.0, 0.0, 1.0]]), np.ones(1))


def _legendre_coeffs(kernel, nmax):
    """lambda_n = 2 pi int_{-1}^{1} G(t) P_n(t) dt (Funk-Hecke), t = 1 - 2 s^2."""
    xg, wg = np.polynomial.legendre.leggauss(40)
    edges = [0.0, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2, 0.05, 0.2, 0.5, 0.8, 1.0]
    S, W = [], []
    for a, b in zip(edges, edges[1:]):
        S.append(0.5 * (b - a) * xg + 0.5 * (a + b))
        W.append(0.5 * (b - a) * wg)
    S, W = np.concatenate(S), np.concatenate(W)
    G = _kernel_profile(kernel, S)
    t = 1 - 2 * S * S
    out = []
    for n in range(nmax + 1):
        Pn = np.polynomial.legendre.legval(t, [0] * n + [1])
        out.append(2 * math.pi * np.sum(W * G * Pn * 4 * S))
    return np.array(out)


def test_P7_biharmonic_legendre_coefficients():
    """Delta^2 Y_n = n^2 (n+1)^2 Y_n (§2.2): G_B has coefficients 1/(n^2 (n+1)^2)."""
    lam = _legendre_coeffs(4, 8)
    assert abs(lam[0] - (math.pi ** 2 / 6 - 1)) < 1e-13  # int_0^1 dilog(u) du
    for n in range(1, 9):
        ref = 1.0 / (n * n * (n + 1) ** 2)
        assert abs(lam[n] - ref) <= 1e-11 * ref + 1e-15, (n, lam[n], ref)


def test_P8_sal_legendre_coefficients():
    """eq. (G_SAL) with k'_n = a1/n, h'_n = b0 + b1/n and eq. (Legendre):
    coefficient of P_n is (3 rw/(4 pi re)) ((1 - b0) + (a1 - b1)/n), so the
    convolution multiplier is (3 rw/re) ((1 - b0) + (a1 - b1)/n)/(2n + 1)
    (eq. salsh with the fit), and (3 rw/re)(1 - b0) for n = 0."""
    lam = _legendre_coeffs(5, 8)
    assert abs(lam[0] - 3 * SAL_RHO * (1 - SAL_B0)) < 1e-12
    for n in range(1, 9):
        ref = 3 * SAL_RHO * ((1 - SAL_B0) + (SAL_A1 - SAL_B1) / n) / (2 * n + 1)
        assert abs(lam[n] - ref) <= 1e-11 * abs(ref), (n, lam[n], ref)


def test_P9_dilog_closed_form_values():
    c = 1 / (4 * math.pi)
    # x.y = 0: dilog(1/2) = pi^2/12 - ln(2)^2/2; antipodes: dilog(0) = 0
    G = _kernel_profile(4, np.array([math.sqrt(0.5), 1.0]))
    assert abs(G[0] - c * (math.pi ** 2 / 12 - math.log(2) ** 2 / 2)) < 1e-16
    assert abs(G[1]) < 1e-17
    # coincident limit pi^2/6 (continuous kernel), approached at |x-y| = 2e-8
    G0 = _kernel_profile(4, np.array([1e-8]))
    assert abs(G0[0] - c * math.pi ** 2 / 6) < 1e-14
    # golden-ratio value dilog((3 - sqrt5)/2) = pi^2/15 - ln(phi)^2
    phi = (1 + math.sqrt(5)) / 2
    u = (3 - math.sqrt(5)) / 2          # (1 + t)/2 = u  ->  s^2 = 1 - u
    Gu = _kernel_profile(4, np.array([math.sqrt(1 - u)]))
    assert abs(Gu[0] - c * (math.pi ** 2 / 15 - math.log(phi) ** 2)) < 1e-15


def test_P10_biharmonic_eigenrelation_on_grid():
    """sum_j G_B(x_i, y_j) f_j A_j -> Y/(n^2(n+1)^2) for f = Y_2,1 (n = 2, 1/36),
    second order: the omitted i = j term of a continuous kernel is O(A)."""
    errs, fixed = [], []
    for E in (8, 16, 32):
        P, A = cubed_sphere_grid(E)
        f = real_sph_harm_all(P, 2)[:, 5]   # a degree-2 harmonic
        phi = direct(4, P, P, f * A)
        ref = f / 36.0
        errs.append(_rel_err(phi, ref, A, ref))
        # adding back the omitted diagonal G_B(x,x) f_i A_i removes the leading term
        fixed.append(_rel_err(phi + math.pi / 24 * f * A, ref, A, ref))
    for a, b in zip(errs, errs[1:]):
        assert 3.5 <= a / b <= 4.5, errs
    assert all(x < 0.2 * e for x, e in zip(fixed, errs)), (fixed, errs)
    assert fixed[-1] < 1e-3

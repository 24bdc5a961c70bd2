"""The biharmonic (eq. G_B) and SAL (eq. G_SAL_approx) kernels at full size on
the GPU: the Poisson workload's grid (E=256, N=393,216) and field, p=8,
theta=0.7, leaf 128, both precision forms, checked against the oracle's direct
sum at 1,024 seeded targets; and the biharmonic eigenrelation
G_B * Y_n = Y_n/(n^2 (n+1)^2) (§2.2) for a degree-2 harmonic, where the
method's error must sit below the grid's own quadrature error.

Gates (relative L2 over the sampled targets): 1e-5 for both forms and both
kernels; biharmonic eigenrelation 5e-6 after the omitted diagonal term
G_B(x,x) f_i A_i = (pi/24) f_i A_i is added back (the remaining midpoint-rule
error at this grid is about 2e-6, second order).
"""

import math

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from workloads import make_config, config_subset, real_sph_harm_all
from oracle import direct as odirect

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def tdev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def say(msg):
    print("\n[gpu case] " + msg, flush=True)


@pytest.fixture(scope="module")
def grid256():
    say("E=256 grid and field")
    c = make_config(2)
    S = config_subset(c["sources"].shape[0], 1024, 2004)
    return c, S


@pytest.mark.parametrize("kernel", [cs.BIHARMONIC, cs.SAL])
def test_full_size_against_oracle(grid256, kernel):
    c, S = grid256
    P, w = c["sources"], c["weights"]
    ref = odirect(kernel, P[S], P, w)
    T, W = tdev(P), tdev(w)
    for fp32 in (False, True):
        say("kernel %d E=256 p=8 fp32=%s" % (kernel, fp32))
        pl = cs.Plan(T, None, kernel=kernel, p=8, theta=0.7, leaf_size=128, fp32=fp32)
        out = pl.eval(W).cpu().numpy()
        pl.close()
        err = rel_l2(out[S], ref)
        print("rel_l2 %.3e" % err, flush=True)
        assert err <= 1e-5


def test_biharmonic_eigenrelation_full_size(grid256):
    c, _ = grid256
    P, A = c["sources"], c["areas"]
    f = real_sph_harm_all(P, 2)[:, 5]       # a degree-2 harmonic
    exact = f / 36.0                         # 1/(n^2 (n+1)^2) at n = 2
    T, W = tdev(P), tdev(f * A)
    for fp32 in (False, True):
        say("biharmonic eigenrelation E=256 fp32=%s" % fp32)
        pl = cs.Plan(T, None, kernel=cs.BIHARMONIC, p=8, theta=0.7, leaf_size=128, fp32=fp32)
        out = pl.eval(W).cpu().numpy()
        pl.close()
        fixed = out + math.pi / 24.0 * f * A
        e_raw = math.sqrt(np.sum((out - exact) ** 2 * A) / np.sum(exact ** 2 * A))
        e_fix = math.sqrt(np.sum((fixed - exact) ** 2 * A) / np.sum(exact ** 2 * A))
        print("raw %.3e  with diagonal %.3e" % (e_raw, e_fix), flush=True)
        assert e_fix < 5e-6 and e_fix < 0.05 * e_raw


@pytest.mark.parametrize("kernel,tol", [(cs.POISSON, 1e-15), (cs.BIOT_SAVART, 2e-15),
                                        (cs.INV_DIST, 1e-15), (cs.BIHARMONIC, 1e-14),
                                        (cs.SAL, 1e-15)])
def test_fp64_kernel_values_one_pair_at_a_time(kernel, tol):
    """The FP64 kernel values of the library's own logarithm, reciprocal and
    reciprocal square root, one (target, source) pair per output: one source,
    200,000 targets at distances from 1e-9 to the antipode (and around the
    zero of the Poisson logarithm, |x - y| = sqrt(2)), against the oracle's
    libm values element by element: |got - ref| <= tol (|ref| + median |ref|)
    (vector norms for Biot-Savart, plus the oracle's own rounding: it forms
    x cross y, whose components lose about 4e-16 absolute, so about
    4e-16 / |x - y| of |ref| for close pairs)."""
    say("one-pair kernel values, kernel %d" % kernel)
    from workloads import random_sphere_points
    rng = np.random.default_rng(61)
    y = np.array([[0.36, -0.48, 0.8]])
    X = random_sphere_points(150000, 62)
    # targets close to the source, down to 1e-9 away
    d = 10.0 ** rng.uniform(-9, -1, 40000)
    u = rng.standard_normal((40000, 3))
    u -= (u @ y[0])[:, None] * y
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    Xc = y + d[:, None] * u
    # targets near |x - y| = sqrt(2) (the great circle 90 degrees away)
    Xq = u[:10000] + rng.uniform(-1e-6, 1e-6, (10000, 1)) * y
    X = np.concatenate([X, Xc, Xq])
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    w = np.array([0.75])
    got = cs.direct(tdev(X), tdev(y), tdev(w), kernel=kernel).cpu().numpy()
    ref = odirect(kernel, X, y, w)
    if kernel == cs.BIOT_SAVART:
        err = np.linalg.norm(got - ref, axis=1)
        mag = np.linalg.norm(ref, axis=1)
    else:
        err, mag = np.abs(got - ref), np.abs(ref)
    bound = tol * (mag + np.median(mag))
    if kernel == cs.BIOT_SAVART:
        bound = bound + 1e-15 * mag / np.linalg.norm(X - y, axis=1)
    worst = float(np.max(err / bound)) * tol
    print("kernel %d worst scaled error %.3e (tol %.0e)" % (kernel, worst, tol), flush=True)
    assert np.all(np.isfinite(got))
    assert np.all(err <= bound)

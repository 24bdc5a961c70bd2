"""Pins of the nonuniform input meshes (no GPU): icosahedral sizes against
the particle counts of paper Table 3, Euler's formula, areas adding up to
4 pi, unit norms, second-order quadrature of a harmonic; exact latitude-
longitude areas."""

import math
import os

import numpy as np

from workloads import icosahedral_grid, latlon_grid, real_y43

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_icosahedral_sizes_match_table3():
    ns = None
    for line in open(os.path.join(GOLDEN, "table3_runtimes.txt")):
        if line.startswith("# method"):
            ns = [int(t.split("=")[1]) for t in line.split()[3:]]
    assert ns == [10 * 4 ** k + 2 for k in range(4, 10)]
    for k in range(0, 6):
        P, A, F = icosahedral_grid(k, return_faces=True)
        assert P.shape[0] == 10 * 4 ** k + 2
        edges = F.shape[0] * 3 // 2
        assert P.shape[0] - edges + F.shape[0] == 2        # Euler
        assert abs(A.sum() - 4 * math.pi) < 1e-13
        assert np.max(np.abs(np.linalg.norm(P, axis=1) - 1)) < 4e-16
        assert np.unique(P, axis=0).shape[0] == P.shape[0]


def test_icosahedral_quadrature_converges():
    errs = []
    for k in (3, 4, 5):
        P, A = icosahedral_grid(k)
        # Re Y_4^3 has mean 0 and mean square 1/2 over the sphere
        errs.append(abs(np.sum(real_y43(P) * A)) + abs(np.sum(real_y43(P) ** 2 * A) - 0.5))
    assert errs[-1] < 5e-6
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5   # second order in the spacing


def test_latlon_areas_and_points():
    P, A = latlon_grid(90, 180)
    assert P.shape == (16200, 3)
    assert abs(A.sum() - 4 * math.pi) < 1e-12
    band = A.reshape(90, 180)
    lat_e = np.radians(np.arange(-90, 91, 2))
    exact = (np.sin(lat_e[1:]) - np.sin(lat_e[:-1])) * 2 * math.pi / 180
    assert np.allclose(band, exact[:, None], rtol=1e-13, atol=0)
    assert np.max(np.abs(np.linalg.norm(P, axis=1) - 1)) < 4e-16
    # strongly nonuniform: polar cells are ~57 times smaller than equatorial ones
    assert 50 < A.max() / A.min() < 60

"""Pins of the BVE oracle (no GPU): the Rossby-Haurwitz wave of eq.
(RH_initial) is stationary, so its vorticity error (eq. bveerr) after 0.1
day is pure discretization error and falls at second order in the grid
spacing (the paper's O(dphi^2)); a solid-body rotation zeta = 2 w z without
planetary rotation turns the particles rigidly about the z axis at rate w
(to first order in the spacing on this mesh: a vertex is not the centroid of
its cell, so the omitted singular self cell no longer cancels)."""

import math

import numpy as np

from workloads import icosahedral_grid
from oracle import bve


def test_rossby_haurwitz_stationary_second_order():
    errs = []
    for k in (3, 4, 5):
        P, A = icosahedral_grid(k)
        x, z = bve.run(P, A, 10)
        errs.append(bve.vorticity_error(x, z, A))
        assert np.max(np.abs(x - P)) > 0.1   # the particles do move
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 4.5, errs
    assert errs[-1] < 1.5e-3


def test_solid_body_rotation_is_rigid():
    w = 1.5  # rad per day
    res = []
    for k in (3, 4):
        P, A = icosahedral_grid(k)
        x, zeta = P.copy(), 2.0 * w * P[:, 2]
        for _ in range(10):
            x, zeta = bve.rk4_step(x, zeta, A, 0.01, omega=0.0)
        ang = w * 0.1
        R = np.array([[math.cos(ang), -math.sin(ang), 0], [math.sin(ang), math.cos(ang), 0],
                      [0, 0, 1.0]])
        res.append(np.max(np.abs(x - P @ R.T)))
        # vorticity is unchanged without planetary rotation
        assert np.array_equal(zeta, 2.0 * w * P[:, 2])
    assert res[-1] < 1e-3 and 1.7 < res[0] / res[1] < 2.5


def test_rh_vorticity_closed_form():
    # with z = sin(lat): cos(lat)^4 cos(4 lon) = x^4 - 6 x^2 y^2 + y^4, so
    # zeta_0 = (2 pi/7) z + 30 z (x^4 - 6 x^2 y^2 + y^4)
    P, A = icosahedral_grid(4)
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    ref = (2 * math.pi / 7) * z + 30 * z * (x ** 4 - 6 * x * x * y * y + y ** 4)
    assert np.max(np.abs(bve.rh_vorticity(P) - ref)) < 1e-13
    assert abs(np.sum(bve.rh_vorticity(P) * A)) < 1e-12   # odd in z

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


# ---- remeshing (paper §12; the oracle's reading: backward remap onto the
# equiangular cubed-sphere grid by local biquadratic interpolation)

from workloads import cubed_sphere_grid, rh_vorticity
from workloads.grid import CUBE_FACES


def _angles(P):
    F = np.asarray(CUBE_FACES)
    f = np.argmax(P @ F[:, 0].T, axis=1)
    an = np.einsum("ij,ij->i", P, F[f, 0])
    return (f, np.arctan(np.einsum("ij,ij->i", P, F[f, 1]) / an),
            np.arctan(np.einsum("ij,ij->i", P, F[f, 2]) / an))


def _rotation(ang, axis):
    u = np.asarray(axis, dtype=np.float64)
    u /= np.linalg.norm(u)
    K = np.array([[0, -u[2], u[1]], [u[2], 0, -u[0]], [-u[1], u[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def test_remesh_without_motion_returns_the_field():
    for E in (3, 8, 17):
        P, A = cubed_sphere_grid(E)
        z = np.sin(3 * P[:, 0]) + P[:, 1] * P[:, 2]
        assert np.max(np.abs(bve.remesh(P, E, P, z, omega=2.0) - z)) < 1e-13


def test_biquadratic_reproduces_biquadratic_fields_inside_faces():
    """A field of degree <= 2 in each face angle (different on every face) is
    reproduced exactly wherever the stencil stays on the face; the weights,
    node indices and face frames all enter."""
    E = 16
    P, A = cubed_sphere_grid(E)
    d = (math.pi / 2) / E

    def field(f, x, y):
        return 1 + f + (2 - f) * x - y + 3 * x * y + (1 + f) * x * x * y * y - 0.5 * y * y * x

    fP, xP, yP = _angles(P)
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((4000, 3))
    Q /= np.linalg.norm(Q, axis=1)[:, None]
    fQ, xQ, yQ = _angles(Q)
    inner = (np.abs(xQ) < math.pi / 4 - 1.5 * d) & (np.abs(yQ) < math.pi / 4 - 1.5 * d)
    got = bve.biquadratic(field(fP, xP, yP), E, Q[inner])
    assert inner.sum() > 2000
    assert np.max(np.abs(got - field(fQ, xQ, yQ)[inner])) < 1e-12


def test_ghost_nodes_lie_on_node_lines_of_the_neighbour_face():
    """The reading's ghost values: the node one angle step beyond a face edge
    lies on a node line of the face across that edge (gnomonic projection),
    so interpolating it there is a quadratic along that line."""
    E = 12
    d = (math.pi / 2) / E
    F = np.asarray(CUBE_FACES)
    nodes = -math.pi / 4 + (np.arange(E) + 0.5) * d
    for f in range(6):
        for i in (-1, E):
            ta = math.tan(-math.pi / 4 + (i + 0.5) * d)
            tb = np.tan(nodes)
            p = F[f, 0] + ta * F[f, 1] + tb[:, None] * F[f, 2]
            p /= np.linalg.norm(p, axis=1)[:, None]
            g, x, y = _angles(p)
            assert np.all(g != f)
            on = np.minimum(np.abs((x + math.pi / 4) / d - 0.5 - np.rint((x + math.pi / 4) / d - 0.5)),
                            np.abs((y + math.pi / 4) / d - 0.5 - np.rint((y + math.pi / 4) / d - 0.5)))
            assert np.max(on) < 1e-12


def test_remesh_of_a_rigid_rotation_converges_at_third_order():
    """Particles turned rigidly (0.4 of a cell's angle about a skew axis)
    carry the absolute vorticity q = f(start point); the remeshed vorticity
    is f(R^-1 y) - 2 Omega z(y) up to the interpolation error, O(h^3) when
    the displacement is a fixed fraction of the cell."""
    om = 2 * math.pi
    errs = []
    for E in (16, 32, 64):
        R = _rotation(0.4 * (math.pi / 2) / E, (0.3, -0.5, 0.8))
        P, A = cubed_sphere_grid(E)
        X = P @ R.T
        f = np.exp(P[:, 0]) * np.cos(2 * P[:, 1]) + P[:, 2] ** 2
        got = bve.remesh(P, E, X, f - 2 * om * X[:, 2], omega=om)
        B = P @ R
        want = np.exp(B[:, 0]) * np.cos(2 * B[:, 1]) + B[:, 2] ** 2 - 2 * om * P[:, 2]
        errs.append(np.max(np.abs(got - want)))
    assert errs[-1] < 5e-5
    for a, b in zip(errs, errs[1:]):
        assert a / b > 7.0, errs


def test_remeshed_rossby_haurwitz_second_order():
    """The stationary Rossby-Haurwitz wave remeshed after each of 10 steps:
    the vorticity error at the cell centres falls at second order (the
    quadrature's; a remesh adds O(h^2) times the step's displacement)."""
    errs = []
    for E in (8, 16, 32):
        P, A = cubed_sphere_grid(E)
        errs.append(bve.vorticity_error(P, bve.run_remeshed(P, A, E, 10), A))
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs
    assert errs[-1] < 1.2e-3

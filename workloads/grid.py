"""Point sets on the unit sphere.

* The equiangular gnomonic cubed-sphere grid (paper §3 and Fig. 1b, read as
  equiangular: the cells are the images of a uniform grid in the local angles
  (xi, eta) of each cube face).  Quadrature points are the cell centres, the
  areas A_j are the exact geodesic areas of the cells (paper eq. nbodysum).
* Seeded uniform random points (normalised standard Gaussians).
"""

import numpy as np

# The six cube faces as (outward normal, first tangent, second tangent).  The
# grid is symmetric under every rotation of the cube, so the frame chosen here
# only fixes the order in which the points are listed.
_FACES = (
    ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)),
    ((-1.0, 0.0, 0.0), (0.0, 0.0, 1.0), (0.0, 1.0, 0.0)),
    ((0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (1.0, 0.0, 0.0)),
    ((0.0, -1.0, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0)),
    ((0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)),
    ((0.0, 0.0, -1.0), (0.0, 1.0, 0.0), (1.0, 0.0, 0.0)),
)
# Public name of the face order: point f E^2 + i E + j of cubed_sphere_grid(E)
# is the centre of cell (i, j) of face f, i along the first tangent.
CUBE_FACES = _FACES


def _solid_angle_corner(X, Y):
    """Solid angle of the plane rectangle [0,X]x[0,Y] on z=1 seen from 0."""
    return np.arctan(X * Y / np.sqrt(1.0 + X * X + Y * Y))


def cubed_sphere_grid(E):
    """Cell centres and exact areas of the equiangular cubed sphere.

    E cells per face edge, N = 6 E^2 cells (paper Table 1 lists E = 2^L).
    Returns (points [N,3] float64 with unit norm, areas [N] float64).
    """
    E = int(E)
    if E < 1:
        raise ValueError("E must be >= 1")
    d = (np.pi / 2.0) / E
    edges = -np.pi / 4.0 + d * np.arange(E + 1)
    mids = -np.pi / 4.0 + d * (np.arange(E) + 0.5)
    T = np.tan(edges)
    tm = np.tan(mids)
    # exact cell areas on one face (identical on all six)
    F = _solid_angle_corner(T[:, None], T[None, :])
    area = F[1:, 1:] - F[:-1, 1:] - F[1:, :-1] + F[:-1, :-1]
    a = np.repeat(tm, E)          # first local tangent coordinate
    b = np.tile(tm, E)            # second local tangent coordinate
    inv = 1.0 / np.sqrt(1.0 + a * a + b * b)
    pts = []
    for n, e1, e2 in _FACES:
        n = np.asarray(n)
        e1 = np.asarray(e1)
        e2 = np.asarray(e2)
        p = (n[None, :] + a[:, None] * e1[None, :] + b[:, None] * e2[None, :]) * inv[:, None]
        pts.append(p)
    P = np.concatenate(pts, axis=0)
    # one more normalisation so that |x| = 1 to the last bit or two
    P /= np.sqrt(np.einsum("ij,ij->i", P, P))[:, None]
    A = np.tile(area.reshape(-1), 6)
    return np.ascontiguousarray(P), np.ascontiguousarray(A)


def random_sphere_points(n, seed):
    """n points uniform on the unit sphere: normalised N(0, I3) draws (PCG64)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((int(n), 3))
    g /= np.sqrt(np.einsum("ij,ij->i", g, g))[:, None]
    return np.ascontiguousarray(g)

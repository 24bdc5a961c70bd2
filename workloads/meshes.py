"""Nonuniform point sets on the unit sphere.

* Icosahedral grids (the paper's timing grid, §10): the twelve vertices of
  the regular icosahedron, each triangle split into four by its edge
  midpoints k times with the new vertices projected onto the sphere;
  N = 10 * 4^k + 2 (k = 8 gives the paper's N = 655,362).  A vertex carries a
  third of the area of every spherical triangle it belongs to, so the areas
  add up to 4 pi.
* Latitude-longitude grids: cell centres of an nlat x nlon grid, uniform in
  latitude and longitude, with exact cell areas; the points crowd together
  towards the poles (a strongly nonuniform set for the adaptive tree).
"""

import numpy as np


def _icosahedron():
    t = (1.0 + np.sqrt(5.0)) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return V / np.linalg.norm(V, axis=1, keepdims=True), F


def _subdivide(V, F):
    """Split every triangle into four; midpoints projected onto the sphere."""
    E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    E.sort(axis=1)
    key = E[:, 0] * (V.shape[0] + 1) + E[:, 1]
    uniq, inv = np.unique(key, return_inverse=True)
    a, b = uniq // (V.shape[0] + 1), uniq % (V.shape[0] + 1)
    M = V[a] + V[b]
    M /= np.linalg.norm(M, axis=1, keepdims=True)
    m = inv.reshape(3, -1) + V.shape[0]  # midpoints of edges 01, 12, 20
    m01, m12, m20 = m[0], m[1], m[2]
    F2 = np.concatenate([
        np.stack([F[:, 0], m01, m20], axis=1),
        np.stack([F[:, 1], m12, m01], axis=1),
        np.stack([F[:, 2], m20, m12], axis=1),
        np.stack([m01, m12, m20], axis=1)])
    return np.concatenate([V, M]), F2


def _spherical_triangle_area(A, B, C):
    """Area of the spherical triangles ABC (unit vectors), from
    tan(E/2) = |A.(B x C)| / (1 + A.B + B.C + C.A)."""
    num = np.abs(np.einsum("ij,ij->i", A, np.cross(B, C)))
    den = 1.0 + np.einsum("ij,ij->i", A, B) + np.einsum("ij,ij->i", B, C) + \
        np.einsum("ij,ij->i", C, A)
    return 2.0 * np.arctan2(num, den)


def icosahedral_grid(k, return_faces=False):
    """Vertices of the k-times subdivided icosahedron and their areas.

    Returns (points [N,3], areas [N]) with N = 10 * 4^k + 2 (and the
    triangles [20 * 4^k, 3] if return_faces).
    """
    k = int(k)
    if k < 0:
        raise ValueError("k must be >= 0")
    V, F = _icosahedron()
    for _ in range(k):
        V, F = _subdivide(V, F)
    tri = _spherical_triangle_area(V[F[:, 0]], V[F[:, 1]], V[F[:, 2]])
    area = np.zeros(V.shape[0])
    for c in range(3):
        np.add.at(area, F[:, c], tri / 3.0)
    if return_faces:
        return V, area, F
    return V, area


def latlon_grid(nlat, nlon):
    """Cell centres of a uniform latitude-longitude grid and exact areas.

    Cells [lat_i, lat_i+1] x [lon_j, lon_j+1]; the centre is at the middle
    latitude and longitude.  Returns (points [nlat*nlon, 3], areas).
    """
    nlat, nlon = int(nlat), int(nlon)
    if nlat < 1 or nlon < 1:
        raise ValueError("nlat, nlon must be >= 1")
    lat_e = np.linspace(-np.pi / 2.0, np.pi / 2.0, nlat + 1)
    lon_e = np.linspace(0.0, 2.0 * np.pi, nlon + 1)
    lat = 0.5 * (lat_e[:-1] + lat_e[1:])
    lon = 0.5 * (lon_e[:-1] + lon_e[1:])
    LAT, LON = np.meshgrid(lat, lon, indexing="ij")
    P = np.stack([np.cos(LAT) * np.cos(LON), np.cos(LAT) * np.sin(LON), np.sin(LAT)], axis=-1)
    P = P.reshape(-1, 3)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    band = (np.sin(lat_e[1:]) - np.sin(lat_e[:-1])) * (2.0 * np.pi / nlon)
    A = np.repeat(band, nlon)
    return P, A

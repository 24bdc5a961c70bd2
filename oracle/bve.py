"""ORACLE -- test infrastructure only.

The barotropic vorticity equation on the rotating sphere (paper §2.3,
eqs. BVE and BVE_ODEs; §12) by the Lagrangian vortex method, stepped with the
classical 4th order Runge-Kutta method, the velocity from the FP64 direct-sum
oracle.  Plain NumPy; shares no code with the GPU library.

The Rossby-Haurwitz initial vorticity is an input and comes from the
workloads package (with theta of eq. RH_initial read as the latitude: the
solid-body term is then the rotation omega = pi/7 per day = Omega/14 that
makes the degree-5 wave stationary for Omega = 2 pi per day, phase speed
(n(n+1) omega - 2(Omega + omega))/(n(n+1)) = 0 for n = 5).

Readings:
  * Particles stay on the sphere: after every Runge-Kutta stage and step the
    positions are projected back onto it (x / |x|).
  * Between remeshings the particles keep their areas A_j (the flow is
    incompressible, so a Lagrangian particle's area is constant).
  * Remeshing (§12: every step, by local biquadratic interpolation) is read
    as a backward remap onto the equiangular cubed-sphere grid the step
    started from (a tensor-product grid on each face, where biquadratic
    interpolation is defined).  Particle g started at cell centre y_g and
    ended at x_g.  The flow map of the step is represented by biquadratic
    interpolation of the displacement D_g = x_g - y_g over the grid, and each
    cell centre's departure point a_g solves normalize(a + D(a)) = y_g, found
    by the fixed-point iteration a <- normalize(y_g - D(a)) from a = y_g,
    REMESH_ITERS times.  The particles carry the absolute vorticity
    q_g = zeta_g + 2 Omega z(x_g) (eq. BVE_ODEs makes it constant along a
    trajectory), so the new vorticity at y_g is q(a_g) - 2 Omega z(y_g),
    q(a) again by biquadratic interpolation.  Interpolation at a point takes
    the face whose normal is closest to it, the face angles
    (xi, eta) = (atan(a.e1 / a.n), atan(a.e2 / a.n)), the 3 x 3 stencil centred
    on the nearest node and the product of the three-point Lagrange weights in
    the uniform angle spacing.  Stencil nodes beyond the face edge are ghost
    nodes at the same angle spacing; in the gnomonic projection a ghost node
    lies on a node line of the face across that edge, and its value is
    interpolated there with the stencil clamped to that face (a quadratic
    along the line).  A corner ghost (beyond both edges) is equidistant from
    the faces across the two edges and takes the one across its first
    angle's edge.  (Stencils clamped at the edges instead, one-sided,
    amplify a node-to-node zigzag when a step moves points more than a
    quarter cell, and remeshing every step makes that grow.)  After the
    remap the particles sit at the cell centres again.  parity pinned by
    tests: exact at nodes, exact for biquadratic fields away from edges,
    ghost nodes on the neighbouring face's node lines, third-order
    convergence under a rigid rotation, second order of the remeshed
    Rossby-Haurwitz run.
"""

import numpy as np

from workloads import rh_vorticity
from workloads.grid import CUBE_FACES

from .direct import direct

KERNEL_BIOT_SAVART = 2
OMEGA = 2.0 * np.pi  # per day


def _project(x):
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def rhs(x, zeta, area, omega=OMEGA):
    """eq. (BVE_ODEs): dx/dt = sum_j K_BS(x, x_j) zeta_j A_j, dzeta/dt = -2 Omega dz/dt."""
    u = direct(KERNEL_BIOT_SAVART, x, x, zeta * area)
    return u, -2.0 * omega * u[:, 2]


def rk4_step(x, zeta, area, dt, omega=OMEGA):
    k1x, k1z = rhs(x, zeta, area, omega)
    k2x, k2z = rhs(_project(x + 0.5 * dt * k1x), zeta + 0.5 * dt * k1z, area, omega)
    k3x, k3z = rhs(_project(x + 0.5 * dt * k2x), zeta + 0.5 * dt * k2z, area, omega)
    k4x, k4z = rhs(_project(x + dt * k3x), zeta + dt * k3z, area, omega)
    x = _project(x + (dt / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x))
    zeta = zeta + (dt / 6.0) * (k1z + 2.0 * k2z + 2.0 * k3z + k4z)
    return x, zeta


def vorticity_error(x, zeta, area):
    """eq. (bveerr): E_zeta against the stationary Rossby-Haurwitz vorticity."""
    z0 = rh_vorticity(x)
    return float(np.sqrt(np.sum((zeta - z0) ** 2 * area) / np.sum(z0 ** 2 * area)))


def run(points, area, steps, dt=0.01, omega=OMEGA):
    """Integrate the Rossby-Haurwitz wave from `points`; returns (x, zeta)."""
    x = np.array(points, dtype=np.float64)
    zeta = rh_vorticity(x)
    for _ in range(steps):
        x, zeta = rk4_step(x, zeta, area, dt, omega)
    return x, zeta


REMESH_ITERS = 8


def _faces():
    F = np.asarray(CUBE_FACES, dtype=np.float64)   # [6][normal, e1, e2][3]
    return F[:, 0], F[:, 1], F[:, 2]


def _face_angles(a, f=None):
    n, e1, e2 = _faces()
    if f is None:
        f = np.argmax(a @ n.T, axis=1)
    an = np.einsum("ij,ij->i", a, n[f])
    xi = np.arctan(np.einsum("ij,ij->i", a, e1[f]) / an)
    eta = np.arctan(np.einsum("ij,ij->i", a, e2[f]) / an)
    return f, xi, eta


def _lagrange3(s):
    return (0.5 * s * (s - 1.0), (1.0 - s) * (1.0 + s), 0.5 * s * (s + 1.0))


def _stencil(ang, d, lo, hi):
    c = np.clip(np.rint((ang + np.pi / 4.0) / d - 0.5), lo, hi).astype(np.int64)
    return c, _lagrange3((ang - (-np.pi / 4.0 + (c + 0.5) * d)) / d)


def biquadratic_clamped(values, E, a, face=None):
    """Biquadratic interpolation on the face of a (or on `face`), the stencil
    clamped to that face (one-sided within a cell of its edges)."""
    E = int(E)
    d = (np.pi / 2.0) / E
    f, xi, eta = _face_angles(a, face)
    (ci, wi), (cj, wj) = _stencil(xi, d, 1, E - 2), _stencil(eta, d, 1, E - 2)
    V = np.asarray(values, dtype=np.float64)
    out = 0.0
    for di in range(3):
        for dj in range(3):
            k = f * E * E + (ci + di - 1) * E + (cj + dj - 1)
            w = wi[di] * wj[dj]
            out = out + (w[:, None] * V[k] if V.ndim == 2 else w * V[k])
    return out


def biquadratic(values, E, a):
    """Local biquadratic interpolation of grid values [6 E^2, ...] at unit
    vectors a [m, 3]: the 3 x 3 stencil centred on the nearest node of a's
    face; a stencil node beyond the face edge (angle index -1 or E) takes the
    value at its own position, which lies on a node line of the face across
    that edge, by biquadratic_clamped there.  A corner node (both indices
    beyond) is as far from the faces across either edge; it takes the face
    across its first angle's edge, so that no rounding decides."""
    E = int(E)
    n, e1, e2 = _faces()
    d = (np.pi / 2.0) / E
    f, xi, eta = _face_angles(a)
    (ci, wi), (cj, wj) = _stencil(xi, d, 0, E - 1), _stencil(eta, d, 0, E - 1)
    V = np.asarray(values, dtype=np.float64)
    out = 0.0
    for di in range(3):
        for dj in range(3):
            i, j = ci + di - 1, cj + dj - 1
            inside = (i >= 0) & (i < E) & (j >= 0) & (j < E)
            v = np.zeros((a.shape[0],) + V.shape[1:])
            k = f[inside] * E * E + i[inside] * E + j[inside]
            v[inside] = V[k]
            g = ~inside
            if np.any(g):
                ta = np.tan(-np.pi / 4.0 + (i[g] + 0.5) * d)
                tb = np.tan(-np.pi / 4.0 + (j[g] + 0.5) * d)
                p = n[f[g]] + ta[:, None] * e1[f[g]] + tb[:, None] * e2[f[g]]
                # the face across the edge: normal -e1 / +e1 if the first
                # index is beyond, else -e2 / +e2
                across = np.where((i[g] < 0)[:, None], -e1[f[g]],
                                  np.where((i[g] >= E)[:, None], e1[f[g]],
                                           np.where((j[g] < 0)[:, None], -e2[f[g]], e2[f[g]])))
                v[g] = biquadratic_clamped(V, E, _project(p), face=np.argmax(across @ n.T, axis=1))
            w = wi[di] * wj[dj]
            out = out + (w[:, None] * v if V.ndim == 2 else w * v)
    return out


def remesh(grid, E, x, zeta, omega=OMEGA, iters=REMESH_ITERS, sample=None):
    """Remap particles that started a step at the cell centres `grid`
    (cubed_sphere_grid(E) order) and ended at x with vorticity zeta back onto
    the cell centres; returns the new vorticity there (the positions are the
    grid again), or at the cell centres grid[sample] only."""
    Y = np.asarray(grid, dtype=np.float64)
    D = np.asarray(x, dtype=np.float64) - Y
    q = np.asarray(zeta, dtype=np.float64) + 2.0 * omega * np.asarray(x)[:, 2]
    y = Y if sample is None else Y[sample]
    a = y.copy()
    for _ in range(iters):
        a = _project(y - biquadratic(D, E, a))
    return biquadratic(q, E, a) - 2.0 * omega * y[:, 2]


def run_remeshed(grid, area, E, steps, dt=0.01, omega=OMEGA):
    """The Rossby-Haurwitz wave on the cubed-sphere grid, remeshed after
    every step; returns the vorticity at the cell centres."""
    y = np.array(grid, dtype=np.float64)
    zeta = rh_vorticity(y)
    for _ in range(steps):
        x, z = rk4_step(y, zeta, area, dt, omega)
        zeta = remesh(y, E, x, z, omega)
    return zeta

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
  * No remeshing: the particles keep their areas A_j (the flow is
    incompressible, so a Lagrangian particle's area is constant).
"""

import numpy as np

from workloads import rh_vorticity

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

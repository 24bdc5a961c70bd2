"""Initial conditions of the barotropic vorticity examples (paper §12).

rh_vorticity: the Rossby-Haurwitz wave of eq. (RH_initial),
    zeta_0 = (2 pi/7) sin(lat) + 30 sin(lat) cos(lat)^4 cos(4 lon),
with theta read as the latitude (z = sin theta): the solid-body part then
rotates at omega = pi/7 per day = Omega/14, which makes the degree-5 wave
stationary on a sphere rotating at Omega = 2 pi per day.
"""

import numpy as np


def rh_vorticity(P):
    """Rossby-Haurwitz initial vorticity at unit vectors P [N,3]."""
    P = np.asarray(P, dtype=np.float64)
    lat = np.arcsin(np.clip(P[:, 2], -1.0, 1.0))
    lon = np.arctan2(P[:, 1], P[:, 0])
    return (2.0 * np.pi / 7.0) * np.sin(lat) + 30.0 * np.sin(lat) * np.cos(lat) ** 4 * np.cos(4.0 * lon)

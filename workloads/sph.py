"""Real orthonormal spherical harmonics on the unit sphere (inputs only).

Y_{n,0} = P_n0(z), Y_{n,m} = sqrt(2) P_nm(z) cos(m lam), Y_{n,-m} = sqrt(2)
P_nm(z) sin(m lam) for m > 0, where P_nm is the associated Legendre function
normalised so that every Y has unit L2 norm on the sphere (no Condon-Shortley
phase; the sign of a basis function does not matter for random fields).  The
paper's real harmonics (section 2.1) are Y_{n,m} = sqrt(2) Re Y_n^m.

The normalised functions come from the standard three-term recurrence in n
at fixed m, which is stable to the degrees used here (n <= 64).
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _legendre_rows(z, s, nmax):
    """Yield (m, P[n=m..nmax]) with P normalised as described above."""
    pmm = np.full_like(z, 1.0 / np.sqrt(4.0 * np.pi))
    for m in range(nmax + 1):
        if m > 0:
            pmm = pmm * s * np.sqrt((2.0 * m + 1.0) / (2.0 * m))
        rows = [pmm]
        if m + 1 <= nmax:
            rows.append(np.sqrt(2.0 * m + 3.0) * z * pmm)
        for n in range(m + 2, nmax + 1):
            a = np.sqrt((4.0 * n * n - 1.0) / (n * n - m * m))
            b = np.sqrt(((n - 1.0) ** 2 - m * m) / (4.0 * (n - 1.0) ** 2 - 1.0))
            rows.append(a * (z * rows[-1] - b * rows[-2]))
        yield m, rows


def _index(n, m):
    """Column of Y_{n,m} in the (n, m = -n..n) ordering."""
    return n * n + n + m


def real_sph_harm_all(points, nmax):
    """Matrix [N, (nmax+1)^2] of all real orthonormal Y_{n,m}, n <= nmax."""
    P = np.asarray(points, dtype=np.float64)
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    s = np.sqrt(np.maximum(0.0, x * x + y * y))
    lam = np.arctan2(y, x)
    out = np.empty((P.shape[0], (nmax + 1) ** 2))
    for m, rows in _legendre_rows(z, s, nmax):
        for k, pnm in enumerate(rows):
            n = m + k
            if m == 0:
                out[:, _index(n, 0)] = pnm
            else:
                out[:, _index(n, m)] = np.sqrt(2.0) * pnm * np.cos(m * lam)
                out[:, _index(n, -m)] = np.sqrt(2.0) * pnm * np.sin(m * lam)
    return out


def bandlimited_field(points, nmax, sigma, seed, nmin=0, chunk=1 << 16):
    """f = sum_{n=nmin..nmax} sum_m a_nm Y_{n,m}, a_nm ~ N(0, sigma(n)^2).

    The coefficients are drawn in (n, m = -n..n) order from PCG64(seed) for
    every n in 0..nmax (so that nmin does not change the draws of higher
    degrees), then those with n < nmin are set to zero.
    """
    rng = np.random.default_rng(seed)
    ncoef = (nmax + 1) ** 2
    a = rng.standard_normal(ncoef)
    for n in range(nmax + 1):
        sl = slice(n * n, (n + 1) * (n + 1))
        a[sl] *= sigma(n) if n >= nmin else 0.0
    P = np.asarray(points, dtype=np.float64)
    f = np.zeros(P.shape[0])

    def one_chunk(lo):
        Q = P[lo:lo + chunk]
        x, y, z = Q[:, 0], Q[:, 1], Q[:, 2]
        s = np.sqrt(np.maximum(0.0, x * x + y * y))
        lam = np.arctan2(y, x)
        acc = np.zeros(Q.shape[0])
        for m, rows in _legendre_rows(z, s, nmax):
            if m == 0:
                for k, pnm in enumerate(rows):
                    acc += a[_index(m + k, 0)] * pnm
            else:
                c = np.sqrt(2.0) * np.cos(m * lam)
                sn = np.sqrt(2.0) * np.sin(m * lam)
                for k, pnm in enumerate(rows):
                    n = m + k
                    acc += pnm * (a[_index(n, m)] * c + a[_index(n, -m)] * sn)
        f[lo:lo + chunk] = acc

    # chunks are independent; NumPy releases the GIL inside its loops
    starts = list(range(0, P.shape[0], chunk))
    workers = max(1, min(16, os.cpu_count() or 1, len(starts)))
    if workers == 1:
        for lo in starts:
            one_chunk(lo)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one_chunk, starts))
    return f


def real_y43(points):
    """Re Y_4^3 = -(3/8) sqrt(35/pi) z (x^3 - 3 x y^2) on the unit sphere."""
    P = np.asarray(points, dtype=np.float64)
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    return -(3.0 / 8.0) * np.sqrt(35.0 / np.pi) * z * (x ** 3 - 3.0 * x * y * y)


def real_y41(points):
    """Re Y_4^1 = -(3/8) sqrt(5/pi) x z (7 z^2 - 3) on the unit sphere."""
    P = np.asarray(points, dtype=np.float64)
    x, z = P[:, 0], P[:, 2]
    return -(3.0 / 8.0) * np.sqrt(5.0 / np.pi) * x * z * (7.0 * z * z - 3.0)

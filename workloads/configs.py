"""The five workloads: point sets, weights and method parameters.

Every input is synthetic and seeded.  Grids are equiangular cubed spheres
with E x E cells per face (N = 6 E^2); weights are w_j = f(x_j) A_j
(paper eq. nbodysum) for a field f given by spherical harmonics.

  1  Poisson log kernel, E=32 (N=6,144), f = Re Y_4^3, p=8, theta=0.7, leaf 64.
  2  Poisson log kernel, E=256 (N=393,216), f = sum_{n=1..32} a_nm Y_nm with
     a_nm ~ N(0, 1/(n+1)^2) (seed 2002) minus its area-weighted mean;
     p in {6, 8, 10}, theta=0.7, leaf 128; sampled targets: seed 2003.
  3  Biot-Savart, E=512 (N=1,572,864), vorticity Re Y_4^1 plus Gaussian noise
     of standard deviation 1e-3 * RMS(Re Y_4^1) (seed 3003); p=8, theta=0.6,
     leaf 128; sampled targets: seed 3004.
  4  1/|x-y|, sources E=1024 (N=6,291,456) with f = sum_{n=0..64} a_nm Y_nm,
     a_nm ~ N(0, 1/(n+1)^3) (seed 4004); 1,000,000 uniform random targets
     (seed 4005); p=10, theta=0.6, leaf 128; sampled targets: seed 4006.
  5  serving stream of 2,000 requests (see the serving module).

Kernel ids follow the library: 1 Poisson log, 2 Biot-Savart, 3 1/|x-y|,
4 biharmonic, 5 SAL closed form.
"""

import numpy as np

from .grid import cubed_sphere_grid, random_sphere_points
from .sph import bandlimited_field, real_y43, real_y41

KERNEL_POISSON = 1
KERNEL_BIOT_SAVART = 2
KERNEL_INV_DIST = 3

CONFIGS = {
    1: dict(name="poisson_E32", E=32, kernel=KERNEL_POISSON, p=8, theta=0.7, leaf=64,
            subset=None, subset_seed=None),
    2: dict(name="poisson_E256", E=256, kernel=KERNEL_POISSON, p=8, theta=0.7, leaf=128,
            subset=4096, subset_seed=2003, field_seed=2002),
    3: dict(name="biot_savart_E512", E=512, kernel=KERNEL_BIOT_SAVART, p=8, theta=0.6, leaf=128,
            subset=4096, subset_seed=3004, field_seed=3003),
    4: dict(name="invdist_src_E1024_tgt_1M", E=1024, n_targets=1_000_000,
            kernel=KERNEL_INV_DIST, p=10, theta=0.6, leaf=128,
            subset=4096, subset_seed=4006, field_seed=4004, target_seed=4005),
}


def make_config(cid, E=None):
    """Inputs of workload `cid` (optionally at another grid size E).

    Returns a dict with float64 arrays: sources [Ns,3], targets [Nt,3] or
    None (same set), weights [Ns], areas [Ns] (source cell areas), and the
    parameters kernel, p, theta, leaf.
    """
    c = dict(CONFIGS[cid])
    if E is not None:
        c["E"] = int(E)
    pts, area = cubed_sphere_grid(c["E"])
    if cid == 1:
        f = real_y43(pts)
    elif cid == 2:
        f = bandlimited_field(pts, 32, lambda n: 1.0 / (n + 1.0), c["field_seed"], nmin=1)
        f = f - np.sum(f * area) / np.sum(area)
    elif cid == 3:
        f = real_y41(pts)
        rms = np.sqrt(np.mean(f * f))
        rng = np.random.default_rng(c["field_seed"])
        f = f + rng.standard_normal(f.shape[0]) * (1e-3 * rms)
    elif cid == 4:
        f = bandlimited_field(pts, 64, lambda n: (n + 1.0) ** -1.5, c["field_seed"])
    else:
        raise KeyError(cid)
    c["sources"] = pts
    c["areas"] = area
    c["field"] = f
    c["weights"] = np.ascontiguousarray(f * area)
    if cid == 4:
        c["targets"] = random_sphere_points(c["n_targets"], c["target_seed"])
    else:
        c["targets"] = None
    return c


def config_subset(n_targets, size, seed):
    """Sorted seeded sample of `size` distinct target indices (PCG64)."""
    rng = np.random.default_rng(seed)
    size = min(int(size), int(n_targets))
    return np.sort(rng.choice(int(n_targets), size=size, replace=False))

"""The barotropic vorticity equation stepped on the GPU (csfmm_bve_rk4_step)
against the BVE oracle: with the direct-sum velocity the trajectories and
vorticities agree to rounding after 10 RK4 steps; with the CSFMM velocity
(MAC 0.7, n = 6, the paper's §12 setting) the Rossby-Haurwitz vorticity error
equals the direct-sum one to within 1%, as the paper reports."""

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from workloads import icosahedral_grid
from oracle import bve as obve

pytestmark = pytest.mark.gpu


def say(msg):
    print("\n[gpu case] " + msg, flush=True)


def _state(P):
    x = torch.tensor(P, dtype=torch.float64, device="cuda")
    z = torch.tensor(obve.rh_vorticity(P), dtype=torch.float64, device="cuda")
    return x, z


def test_bve_direct_matches_oracle():
    say("bve direct velocity, icosahedral k=3, 10 steps")
    P, A = icosahedral_grid(3)
    x, z = _state(P)
    a = torch.tensor(A, dtype=torch.float64, device="cuda")
    for _ in range(10):
        cs.bve_rk4_step(x, z, a, 0.01, use_direct=True)
    xr, zr = obve.run(P, A, 10)
    xg, zg = x.cpu().numpy(), z.cpu().numpy()
    print("x diff %.3e zeta rel %.3e" % (np.abs(xg - xr).max(),
                                          np.abs(zg - zr).max() / np.abs(zr).max()), flush=True)
    assert np.abs(xg - xr).max() < 1e-12
    assert np.abs(zg - zr).max() < 1e-12 * np.abs(zr).max()


@pytest.mark.parametrize("k", [4, 5])
def test_bve_csfmm_error_equals_direct(k):
    say("bve csfmm vs direct velocity, icosahedral k=%d, 10 steps" % k)
    P, A = icosahedral_grid(k)
    a = torch.tensor(A, dtype=torch.float64, device="cuda")
    res = {}
    for direct in (True, False):
        x, z = _state(P)
        for _ in range(10):
            cs.bve_rk4_step(x, z, a, 0.01, p=6, theta=0.7, leaf_size=64, use_direct=direct)
        xg, zg = x.cpu().numpy(), z.cpu().numpy()
        res[direct] = (xg, zg, obve.vorticity_error(xg, zg, A))
    e_dir, e_fmm = res[True][2], res[False][2]
    print("E_zeta direct %.4e csfmm %.4e, x diff %.2e" % (
        e_dir, e_fmm, np.abs(res[True][0] - res[False][0]).max()), flush=True)
    assert abs(e_fmm - e_dir) < 0.01 * e_dir
    assert np.abs(res[True][0] - res[False][0]).max() < 1e-5
    assert e_dir < (1.5e-2 if k == 4 else 1.5e-3)

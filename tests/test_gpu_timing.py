"""Stage timing through the C ABI (csfmm_plan_timing / _timing_read): six
sums, the interaction span holding both interaction launches, and the two
levels recording what they say."""

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from workloads import cubed_sphere_grid, random_sphere_points

pytestmark = pytest.mark.gpu


def test_stage_sums_and_interaction_span():
    print("\n[gpu case] timing: 200,000 random targets x E=96 grid, p=8", flush=True)
    S, _ = cubed_sphere_grid(96)
    X = random_sphere_points(200000, 81)
    w = np.random.default_rng(82).standard_normal(S.shape[0])
    T = torch.tensor(X, device="cuda")
    Sd = torch.tensor(S, device="cuda")
    W = torch.tensor(w, device="cuda")
    pl = cs.Plan(T, Sd, kernel=cs.INV_DIST, p=8, theta=0.6, leaf_size=128)
    out = pl.eval(W)
    assert cs.STAGES == ("p2m", "m2m", "near_pp", "pc_far", "l2l_l2p", "interaction_span")
    for level in (1, 2):
        pl.timing(level)
        for _ in range(5):
            pl.eval(W, out=out)
        n, st = pl.timing_read()
        pl.timing(False)
        print(level, n, {k: round(v / n, 4) for k, v in st.items()}, flush=True)
        assert n == 5
        assert st["near_pp"] > 0 and st["pc_far"] > 0
        # the span runs from the PP launch's start to the join after both
        assert st["interaction_span"] >= max(st["near_pp"], st["pc_far"]) * (1 - 1e-6)
        if level == 2:
            assert st["p2m"] == 0 and st["m2m"] == 0 and st["l2l_l2p"] == 0
        else:
            assert min(st.values()) > 0
    pl.close()

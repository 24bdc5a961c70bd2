"""csfmm_direct_noalloc (the entry point for callers that cannot allocate)
against csfmm_direct through the C ABI: the same kernels and source splits,
so the results agree bit for bit; two calls in a row on one GPU's scratch,
the second smaller, and the size limit rejected before any launch."""

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from workloads import cubed_sphere_grid, random_sphere_points

pytestmark = pytest.mark.gpu


def tdev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("kernel,fp32", [(1, False), (2, True), (3, False)])
def test_noalloc_direct_equals_direct_twice(kernel, fp32):
    print("\n[gpu case] direct_noalloc kernel %d fp32 %s" % (kernel, fp32), flush=True)
    S = tdev(cubed_sphere_grid(24)[0])
    rng = np.random.default_rng(7)
    w = tdev(rng.standard_normal(S.shape[0]))
    vd = 3 if kernel == 2 else 1
    for nt in (5003, 777):   # the second call smaller: stale scratch must not leak in
        X = tdev(random_sphere_points(nt, nt))
        want = cs.direct(X, S, w, kernel=kernel, fp32=fp32)
        out = torch.full((nt, 3) if vd == 3 else (nt,), float("nan"), dtype=torch.float64,
                         device="cuda")
        got = cs.direct_noalloc(X, S, w, out, kernel=kernel, fp32=fp32)
        torch.cuda.synchronize()
        assert torch.equal(got, want)


def test_noalloc_direct_rejects_sizes_beyond_the_scratch():
    print("\n[gpu case] direct_noalloc size limit", flush=True)
    S = tdev(cubed_sphere_grid(4)[0])
    w = torch.ones(S.shape[0], dtype=torch.float64, device="cuda")
    n = (1 << 22) // 3 + 1   # Biot-Savart: three partial sums per target
    X = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    X[:, 2] = 1.0
    out = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(cs.CsfmmError) as ei:
        cs.direct_noalloc(X, S, w, out, kernel=2)
    assert ei.value.status == -1
    assert torch.count_nonzero(out) == 0   # nothing was launched

"""An eval captured into a HIP graph (through torch.cuda.graph): the capture
takes the PP near field's fork onto the workspace side stream and the join
back, and every replay equals the eager eval of the weights the graph reads
at that moment; replays are interleaved with eager work and synchronisation."""

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from workloads import cubed_sphere_grid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kernel,fp32", [(1, True), (2, False)])
def test_eval_graph_replays_match_eager(kernel, fp32):
    print("\n[gpu case] graph capture of eval, kernel %d fp32 %s" % (kernel, fp32), flush=True)
    P, A = cubed_sphere_grid(32)
    rng = np.random.default_rng(12)
    T = torch.tensor(P, dtype=torch.float64, device="cuda")
    W = torch.tensor(rng.standard_normal(P.shape[0]), dtype=torch.float64, device="cuda")
    plan = cs.Plan(T, None, kernel=kernel, p=6, theta=0.7, leaf_size=64, fp32=fp32)
    out = plan.eval(W)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up outside the capture
        plan.eval(W, out=out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.eval(W, out=out)
    for rep in range(4):
        W.copy_(torch.tensor(rng.standard_normal(P.shape[0]), dtype=torch.float64, device="cuda"))
        eager = plan.eval(W).clone()        # eager work between replays
        torch.cuda.synchronize()
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
    del g
    plan.close()

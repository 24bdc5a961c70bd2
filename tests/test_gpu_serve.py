"""Serving on the GPU: packed multi-request evaluation is bitwise identical to
evaluating each request alone, batches larger than one packed launch are
chunked, and a real-time request stream under a tight HBM budget (forcing
queueing and plan eviction) completes with correct results."""

import numpy as np
import pytest
import torch

import paper_2508_13550_amd as cs
from paper_2508_13550_amd.serve import Server, Request, latency_stats
from workloads import cubed_sphere_grid, real_sph_harm_all
from workloads.serving import request_mix, poisson_arrivals
from oracle import direct as odirect

pytestmark = pytest.mark.gpu


def say(msg):
    print("\n[gpu case] " + msg, flush=True)


_GRIDS = {}


def grid(E):
    if E not in _GRIDS:
        P, A = cubed_sphere_grid(E)
        Y = real_sph_harm_all(P, 8)
        _GRIDS[E] = (P, A, Y, torch.tensor(P, dtype=torch.float64, device="cuda"))
    return _GRIDS[E]


def weights(E, coef):
    P, A, Y, _ = grid(E)
    return torch.tensor((Y @ coef) * A, dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("fp32", [True, False])
def test_packed_mixed_near_field_paths_equal_alone_bitwise(fp32):
    """A request on the one-wave-per-leaf near field with symmetric PP pairs
    (6,144 leaves of 9 points) packed with requests on the block path (few
    leaves) and with Biot-Savart (no symmetric pairs): each result is bitwise
    the request evaluated alone, whatever else shares its launches; both
    forms (the FP64 form's symmetric tile has its own column layout)."""
    say("eval_many: wave/symmetric path packed with block-path requests, fp32=%s" % fp32)
    big = cs.Plan(grid(96)[3], None, kernel=1, p=4, theta=0.7, leaf_size=16, fp32=fp32)
    small = cs.Plan(grid(16)[3], None, kernel=1, p=4, theta=0.7, leaf_size=16, fp32=fp32)
    assert big.stats()["near_wave"] == 1 and small.stats()["near_wave"] == 0
    assert big.stats()["pp_sym_pairs"] > 0
    rng = np.random.default_rng(21)
    reqs = [(big, 1), (small, 1), (big, 3), (small, 2), (big, 2)]
    batch, alone = [], []
    for pl, k in reqs:
        E = 96 if pl is big else 16
        w = weights(E, rng.standard_normal(81))
        alone.append(pl.eval(w, kernel=k).cpu().numpy())
        batch.append((pl, cs.Workspace(pl), k, w))
    outs = cs.eval_many(batch)
    torch.cuda.synchronize()
    for a, o in zip(alone, outs):
        assert np.array_equal(a, o.cpu().numpy())
    for _, ws, _, _ in batch:
        ws.close()
    big.close()
    small.close()


@pytest.mark.parametrize("rows_min", [None, "0"])
def test_packed_equals_alone_bitwise(rows_min, monkeypatch):
    """Packed requests of mixed sizes and kernels equal each request alone, bit
    for bit; also with the row-blocked M2M forced onto every level (at full
    size it takes levels of 8,192 parents or more), whose blocks then belong
    to several requests of one launch."""
    if rows_min is not None:
        monkeypatch.setenv("CSFMM_M2M_ROWS_MIN", rows_min)
    say("eval_many vs alone, CSFMM_M2M_ROWS_MIN=%s" % rows_min)
    mix = request_mix(10, seed_mix=11, e_choices=(8, 16, 32))
    plans, alone, batch = {}, [], []
    for E, k, p, c in mix:
        if (E, p) not in plans:
            plans[(E, p)] = cs.Plan(grid(E)[3], None, kernel=1, p=p, theta=0.6, leaf_size=64,
                                    fp32=True)
        pl = plans[(E, p)]
        w = weights(E, c)
        alone.append(pl.eval(w, kernel=k).cpu().numpy())
        batch.append((pl, cs.Workspace(pl), k, w))
    outs = cs.eval_many(batch)
    torch.cuda.synchronize()
    for a, o in zip(alone, outs):
        assert np.array_equal(a, o.cpu().numpy())
    for _, ws, _, _ in batch:
        ws.close()
    for pl in plans.values():
        pl.close()


def test_batches_larger_than_one_launch():
    say("40 requests in one eval_many (two packed chunks)")
    P, A, Y, T = grid(16)
    pl = cs.Plan(T, None, kernel=3, p=6, theta=0.6, leaf_size=32, fp32=False)
    rng = np.random.default_rng(1)
    ws = [cs.Workspace(pl) for _ in range(40)]
    W = [torch.tensor(rng.standard_normal(P.shape[0]), device="cuda") for _ in range(40)]
    outs = cs.eval_many([(pl, ws[i], 3, W[i]) for i in range(40)])
    for i in (0, 17, 31, 32, 39):
        ref = pl.eval(W[i]).cpu().numpy()
        assert np.array_equal(ref, outs[i].cpu().numpy())
    for w_ in ws:
        w_.close()
    pl.close()


def test_served_stream_under_tight_budget():
    say("real-time stream, 60 requests, tight HBM budget")
    n = 60
    mix = request_mix(n, seed_mix=5006, e_choices=(16, 32, 64))
    arr = poisson_arrivals(n, rate=400.0, seed=5005)
    # budget holding about two of the larger plans at once
    big = cs.estimate_bytes(6 * 64 * 64, 6 * 64 * 64, 8, 128, True)
    srv = Server(budget_bytes=int(2.5 * big), theta=0.6, leaf=128, fp32=True, max_batch=8)
    reqs = []
    for i, ((E, k, p, c), t) in enumerate(zip(mix, arr)):
        reqs.append(Request(id=i, geometry=("grid", E), targets=grid(E)[3], sources=None,
                            kernel=k, p=p, weights=weights(E, c), t_arrival=float(t)))
    done = srv.run(reqs)
    st = srv.sched.stats()
    lat = latency_stats(done)
    print("sched", st, "latency", lat, "batches", srv.batch_sizes, flush=True)
    assert len(done) == n and st["completed"] == n and st["rejected"] == 0
    assert st["evictions"] > 0 and st["plan_hits"] > 0
    assert max(srv.batch_sizes) > 1
    # every result equals the request evaluated alone; a sample against the oracle
    for r in done[::7]:
        E = r.geometry[1]
        pl = cs.Plan(grid(E)[3], None, kernel=r.kernel, p=r.p, theta=0.6, leaf_size=128,
                     fp32=True)
        alone = pl.eval(r.weights).cpu().numpy()
        pl.close()
        got = r.out.cpu().numpy()
        assert np.array_equal(alone, got)
        P = grid(E)[0]
        S = np.arange(0, P.shape[0], max(1, P.shape[0] // 256))
        ref = odirect(r.kernel, P[S], P, r.weights.cpu().numpy())
        err = np.sqrt(np.sum((got[S] - ref) ** 2) / np.sum(ref ** 2))
        assert err < 1e-5
    srv.close()


def test_served_stream_at_full_request_sizes():
    """The serving workload's request sizes: E in {16, ..., 512} (N up to
    1,572,864), all three kernels, p in {6, 8}, 36 requests arriving faster
    than they are served, so that batches run beside each other on the
    executor's streams.  Every result equals, bit for bit, the request
    evaluated alone on its resident plan; sampled requests of each kernel, the
    largest among them, match the oracle on 1,024 targets within 1e-5."""
    from workloads import config_subset
    from gates import rel_l2
    say("served stream at full request sizes: 36 requests, E up to 512")
    n = 36
    mix = request_mix(n, seed_mix=5006)
    arr = poisson_arrivals(n, rate=2000.0, seed=5005)
    free, _ = torch.cuda.mem_get_info()
    srv = Server(budget_bytes=int(0.5 * free), theta=0.6, leaf=128, fp32=True, max_batch=16)
    reqs = [Request(id=i, geometry=("grid", E), targets=grid(E)[3], sources=None, kernel=k, p=p,
                    weights=weights(E, c), t_arrival=float(t))
            for i, ((E, k, p, c), t) in enumerate(zip(mix, arr))]
    done = srv.run(reqs)
    st = srv.sched.stats()
    print("sched", st, "latency", latency_stats(done), "batches", srv.batch_sizes, flush=True)
    assert len(done) == n and st["completed"] == n and st["rejected"] == 0
    assert st["evictions"] == 0
    assert srv.max_concurrent >= 2   # batches ran beside each other
    from paper_2508_13550_amd.serve import plan_key
    by_id = {r.id: r for r in done}
    for r in done:
        pl = srv.plans[plan_key(r.geometry, r.p, 0.6, 128, True)]
        alone = pl.eval(r.weights, kernel=r.kernel)
        assert torch.equal(alone, r.out), r.id
    # oracle check: for each kernel its largest request and its first one
    picks = set()
    for k in (1, 2, 3):
        ids = [i for i, m in enumerate(mix) if m[1] == k]
        picks.add(max(ids, key=lambda i: mix[i][0]))
        picks.add(ids[0])
    for i in sorted(picks):
        r = by_id[i]
        E = r.geometry[1]
        P = grid(E)[0]
        S = config_subset(P.shape[0], 1024, 5008)
        say("oracle check of request %d: E=%d kernel %d p=%d" % (i, E, r.kernel, r.p))
        ref = odirect(r.kernel, P[S], P, r.weights.cpu().numpy())
        err = rel_l2(r.out.cpu().numpy()[S], ref)
        print("request %d E=%d kernel %d p=%d rel L2 %.3e" % (i, E, r.kernel, r.p, err), flush=True)
        assert err < 1e-5
    srv.close()


@pytest.mark.parametrize("E,p", [(16, 6), (64, 8), (256, 6), (512, 8)])
def test_admission_estimates_cover_the_bytes_held(E, p):
    """The scheduler admits by estimates made before a plan exists: they must
    cover what the plan and a workspace then hold, in both forms (same-set
    plans of E >= 256 hold the symmetric PP slots, 8 bytes a value in FP64);
    the plan's own workspace figure is exact."""
    from paper_2508_13550_amd.serve import workspace_bytes_estimate
    T = grid(E)[3]
    n = T.shape[0]
    for fp32 in (False, True):
        pl = cs.Plan(T, None, kernel=1, p=p, theta=0.6, leaf_size=128, fp32=fp32)
        ws = cs.Workspace(pl)
        st = pl.stats()
        est_plan = cs.estimate_bytes(n, n, p, 128, fp32)
        est_ws = workspace_bytes_estimate(n, n, p, 128)
        print("E=%d p=%d fp32=%s plan %d <= %d, workspace %d <= %d, sym pairs %d"
              % (E, p, fp32, st["device_bytes"], est_plan, ws.device_bytes, est_ws,
                 st["pp_sym_pairs"]), flush=True)
        assert cs.workspace_bytes(pl) == ws.device_bytes
        assert st["device_bytes"] <= est_plan
        assert ws.device_bytes <= est_ws
        if E >= 256:
            assert st["pp_sym_pairs"] > 0
        ws.close()
        pl.close()

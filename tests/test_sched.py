"""The serving scheduler's policy on the host (no GPU): first-come admission by
HBM footprint, plan cache hits and LRU eviction of idle plans, workspace
pools, batch size limit, rejection of requests that can never fit, and the
budget invariant under a seeded random stream with a fake clock."""

import numpy as np
import pytest

from paper_2508_13550_amd.serve import Scheduler

MB = 1 << 20


def test_batches_and_plan_cache():
    s = Scheduler(budget_bytes=1000 * MB, max_batch=4)
    for i in range(6):
        s.submit(i, plan_key=7, plan_bytes=100 * MB, ws_bytes=10 * MB, t_arrival=0.0)
    d = s.step(0.0)
    assert d["launch"] == [0, 1, 2, 3]            # max_batch
    assert d["build"] == [7]                      # one build for the shared plan
    assert d["new_ws"] == [7, 7, 7, 7]            # pool grows to the peak in flight
    d2 = s.step(0.0)
    assert d2["launch"] == [4, 5] and d2["build"] == []
    st = s.stats()
    assert st["plan_misses"] == 1 and st["plan_hits"] == 5
    for i in range(6):
        s.complete(i, 1.0)
    s.submit(6, 7, 100 * MB, 10 * MB, 2.0)
    d3 = s.step(2.0)
    assert d3["launch"] == [6] and d3["new_ws"] == []   # a pooled workspace is reused
    assert s.stats()["used_bytes"] == (100 + 6 * 10) * MB


def test_arrival_time_and_fifo():
    s = Scheduler(budget_bytes=1000 * MB, max_batch=8)
    s.submit(1, 1, 10 * MB, 1 * MB, 0.5)
    s.submit(2, 2, 10 * MB, 1 * MB, 0.1)   # queue order is submission order
    assert s.step(0.2)["launch"] == []     # the head has not arrived yet
    assert s.step(0.5)["launch"] == [1, 2]


def test_budget_forces_queueing_and_lru_eviction():
    s = Scheduler(budget_bytes=250 * MB, max_batch=8)
    s.submit(0, 100, 200 * MB, 20 * MB, 0.0)
    s.submit(1, 200, 200 * MB, 20 * MB, 0.0)
    d = s.step(0.0)
    assert d["launch"] == [0]                  # plan 200 does not fit next to plan 100
    assert s.step(0.1)["launch"] == []         # 100 is busy: no eviction, 1 waits
    s.complete(0, 0.2)
    d = s.step(0.3)
    assert d["evict"] == [100] and d["build"] == [200] and d["launch"] == [1]
    st = s.stats()
    assert st["evictions"] == 1 and st["used_bytes"] <= st["budget_bytes"]


def test_oldest_request_is_not_overtaken():
    s = Scheduler(budget_bytes=300 * MB, max_batch=8)
    s.submit(0, 1, 200 * MB, 10 * MB, 0.0)
    s.submit(1, 2, 200 * MB, 10 * MB, 0.0)
    s.submit(2, 1, 200 * MB, 10 * MB, 0.0)   # would fit on plan 1, but 1 is older
    assert s.step(0.0)["launch"] == [0]
    assert s.step(0.0)["launch"] == []


def test_reject_request_larger_than_device():
    s = Scheduler(budget_bytes=100 * MB, max_batch=8)
    s.submit(0, 1, 200 * MB, 1 * MB, 0.0)
    s.submit(1, 2, 50 * MB, 1 * MB, 0.0)
    d = s.step(0.0)
    assert d["reject"] == [0] and d["launch"] == [1]
    assert s.stats()["rejected"] == 1


def test_complete_unknown_request_is_an_error():
    s = Scheduler(budget_bytes=100 * MB, max_batch=8)
    with pytest.raises(Exception):
        s.complete(42, 0.0)


def test_random_stream_invariants():
    rng = np.random.default_rng(5)
    budget = 2000 * MB
    s = Scheduler(budget_bytes=budget, max_batch=16)
    sizes = {k: (int(rng.integers(50, 900)) * MB, int(rng.integers(5, 80)) * MB) for k in range(12)}
    t = 0.0
    inflight = []
    done = 0
    n = 400
    for i in range(n):
        k = int(rng.integers(0, 12))
        s.submit(i, k, sizes[k][0], sizes[k][1], t)
        t += float(rng.exponential(0.01))
    clock = 0.0
    resident = set()
    while done < n:
        clock += 0.005
        d = s.step(clock)
        for k in d["evict"]:
            assert k in resident
            resident.discard(k)
        for k in d["build"]:
            assert k not in resident
            resident.add(k)
        st = s.stats()
        assert st["used_bytes"] <= budget
        inflight.extend(d["launch"])
        # finish the oldest half of what is in flight
        m = (len(inflight) + 1) // 2
        for rid in inflight[:m]:
            s.complete(rid, clock)
            done += 1
        inflight = inflight[m:]
    st = s.stats()
    assert st["completed"] == n and st["queued"] == 0 and st["in_flight"] == 0
    assert st["plan_hits"] + st["plan_misses"] == n


def test_cost_classes_form_separate_batches():
    """A batch is the oldest waiting request and the waiting requests within a
    factor 4 of its cost; the others wait for the next batch, which the
    executor may run beside it, so small requests are not held behind a large
    one; within a class the order is first-come."""
    s = Scheduler(budget_bytes=10000 * MB, max_batch=8)
    costs = [1e6, 1e3, 2e3, 3e6, 1.5e3, 8e5]
    for i, c in enumerate(costs):
        s.submit(i, plan_key=i, plan_bytes=10 * MB, ws_bytes=1 * MB, t_arrival=0.0, cost=c)
    assert s.step(0.0)["launch"] == [0, 3, 5]   # the head (1e6) and its class
    assert s.step(0.0)["launch"] == [1, 2, 4]   # the next oldest (1e3) and its class
    assert s.step(0.0)["launch"] == []
    assert s.stats()["batches"] == 2


def test_cost_class_never_overtakes_the_oldest_on_memory():
    s = Scheduler(budget_bytes=300 * MB, max_batch=8)
    s.submit(0, 1, 200 * MB, 10 * MB, 0.0, cost=1e6)
    s.submit(1, 2, 200 * MB, 10 * MB, 0.0, cost=1e3)   # does not fit beside plan 1
    s.submit(2, 3, 20 * MB, 10 * MB, 0.0, cost=1e3)
    assert s.step(0.0)["launch"] == [0]
    # the oldest waiting request (1) does not fit: no batch starts, 2 waits too
    assert s.step(0.0)["launch"] == []
    s.complete(0, 1.0)
    d = s.step(1.0)
    assert d["evict"] == [1] and d["launch"] == [1, 2]

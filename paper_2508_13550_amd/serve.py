"""Serving loop: continuous batching of CSFMM evaluations on one GPU.

Requests (targets, sources, kernel, degree, weights) arrive over time.  The
native scheduler (csfmm_sched_*, see include/csfmm.h) forms batches: the
oldest waiting request and the waiting requests of its cost class, while their
memory fits the HBM budget; plans stay resident in a cache keyed by geometry
and parameters, each with a pool of eval workspaces.  A batch is one packed
csfmm_eval_many (one launch per phase).  The executor keeps several compute
streams of equal priority; whenever one is free it asks the scheduler for the
next batch and launches it there, so batches run beside each other on the
device: requests that arrive while others are on the GPU are admitted as
streams, slots and memory free up, and a small request need not wait for a
large one's launches.  Each launch waits (on the device) for the stream that
produced its requests' inputs.  Plans are built on a separate stream.
Completion times come from HIP events.
"""

import ctypes
import hashlib
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (Plan, Workspace, eval_many, load_library, BIOT_SAVART, _check)


class SchedStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "launched", "completed", "rejected", "batches", "plan_hits", "plan_misses",
        "evictions", "used_bytes", "budget_bytes", "queued", "in_flight", "resident_plans")]


class Decision(ctypes.Structure):
    _fields_ = [
        ("launch_ids", ctypes.POINTER(ctypes.c_int64)), ("cap_launch", ctypes.c_int),
        ("n_launch", ctypes.c_int),
        ("build_keys", ctypes.POINTER(ctypes.c_uint64)), ("cap_build", ctypes.c_int),
        ("n_build", ctypes.c_int),
        ("new_ws_keys", ctypes.POINTER(ctypes.c_uint64)), ("n_new_ws", ctypes.c_int),
        ("evict_keys", ctypes.POINTER(ctypes.c_uint64)), ("cap_evict", ctypes.c_int),
        ("n_evict", ctypes.c_int),
        ("reject_ids", ctypes.POINTER(ctypes.c_int64)), ("cap_reject", ctypes.c_int),
        ("n_reject", ctypes.c_int),
    ]


def _declare(L):
    if getattr(L, "_sched_declared", False):
        return
    vp = ctypes.c_void_p
    L.csfmm_sched_create.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.POINTER(vp)]
    L.csfmm_sched_destroy.argtypes = [vp]
    L.csfmm_sched_submit.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_double]
    L.csfmm_sched_step.argtypes = [vp, ctypes.c_double, ctypes.POINTER(Decision)]
    L.csfmm_sched_complete.argtypes = [vp, ctypes.c_int64, ctypes.c_double]
    L.csfmm_sched_get_stats.argtypes = [vp, ctypes.POINTER(SchedStats)]
    for f in ("csfmm_sched_create", "csfmm_sched_destroy", "csfmm_sched_submit",
              "csfmm_sched_step", "csfmm_sched_complete", "csfmm_sched_get_stats"):
        getattr(L, f).restype = ctypes.c_int
    L._sched_declared = True


class Scheduler:
    """ctypes front end of the native scheduler (host only, no GPU needed)."""

    def __init__(self, budget_bytes, max_batch=32, cap=256):
        self.L = load_library()
        _declare(self.L)
        h = ctypes.c_void_p()
        _check(self.L.csfmm_sched_create(int(budget_bytes), int(max_batch), ctypes.byref(h)))
        self._h = h
        self.cap = cap
        self._launch = (ctypes.c_int64 * cap)()
        self._build = (ctypes.c_uint64 * cap)()
        self._neww = (ctypes.c_uint64 * cap)()
        self._evict = (ctypes.c_uint64 * cap)()
        self._reject = (ctypes.c_int64 * cap)()

    def submit(self, req_id, plan_key, plan_bytes, ws_bytes, t_arrival, cost=1.0):
        _check(self.L.csfmm_sched_submit(self._h, int(req_id), int(plan_key), int(plan_bytes),
                                         int(ws_bytes), float(t_arrival), float(cost)))

    def step(self, now):
        d = Decision(self._launch, self.cap, 0, self._build, self.cap, 0, self._neww, 0,
                     self._evict, self.cap, 0, self._reject, self.cap, 0)
        _check(self.L.csfmm_sched_step(self._h, float(now), ctypes.byref(d)))
        return {"launch": list(self._launch[:d.n_launch]), "build": list(self._build[:d.n_build]),
                "new_ws": list(self._neww[:d.n_new_ws]), "evict": list(self._evict[:d.n_evict]),
                "reject": list(self._reject[:d.n_reject])}

    def complete(self, req_id, now):
        _check(self.L.csfmm_sched_complete(self._h, int(req_id), float(now)))

    def stats(self):
        s = SchedStats()
        _check(self.L.csfmm_sched_get_stats(self._h, ctypes.byref(s)))
        return {n: getattr(s, n) for n, _ in s._fields_}

    def close(self):
        if self._h is not None:
            self.L.csfmm_sched_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_key(geometry, p, theta, leaf, fp32):
    """Stable 64-bit key of a plan: geometry id and method parameters."""
    h = hashlib.blake2b(repr((geometry, int(p), float(theta), int(leaf), bool(fp32))).encode(),
                        digest_size=8)
    return int.from_bytes(h.digest(), "little")


def estimate_cells(n, leaf):
    return 6 + (16 * n) // (3 * leaf) + 64


def workspace_bytes_estimate(n_t, n_s, p, leaf):
    """Upper estimate of one eval workspace (the terms of csfmm_workspace_bytes):
    sorted weights, proxy weights and potentials, two near-field arrays and,
    for same-set plans, the column sums of the symmetric PP pairs (64 values
    per owned pair, 4 bytes in the FP32 form and 8 in FP64, at most 16 pairs
    per leaf)."""
    K = (p + 1) ** 2
    KS = (K + 3) // 4 * 4
    ct, cs = estimate_cells(n_t, leaf), estimate_cells(n_s, leaf)
    return (8 * (n_s + cs * KS + 3 * ct * KS + 6 * n_t) + 8 * 64 * 16 * ct + 1024)


@dataclass
class Request:
    id: int
    geometry: object             # hashable geometry id (equal ids = equal point sets)
    targets: torch.Tensor        # [n_t,3] float64 on the GPU
    sources: object              # [n_s,3] tensor or None (same set)
    kernel: int
    p: int
    weights: torch.Tensor        # [n_s] float64 on the GPU
    t_arrival: float = 0.0
    out: object = None
    t_done: float = field(default=float("nan"))
    ready: object = None         # event on the stream that produced the inputs

    @property
    def n_t(self):
        return self.targets.shape[0]

    @property
    def n_s(self):
        return self.n_t if self.sources is None else self.sources.shape[0]


class Server:
    """Executes the scheduler's decisions on the GPU, one batch per free
    compute stream (all of the default priority)."""

    def __init__(self, budget_bytes, theta=0.6, leaf=128, fp32=True, max_batch=32,
                 n_streams=3, clock=time.perf_counter):
        from . import estimate_bytes
        self._estimate_bytes = estimate_bytes
        self.theta, self.leaf, self.fp32 = float(theta), int(leaf), bool(fp32)
        self.sched = Scheduler(budget_bytes, max_batch)
        self.clock = clock
        self.streams = [torch.cuda.Stream() for _ in range(int(n_streams))]
        self.plan_stream = torch.cuda.Stream()
        self.plans = {}          # key -> Plan
        self.pools = {}          # key -> [free Workspace]
        self.requests = {}       # id -> Request (waiting or in flight)
        self.key_of = {}         # id -> plan key
        self.busy = {}           # stream index -> (event, [request ids], {id: workspace})
        self.done = []
        self.rejected = []
        self.batch_sizes = []
        self.max_concurrent = 0  # most batches in flight at once
        self.host_s = 0.0        # host time spent scheduling and launching
        torch.cuda.synchronize()
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref.record(self.streams[0])
        torch.cuda.synchronize()
        self._t_ref = self.clock()

    def submit(self, req):
        key = plan_key(req.geometry, req.p, self.theta, self.leaf, self.fp32)
        pb = self._estimate_bytes(req.n_t, req.n_s, req.p, self.leaf, self.fp32)
        wb = workspace_bytes_estimate(req.n_t, req.n_s, req.p, self.leaf)
        # the inputs may still be in flight on the caller's stream
        req.ready = torch.cuda.Event()
        req.ready.record(torch.cuda.current_stream())
        self.requests[req.id] = req
        self.key_of[req.id] = key
        self.sched.submit(req.id, key, pb, wb, req.t_arrival, cost=req.n_t + req.n_s)

    def _build(self, key, req):
        self.plan_stream.wait_event(req.ready)
        with torch.cuda.stream(self.plan_stream):
            self.plans[key] = Plan(req.targets, req.sources, kernel=req.kernel, p=req.p,
                                   theta=self.theta, leaf_size=self.leaf, fp32=self.fp32)
        self.pools[key] = []

    def step(self, now=None):
        """One scheduling step: if a compute stream is free, evict, build and
        launch the scheduler's next batch there; returns the launched ids."""
        t0 = time.perf_counter()
        try:
            return self._step(now)
        finally:
            self.host_s += time.perf_counter() - t0

    def _step(self, now):
        self.poll()
        free = [i for i in range(len(self.streams)) if i not in self.busy]
        if not free:
            return []
        now = self.clock() if now is None else now
        d = self.sched.step(now)
        for key in d["evict"]:
            for ws in self.pools.pop(key, []):
                ws.close()
            pl = self.plans.pop(key, None)
            if pl is not None:
                pl.close()
        for rid in d["reject"]:
            self.rejected.append(self.requests.pop(rid))
        if not d["launch"]:
            return []
        first = {}
        for rid in d["launch"]:
            first.setdefault(self.key_of[rid], rid)
        for key in d["build"]:
            self._build(key, self.requests[first[key]])
        with torch.cuda.stream(self.plan_stream):
            for key in d["new_ws"]:
                self.pools[key].append(Workspace(self.plans[key]))
        batch, used = [], {}
        si = free[0]
        stream = self.streams[si]
        stream.wait_stream(self.plan_stream)   # plans and workspaces built there
        for rid in d["launch"]:
            key = self.key_of[rid]
            req = self.requests[rid]
            ws = self.pools[key].pop()
            used[rid] = ws
            stream.wait_event(req.ready)
            batch.append((self.plans[key], ws, req.kernel, req.weights))
        with torch.cuda.stream(stream):
            outs = eval_many(batch)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        for rid, o in zip(d["launch"], outs):
            self.requests[rid].out = o
        self.busy[si] = (ev, list(d["launch"]), used)
        self.batch_sizes.append(len(d["launch"]))
        self.max_concurrent = max(self.max_concurrent, len(self.busy))
        return list(d["launch"])

    def poll(self, wait=False):
        """Retire finished batches (in any order); returns the finished requests."""
        fin = []
        for si in sorted(self.busy):
            ev, ids, used = self.busy[si]
            if wait:
                ev.synchronize()
            elif not ev.query():
                continue
            t_done = self._t_ref + self._ref.elapsed_time(ev) / 1e3
            for rid in ids:
                req = self.requests.pop(rid)
                req.t_done = t_done
                self.pools[self.key_of[rid]].append(used[rid])
                self.sched.complete(rid, t_done)
                fin.append(req)
            del self.busy[si]
        self.done.extend(fin)
        return fin

    def run(self, reqs, idle_sleep=2e-4):
        """Serve a stream of requests in real time (t_arrival relative to now)."""
        t0 = self.clock()
        pending = sorted(reqs, key=lambda r: r.t_arrival)
        for r in pending:
            r.t_arrival += t0
        i = 0
        while i < len(pending) or self.requests:
            now = self.clock()
            while i < len(pending) and pending[i].t_arrival <= now:
                self.submit(pending[i])
                i += 1
            launched = self.step(now)
            if not launched:
                if self.busy:
                    self.poll()
                if i < len(pending) and not self.busy:
                    time.sleep(min(idle_sleep, max(0.0, pending[i].t_arrival - self.clock())))
        self.poll(wait=True)
        return self.done

    def close(self):
        self.poll(wait=True)
        for pool in self.pools.values():
            for ws in pool:
                ws.close()
        for pl in self.plans.values():
            pl.close()
        self.pools.clear()
        self.plans.clear()
        self.sched.close()


def latency_stats(reqs):
    lat = np.array([r.t_done - r.t_arrival for r in reqs if np.isfinite(r.t_done)])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}


def output_shape(req):
    return (req.n_t, 3) if req.kernel == BIOT_SAVART else (req.n_t,)

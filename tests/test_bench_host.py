"""Host logic of the benchmark script, without a GPU: the one-GPU guard, the
freshness rule for committed counter records, and the error measures the
benchmark line reports against the oracle."""

import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert r.stdout == ""
    assert "one GPU" in r.stderr


def test_counter_record_is_used_only_for_the_source_it_was_taken_on(monkeypatch):
    for name in (bench.HEADLINE_RECORD, bench.POISSON_RECORD):
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        sha = rec["tile_hip_sha256"]
        monkeypatch.setattr(bench, "source_sha", lambda name="tile.hip": sha)
        assert bench.recorded_traffic(name) == rec
        monkeypatch.setattr(bench, "source_sha", lambda name="tile.hip": "0" * 64)
        assert bench.recorded_traffic(name) is None
    assert bench.recorded_traffic("no_such_record.json") is None


def test_error_measures_on_a_worked_example():
    ref = np.array([3.0, -4.0, 0.0, 1.0])
    got = ref + np.array([0.0, 0.4, 0.1, 0.0])
    e = bench.errors(got, ref)
    # rel L2 = |(0, .4, .1, 0)| / |(3, -4, 0, 1)| ; max = .4 / 4
    assert np.isclose(e["rel_l2_err"], np.sqrt(0.17 / 26.0))
    assert np.isclose(e["max_err"], 0.1)
    # per target, floored at the RMS sqrt(26/4): the zero target's .1 error
    # counts against the RMS, the -4 target's .4 against 4
    rms = np.sqrt(26.0 / 4.0)
    assert np.isclose(e["elem_max_err"], max(0.4 / 4.0, 0.1 / rms))
    # area weights enter the L2 measure only
    a = np.array([1.0, 2.0, 1.0, 1.0])
    ea = bench.errors(got, ref, a)
    assert np.isclose(ea["rel_l2_err"], np.sqrt((2 * 0.16 + 0.01) / (9 + 32 + 1)))
    assert ea["max_err"] == e["max_err"] and ea["elem_max_err"] == e["elem_max_err"]


def test_vector_errors_use_the_euclidean_norm_per_target():
    ref = np.array([[3.0, 4.0, 0.0], [0.0, 0.0, 1.0]])
    got = ref + np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 0.0]])
    e = bench.errors(got, ref)
    assert np.isclose(e["rel_l2_err"], 0.5 / np.sqrt(26.0))
    assert np.isclose(e["max_err"], 0.5 / 5.0)


def _csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for r in rows:
            f.write("%d,\"%s\",%d,%s,%r\n" % r)


def test_counter_folding(tmp_path, monkeypatch):
    """Counter runs fold into per-launch HBM bytes: rows of one dispatch are
    summed, dispatches of one (kernel, grid) averaged, KiB scaled by what the
    same counter reads for a 256 MiB copy; only the tile kernels are kept, and
    the PP launch is told apart by the instance's last template argument."""
    pp = "void csfmm::(anonymous namespace)::k_tile<3, false, true>(csfmm::Batch)"
    far = "void csfmm::(anonymous namespace)::k_tile<3, false, false>(csfmm::Batch)"
    wave = "void csfmm::(anonymous namespace)::k_tile_wave<1, true>(csfmm::Batch)"
    other = "void csfmm::(anonymous namespace)::k_l2p(csfmm::Batch)"
    copy = "__amd_rocclr_copyBuffer"
    d = tmp_path / "ctr"
    _csv(str(d / "FETCH_SIZE" / "a_counter_collection.csv"),
         [(1, pp, 4096, "FETCH_SIZE", 100.0), (1, pp, 4096, "FETCH_SIZE", 20.0),
          (2, pp, 4096, "FETCH_SIZE", 140.0), (3, far, 8192, "FETCH_SIZE", 50.0),
          (4, wave, 1024, "FETCH_SIZE", 10.0), (5, other, 64, "FETCH_SIZE", 999.0)])
    _csv(str(d / "WRITE_SIZE" / "a_counter_collection.csv"),
         [(1, pp, 4096, "WRITE_SIZE", 8.0), (2, pp, 4096, "WRITE_SIZE", 12.0),
          (3, far, 8192, "WRITE_SIZE", 5.0), (4, wave, 1024, "WRITE_SIZE", 1.0)])
    _csv(str(d / "FETCH_SIZE_copy" / "a_counter_collection.csv"),
         [(1, copy, 65536, "FETCH_SIZE", 2.0 * 262144)])     # reads twice the copy's bytes
    _csv(str(d / "WRITE_SIZE_copy" / "a_counter_collection.csv"),
         [(1, copy, 65536, "WRITE_SIZE", 262144.0)])         # writes exactly them
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_sha", lambda name="tile.hip": "ab" * 32)

    class A:
        counters = str(d)
        record = "rec.json"
    bench.fold_counters(A)
    rec = json.load(open(str(tmp_path / "profiles" / "rec.json")))
    assert rec["tile_hip_sha256"] == "ab" * 32
    assert rec["copy_calibration"]["fetch_factor"] == 0.5
    assert rec["copy_calibration"]["write_factor"] == 1.0
    by = {x["kernel"]: x for x in rec["dispatches"]}
    assert set(by) == {pp, far, wave}
    assert by[pp]["dispatches"] == 2 and by[pp]["fetch_size_kib"] == 130.0
    assert by[pp]["traffic_bytes"] == 130.0 * 1024 * 0.5 + 10.0 * 1024
    assert by[far]["traffic_bytes"] == 50.0 * 1024 * 0.5 + 5.0 * 1024
    assert by[pp]["pp"] and by[wave]["pp"] and not by[far]["pp"]


def test_roofline_of_the_interaction_launches(monkeypatch):
    """The dominant kernel's roofline: both interaction launches' evaluations
    at 11 flops over the span they occupy (never shorter than either launch),
    against the form's vector peak; traffic from the counter record only when
    its PP dispatch has this plan's grid."""
    st = {"evals_pp": 4e9, "evals_pc": 1e9, "evals_cp": 0, "evals_cc": 3e9,
          "n_leaves_t": 1000, "near_wave": 0}
    stage = {"near_pp_timed_region": 5.0, "pc_far_timed_region": 6.0,
             "interaction_span_timed_region": 7.0}
    rec = {"dispatches": [
        {"kernel": "k_tile<3, false, true>", "grid_size": 256 * 1000, "pp": True,
         "traffic_bytes": 3e8},
        {"kernel": "x::k_tile<3, false, false>", "grid_size": 99, "pp": False,
         "traffic_bytes": 4e8}]}
    monkeypatch.setattr(bench, "recorded_traffic", lambda name: rec)
    r = bench.roofline_of({"stats": st, "stage": stage}, False, "rec.json", "k")
    assert np.isclose(r["achieved"], 8e9 * 11 / 7e-3 / 1e12)
    assert r["peak"] == 78.6 and np.isclose(r["frac"], r["achieved"] / 78.6)
    assert r["traffic"] == 7e8 and r["traffic_record"] == "rec.json"
    assert np.isclose(r["launches"]["pp"]["achieved"], 4e9 * 11 / 5e-3 / 1e12)
    assert np.isclose(r["launches"]["pc_far"]["achieved"], 4e9 * 11 / 6e-3 / 1e12)
    # a span shorter than a launch is taken as that launch; FP32 peak
    stage["interaction_span_timed_region"] = 1.0
    r = bench.roofline_of({"stats": st, "stage": stage}, True, "rec.json", "k")
    assert r["span_ms"] == 6.0 and r["peak"] == 157.3
    # a record of another workload (its PP grid differs) gives no traffic
    st["near_wave"] = 1
    r = bench.roofline_of({"stats": st, "stage": stage}, False, "rec.json", "k")
    assert r["traffic"] is None and r["traffic_record"] is None

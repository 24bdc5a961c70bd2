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

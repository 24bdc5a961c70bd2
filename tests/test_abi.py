"""The C ABI without a GPU: every symbol include/csfmm.h declares is exported,
and argument errors come back as status codes before any device work."""

import ctypes
import os
import re

import pytest

import paper_2508_13550_amd as cs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "csfmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(csfmm_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("csfmm_plan", "csfmm_eval", "csfmm_direct", "csfmm_plan_destroy",
                 "csfmm_plan_stats", "csfmm_last_error", "csfmm_estimate_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = cs.load_library()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(cs.EXPORTED) <= set(_declared())


def _plan(L, targets, n_t, sources, n_s, kernel, p, theta, leaf, flags):
    h = ctypes.c_void_p()
    rc = L.csfmm_plan(targets, n_t, sources, n_s, kernel, p, theta, leaf, flags, None,
                      ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("args,what", [
    ((None, 10, None, 0, 1, 8, 0.7, 64, 0), "targets"),
    ((1, 0, None, 0, 1, 8, 0.7, 64, 0), "n_t"),
    ((1, 10, None, 0, 9, 8, 0.7, 64, 0), "kernel"),
    ((1, 10, None, 0, 1, 0, 0.7, 64, 0), "degree"),
    ((1, 10, None, 0, 1, 17, 0.7, 64, 0), "degree"),
    ((1, 10, None, 0, 1, 8, 0.0, 64, 0), "theta"),
    ((1, 10, None, 0, 1, 8, 1.0, 64, 0), "theta"),
    ((1, 10, None, 0, 1, 8, float("nan"), 64, 0), "theta"),
    ((1, 10, None, 0, 1, 8, 0.7, 0, 0), "leaf"),
    ((1, 10, None, 0, 1, 8, 0.7, 64, 4), "flags"),
    ((1, 10, 1, 0, 1, 8, 0.7, 64, 0), "n_s"),
])
def test_plan_argument_errors(args, what):
    L = cs.load_library()
    rc, h = _plan(L, *args)
    assert rc == -1
    assert h.value is None
    msg = L.csfmm_last_error().decode()
    assert what.split("_")[0] in msg.lower() or what in msg.lower()


def test_other_argument_errors():
    L = cs.load_library()
    assert L.csfmm_eval(None, None, None, None) == -1
    assert L.csfmm_direct(None, 1, None, 1, None, 1, 0, None, None) == -1
    assert L.csfmm_direct(1, 1, 1, 1, 1, 7, 0, 1, None) == -1
    assert L.csfmm_plan_destroy(None) == 0
    assert L.csfmm_plan_stats(None, None) == -1
    assert L.csfmm_estimate_bytes(0, 10, 8, 64, 0) == -1
    b1 = L.csfmm_estimate_bytes(393216, 0, 8, 128, 0)
    b2 = L.csfmm_estimate_bytes(6291456, 6291456, 10, 128, 1)
    assert 0 < b1 < b2 < 64 * 2 ** 30


def test_bve_argument_errors():
    L = cs.load_library()
    f = L.csfmm_bve_rk4_step
    assert f(None, None, None, 10, 0.01, 6.28, 6, 0.7, 64, 0, 0, None) == -1
    assert f(1, 1, 1, 0, 0.01, 6.28, 6, 0.7, 64, 0, 0, None) == -1
    assert f(1, 1, 1, 10, 0.0, 6.28, 6, 0.7, 64, 0, 0, None) == -1
    assert f(1, 1, 1, 10, 0.01, 6.28, 6, 0.7, 64, 8, 0, None) == -1
    assert "bve" in L.csfmm_last_error().decode() or "flags" in L.csfmm_last_error().decode()


def test_bve_remesh_argument_errors():
    """Host-side checks of csfmm_bve_remesh; none of these reaches the device."""
    L = cs.load_library()
    f = L.csfmm_bve_remesh
    assert f(None, 4, 1, 1, 6.28, None) == -1
    assert f(4096, 2, 1 << 20, 1 << 21, 6.28, None) == -1        # E < 3
    assert f(4096, 1 << 15, 1 << 40, 1 << 41, 6.28, None) == -1  # E too large
    assert f(4096, 4, 1 << 20, 1 << 21, float("inf"), None) == -1
    assert f(4096, 4, 4096 + 8, 1 << 21, 6.28, None) == -1       # grid overlaps x
    assert f(4096, 4, 1 << 20, 4096 + 8, 6.28, None) == -1       # zeta inside grid
    assert f(4096, 4, 1 << 20, (1 << 20) + 16, 6.28, None) == -1  # zeta inside x
    assert f(4096, 4, 1 << 20, (1 << 20) - 8, 6.28, None) == -1   # zeta runs into x
    assert "remesh" in L.csfmm_last_error().decode()

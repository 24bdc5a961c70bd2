"""ORACLE -- test infrastructure only.  ctypes front end of direct.c."""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle_direct.so")
_lib = None


def build_oracle():
    """Compile direct.c with gcc (plain -O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_direct.restype = ctypes.c_int
        lib.oracle_direct.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def oracle_threads():
    """Number of OpenMP threads the oracle uses by default."""
    return int(_load().oracle_max_threads())


def direct(kernel, targets, sources, weights, nthreads=0):
    """phi_i = sum_j K(x_i, y_j) w_j in FP64, exact coincidences omitted.

    kernel: 1 Poisson log, 2 Biot-Savart (returns [Nt,3]), 3 1/|x-y|,
    4 biharmonic, 5 SAL closed form.
    """
    lib = _load()
    t = np.ascontiguousarray(targets, dtype=np.float64)
    s = np.ascontiguousarray(sources, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    if t.ndim != 2 or t.shape[1] != 3 or s.ndim != 2 or s.shape[1] != 3:
        raise ValueError("points must be [N,3]")
    if w.shape != (s.shape[0],):
        raise ValueError("weights must be [Ns]")
    out = np.zeros((t.shape[0], 3) if kernel == 2 else (t.shape[0],))
    rc = lib.oracle_direct(int(kernel), t.ctypes.data, t.shape[0], s.ctypes.data,
                           s.shape[0], w.ctypes.data, out.ctypes.data, int(nthreads))
    if rc != 0:
        raise ValueError("oracle_direct rejected its arguments (kernel %r)" % (kernel,))
    return out

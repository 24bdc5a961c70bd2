"""Cubed sphere fast multipole method on AMD MI355X (gfx950).

A thin ctypes binding of libcsfmm.so (declared in include/csfmm.h).  PyTorch
tensors supply device memory and the current HIP stream; every step of the
method runs in the library's HIP kernels.  If the library is missing, or no
GPU is present, calls raise instead of falling back to anything else.

    plan = Plan(targets, None, kernel=POISSON, p=8, theta=0.7, leaf_size=64)
    phi = plan.eval(weights)          # phi_i = sum_j K(x_i, x_j) w_j, i != j
    ref = direct(targets, targets, weights, kernel=POISSON)
"""

import ctypes
import os

import torch

POISSON = 1
BIOT_SAVART = 2
INV_DIST = 3
BIHARMONIC = 4
SAL = 5
KERNELS = {"poisson": POISSON, "biot_savart": BIOT_SAVART, "inv_dist": INV_DIST,
           "biharmonic": BIHARMONIC, "sal": SAL}

FP64 = 0
FP32_FORM = 1
SHRINK = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsfmm.so")

LIST_KINDS = ("PP", "PC", "CP", "CC")


class CsfmmError(RuntimeError):
    """A negative status from the library, with its message."""

    def __init__(self, status, msg):
        super().__init__("csfmm error %d: %s" % (status, msg))
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_targets", ctypes.c_int64), ("n_sources", ctypes.c_int64),
        ("same_set", ctypes.c_int32), ("kernel", ctypes.c_int32),
        ("p", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
        ("theta", ctypes.c_double), ("flags", ctypes.c_uint32),
        ("depth_t", ctypes.c_int32), ("depth_s", ctypes.c_int32),
        ("n_cells_t", ctypes.c_int64), ("n_cells_s", ctypes.c_int64),
        ("n_leaves_t", ctypes.c_int64), ("n_leaves_s", ctypes.c_int64),
        ("n_pp", ctypes.c_int64), ("n_pc", ctypes.c_int64),
        ("n_cp", ctypes.c_int64), ("n_cc", ctypes.c_int64),
        ("evals_pp", ctypes.c_int64), ("evals_pc", ctypes.c_int64),
        ("evals_cp", ctypes.c_int64), ("evals_cc", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("max_leaf_t", ctypes.c_int64),
        ("pp_sym_pairs", ctypes.c_int64), ("pp_one_way", ctypes.c_int64),
        ("pp_close", ctypes.c_int64), ("near_wave", ctypes.c_int64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None

EXPORTED = (
    "csfmm_plan", "csfmm_eval", "csfmm_eval_kernel", "csfmm_direct", "csfmm_plan_destroy",
    "csfmm_plan_stats", "csfmm_estimate_bytes", "csfmm_last_error", "csfmm_plan_cells",
    "csfmm_plan_proxies", "csfmm_plan_permutation", "csfmm_plan_list", "csfmm_eval_stages",
    "csfmm_plan_timing", "csfmm_plan_timing_read", "csfmm_workspace_create",
    "csfmm_workspace_destroy", "csfmm_workspace_bytes", "csfmm_eval_many",
    "csfmm_eval_treecode", "csfmm_bve_rk4_step", "csfmm_bve_remesh", "csfmm_direct_noalloc",
    "csfmm_workspace_device_bytes",
)

STAGES = ("p2m", "m2m", "near_pp", "pc_far", "l2l_l2p", "interaction_span")


def load_library(path=LIB_PATH):
    """Load libcsfmm.so and declare its C signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libcsfmm.so not found at %s; build it with "
                           "`python -m paper_2508_13550_amd.build`" % path)
    L = ctypes.CDLL(path)
    vp, i64, i32p, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    L.csfmm_plan.argtypes = [dp, i64, dp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                             ctypes.c_int, ctypes.c_uint, vp, ctypes.POINTER(vp)]
    L.csfmm_eval.argtypes = [vp, dp, dp, vp]
    L.csfmm_eval_kernel.argtypes = [vp, ctypes.c_int, dp, dp, vp]
    L.csfmm_eval_stages.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp, dp, vp]
    L.csfmm_eval_treecode.argtypes = [vp, ctypes.c_int, dp, dp, vp]
    L.csfmm_bve_rk4_step.argtypes = [dp, dp, dp, i64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_uint,
                                     ctypes.c_int, vp]
    L.csfmm_bve_remesh.argtypes = [dp, i64, dp, dp, ctypes.c_double, vp]
    L.csfmm_direct.argtypes = [dp, i64, dp, i64, dp, ctypes.c_int, ctypes.c_uint, dp, vp]
    L.csfmm_direct_noalloc.argtypes = L.csfmm_direct.argtypes
    L.csfmm_plan_destroy.argtypes = [vp]
    L.csfmm_plan_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.csfmm_estimate_bytes.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    L.csfmm_estimate_bytes.restype = ctypes.c_int64
    L.csfmm_last_error.restype = ctypes.c_char_p
    L.csfmm_plan_cells.argtypes = [vp, ctypes.c_int] + [i32p] * 7 + [dp, dp]
    L.csfmm_plan_proxies.argtypes = [vp, ctypes.c_int, dp]
    L.csfmm_plan_permutation.argtypes = [vp, ctypes.c_int, dp]
    L.csfmm_plan_list.argtypes = [vp, ctypes.c_int, i32p, i32p, i64]
    L.csfmm_plan_timing.argtypes = [vp, ctypes.c_int]
    L.csfmm_workspace_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
    L.csfmm_workspace_destroy.argtypes = [vp]
    L.csfmm_workspace_bytes.argtypes = [vp]
    L.csfmm_workspace_bytes.restype = ctypes.c_int64
    L.csfmm_workspace_device_bytes.argtypes = [vp]
    L.csfmm_workspace_device_bytes.restype = ctypes.c_int64
    L.csfmm_eval_many.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(vp),
                                  ctypes.POINTER(vp), vp]
    L.csfmm_plan_timing_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTED:
        f = getattr(L, name)
        if name not in ("csfmm_estimate_bytes", "csfmm_last_error", "csfmm_workspace_bytes",
                        "csfmm_workspace_device_bytes"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        msg = _lib.csfmm_last_error().decode(errors="replace")
        raise CsfmmError(rc, msg)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("csfmm needs an AMD GPU (gfx950); none is visible")
    load_library()


def _points(x, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if x.dtype != torch.float64 or x.device.type != "cuda" or x.dim() != 2 or x.shape[1] != 3:
        raise ValueError("%s must be a float64 [N,3] tensor on the GPU" % name)
    return x.contiguous()


def _vec(x, n, name):
    if not isinstance(x, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if x.dtype != torch.float64 or x.device.type != "cuda" or x.shape != (n,):
        raise ValueError("%s must be a float64 [%d] tensor on the GPU" % (name, n))
    return x.contiguous()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def estimate_bytes(n_t, n_s, p, leaf_size, fp32=False):
    """Upper estimate of a plan's device bytes (csfmm_estimate_bytes)."""
    L = load_library()
    return int(L.csfmm_estimate_bytes(int(n_t), int(n_s), int(p), int(leaf_size),
                                      FP32_FORM if fp32 else FP64))


class Plan:
    """csfmm_plan: trees, proxies, interpolation operators and lists."""

    def __init__(self, targets, sources=None, kernel=POISSON, p=8, theta=0.7, leaf_size=64,
                 fp32=False, shrink=False):
        _require_gpu()
        self.targets = _points(targets, "targets")
        self.sources = None if sources is None else _points(sources, "sources")
        self.kernel = int(kernel)
        self.p = int(p)
        self.theta = float(theta)
        self.leaf_size = int(leaf_size)
        self.fp32 = bool(fp32)
        self.shrink = bool(shrink)
        self.n_t = self.targets.shape[0]
        self.n_s = self.n_t if self.sources is None else self.sources.shape[0]
        h = ctypes.c_void_p()
        src_ptr = None if self.sources is None else self.sources.data_ptr()
        _check(_lib.csfmm_plan(self.targets.data_ptr(), self.n_t, src_ptr, self.n_s,
                               self.kernel, self.p, self.theta, self.leaf_size,
                               (FP32_FORM if self.fp32 else FP64) | (SHRINK if self.shrink else 0),
                               _stream(), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan was destroyed")
        return self._h

    def _out(self, kernel, out):
        shape = (self.n_t, 3) if kernel == BIOT_SAVART else (self.n_t,)
        if out is None:
            return torch.empty(shape, dtype=torch.float64, device=self.targets.device)
        if out.shape != shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape %s" % (shape,))
        return out

    def eval(self, weights, kernel=None, out=None):
        """csfmm_eval / csfmm_eval_kernel: phi at the targets (caller order)."""
        k = self.kernel if kernel is None else int(kernel)
        w = _vec(weights, self.n_s, "weights")
        out = self._out(k, out)
        _check(_lib.csfmm_eval_kernel(self.handle, k, w.data_ptr(), out.data_ptr(), _stream()))
        return out

    def eval_treecode(self, weights, kernel=None, out=None):
        """csfmm_eval_treecode: the cubed sphere treecode (Algorithm 1), FP64."""
        k = self.kernel if kernel is None else int(kernel)
        w = _vec(weights, self.n_s, "weights")
        out = self._out(k, out)
        _check(_lib.csfmm_eval_treecode(self.handle, k, w.data_ptr(), out.data_ptr(), _stream()))
        return out

    def eval_stages(self, weights, kernel=None):
        """csfmm_eval_stages: (phi, proxy weights, proxy potentials, near field)."""
        k = self.kernel if kernel is None else int(kernel)
        st = self.stats()
        KS = ((self.p + 1) ** 2 + 3) // 4 * 4
        vd = 3 if k == BIOT_SAVART else 1
        w = _vec(weights, self.n_s, "weights")
        out = self._out(k, None)
        dev = self.targets.device
        wbar = torch.empty((st["n_cells_s"], KS), dtype=torch.float64, device=dev)
        psi = torch.empty((vd, st["n_cells_t"], KS), dtype=torch.float64, device=dev)
        near = torch.empty((self.n_t, vd), dtype=torch.float64, device=dev)
        _check(_lib.csfmm_eval_stages(self.handle, k, w.data_ptr(), out.data_ptr(),
                                      wbar.data_ptr(), psi.data_ptr(), near.data_ptr(), _stream()))
        K = (self.p + 1) ** 2
        return out, wbar[:, :K], psi[:, :, :K], near

    def stats(self):
        s = Stats()
        _check(_lib.csfmm_plan_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    def timing(self, enable=True):
        """Per-stage event timing: True/1 every stage, 2 the PP and the PC + far
        launches only, False/0 off; on resets the sums."""
        level = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        _check(_lib.csfmm_plan_timing(self.handle, level))

    def timing_read(self):
        """(number of timed evals, {stage: summed ms}) for the evals since timing(True)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int64()
        _check(_lib.csfmm_plan_timing_read(self.handle, ms, ctypes.byref(n)))
        return int(n.value), dict(zip(STAGES, list(ms)))

    def cells(self, which=0):
        """Cell arrays of the target (0) or source (1) tree, as NumPy arrays."""
        import numpy as np
        st = self.stats()
        n = st["n_cells_t"] if which == 0 else st["n_cells_s"]
        arrs = {k: np.empty(n, dtype=np.int32)
                for k in ("level", "face", "ci", "cj", "begin", "count", "child0")}
        center = np.empty((n, 3))
        radius = np.empty(n)
        _check(_lib.csfmm_plan_cells(self.handle, which,
                                     *[arrs[k].ctypes.data for k in
                                       ("level", "face", "ci", "cj", "begin", "count", "child0")],
                                     center.ctypes.data, radius.ctypes.data))
        arrs["center"] = center
        arrs["radius"] = radius
        return arrs

    def proxies(self, which=0):
        import numpy as np
        st = self.stats()
        n = st["n_cells_t"] if which == 0 else st["n_cells_s"]
        out = np.empty((n, (self.p + 1) ** 2, 3))
        _check(_lib.csfmm_plan_proxies(self.handle, which, out.ctypes.data))
        return out

    def permutation(self, which=0):
        import numpy as np
        n = self.n_t if which == 0 else self.n_s
        out = np.empty(n, dtype=np.int64)
        _check(_lib.csfmm_plan_permutation(self.handle, which, out.ctypes.data))
        return out

    def lists(self):
        """{"PP": (tgt, src), ...} cell-index pairs sorted by target then source."""
        import numpy as np
        st = self.stats()
        res = {}
        for kind, name in enumerate(LIST_KINDS):
            n = st["n_" + name.lower()]
            t = np.empty(max(n, 1), dtype=np.int32)
            s = np.empty(max(n, 1), dtype=np.int32)
            _check(_lib.csfmm_plan_list(self.handle, kind, t.ctypes.data, s.ctypes.data, n))
            res[name] = (t[:n], s[:n])
        return res

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.csfmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """csfmm_workspace_create: eval buffers of one in-flight request on a plan."""

    def __init__(self, plan):
        _require_gpu()
        self.plan = plan
        h = ctypes.c_void_p()
        _check(_lib.csfmm_workspace_create(plan.handle, _stream(), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("workspace was destroyed")
        return self._h

    @property
    def device_bytes(self):
        """Device bytes this workspace holds."""
        return int(_lib.csfmm_workspace_device_bytes(self.handle))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.csfmm_workspace_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(plan):
    """Device bytes of one workspace for this plan."""
    return int(load_library().csfmm_workspace_bytes(plan.handle))


def eval_many(requests, outs=None):
    """csfmm_eval_many over [(plan, workspace, kernel, weights), ...] -> outputs.

    One packed launch per phase serves all requests (near and far field: one
    per kernel id and form).  Returns the list of output tensors.
    """
    _require_gpu()
    n = len(requests)
    P = (ctypes.c_void_p * n)()
    W = (ctypes.c_void_p * n)()
    K = (ctypes.c_int * n)()
    WP = (ctypes.c_void_p * n)()
    OP = (ctypes.c_void_p * n)()
    res = []
    keep = []
    for i, (plan, ws, kernel, weights) in enumerate(requests):
        if ws.plan is not plan:
            raise ValueError("request %d: workspace belongs to another plan" % i)
        k = plan.kernel if kernel is None else int(kernel)
        w = _vec(weights, plan.n_s, "weights")
        o = plan._out(k, None if outs is None else outs[i])
        keep.append(w)
        res.append(o)
        P[i] = plan.handle.value
        W[i] = ws.handle.value
        K[i] = k
        WP[i] = w.data_ptr()
        OP[i] = o.data_ptr()
    _check(_lib.csfmm_eval_many(n, P, W, K, WP, OP, _stream()))
    return res


def bve_rk4_step(x, zeta, area, dt, omega=2.0 * 3.141592653589793, p=6, theta=0.7,
                 leaf_size=128, fp32=False, use_direct=False):
    """csfmm_bve_rk4_step: one RK4 step of the barotropic vorticity equation;
    x [n,3] and zeta [n] (float64, on the GPU) are updated in place."""
    _require_gpu()
    xp = _points(x, "x")
    n = xp.shape[0]
    z = _vec(zeta, n, "zeta")
    a = _vec(area, n, "area")
    if xp.data_ptr() != x.data_ptr() or z.data_ptr() != zeta.data_ptr():
        raise ValueError("x and zeta must be contiguous float64 CUDA tensors (updated in place)")
    _check(_lib.csfmm_bve_rk4_step(xp.data_ptr(), z.data_ptr(), a.data_ptr(), n, float(dt),
                                   float(omega), int(p), float(theta), int(leaf_size),
                                   FP32_FORM if fp32 else FP64, 1 if use_direct else 0,
                                   _stream()))
    return x, zeta


def bve_remesh(grid, E, x, zeta, omega=2.0 * 3.141592653589793):
    """csfmm_bve_remesh: map particles that started a step at the cells of
    the equiangular cubed-sphere grid `grid` (cubed_sphere_grid(E) order) back
    onto them; x becomes grid and zeta the remeshed vorticity (in place)."""
    _require_gpu()
    E = int(E)
    n = 6 * E * E
    g = _points(grid, "grid")
    xp = _points(x, "x")
    z = _vec(zeta, n, "zeta")
    if g.shape[0] != n or xp.shape[0] != n:
        raise ValueError("grid and x must hold 6 E^2 = %d points" % n)
    if xp.data_ptr() != x.data_ptr() or z.data_ptr() != zeta.data_ptr():
        raise ValueError("x and zeta must be contiguous float64 CUDA tensors (updated in place)")
    _check(_lib.csfmm_bve_remesh(g.data_ptr(), E, xp.data_ptr(), z.data_ptr(), float(omega),
                                 _stream()))
    return x, zeta


def direct(targets, sources, weights, kernel=POISSON, fp32=False, out=None):
    """csfmm_direct: phi_i = sum_j K(x_i, y_j) w_j over all pairs (coincidences omitted)."""
    _require_gpu()
    t = _points(targets, "targets")
    s = _points(sources, "sources")
    w = _vec(weights, s.shape[0], "weights")
    shape = (t.shape[0], 3) if int(kernel) == BIOT_SAVART else (t.shape[0],)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=t.device)
    _check(_lib.csfmm_direct(t.data_ptr(), t.shape[0], s.data_ptr(), s.shape[0], w.data_ptr(),
                             int(kernel), FP32_FORM if fp32 else FP64, out.data_ptr(), _stream()))
    return out


def direct_noalloc(targets, sources, weights, out, kernel=POISSON, fp32=False):
    """csfmm_direct_noalloc: the direct sum into a caller-provided `out`, with
    no device allocation by the library (static scratch; calls that overlap
    on one GPU race)."""
    _require_gpu()
    t = _points(targets, "targets")
    s = _points(sources, "sources")
    w = _vec(weights, s.shape[0], "weights")
    shape = (t.shape[0], 3) if int(kernel) == BIOT_SAVART else (t.shape[0],)
    if (not isinstance(out, torch.Tensor) or out.dtype != torch.float64 or
            out.device.type != "cuda" or tuple(out.shape) != shape or not out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 GPU tensor of shape %s" % (shape,))
    _check(_lib.csfmm_direct_noalloc(t.data_ptr(), t.shape[0], s.data_ptr(), s.shape[0],
                                     w.data_ptr(), int(kernel), FP32_FORM if fp32 else FP64,
                                     out.data_ptr(), _stream()))
    return out

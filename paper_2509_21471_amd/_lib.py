"""ctypes binding of libdmk_stokes.so (argument marshalling only).

Every computation runs in the HIP library; torch is used only to own device
memory and to name the stream.  Importing works without a GPU (host-only
diagnostics are callable); plan/eval raise if the library or a GPU is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libdmk_stokes.so")

DMK_OK = 0
STATUS = {0: "DMK_OK", -1: "DMK_ERR_ARG", -2: "DMK_ERR_UNSUPPORTED", -3: "DMK_ERR_DOMAIN",
          -4: "DMK_ERR_NONFINITE", -5: "DMK_ERR_TOL", -6: "DMK_ERR_OOM", -7: "DMK_ERR_HIP"}
PREC_FP64, PREC_MIXED = 0, 1
KERNEL_STOKESLET, KERNEL_STRESSLET = 0, 1
METHOD_DMK, METHOD_EWALD = 0, 1

SYMBOLS = ["dmk_stokes_ewald_params", "dmk_stokes_radial_stresslet", "dmk_stokes_params_ex", "dmk_stokes_params_kernel", "dmk_stokes_eval_stresslet",
           "dmk_stokes_residual_sum_stresslet", "dmk_stokes_plan", "dmk_stokes_plan_ex", "dmk_stokes_plan_batch", "dmk_stokes_plan_targets", "dmk_stokes_autotune", "dmk_stokes_eval", "dmk_stokes_plan_info",
           "dmk_stokes_tree_leaves", "dmk_stokes_destroy", "dmk_last_error", "dmk_stokes_params",
           "dmk_stokes_radial", "dmk_stokes_mollifier", "dmk_stokes_residual_sum", "dmk_stokes_phase_ms",
           "dmk_stokes_residual_sum_noalloc",
           "dmk_stokes_near_stats", "dmk_stokes_release_cached_memory", "dmk_stokes_host_tree"]
PHASES = ["anterp", "merge", "outgoing", "translate", "incoming", "root", "interp", "leaf_eval", "near",
          "finalize"]
FLAG_PHASE_TIMING = 1
FLAG_CONCURRENT_PLAN = 2
FLAG_GRAPH = 4
FLAG_MORTON_ORDER = 8
FLAG_HOST_TREE = 16


class DMKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("leaf_size", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("mem_cap_bytes", ctypes.c_size_t), ("flags", ctypes.c_int), ("near_lanes", ctypes.c_int),
                ("q", ctypes.c_int), ("p", ctypes.c_int), ("rhs_batch", ctypes.c_int), ("window", ctypes.c_int),
                ("kernel", ctypes.c_int), ("method", ctypes.c_int), ("stage_rows", ctypes.c_int),
                ("eval_points", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("c", ctypes.c_double), ("q", ctypes.c_int), ("p", ctypes.c_int),
                ("n1", ctypes.c_int), ("nper", ctypes.c_int), ("leaf_size", ctypes.c_int),
                ("deg_P", ctypes.c_int), ("deg_Q", ctypes.c_int), ("levels", ctypes.c_int),
                ("periodic", ctypes.c_int), ("n_points", ctypes.c_int64), ("n_boxes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_nonempty_boxes", ctypes.c_int64),
                ("n_nonempty_leaves", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
                ("n_senders", ctypes.c_int64), ("n_receivers", ctypes.c_int64),
                ("center", ctypes.c_double * 3), ("box_len", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t), ("plan_ms", ctypes.c_double),
                ("plan_phase_ms", ctypes.c_double * 6), ("near_lanes", ctypes.c_int), ("precision", ctypes.c_int),
                ("window", ctypes.c_int), ("sigma", ctypes.c_double), ("kernel", ctypes.c_int),
                ("method", ctypes.c_int), ("ewald_grid", ctypes.c_int), ("ewald_modes", ctypes.c_int),
                ("ewald_width", ctypes.c_int), ("no_coincident", ctypes.c_int)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name in ("center", "plan_phase_ms") else v
        return d


_lib = None


def lib():
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: run paper_2509_21471_amd.build.build() first")
        L = ctypes.CDLL(SO_PATH)
        vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
        L.dmk_stokes_plan.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(vp)]
        L.dmk_stokes_plan_ex.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.dmk_stokes_plan_targets.argtypes = [vp, i64, vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                              ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.dmk_stokes_plan_batch.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.POINTER(Opts), ctypes.POINTER(vp)]
        L.dmk_stokes_autotune.argtypes = [vp, i64, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.POINTER(Opts), ctypes.c_int, ctypes.POINTER(Opts),
                                          ctypes.POINTER(ctypes.c_double)]
        L.dmk_stokes_eval.argtypes = [vp, vp, ctypes.c_int, vp]
        L.dmk_stokes_eval_stresslet.argtypes = [vp, vp, vp, ctypes.c_int, vp]
        L.dmk_stokes_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.dmk_stokes_tree_leaves.argtypes = [vp, vp, vp, vp, vp]
        L.dmk_stokes_destroy.argtypes = [vp]
        L.dmk_stokes_destroy.restype = None
        L.dmk_last_error.argtypes = []
        L.dmk_last_error.restype = ctypes.c_char_p
        L.dmk_stokes_params.argtypes = [ctypes.c_double, ctypes.POINTER(PlanInfo)]
        L.dmk_stokes_params_ex.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.POINTER(PlanInfo)]
        L.dmk_stokes_params_kernel.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(PlanInfo)]
        L.dmk_stokes_radial.argtypes = [ctypes.c_double, dp, i64, dp]
        L.dmk_stokes_mollifier.argtypes = [ctypes.c_double, dp, i64, dp]
        L.dmk_stokes_radial_stresslet.argtypes = [ctypes.c_double, dp, i64, dp]
        L.dmk_stokes_ewald_params.argtypes = [ctypes.c_double, i64, ctypes.c_int, ctypes.POINTER(PlanInfo)]
        L.dmk_stokes_residual_sum.argtypes = [vp, i64, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp, vp]
        L.dmk_stokes_residual_sum_noalloc.argtypes = [vp, i64, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp,
                                                      vp]
        L.dmk_stokes_residual_sum_stresslet.argtypes = [vp, i64, vp, vp, vp, i64, ctypes.c_double,
                                                        ctypes.c_double, vp, vp]
        L.dmk_stokes_phase_ms.argtypes = [vp, dp]
        L.dmk_stokes_near_stats.argtypes = [vp, vp, vp, vp]
        L.dmk_stokes_host_tree.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, i64, vp, vp, vp, vp, vp]
        L.dmk_stokes_release_cached_memory.argtypes = []
        L.dmk_stokes_release_cached_memory.restype = None
        for s in SYMBOLS:
            if s not in ("dmk_stokes_destroy", "dmk_last_error", "dmk_stokes_release_cached_memory"):
                getattr(L, s).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != DMK_OK:
        raise DMKError(rc, lib().dmk_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---- host-only diagnostics ------------------------------------------------------
def params(tol: float, window: int = 0, kernel: int = KERNEL_STOKESLET) -> dict:
    info = PlanInfo()
    _check(lib().dmk_stokes_params_kernel(float(tol), int(window), int(kernel), ctypes.byref(info)))
    return info.as_dict()


def radial(tol: float, rho) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
    out = np.zeros((rho.size, 4))
    _check(lib().dmk_stokes_radial(float(tol), _dp(rho), rho.size, _dp(out)))
    return out


def ewald_params(tol: float, n: int, leaf_size: int = 0) -> dict:
    """Split level and grid a spectral Ewald plan would use (host only)."""
    info = PlanInfo()
    _check(lib().dmk_stokes_ewald_params(float(tol), int(n), int(leaf_size), ctypes.byref(info)))
    return info.as_dict()


def radial_stresslet(tol: float, rho) -> np.ndarray:
    """(A, D) of the residual stresslet's near-field fits at rho^2, shape (n, 2)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
    out = np.zeros((rho.size, 2))
    _check(lib().dmk_stokes_radial_stresslet(float(tol), _dp(rho), rho.size, _dp(out)))
    return out


def mollifier(tol: float, k) -> np.ndarray:
    k = np.ascontiguousarray(k, dtype=np.float64).ravel()
    out = np.zeros((k.size, 2))
    _check(lib().dmk_stokes_mollifier(float(tol), _dp(k), k.size, _dp(out)))
    return out


def host_tree(points, leaf_size: int, periodic: bool = False):
    """Leaves of the octree built on the host: (levels, coords (L,3), counts, near_pairs)."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n = pts.shape[0]
    nl, npairs = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().dmk_stokes_host_tree(pts.ctypes.data, n, int(leaf_size), int(bool(periodic)), 0, None, None, None,
                                    ctypes.byref(nl), ctypes.byref(npairs))
    cap = nl.value
    lev = np.zeros(cap, dtype=np.int32)
    crd = np.zeros((cap, 3), dtype=np.int64)
    cnt = np.zeros(cap, dtype=np.int64)
    _check(lib().dmk_stokes_host_tree(pts.ctypes.data, n, int(leaf_size), int(bool(periodic)), cap,
                                      lev.ctypes.data, crd.ctypes.data, cnt.ctypes.data, ctypes.byref(nl),
                                      ctypes.byref(npairs)))
    return lev, crd, cnt, npairs.value


# ---- device entry points --------------------------------------------------------
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the DMK library runs on gfx950 only")
    return torch


def _dev_f64(t, shape_last=3):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        t = t.to(device="cuda", dtype=torch.float64).contiguous()
    if t.shape[-1] != shape_last:
        raise ValueError(f"last dimension must be {shape_last}")
    return t


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A DMK plan over device points (sources = targets)."""

    def __init__(self, points, periodic: bool = False, tol: float = 1e-6, precision: int = PREC_FP64,
                 leaf_size: int = 0, stream=None, mem_cap_bytes: int = 0, timing: bool = False,
                 near_lanes: int = 0, q: int = 0, p: int = 0, rhs_batch: int = 0, concurrent: bool = False,
                 offsets=None, graph: bool = False, targets=None, window: int = 0,
                 kernel: int = KERNEL_STOKESLET, method: int = METHOD_DMK, leaf_order: bool = True,
                 host_tree: bool = False, stage_rows: int = 0, eval_points: int = 0):
        """offsets (host int sequence, n_problems + 1 entries) makes a batched
        plan over independent problems (dmk_stokes_plan_batch); targets (device
        (m,3)) makes a plan evaluating the sums at a separate target set
        (dmk_stokes_plan_targets): forces (n_rhs, n, 3) -> velocities (n_rhs, m, 3).
        kernel = KERNEL_STRESSLET makes a stresslet plan, evaluated with
        eval_stresslet.  method = METHOD_EWALD makes a single-level spectral
        Ewald plan (periodic, one problem).  leaf_order = False keeps the
        points of every leaf in Morton order (DMK_FLAG_MORTON_ORDER).
        host_tree = True builds the octree and lists on the host
        (DMK_FLAG_HOST_TREE, the reference construction)."""
        torch = _torch()
        pts = _dev_f64(points)
        self.n = int(pts.shape[0])
        self.n_out = self.n
        self.stream = stream
        opts = Opts(int(precision), int(leaf_size), _stream_ptr(stream), int(mem_cap_bytes),
                    (FLAG_PHASE_TIMING if timing else 0) | (FLAG_CONCURRENT_PLAN if concurrent else 0)
                    | (FLAG_GRAPH if graph else 0) | (0 if leaf_order else FLAG_MORTON_ORDER)
                    | (FLAG_HOST_TREE if host_tree else 0),
                    int(near_lanes), int(q), int(p), int(rhs_batch), int(window), int(kernel),
                    int(method), int(stage_rows), int(eval_points))
        h = ctypes.c_void_p()
        if targets is not None:
            if offsets is not None:
                raise ValueError("targets and offsets cannot be combined")
            tg = _dev_f64(targets)
            self.n_out = int(tg.shape[0])
            _check(lib().dmk_stokes_plan_targets(ctypes.c_void_p(pts.data_ptr()), self.n,
                                                 ctypes.c_void_p(tg.data_ptr()), self.n_out, 3,
                                                 int(bool(periodic)), float(tol), ctypes.byref(opts),
                                                 ctypes.byref(h)))
        elif offsets is None:
            _check(lib().dmk_stokes_plan_ex(ctypes.c_void_p(pts.data_ptr()), self.n, 3, int(bool(periodic)),
                                            float(tol), ctypes.byref(opts), ctypes.byref(h)))
        else:
            off = np.ascontiguousarray(offsets, dtype=np.int64)
            if off.ndim != 1 or off.size < 2 or off[-1] != self.n:
                raise ValueError("offsets must hold n_problems + 1 entries ending at n")
            _check(lib().dmk_stokes_plan_batch(ctypes.c_void_p(pts.data_ptr()),
                                               off.ctypes.data_as(ctypes.c_void_p), int(off.size - 1), 3,
                                               int(bool(periodic)), float(tol), ctypes.byref(opts),
                                               ctypes.byref(h)))
        self._h = h
        self._torch = torch

    def eval(self, forces, out=None):
        torch = self._torch
        f = _dev_f64(forces)
        n_rhs = 1 if f.dim() == 2 else int(f.shape[0])
        if f.shape[-2] != self.n:
            raise ValueError("forces must have shape (n,3) or (n_rhs,n,3)")
        if out is None:
            shape = (self.n_out, 3) if f.dim() == 2 else (n_rhs, self.n_out, 3)
            out = torch.empty(shape, dtype=f.dtype, device=f.device)
        _check(lib().dmk_stokes_eval(self._h, ctypes.c_void_p(f.data_ptr()), n_rhs,
                                     ctypes.c_void_p(out.data_ptr())))
        return out

    def eval_stresslet(self, forces, normals, out=None):
        """Stresslet sums u_j = sum T_jlm f_l n_m (dmk_stokes_eval_stresslet)."""
        torch = self._torch
        f = _dev_f64(forces)
        nv = _dev_f64(normals)
        if f.shape != nv.shape:
            raise ValueError("forces and normals must have the same shape")
        n_rhs = 1 if f.dim() == 2 else int(f.shape[0])
        if f.shape[-2] != self.n:
            raise ValueError("forces must have shape (n,3) or (n_rhs,n,3)")
        if out is None:
            shape = (self.n_out, 3) if f.dim() == 2 else (n_rhs, self.n_out, 3)
            out = torch.empty(shape, dtype=f.dtype, device=f.device)
        _check(lib().dmk_stokes_eval_stresslet(self._h, ctypes.c_void_p(f.data_ptr()),
                                               ctypes.c_void_p(nv.data_ptr()), n_rhs,
                                               ctypes.c_void_p(out.data_ptr())))
        return out

    def info(self) -> dict:
        info = PlanInfo()
        _check(lib().dmk_stokes_plan_info(self._h, ctypes.byref(info)))
        return info.as_dict()

    def phase_ms(self) -> dict:
        out = np.zeros(len(PHASES))
        _check(lib().dmk_stokes_phase_ms(self._h, _dp(out)))
        return dict(zip(PHASES, out.tolist()))

    def near_stats(self) -> dict:
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().dmk_stokes_near_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"listed": a.value, "evaluated": b.value, "in_support": c.value}

    def tree_leaves(self):
        info = self.info()
        L = int(info["n_leaves"])
        lev = np.zeros(L, dtype=np.int32)
        crd = np.zeros((L, 3), dtype=np.int64)
        cnt = np.zeros(L, dtype=np.int64)
        pl = np.zeros(self.n, dtype=np.int64)
        _check(lib().dmk_stokes_tree_leaves(self._h, lev.ctypes.data, crd.ctypes.data, cnt.ctypes.data,
                                            pl.ctypes.data))
        return lev, crd, cnt, pl

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dmk_stokes_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(points, periodic: bool = False, tol: float = 1e-6, precision: int = PREC_FP64, offsets=None,
             n_rhs: int = 1, leaf_size: int = 0, stream=None) -> dict:
    """dmk_stokes_autotune: the leaf size, near-field lane split and far-field
    tile shapes (stage_rows, eval_points) to pass to Plan for this workload, and
    the best trial's plan + eval milliseconds."""
    pts = _dev_f64(points)
    n = int(pts.shape[0])
    opts = Opts(int(precision), int(leaf_size), _stream_ptr(stream), 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0)
    tuned = Opts()
    ms = ctypes.c_double()
    off = None
    nprob = 0
    if offsets is not None:
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        nprob = int(off.size - 1)
    _check(lib().dmk_stokes_autotune(ctypes.c_void_p(pts.data_ptr()), n,
                                     None if off is None else off.ctypes.data_as(ctypes.c_void_p), nprob, 3,
                                     int(bool(periodic)), float(tol), ctypes.byref(opts), int(n_rhs),
                                     ctypes.byref(tuned), ctypes.byref(ms)))
    return {"leaf_size": tuned.leaf_size, "near_lanes": tuned.near_lanes, "stage_rows": tuned.stage_rows,
            "eval_points": tuned.eval_points, "ms": ms.value}


def residual_sum(targets, sources, forces, r_lambda: float, tol: float, stream=None):
    torch = _torch()
    t = _dev_f64(targets)
    s = _dev_f64(sources)
    f = _dev_f64(forces)
    out = torch.empty_like(t)
    _check(lib().dmk_stokes_residual_sum(ctypes.c_void_p(t.data_ptr()), int(t.shape[0]),
                                         ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                         int(s.shape[0]), float(r_lambda), float(tol), _stream_ptr(stream),
                                         ctypes.c_void_p(out.data_ptr())))
    return out


def residual_sum_noalloc(targets, sources, forces, r_lambda: float, tol: float, out, stream=None):
    """dmk_stokes_residual_sum_noalloc: the library allocates nothing; `out`
    (m, 3) float64 on the device is caller-provided.  Stream-ordered, no
    synchronisation."""
    t = _dev_f64(targets)
    s = _dev_f64(sources)
    f = _dev_f64(forces)
    _check(lib().dmk_stokes_residual_sum_noalloc(ctypes.c_void_p(t.data_ptr()), int(t.shape[0]),
                                                 ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                                 int(s.shape[0]), float(r_lambda), float(tol), _stream_ptr(stream),
                                                 ctypes.c_void_p(out.data_ptr())))
    return out


def residual_sum_stresslet(targets, sources, forces, normals, r_lambda: float, tol: float, stream=None):
    torch = _torch()
    t = _dev_f64(targets)
    s = _dev_f64(sources)
    f = _dev_f64(forces)
    nv = _dev_f64(normals)
    out = torch.empty_like(t)
    _check(lib().dmk_stokes_residual_sum_stresslet(ctypes.c_void_p(t.data_ptr()), int(t.shape[0]),
                                                   ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                                   ctypes.c_void_p(nv.data_ptr()), int(s.shape[0]),
                                                   float(r_lambda), float(tol), _stream_ptr(stream),
                                                   ctypes.c_void_p(out.data_ptr())))
    return out

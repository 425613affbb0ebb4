"""CPU oracle for the Stokeslet point sums -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2509_21471_amd``) never imports, links or calls it, and the two share
no code: the oracle is the plain definition of the sums (direct O(N^2) sum,
converged Gaussian-Ewald sum for the periodic cell) plus an independent
evaluation of the kernel-splitting functions used to pin the method's pieces.

Modules
-------
direct.c     compiled to ``liboracle.so`` (OpenMP): direct free-space Stokeslet
             and stresslet sums and the real-space half of the Gaussian Ewald sum.
ewald.py     periodic sum: Fourier half (structure factor by numpy matmul),
             self term, real half via the C routine.
splitting.py PSWF window (Chebyshev collocation of the prolate differential
             operator, lowest eigenfunction), phi, Phi, the biharmonic
             mollifier, residual / mollified Stokeslets and a brute force
             residual pair sum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "direct.c")
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, src, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        L.oracle_stokeslet_direct.argtypes = [dp, dp, ctypes.c_int64, ip, ctypes.c_int64, dp]
        L.oracle_stokeslet_direct.restype = None
        L.oracle_stokeslet_ewald_real.argtypes = [dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                                  ctypes.c_double, ctypes.c_double, dp]
        L.oracle_stokeslet_ewald_real.restype = ctypes.c_int
        L.oracle_stresslet_direct.argtypes = [dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64, dp]
        L.oracle_stresslet_direct.restype = None
        L.oracle_stresslet_ewald_real.argtypes = [dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                                  ctypes.c_double, ctypes.c_double, dp]
        L.oracle_stresslet_ewald_real.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(nt: int) -> None:
    """Threads of later oracle calls (timing only: results do not depend on it)."""
    lib().oracle_set_num_threads(int(nt))


def direct(x, f, targets=None):
    """Free-space Stokeslet sum u_b = sum_{a != b} S(x_b - x_a) f_a at the
    listed target indices (all points if None).  Returns (m,3)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = x.shape[0]
    tg = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    u = np.zeros((tg.shape[0], 3))
    lib().oracle_stokeslet_direct(_dp(x), _dp(f), n, _ip(tg), tg.shape[0], _dp(u))
    return u


def ewald_real(x, f, targets, xi, rc):
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    tg = np.ascontiguousarray(targets, dtype=np.int64)
    u = np.zeros((tg.shape[0], 3))
    rc_ = lib().oracle_stokeslet_ewald_real(_dp(x), _dp(f), x.shape[0], _ip(tg), tg.shape[0],
                                            float(xi), float(rc), _dp(u))
    if rc_ != 0:
        raise ValueError("ewald_real: need 0 < rc <= 1/2 and xi > 0")
    return u


def rel_l2(u, ref):
    """Relative l2 error over all (target, component) entries."""
    u = np.asarray(u, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((u - ref).ravel()) / np.linalg.norm(ref.ravel()))


def stresslet_direct(x, f, nv, targets=None):
    """Free-space stresslet sum u_b = sum_{a != b} T(x_b - x_a) : (f_a n_a) at
    the listed target indices (all points if None).  Returns (m,3)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nv = np.ascontiguousarray(nv, dtype=np.float64)
    n = x.shape[0]
    t = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    u = np.zeros((t.size, 3))
    lib().oracle_stresslet_direct(_dp(x), _dp(f), _dp(nv), n, _ip(t), t.size, _dp(u))
    return u


def stresslet_ewald_real(x, f, nv, targets, xi, rc):
    """Real-space half of the Gaussian Ewald split of the periodic stresslet
    sum (minimum-image pairs within rc), at the listed target indices."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nv = np.ascontiguousarray(nv, dtype=np.float64)
    tg = np.ascontiguousarray(targets, dtype=np.int64)
    u = np.zeros((tg.size, 3))
    rc_ = lib().oracle_stresslet_ewald_real(_dp(x), _dp(f), _dp(nv), x.shape[0], _ip(tg), tg.size, float(xi),
                                            float(rc), _dp(u))
    if rc_ != 0:
        raise ValueError("stresslet_ewald_real: need 0 < rc <= 1/2 and xi > 0")
    return u

"""Multi-core CPU baseline of the decomposed sweep (OpenMP over subdomains; see psw_cpu_omp.c).

bench.py reports it beside the single-threaded oracle; tests/test_cpu_parallel.py holds it to the oracle.
It is not part of the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psw_cpu_omp.c")
_SO = os.path.join(_HERE, "libpsw_cpu_omp.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        subprocess.run(["gcc", "-O3", "-fopenmp", "-std=c99", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"], check=True)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        L.cpu_dsweep.argtypes = [ctypes.c_int, P(ctypes.c_int64), P(ctypes.c_int), P(ctypes.c_int8), P(dp), dp, dp,
                                 dp, dp, dp]
        L.cpu_dsweep.restype = ctypes.c_int
        L.cpu_threads.restype = ctypes.c_int
        L.cpu_triad_bytes_per_s.argtypes = [ctypes.c_int64, ctypes.c_int]
        L.cpu_triad_bytes_per_s.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def dsweep(dim, n, p, dirs, diags, f, uold=None, piv=None, omega=None):
    """One decomposed sweep (stationary with uold and omega per start corner, or a start-coupled
    preconditioner half-sweep with piv); the arguments follow oracle.dsweep."""
    n3 = (ctypes.c_int64 * 3)(*(list(n) + [1] * (3 - dim)))
    p3 = (ctypes.c_int * 3)(*(list(p) + [1] * (3 - dim)))
    arr = [np.ascontiguousarray(d, dtype=np.float64) for d in diags]
    pp = (ctypes.POINTER(ctypes.c_double) * len(arr))(*[_dp(a) for a in arr])
    f = np.ascontiguousarray(f, dtype=np.float64)
    uold = None if uold is None else np.ascontiguousarray(uold, dtype=np.float64)
    piv = None if piv is None else np.ascontiguousarray(piv, dtype=np.float64)
    om = None
    if omega is not None:
        om = np.ascontiguousarray(np.broadcast_to(np.asarray(omega, np.float64).reshape(-1), (1 << dim,))
                                  if np.size(omega) == 1 else np.asarray(omega, np.float64))
    dirs = np.ascontiguousarray(dirs, np.int8)
    out = np.empty_like(f)
    st = lib().cpu_dsweep(dim, n3, p3, dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), pp, _dp(om), _dp(piv),
                          _dp(uold), _dp(f), _dp(out))
    if st:
        raise RuntimeError(f"cpu_dsweep failed ({st})")
    return out


def threads() -> int:
    return int(lib().cpu_threads())


def triad_gbs(n=1 << 26, reps=5) -> float:
    """Host STREAM triad (a = b + 3 c, 24 bytes per element), best of reps, in GB/s."""
    return lib().cpu_triad_bytes_per_s(int(n), int(reps)) / 1e9

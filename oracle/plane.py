"""ctypes front-end of the direct-correlation oracle (direct.c).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline may use this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_direct.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile direct.c with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.fdas_oracle_plane.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_int64, P]
        lib.fdas_oracle_cells.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32,
                                          P, P, ctypes.c_int64, P, P]
        lib.fdas_oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    return int(_load().fdas_oracle_threads())


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def plane(spec, taps, r0: int = 0, r1: int | None = None) -> np.ndarray:
    """P[j, r] for r in [r0, r1) (all rows of ``taps``), float64 (n_z, r1 - r0)."""
    x = _c128(spec)
    g = _c128(taps)
    n = x.size
    r1 = n if r1 is None else r1
    n_z, m = g.shape
    out = np.empty((n_z, max(r1 - r0, 0)), dtype=np.float64)
    if r1 > r0:
        _load().fdas_oracle_plane(x.ctypes.data, n, g.ctypes.data, n_z, m,
                                  r0, r1, out.ctypes.data)
    return out


def cells(spec, taps, j, r, with_amp: bool = False):
    """Power (and complex sum) at individual cells (j[i], r[i])."""
    x = _c128(spec)
    g = _c128(taps)
    j = np.ascontiguousarray(j, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.int64)
    p = np.empty(j.size, dtype=np.float64)
    a = np.empty(j.size, dtype=np.complex128) if with_amp else None
    _load().fdas_oracle_cells(x.ctypes.data, x.size, g.ctypes.data, g.shape[1],
                              j.ctypes.data, r.ctypes.data, j.size, p.ctypes.data,
                              a.ctypes.data if with_amp else None)
    return (p, a) if with_amp else p

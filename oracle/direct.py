"""Python entry points of the C direct-sum oracle (``direct.c``).

TEST INFRASTRUCTURE ONLY.  ``build()`` compiles ``direct.c`` with gcc into
``liboracle.so`` next to this file; ``direct_grid`` and ``direct_points``
call it through ctypes.  Appendix A, eq. greenSum / eq. green2D.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SELF_SKIP = 0
SELF_CELLAVG = 1


def build(force: bool = True) -> str:
    """Compile the oracle (plain FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                        "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d = ctypes.POINTER(ctypes.c_double)
        lib.oracle_direct_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, d, ctypes.c_int64, d, d, ctypes.c_int32, d]
        lib.oracle_direct_grid.restype = ctypes.c_int
        lib.oracle_direct_points.argtypes = [ctypes.c_int64, d, d, d, ctypes.c_int64, d, d, d]
        lib.oracle_direct_points.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_get_threads.argtypes = []
        lib.oracle_get_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the target loop (0 restores the OpenMP default); results do not depend on it."""
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def direct_grid(f, h: float, tx, ty, x0: float = 0.0, y0: float = 0.0, self_mode: int = SELF_SKIP) -> np.ndarray:
    """P at targets from grid sources f[j, i] at (x0+(i+.5)h, y0+(j+.5)h)."""
    lib = _load()
    f = _f64(f)
    if f.ndim != 2:
        raise ValueError("f must be a (ny, nx) array")
    ny, nx = f.shape
    tx = _f64(tx).ravel()
    ty = _f64(ty).ravel()
    if tx.shape != ty.shape:
        raise ValueError("tx and ty differ in length")
    out = np.empty(tx.size, dtype=np.float64)
    rc = lib.oracle_direct_grid(nx, ny, float(x0), float(y0), float(h), _ptr(f), tx.size, _ptr(tx), _ptr(ty),
                                int(self_mode), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_direct_grid rejected its arguments")
    return out


def direct_points(sx, sy, w, tx, ty) -> np.ndarray:
    """P at targets from scattered sources with weights w = f h^2 (coincident sources skipped)."""
    lib = _load()
    sx, sy, w = _f64(sx).ravel(), _f64(sy).ravel(), _f64(w).ravel()
    tx, ty = _f64(tx).ravel(), _f64(ty).ravel()
    if not (sx.size == sy.size == w.size) or tx.size != ty.size:
        raise ValueError("length mismatch")
    out = np.empty(tx.size, dtype=np.float64)
    rc = lib.oracle_direct_points(sx.size, _ptr(sx), _ptr(sy), _ptr(w), tx.size, _ptr(tx), _ptr(ty), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_direct_points rejected its arguments")
    return out

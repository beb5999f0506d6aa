"""ctypes loader for the plain C Jacobi eigensolver (oracle; test use only)."""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        so = _build.SO if os.path.exists(_build.SO) else _build.build()
        lib = ctypes.CDLL(so)
        lib.oracle_jacobi_eigh.restype = ctypes.c_int
        lib.oracle_jacobi_eigh.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        _lib = lib
    return _lib


def jacobi_eigh(h: np.ndarray, rel_tol: float = 1e-15, max_sweeps: int = 60):
    """Eigenpairs of symmetric h by cyclic Jacobi, sorted ascending.
    Returns (w, V) with h ~= V diag(w) V^T."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    a = np.ascontiguousarray(h.copy())
    w = np.empty(n)
    v = np.empty((n, n))
    sweeps = _load().oracle_jacobi_eigh(n, a.ctypes.data, w.ctypes.data, v.ctypes.data,
                                        rel_tol, max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    order = np.argsort(w, kind="stable")
    return w[order], v[:, order]

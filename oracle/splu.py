"""ctypes wrapper of the oracle's C sparse LU (``splu.c``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.splu_factor.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_double, ctypes.POINTER(ctypes.c_void_p),
                                    ctypes.POINTER(ctypes.c_int64)]
        lib.splu_factor.restype = ctypes.c_int
        lib.splu_solve.argtypes = [ctypes.c_void_p, P, P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, P]
        lib.splu_solve.restype = ctypes.c_int
        lib.splu_free.argtypes = [ctypes.c_void_p]
        lib.splu_nnz_l.argtypes = [ctypes.c_void_p]
        lib.splu_nnz_l.restype = ctypes.c_int64
        lib.splu_nnz_u.argtypes = [ctypes.c_void_p]
        lib.splu_nnz_u.restype = ctypes.c_int64
        _lib = lib
    return _lib


class SingularError(RuntimeError):
    pass


class SparseLU:
    """P Q^T A Q = L U by left-looking partial pivoting; solve() refines in FP64.

    tau = 1 is true partial pivoting; tau < 1 keeps the diagonal of Q^T A Q when
    it is within tau of the column maximum (less fill on large systems)."""

    def __init__(self, n, rowptr, colind, values, q=None, tau=1.0):
        lib = _load()
        self.n = int(n)
        self._rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._ci = np.ascontiguousarray(colind, dtype=np.int32)
        self._v = np.ascontiguousarray(values, dtype=np.float64)
        self._q = None if q is None else np.ascontiguousarray(q, dtype=np.int32)
        h = ctypes.c_void_p()
        fail = ctypes.c_int64(-1)
        rc = lib.splu_factor(self.n, self._rp.ctypes.data, self._ci.ctypes.data, self._v.ctypes.data,
                             None if self._q is None else self._q.ctypes.data, float(tau), ctypes.byref(h), ctypes.byref(fail))
        if rc == -4:
            raise SingularError(f"zero pivot column {fail.value}")
        if rc != 0:
            raise RuntimeError(f"splu_factor failed: {rc}")
        self._h = h

    @property
    def nnz_lu(self) -> int:
        lib = _load()
        return int(lib.splu_nnz_l(self._h) + lib.splu_nnz_u(self._h))

    def solve(self, b, tol=1e-14, max_steps=3):
        """Solve A x = b (b: (n,) or (nrhs, n)); returns x, omega per rhs, steps per rhs."""
        lib = _load()
        b = np.asarray(b, dtype=np.float64)
        one = b.ndim == 1
        B = np.ascontiguousarray(b.reshape(1, -1) if one else b)
        nrhs = B.shape[0]
        X = np.zeros_like(B)
        om = np.zeros(nrhs)
        st = np.zeros(nrhs, dtype=np.int32)
        rc = lib.splu_solve(self._h, B.ctypes.data, X.ctypes.data, nrhs, tol, max_steps,
                            om.ctypes.data, st.ctypes.data)
        if rc != 0:
            raise RuntimeError(f"splu_solve failed: {rc}")
        return (X[0] if one else X), om, st

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.splu_free(self._h)
            self._h = None

"""Independent checks that pin the oracle, and the backward-error measures.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper relies on a direct solver to satisfy the constraints "to machine
precision" (Sec. 3.3), which is what the backward-error measures below
quantify:

* componentwise (Oettli-Prager) omega = max_i |b - A x|_i / (|A||x| + |b|)_i
* normwise (Rigal-Gaches) eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.sparse as sp


def csr(n, rowptr, colind, values):
    return sp.csr_matrix((np.asarray(values, dtype=np.float64), np.asarray(colind), np.asarray(rowptr)),
                         shape=(n, n))


def omega(A, x, b):
    """Componentwise backward error, 0/0 counted as 0; exact-sum residual (math.fsum per row)."""
    A = A.tocsr()
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = residual_exact(A, x, b)
    d = abs(A) @ np.abs(x) + np.abs(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(d > 0, np.abs(r) / np.where(d > 0, d, 1.0), np.where(r == 0, 0.0, np.inf))
    return float(w.max()) if w.size else 0.0


def eta(A, x, b):
    """Normwise backward error."""
    A = A.tocsr()
    r = residual_exact(A, x, b)
    nA = float(abs(A).sum(axis=1).max()) if A.shape[0] else 0.0
    den = nA * float(np.abs(x).max(initial=0.0)) + float(np.abs(b).max(initial=0.0))
    return float(np.abs(r).max(initial=0.0)) / den if den > 0 else 0.0


def residual_exact(A, x, b):
    """r = b - A x with each row summed by an error-free method (math.fsum of the
    exact products' two-sum splitting would be overkill: products are rounded once,
    the row sum is exact)."""
    A = A.tocsr()
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    prod = A.data * x[A.indices]
    r = np.empty(A.shape[0])
    ip = A.indptr
    for i in range(A.shape[0]):
        r[i] = math.fsum([b[i], *(-prod[ip[i]:ip[i + 1]])])
    return r


def residual(A, x, b):
    """Fast FP64 residual (ordinary summation), for large systems."""
    return np.asarray(b, dtype=np.float64) - A.tocsr() @ np.asarray(x, dtype=np.float64)


def omega_fast(A, x, b):
    A = A.tocsr()
    r = residual(A, x, b)
    d = abs(A) @ np.abs(x) + np.abs(b)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(d > 0, np.abs(r) / np.where(d > 0, d, 1.0), np.where(r == 0, 0.0, np.inf))
    return float(w.max()) if w.size else 0.0


def dense_gepp_solve(A, b):
    """Dense LU with partial pivoting (LAPACK gesv through numpy)."""
    return np.linalg.solve(np.asarray(A.todense() if sp.issparse(A) else A, dtype=np.float64), b)


def fraction_solve(A_int, b_int):
    """Exact solution of A x = b by Gaussian elimination over the rationals."""
    n = len(A_int)
    M = [[Fraction(int(v)) for v in row] + [Fraction(int(bv))] for row, bv in zip(A_int, b_int)]
    for k in range(n):
        p = next((i for i in range(k, n) if M[i][k] != 0), None)
        if p is None:
            raise ZeroDivisionError("singular")
        M[k], M[p] = M[p], M[k]
        for i in range(k + 1, n):
            if M[i][k] != 0:
                f = M[i][k] / M[k][k]
                M[i] = [a - f * c for a, c in zip(M[i], M[k])]
    x = [Fraction(0)] * n
    for k in range(n - 1, -1, -1):
        s = M[k][n] - sum(M[k][j] * x[j] for j in range(k + 1, n))
        x[k] = s / M[k][k]
    return x

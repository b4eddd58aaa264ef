"""Binding of the ALE Newton assembly (include/ale.h): argument marshalling only.

``Assembly(problem)`` uploads a problem description (anything with the fields
of ``vivjac.ale2d.AleProblem``) once; ``residual(U)`` and ``jacobian(U)``
evaluate NL(U) and J(U) on the GPU.  ``newton`` runs the paper's Newton-Raphson
iteration (Sec. 3.4, eq. NR_iteration) with every step on the device: assembly
here, factorization and solve in libmf.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import MF_OK, MFError, Symbolic, _check, _stream_ptr, check_vectors, lib

P = ctypes.c_void_p


class ale_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnodes", ctypes.c_int32), ("nvert", ctypes.c_int32),
                ("nelem", ctypes.c_int32), ("nedge", ctypes.c_int32),
                ("tri", P), ("vtx", P), ("gedge", P), ("gvtx", P), ("u_dof", P), ("p_dof", P), ("x_dof", P),
                ("lam_dof", P), ("s_dof", P), ("gamma_vertex", P), ("u_bc", P), ("u_prev", P), ("x_ref", P),
                ("x_prev", P), ("lam_s", P), ("nu", ctypes.c_double), ("dt", ctypes.c_double),
                ("k", ctypes.c_double), ("rowptr", P), ("colind", P)]


def _bind():
    L = lib()
    if not getattr(L, "_ale_bound", False):
        L.ale_create.argtypes = [ctypes.POINTER(ale_desc), ctypes.POINTER(ctypes.c_void_p)]
        L.ale_create.restype = ctypes.c_int
        L.ale_residual.argtypes = [ctypes.c_void_p, P, P, P]
        L.ale_residual.restype = ctypes.c_int
        L.ale_jacobian.argtypes = [ctypes.c_void_p, P, P, P, P]
        L.ale_jacobian.restype = ctypes.c_int
        L.ale_device_bytes.argtypes = [ctypes.c_void_p]
        L.ale_device_bytes.restype = ctypes.c_int64
        L.ale_release.argtypes = [ctypes.c_void_p]
        L.ale_release.restype = None
        L._ale_bound = True
    return L


class Assembly:
    def __init__(self, prob):
        L = _bind()
        self.n, self.nnz = int(prob.n), int(prob.rowptr[-1])
        keep = {
            "tri": np.ascontiguousarray(prob.tri, dtype=np.int32),
            "vtx": np.ascontiguousarray(prob.vtx, dtype=np.int32),
            "gedge": np.ascontiguousarray(prob.gedge, dtype=np.int32),
            "gvtx": np.ascontiguousarray(prob.gvtx, dtype=np.int32),
            "u_dof": np.ascontiguousarray(prob.u_dof, dtype=np.int64),
            "p_dof": np.ascontiguousarray(prob.p_dof, dtype=np.int64),
            "x_dof": np.ascontiguousarray(prob.x_dof, dtype=np.int64),
            "lam_dof": np.ascontiguousarray(prob.lam_dof, dtype=np.int64),
            "s_dof": np.ascontiguousarray(prob.s_dof, dtype=np.int64),
            "gamma_vertex": np.ascontiguousarray(prob.gamma_vertex, dtype=np.uint8),
            "u_bc": np.ascontiguousarray(prob.u_bc, dtype=np.float64),
            "u_prev": np.ascontiguousarray(prob.u_prev, dtype=np.float64),
            "x_ref": np.ascontiguousarray(prob.vX, dtype=np.float64),
            "x_prev": np.ascontiguousarray(prob.x_prev, dtype=np.float64),
            "lam_s": np.ascontiguousarray(prob.lam_s, dtype=np.float64),
            "rowptr": np.ascontiguousarray(prob.rowptr, dtype=np.int64),
            "colind": np.ascontiguousarray(prob.colind, dtype=np.int32),
        }
        d = ale_desc(n=self.n, nnodes=int(prob.u_dof.shape[0]), nvert=int(prob.vX.shape[0]),
                     nelem=int(prob.tri.shape[0]), nedge=int(prob.gedge.shape[0]),
                     nu=float(prob.nu), dt=float(prob.dt), k=float(prob.k),
                     **{k: v.ctypes.data for k, v in keep.items()})
        h = ctypes.c_void_p()
        _check(L.ale_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    @property
    def device_bytes(self) -> int:
        return int(_bind().ale_device_bytes(self._h))

    def residual(self, U, R=None, stream=None):
        import torch
        check_vectors(U, self.n, "U", nrhs=1)
        if R is None:
            R = torch.empty_like(U)
        else:
            check_vectors(R, self.n, "R", nrhs=1)
        _check(_bind().ale_residual(self._h, P(U.data_ptr()), P(R.data_ptr()), _stream_ptr(stream)))
        return R

    def jacobian(self, U, values=None, R=None, stream=None):
        """J(U) in the pattern's CSR order (and NL(U) into R when given)."""
        import torch
        check_vectors(U, self.n, "U", nrhs=1)
        if values is None:
            values = torch.empty(self.nnz, dtype=torch.float64, device=U.device)
        elif not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == torch.float64
                  and values.is_contiguous() and values.numel() == self.nnz):
            raise TypeError("values must be a contiguous float64 CUDA tensor with nnz entries")
        if R is not None:
            check_vectors(R, self.n, "R", nrhs=1)
        _check(_bind().ale_jacobian(self._h, P(U.data_ptr()), P(values.data_ptr()),
                                    P(R.data_ptr()) if R is not None else None, _stream_ptr(stream)))
        return values

    def release(self):
        if getattr(self, "_h", None):
            _bind().ale_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def newton(prob, U0=None, iters=8, tol=1e-10, prec="fp64", target_omega=1e-12, stream=None, assembly=None,
           symbolic=None):
    """Newton-Raphson on NL(U) = 0 with every step on the GPU: assemble J(U_m)
    and NL(U_m), factor J (analysis once, reused), solve J dU = -NL, update.
    Stops when max |NL| <= tol.  Every call runs on ``stream`` (torch's current
    stream by default).  Returns (U, [max |NL| per iterate], [solve info])."""
    import torch
    if stream is not None:
        with torch.cuda.stream(stream):
            return newton(prob, U0, iters, tol, prec, target_omega, None, assembly, symbolic)
    dev = torch.device("cuda:0")
    A = assembly or Assembly(prob)
    S = symbolic or Symbolic(prob.n, prob.rowptr, prob.colind, prob.root)
    U = torch.from_numpy(np.asarray(prob.initial_guess() if U0 is None else U0, dtype=np.float64)).to(dev)
    vals = torch.empty(A.nnz, dtype=torch.float64, device=dev)
    R = torch.empty_like(U)
    dU = torch.empty_like(U)
    num = None
    norms, infos = [], []
    for m in range(iters + 1):
        A.jacobian(U, values=vals, R=R, stream=stream)
        norms.append(float(R.abs().max()))
        if norms[-1] <= tol or m == iters:
            break
        num = S.factor(vals, numeric=num, stream=stream, prec=prec, target_omega=target_omega)
        R.neg_()
        _, info = num.solve(R, x=dU, stream=stream)
        infos.append(info)
        U.add_(dU)
    if num is not None:
        num.release()
    if assembly is None:
        A.release()
    return U, norms, infos


__all__ = ["Assembly", "newton", "ale_desc", "MF_OK", "MFError"]

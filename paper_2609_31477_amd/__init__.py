"""Python binding of libmf, the MI355X multifrontal solver for the coupled VIV Newton Jacobian.

Argument marshalling only: every step of analysis, factorization and solve runs
inside libmf.so (host C++ symbolic phase, gfx950 HIP kernels).  PyTorch provides
device memory and the stream.  There is no fallback: if the library is not
built, importing the binding's solver classes raises.

    sym = Symbolic(n, rowptr, colind, root, leaf_max=64)       # mf_analyze
    num = sym.factor(values_tensor_on_cuda)                     # mf_factor
    x, info = num.solve(b_tensor_on_cuda)                       # mf_solve
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmf.so")

MF_OK, MF_ERR_ARG, MF_ERR_PATTERN, MF_ERR_OOM, MF_ERR_SINGULAR, MF_ERR_DEVICE, MF_ERR_NOT_CONVERGED, MF_ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
MF_FP64, MF_FP32, MF_BF16 = 0, 1, 2
PRECISIONS = {"fp64": MF_FP64, "fp32": MF_FP32, "bf16": MF_BF16}

# every entry point declared in include/mf.h
EXPORTS = ["mf_default_options", "mf_analyze", "mf_symbolic_export", "mf_factor", "mf_get_factor_info",
           "mf_solve", "mf_batch_analyze", "mf_factor_batched", "mf_solve_batched", "mf_footprint_bytes",
           "mf_debug_front", "mf_release", "mf_last_error", "mf_solve_noalloc", "mf_set_operator",
           "mf_set_operator_batched"]


class mf_options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("pivot_u", ctypes.c_double), ("leaf_max", ctypes.c_int32),
                ("target_omega", ctypes.c_double), ("max_outer", ctypes.c_int32), ("gmres_m", ctypes.c_int32),
                ("gmres_tol", ctypes.c_double), ("refine", ctypes.c_int32), ("panel_nb", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("scale", ctypes.c_int32), ("plan", ctypes.c_int32),
                ("tune", ctypes.c_int32), ("fallback", ctypes.c_int32), ("sweep", ctypes.c_int32)]


class mf_symbolic_view(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nfronts", ctypes.c_int32), ("leaf_max", ctypes.c_int32),
                ("spec_version", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("perm", ctypes.POINTER(ctypes.c_int32)), ("front_ptr", ctypes.POINTER(ctypes.c_int32)),
                ("front_parent", ctypes.POINTER(ctypes.c_int32)), ("rows_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("rows", ctypes.POINTER(ctypes.c_int32)), ("var_etree", ctypes.POINTER(ctypes.c_int32)),
                ("nominal_flops", ctypes.c_double), ("nominal_nnz_lu", ctypes.c_double)]


class mf_factor_info(ctypes.Structure):
    _fields_ = [("delayed_pivots", ctypes.c_int64), ("max_front", ctypes.c_int32), ("root_order", ctypes.c_int32),
                ("factor_flops", ctypes.c_double), ("actual_flops", ctypes.c_double),
                ("factor_bytes", ctypes.c_int64), ("t_assemble_ms", ctypes.c_double),
                ("t_panel_ms", ctypes.c_double), ("t_schur_ms", ctypes.c_double), ("t_finalize_ms", ctypes.c_double),
                ("schur_flops", ctypes.c_double), ("schur_launches", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("t_panel_kernel_ms", ctypes.c_double), ("panel_flops", ctypes.c_double),
                ("panel_launches", ctypes.c_int32), ("planned", ctypes.c_int32),
                ("plan_fallbacks", ctypes.c_int32), ("tuned", ctypes.c_int32)]


class mf_solve_info(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("omega0", ctypes.c_double), ("outer_iters", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("eta", ctypes.c_double), ("delayed_pivots", ctypes.c_int64),
                ("fp64_fallback", ctypes.c_int32)]


class MFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mf status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libmf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.mf_default_options.argtypes = [ctypes.POINTER(mf_options)]
        L.mf_default_options.restype = None
        L.mf_analyze.argtypes = [ctypes.c_int64, P, P, ctypes.c_int32, P, ctypes.POINTER(mf_options),
                                 ctypes.POINTER(ctypes.c_void_p)]
        L.mf_analyze.restype = ctypes.c_int
        L.mf_symbolic_export.argtypes = [ctypes.c_void_p, ctypes.POINTER(mf_symbolic_view)]
        L.mf_symbolic_export.restype = ctypes.c_int
        L.mf_factor.argtypes = [ctypes.c_void_p, P, ctypes.POINTER(mf_options), P, ctypes.POINTER(ctypes.c_void_p)]
        L.mf_factor.restype = ctypes.c_int
        L.mf_get_factor_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(mf_factor_info)]
        L.mf_get_factor_info.restype = ctypes.c_int
        L.mf_solve.argtypes = [ctypes.c_void_p, P, P, ctypes.c_int32, ctypes.c_int64, P,
                               ctypes.POINTER(mf_solve_info)]
        L.mf_solve.restype = ctypes.c_int
        L.mf_solve_noalloc.argtypes = [ctypes.c_void_p, P, P, ctypes.c_int32, ctypes.c_int64, P,
                                       ctypes.POINTER(mf_solve_info)]
        L.mf_solve_noalloc.restype = ctypes.c_int
        L.mf_set_operator.argtypes = [ctypes.c_void_p, P, ctypes.POINTER(mf_options), P]
        L.mf_set_operator.restype = ctypes.c_int
        L.mf_set_operator_batched.argtypes = [ctypes.c_void_p, P, ctypes.POINTER(mf_options), P]
        L.mf_set_operator_batched.restype = ctypes.c_int
        L.mf_footprint_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(mf_options), ctypes.c_double]
        L.mf_footprint_bytes.restype = ctypes.c_int64
        L.mf_batch_analyze.argtypes = [ctypes.c_int32, P, ctypes.POINTER(ctypes.c_void_p)]
        L.mf_batch_analyze.restype = ctypes.c_int
        L.mf_factor_batched.argtypes = [ctypes.c_void_p, P, ctypes.POINTER(mf_options), P,
                                        ctypes.POINTER(ctypes.c_void_p)]
        L.mf_factor_batched.restype = ctypes.c_int
        L.mf_solve_batched.argtypes = [ctypes.c_void_p, P, P, P, P, ctypes.POINTER(mf_solve_info)]
        L.mf_solve_batched.restype = ctypes.c_int
        L.mf_debug_front.argtypes = [ctypes.c_void_p, ctypes.c_int32, P, P, P]
        L.mf_debug_front.restype = ctypes.c_int
        L.mf_release.argtypes = [ctypes.c_void_p]
        L.mf_release.restype = None
        L.mf_last_error.argtypes = []
        L.mf_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(st):
    if st != MF_OK:
        raise MFError(st, lib().mf_last_error().decode())


def default_options(**kw) -> mf_options:
    o = mf_options()
    lib().mf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(o, k, v)
    return o


def check_vectors(t, n, name, nrhs=None, require_cuda=True):
    """Validate a right-hand-side or solution tensor before its pointer crosses the
    ABI (the library cannot check device buffer sizes): float64, contiguous, on
    the GPU, shaped (n,) or (nrhs, n).  Returns its number of columns."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if require_cuda and not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if t.dim() not in (1, 2) or t.shape[-1] != n:
        raise ValueError(f"{name} must have shape ({n},) or (nrhs, {n}), got {tuple(t.shape)}")
    cols = 1 if t.dim() == 1 else int(t.shape[0])
    if nrhs is not None and cols != nrhs:
        raise ValueError(f"{name} has {cols} columns, expected {nrhs}")
    return cols


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


@dataclass
class SymbolicView:
    n: int
    nfronts: int
    nlevels: int
    leaf_max: int
    spec_version: int
    perm: np.ndarray
    front_ptr: np.ndarray
    front_parent: np.ndarray
    rows_ptr: np.ndarray
    rows: np.ndarray
    var_etree: np.ndarray
    nominal_flops: float
    nominal_nnz_lu: float


class Symbolic:
    """mf_analyze: the specified nested-dissection analysis of one sparsity pattern."""

    def __init__(self, n, rowptr, colind, root=(), leaf_max=64, **opts):
        L = lib()
        self.n = int(n)
        rp = np.ascontiguousarray(rowptr, dtype=np.int64)
        ci = np.ascontiguousarray(colind, dtype=np.int32)
        rt = np.ascontiguousarray(np.asarray(root, dtype=np.int32).ravel())
        self.nnz = int(rp[-1]) if rp.size else 0
        self.options = default_options(leaf_max=leaf_max, **opts)
        h = ctypes.c_void_p()
        st = L.mf_analyze(self.n, rp.ctypes.data, ci.ctypes.data, int(rt.size),
                          rt.ctypes.data if rt.size else None, ctypes.byref(self.options), ctypes.byref(h))
        _check(st)
        self._h = h

    def export(self) -> SymbolicView:
        v = mf_symbolic_view()
        _check(lib().mf_symbolic_export(self._h, ctypes.byref(v)))
        nf = v.nfronts

        def arr(p, cnt, dt):
            if cnt == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(p, shape=(cnt,)).astype(dt, copy=True)

        rows_ptr = arr(v.rows_ptr, nf + 1, np.int64) if nf else np.zeros(1, np.int64)
        return SymbolicView(n=v.n, nfronts=nf, nlevels=v.nlevels, leaf_max=v.leaf_max, spec_version=v.spec_version,
                            perm=arr(v.perm, v.n, np.int32),
                            front_ptr=arr(v.front_ptr, nf + 1, np.int32) if nf else np.zeros(1, np.int32),
                            front_parent=arr(v.front_parent, nf, np.int32), rows_ptr=rows_ptr,
                            rows=arr(v.rows, int(rows_ptr[-1]), np.int32), var_etree=arr(v.var_etree, v.n, np.int32),
                            nominal_flops=v.nominal_flops, nominal_nnz_lu=v.nominal_nnz_lu)

    def footprint_bytes(self, prec="fp64", margin=0.5) -> int:
        o = default_options(prec=prec)
        return int(lib().mf_footprint_bytes(self._h, ctypes.byref(o), float(margin)))

    def factor(self, values, numeric=None, stream=None, **opts):
        """values: torch float64 tensor on the GPU (nnz entries in CSR order)."""
        return Numeric.factor(self, values, numeric=numeric, stream=stream, **opts)

    def release(self):
        if getattr(self, "_h", None):
            lib().mf_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Numeric:
    """mf_factor / mf_solve on one symbolic handle (factors stay on the device)."""

    def __init__(self, sym):
        self.sym = sym
        self._h = ctypes.c_void_p()

    @classmethod
    def factor(cls, sym, values, numeric=None, stream=None, **opts):
        import torch
        if not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == torch.float64):
            raise TypeError("values must be a float64 CUDA tensor")
        if values.numel() != sym.nnz or not values.is_contiguous():
            raise ValueError("values must be contiguous with nnz entries")
        num = numeric if numeric is not None else cls(sym)
        num._opts = dict(opts)
        o = default_options(leaf_max=sym.options.leaf_max, **opts) if opts else None
        st = lib().mf_factor(sym._h, ctypes.c_void_p(values.data_ptr()), ctypes.byref(o) if o is not None else None,
                             _stream_ptr(stream), ctypes.byref(num._h))
        _check(st)
        return num

    def info(self) -> mf_factor_info:
        inf = mf_factor_info()
        _check(lib().mf_get_factor_info(self._h, ctypes.byref(inf)))
        return inf

    def set_operator(self, values, stream=None, **refine_opts):
        """mf_set_operator: later solves use these values (same pattern) as the
        operator and the current factors as the preconditioner; refine_opts
        (target_omega, max_outer, gmres_m, gmres_tol, fallback, refine) replace the
        factorization's refinement settings for those solves."""
        import torch
        if not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == torch.float64):
            raise TypeError("values must be a float64 CUDA tensor")
        if values.numel() != self.sym.nnz or not values.is_contiguous():
            raise ValueError("values must be contiguous with nnz entries")
        o = self._refine_options(refine_opts, getattr(self, "_opts", {}))
        _check(lib().mf_set_operator(self._h, ctypes.c_void_p(values.data_ptr()),
                                     ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))
        return self

    _REFINE_KEYS = ("target_omega", "max_outer", "gmres_m", "gmres_tol", "fallback", "refine")

    @staticmethod
    def _refine_options(kw, factor_opts):
        """The refinement fields of an mf_options for mf_set_operator: the given
        ones, the rest as the last factorization set them (or the defaults)."""
        bad = set(kw) - set(Numeric._REFINE_KEYS)
        if bad:
            raise TypeError(f"set_operator takes only refinement options, not {sorted(bad)}")
        if not kw:
            return None
        full = {k: factor_opts[k] for k in Numeric._REFINE_KEYS if k in factor_opts}
        full.update(kw)
        full.setdefault("refine", -1)
        return default_options(**full)

    def solve(self, b, x=None, stream=None, check=True):
        """b: float64 CUDA tensor (n,) or (nrhs, n) -- row r is right-hand side r
        (i.e. column-major n x nrhs with ld = n).  Returns (x, mf_solve_info)."""
        import torch
        n = self.sym.n
        nrhs = check_vectors(b, n, "b")
        if x is None:
            x = torch.empty_like(b)
        else:
            check_vectors(x, n, "x", nrhs=nrhs)
            if x.shape != b.shape:
                raise ValueError("x must have the shape of b")
            if x.numel() > 0 and x.data_ptr() == b.data_ptr():
                raise ValueError("x and b must be distinct buffers")
        inf = mf_solve_info()
        st = lib().mf_solve(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs, n,
                            _stream_ptr(stream), ctypes.byref(inf))
        if check or st != MF_ERR_NOT_CONVERGED:
            _check(st)
        return x, inf

    def solve_noalloc(self, b, x, stream=None, check=True):
        """mf_solve_noalloc: as solve(), into a caller-provided x, with the library's
        static scratch instead of any allocation."""
        n = self.sym.n
        nrhs = check_vectors(b, n, "b")
        check_vectors(x, n, "x", nrhs=nrhs)
        if x.shape != b.shape:
            raise ValueError("x must have the shape of b")
        if x.numel() > 0 and x.data_ptr() == b.data_ptr():
            raise ValueError("x and b must be distinct buffers")
        inf = mf_solve_info()
        st = lib().mf_solve_noalloc(self._h, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs, n,
                                    _stream_ptr(stream), ctypes.byref(inf))
        if check or st != MF_ERR_NOT_CONVERGED:
            _check(st)
        return x, inf

    def debug_front(self, front):
        """(meta dict, F (m x m, column-major as a numpy array F[i, j]), iv dict) of one front."""
        meta = np.zeros(8, dtype=np.int32)
        _check(lib().mf_debug_front(self._h, int(front), meta.ctypes.data, None, None))
        m, P = int(meta[0]), int(meta[1])
        F = np.zeros(m * m, dtype=np.float64)
        iv = np.zeros(3 * P + m, dtype=np.int32)
        _check(lib().mf_debug_front(self._h, int(front), meta.ctypes.data, F.ctypes.data, iv.ctypes.data))
        keys = ["m", "P", "din", "k", "npiv", "mnom", "prec", "slot"]
        return (dict(zip(keys, meta.tolist())), F.reshape(m, m).T.copy(),
                dict(rowpiv=iv[:P], colperm=iv[P:2 * P], rowperm=iv[2 * P:3 * P], colvar=iv[3 * P:]))

    def release(self):
        if getattr(self, "_h", None):
            lib().mf_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Batch:
    """mf_batch_analyze / mf_factor_batched / mf_solve_batched over several analyzed systems."""

    def __init__(self, syms):
        L = lib()
        self.syms = list(syms)
        self.ns = [s.n for s in self.syms]
        self.nnzs = [s.nnz for s in self.syms]
        arr = (ctypes.c_void_p * len(self.syms))(*[s._h.value for s in self.syms])
        h = ctypes.c_void_p()
        _check(L.mf_batch_analyze(len(self.syms), ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(h)))
        self._h = h
        self._num = ctypes.c_void_p()
        self.n = sum(self.ns)
        self.nnz = sum(self.nnzs)

    def export(self) -> SymbolicView:
        return Symbolic.export(self)

    def factor(self, values, stream=None, **opts):
        """values: list of float64 CUDA tensors, one per system."""
        import torch
        if len(values) != len(self.syms):
            raise ValueError("one values tensor per system")
        for v, nz in zip(values, self.nnzs):
            if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
                    and v.numel() == nz):
                raise TypeError("values[i] must be a contiguous float64 CUDA tensor with nnz_i entries")
        ptrs = (ctypes.c_void_p * len(values))(*[v.data_ptr() for v in values])
        self._opts = dict(opts)
        o = default_options(leaf_max=self.syms[0].options.leaf_max, **opts) if opts else None
        _check(lib().mf_factor_batched(self._h, ctypes.cast(ptrs, ctypes.c_void_p),
                                       ctypes.byref(o) if o is not None else None, _stream_ptr(stream),
                                       ctypes.byref(self._num)))
        return self

    def info(self) -> mf_factor_info:
        inf = mf_factor_info()
        _check(lib().mf_get_factor_info(self._num, ctypes.byref(inf)))
        return inf

    def set_operator(self, values, stream=None, **refine_opts):
        """mf_set_operator_batched: one float64 CUDA tensor per system (nnz_i entries)."""
        import torch
        if len(values) != len(self.syms):
            raise ValueError("one values tensor per system")
        for v, nz in zip(values, self.nnzs):
            if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
                    and v.numel() == nz):
                raise TypeError("values[i] must be a contiguous float64 CUDA tensor with nnz_i entries")
        ptrs = (ctypes.c_void_p * len(values))(*[v.data_ptr() for v in values])
        o = Numeric._refine_options(refine_opts, getattr(self, "_opts", {}))
        _check(lib().mf_set_operator_batched(self._num, ctypes.cast(ptrs, ctypes.c_void_p),
                                             ctypes.byref(o) if o is not None else None, _stream_ptr(stream)))
        return self

    def solve(self, bs, xs=None, stream=None, check=True):
        """bs: list of float64 CUDA tensors, system i's shaped (n_i,) or (nrhs_i, n_i);
        the systems may have different numbers of right-hand sides.  Returns
        (xs, [mf_solve_info])."""
        import torch
        if len(bs) != len(self.syms):
            raise ValueError("one right-hand-side tensor per system")
        nrhs = [check_vectors(b, n, f"bs[{i}]") for i, (b, n) in enumerate(zip(bs, self.ns))]
        if xs is None:
            xs = [torch.empty_like(b) for b in bs]
        else:
            if len(xs) != len(bs):
                raise ValueError("one solution tensor per system")
            for i, (x, b, n, k) in enumerate(zip(xs, bs, self.ns, nrhs)):
                check_vectors(x, n, f"xs[{i}]", nrhs=k)
                if x.shape != b.shape:
                    raise ValueError(f"xs[{i}] must have the shape of bs[{i}]")
                if x.numel() > 0 and x.data_ptr() == b.data_ptr():
                    raise ValueError(f"xs[{i}] and bs[{i}] must be distinct buffers")
        bp = (ctypes.c_void_p * len(bs))(*[b.data_ptr() for b in bs])
        xp = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        nr = (ctypes.c_int32 * len(bs))(*nrhs)
        infos = (mf_solve_info * len(bs))()
        st = lib().mf_solve_batched(self._num, ctypes.cast(bp, ctypes.c_void_p), ctypes.cast(xp, ctypes.c_void_p),
                                    ctypes.cast(nr, ctypes.c_void_p), _stream_ptr(stream), infos)
        if check or st != MF_ERR_NOT_CONVERGED:
            _check(st)
        return xs, list(infos)

    def release(self):
        if getattr(self, "_num", None) and self._num.value:
            lib().mf_release(self._num)
            self._num = ctypes.c_void_p()
        if getattr(self, "_h", None):
            lib().mf_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

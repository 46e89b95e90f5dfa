"""Python binding of libofm (ctypes; argument marshalling only).

Every computation runs in the HIP library.  Tensors are torch CUDA (ROCm)
tensors; pointers and the current stream are handed to the C ABI declared in
include/ofm.h.  If the compiled library is missing this module raises: there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libofm.so")

OFM_F1, OFM_TRI_F1, OFM_F2, OFM_TRI_F2 = 0, 1, 2, 3
OFM_FP64, OFM_FP32, OFM_FP32_BF16X = 0, 1, 2
OFM_LAP_VALIDATE = 1
OFM_LAP_NO_REORDER = 2
OFM_LAP_NO_UPPER = 4

STATUS = {
    0: "OFM_OK", -1: "OFM_E_INVALID_ARG", -2: "OFM_E_SHAPE", -3: "OFM_E_GRAPH",
    -4: "OFM_E_NONFINITE", -5: "OFM_E_NUMERIC", -6: "OFM_E_HIP", -7: "OFM_E_NOMEM",
    -8: "OFM_E_UNSUPPORTED", -9: "OFM_E_NO_ROOT",
}

VARIANTS = {"f1": OFM_F1, "tri-f1": OFM_TRI_F1, "f2": OFM_F2, "tri-f2": OFM_TRI_F2}


class OfmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


# ofm_opts.gather
GATHER_AUTO, GATHER_DEFAULT, GATHER_HOT_COLD = 0, 1, 2


class Opts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("first_step", ctypes.c_int),
        ("restart", ctypes.c_int),
        ("alpha0", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("graph", ctypes.c_int),
        ("recur", ctypes.c_int),
        ("gather", ctypes.c_int),
        ("freeze_eps", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("relres", ctypes.c_double),
        ("objective", ctypes.c_double),
        ("relres_iter", ctypes.c_int64),
        ("gather", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double

_SIGS = {
    "ofm_status_string": (ctypes.c_char_p, [_I]),
    "ofm_version": (ctypes.c_char_p, []),
    "ofm_build_laplacian": (_I, [_I64, _I64, _P, _P, _P, _I, ctypes.c_uint, _P,
                                 ctypes.POINTER(_P)]),
    "ofm_build_laplacian_grouped": (_I, [_I64, _I64, _P, _P, _P, _I, ctypes.c_uint, _P, _P,
                                         ctypes.POINTER(_P)]),
    "ofm_select_roots": (_I, [_I, _I64, _P, _P, _P, _P]),
    "ofm_gather_rows": (_I, [_I64, _I, _I, _P, _P, _I64, _P, _P]),
    "ofm_grouped_order": (_I, [_I64, _P, _P, _P, _P]),
    "ofm_laplacian_destroy": (_I, [_P]),
    "ofm_laplacian_info": (_I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                ctypes.POINTER(_D), _P]),
    "ofm_laplacian_upper": (_I, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "ofm_apply_A": (_I, [_P, _I, _I, _P, _P, _P]),
    "ofm_workspace_create": (_I, [_P, _I, ctypes.POINTER(Opts), ctypes.POINTER(_P)]),
    "ofm_workspace_destroy": (_I, [_P]),
    "ofm_init": (_I, [_P, _P, _P]),
    "ofm_step": (_I, [_P, _P, _P]),
    "ofm_solve": (_I, [_P, _P, _P, ctypes.POINTER(Stats)]),
    "ofm_residual": (_I, [_P, _P, _P, ctypes.POINTER(Stats)]),
    "ofm_get_stats": (_I, [_P, _P, ctypes.POINTER(Stats)]),
    "ofm_get_state": (_I, [_P, _P, _P, _P]),
    "ofm_set_state": (_I, [_P, _P, _P, _P, _I64, _P]),
    "ofm_get_step_info": (_I, [_P, _P, _P, _P, _P, _P]),
    "ofm_get_products": (_I, [_P, _I, _P, _P]),
    "ofm_objective": (_I, [_P, _P, _P, _P, _P]),
    "ofm_set_timing": (_I, [_P, ctypes.c_uint]),
    "ofm_get_timing": (_I, [_P, _P, _P, _I]),
    "ofm_batch_create": (_I, [_I, _P, _P, ctypes.POINTER(Opts), ctypes.POINTER(_P)]),
    "ofm_batch_destroy": (_I, [_P]),
    "ofm_batch_solve": (_I, [_P, _P, _P, _P]),
    "ofm_batch_schedule": (_I, [_P, _I, _P, _P, _P, _P, _P, _P]),
    "ofm_batch_phases": (_I, [_P, _P, _P, _P]),
    "ofm_batch_init": (_I, [_P, _P, _P]),
    "ofm_batch_set_schedule": (_I, [_P, _I, _I]),
    "ofm_batch_set_persistent": (_I, [_P, _I]),
    "ofm_batch_persist_info": (_I, [_P, _P, _P]),
    "ofm_batch_step": (_I, [_P, _P]),
    "ofm_batch_get_state": (_I, [_P, _I, _P, _P, _P]),
    "ofm_batch_get_step_info": (_I, [_P, _I, _P, _P, _P, _P, _P]),
    "ofm_scale": (_I, [_I64, _I, _P, _P, _P, _P]),
    "ofm_row_normalize": (_I, [_I64, _I, _I, _P, _P, _P]),
    "ofm_kmeans_assign": (_I, [_I64, _I, _I, _P, _P, _P, _P, _P]),
    "ofm_kmeans": (_I, [_I64, _I, _I, _P, _P, _I, _P, _P, _P, _P]),
    "ofm_kmeans_noalloc": (_I, [_I64, _I, _I, _P, _P, _I, _P, _P, _P, _P]),
    "ofm_kmeans_static_bytes": (ctypes.c_size_t, [_I64, _I, _I]),
}


def load(path: str = LIB_PATH):
    """Load libofm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libofm.so not built at {path}; run paper_2305_10356_amd.build.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        raise OfmError(status, where)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _prec(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return OFM_FP64
    if t.dtype == torch.float32:
        return OFM_FP32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev_block(t, k: Optional[int] = None):
    torch = _torch()
    if not (t.is_cuda and t.dim() == 2 and t.is_contiguous()):
        raise ValueError("expected a contiguous 2-D device tensor")
    if t.dtype not in (torch.float32, torch.float64):
        raise TypeError("expected float32 or float64")
    if k is not None and t.shape[1] != k:
        raise ValueError(f"expected {k} columns")
    return t


class Laplacian:
    """Handle of the shifted normalized Laplacian A = L - 2I of a graph."""

    def __init__(self, row_ptr, col_idx, vals=None, validate: bool = False,
                 reorder: bool = True, groups=None, stream=None, upper: bool = True):
        """``vals``: optional edge weights, FP64 or FP32 (a tensor keeps its
        dtype; anything else is taken as FP64).  ``groups``: optional
        int32[n] (a host array or a tensor, e.g. the cluster labels of an
        earlier solve; negative = none) that lays the row-processing order out
        for the XCDs (``ofm_build_laplacian_grouped``).  ``upper=False``
        builds no upper-triangle copy (``OFM_LAP_NO_UPPER``): the f1 line
        searches then take diag(V^T A V) from the full product A V."""
        torch = _torch()
        lib = load()
        self._lib = lib
        rp = torch.as_tensor(row_ptr, dtype=torch.int32).contiguous().cuda()
        ci = torch.as_tensor(col_idx, dtype=torch.int32).contiguous().cuda()
        vv, vdt = None, OFM_FP64
        if vals is not None:
            if hasattr(vals, "dtype") and vals.dtype in (torch.float32, np.float32):
                vv, vdt = torch.as_tensor(vals, dtype=torch.float32).contiguous().cuda(), OFM_FP32
            else:
                vv = torch.as_tensor(vals, dtype=torch.float64).contiguous().cuda()
        n = rp.numel() - 1
        flags = ((OFM_LAP_VALIDATE if validate else 0) | (0 if reorder else OFM_LAP_NO_REORDER)
                 | (0 if upper else OFM_LAP_NO_UPPER))
        h = ctypes.c_void_p()
        if groups is None:
            st = lib.ofm_build_laplacian(n, ci.numel(), _ptr(rp), _ptr(ci) if ci.numel() else None,
                                         _ptr(vv) if vv is not None else None, vdt, flags,
                                         _stream(stream), ctypes.byref(h))
            _check(st, "ofm_build_laplacian")
        else:
            if hasattr(groups, "detach"):  # a torch tensor, possibly on the device
                groups = groups.detach().cpu().numpy()
            gr = np.ascontiguousarray(np.asarray(groups), dtype=np.int32)
            if gr.shape != (n,):
                raise ValueError("groups must hold one entry per node")
            st = lib.ofm_build_laplacian_grouped(
                n, ci.numel(), _ptr(rp), _ptr(ci) if ci.numel() else None,
                _ptr(vv) if vv is not None else None, vdt, flags,
                gr.ctypes.data_as(ctypes.c_void_p),
                _stream(stream), ctypes.byref(h))
            _check(st, "ofm_build_laplacian_grouped")
        self.grouped = groups is not None
        self.handle = h
        self.n = n
        self.nnz = ci.numel()

    def info(self):
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        na = ctypes.c_double()
        deg = np.zeros(self.n, dtype=np.float64)
        _check(self._lib.ofm_laplacian_info(self.handle, ctypes.byref(n), ctypes.byref(nnz),
                                            ctypes.byref(na), deg.ctypes.data_as(ctypes.c_void_p)),
               "ofm_laplacian_info")
        return {"n": n.value, "nnz": nnz.value, "normA2": na.value, "degrees": deg}

    def upper(self):
        """(rows, entries) of the upper-triangle copy; (0, 0) when none."""
        r = ctypes.c_int64()
        e = ctypes.c_int64()
        _check(self._lib.ofm_laplacian_upper(self.handle, ctypes.byref(r), ctypes.byref(e)),
               "ofm_laplacian_upper")
        return r.value, e.value

    def apply(self, Z, Y=None, stream=None):
        """Y = A Z (same dtype as Z)."""
        torch = _torch()
        _dev_block(Z)
        if Y is None:
            Y = torch.empty_like(Z)
        _check(self._lib.ofm_apply_A(self.handle, Z.shape[1], _prec(Z), _ptr(Z), _ptr(Y),
                                     _stream(stream)), "ofm_apply_A")
        return Y

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.ofm_laplacian_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """Iteration state of Algorithm 2 for one graph, k and option set."""

    def __init__(self, lap: Laplacian, k: int, variant="f1", precision=OFM_FP32,
                 max_iter: int = 1000, check_every: int = 10, first_step: int = 0,
                 restart: bool = False, alpha0: float = 0.0, tol: float = 0.0,
                 graph: bool = False, recur: bool = False, gather: int = GATHER_AUTO,
                 freeze_eps: float = 0.0):
        lib = load()
        self._lib = lib
        self.lap = lap
        self.k = k
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self.opts = Opts(v, int(precision), int(max_iter), int(check_every), int(first_step),
                         1 if restart else 0, float(alpha0), float(tol), 1 if graph else 0,
                         1 if recur else 0, int(gather), float(freeze_eps))
        h = ctypes.c_void_p()
        _check(lib.ofm_workspace_create(lap.handle, k, ctypes.byref(self.opts), ctypes.byref(h)),
               "ofm_workspace_create")
        self.handle = h

    @property
    def dtype(self):
        torch = _torch()
        return torch.float64 if self.opts.precision == OFM_FP64 else torch.float32

    def _x(self, X):
        _dev_block(X, self.k)
        if X.dtype != self.dtype or X.shape[0] != self.lap.n:
            raise ValueError("X must be N x k of the workspace precision")
        return X

    def init(self, X, stream=None):
        _check(self._lib.ofm_init(self.handle, _ptr(self._x(X)), _stream(stream)), "ofm_init")

    def step(self, X, stream=None):
        _check(self._lib.ofm_step(self.handle, _ptr(self._x(X)), _stream(stream)), "ofm_step")

    def solve(self, X, stream=None) -> dict:
        st = Stats()
        r = self._lib.ofm_solve(self.handle, _ptr(self._x(X)), _stream(stream), ctypes.byref(st))
        if r not in (0, -4, -5):
            _check(r, "ofm_solve")
        return st.as_dict()

    def residual(self, X, stream=None) -> dict:
        st = Stats()
        r = self._lib.ofm_residual(self.handle, _ptr(self._x(X)), _stream(stream), ctypes.byref(st))
        if r not in (0, -4, -5):
            _check(r, "ofm_residual")
        return st.as_dict()

    def stats(self, stream=None) -> dict:
        st = Stats()
        self._lib.ofm_get_stats(self.handle, _stream(stream), ctypes.byref(st))
        return st.as_dict()

    def get_state(self, stream=None):
        torch = _torch()
        Vp = torch.empty((self.lap.n, self.k), dtype=self.dtype, device="cuda")
        Gp = torch.empty_like(Vp)
        _check(self._lib.ofm_get_state(self.handle, _ptr(Vp), _ptr(Gp), _stream(stream)),
               "ofm_get_state")
        return Vp, Gp

    def set_state(self, X, V_prev, G_prev, t: int, stream=None):
        for a in (X, V_prev, G_prev):
            self._x(a)
        _check(self._lib.ofm_set_state(self.handle, _ptr(X), _ptr(V_prev), _ptr(G_prev), int(t),
                                       _stream(stream)), "ofm_set_state")

    def step_info(self, stream=None) -> dict:
        k = self.k
        alpha = np.zeros(k)
        beta = np.zeros(k)
        coef = np.zeros(4 * k)
        nr = np.zeros(k, dtype=np.int32)
        _check(self._lib.ofm_get_step_info(
            self.handle, alpha.ctypes.data_as(ctypes.c_void_p), beta.ctypes.data_as(ctypes.c_void_p),
            coef.ctypes.data_as(ctypes.c_void_p), nr.ctypes.data_as(ctypes.c_void_p),
            _stream(stream)), "ofm_get_step_info")
        return {"alpha": alpha, "beta": beta, "coeffs": coef.reshape(k, 4).T.copy(), "nroots": nr}

    def objective(self, X, grad=None, stream=None):
        """(f(X) as a 1-element FP64 device tensor, grad f(X) or None)."""
        torch = _torch()
        self._x(X)
        f = torch.empty(1, dtype=torch.float64, device=X.device)
        if grad is not None:
            self._x(grad)
        _check(self._lib.ofm_objective(self.handle, _ptr(X), _ptr(f),
                                       _ptr(grad) if grad is not None else None,
                                       _stream(stream)), "ofm_objective")
        return f, grad

    PASSES = ["spmm_x", "g", "v", "spmm_v", "linesearch", "update", "reduce", "residual", "other"]

    def set_timing(self, enable=True):
        """True: time every pass; False: off; a list of pass names: those only."""
        if enable is True:
            mask = (1 << len(self.PASSES)) - 1
        elif not enable:
            mask = 0
        else:
            mask = 0
            for p in enable:
                mask |= 1 << self.PASSES.index(p)
        _check(self._lib.ofm_set_timing(self.handle, mask), "ofm_set_timing")

    def timing(self, reset: bool = True) -> dict:
        """{pass: (total ms, launches)} since the last reset (synchronizing)."""
        ms = np.zeros(len(self.PASSES))
        cnt = np.zeros(len(self.PASSES), dtype=np.int64)
        _check(self._lib.ofm_get_timing(self.handle, ms.ctypes.data_as(ctypes.c_void_p),
                                        cnt.ctypes.data_as(ctypes.c_void_p), 1 if reset else 0),
               "ofm_get_timing")
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(self.PASSES)}

    PRODUCTS = {"M": 0, "H": 1, "K": 2, "P": 3, "C": 4, "E": 5, "F": 6}

    def product(self, name: str, stream=None) -> np.ndarray:
        """Host copy of one k x k product (X^T X = "M", X^T A X = "H", ...)."""
        out = np.zeros((self.k, self.k))
        _check(self._lib.ofm_get_products(self.handle, self.PRODUCTS[name],
                                          out.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "ofm_get_products")
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.ofm_workspace_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent graphs solved together (one launch per pass and width
    group).  ``laps``: Laplacian handles; ``ks``: their widths."""

    def __init__(self, laps, ks, variant="f1", precision=OFM_FP32, max_iter: int = 1000,
                 check_every: int = 10, tol: float = 1e-4, restart: bool = False,
                 first_step: int = 0, alpha0: float = 0.0, recur: bool = False,
                 freeze_eps: float = 0.0, graph: bool = False):
        lib = load()
        self._lib = lib
        self.laps = list(laps)
        self.ks = [int(k) for k in ks]
        v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self.opts = Opts(v, int(precision), int(max_iter), int(check_every), int(first_step),
                         1 if restart else 0, float(alpha0), float(tol), 1 if graph else 0,
                         1 if recur else 0, GATHER_DEFAULT, float(freeze_eps))
        n = len(self.laps)
        handles = (ctypes.c_void_p * n)(*[l.handle.value for l in self.laps])
        kk = (ctypes.c_int * n)(*self.ks)
        h = ctypes.c_void_p()
        _check(lib.ofm_batch_create(n, handles, kk, ctypes.byref(self.opts), ctypes.byref(h)),
               "ofm_batch_create")
        self.handle = h

    def _ptrs(self, Xs):
        n = len(self.laps)
        if len(Xs) != n:
            raise ValueError(f"expected {n} blocks")
        for X, lap, k in zip(Xs, self.laps, self.ks):
            _dev_block(X, k)
            if X.dtype != _torch().float32 or X.shape[0] != lap.n:
                raise ValueError("X must be N x k FP32")
        return (ctypes.c_void_p * n)(*[X.data_ptr() for X in Xs])

    def init(self, Xs, stream=None):
        """Set-up step of Algorithm 2 on every graph (the blocks are kept)."""
        self._held = list(Xs)
        _check(self._lib.ofm_batch_init(self.handle, self._ptrs(Xs), _stream(stream)),
               "ofm_batch_init")

    def step(self, stream=None):
        """One lockstep loop iteration of every active graph."""
        _check(self._lib.ofm_batch_step(self.handle, _stream(stream)), "ofm_batch_step")

    def get_state(self, i: int, stream=None):
        """(V_prev, G_prev) of graph i, FP32 device tensors."""
        torch = _torch()
        Vp = torch.empty((self.laps[i].n, self.ks[i]), dtype=torch.float32, device="cuda")
        Gp = torch.empty_like(Vp)
        _check(self._lib.ofm_batch_get_state(self.handle, int(i), _ptr(Vp), _ptr(Gp),
                                             _stream(stream)), "ofm_batch_get_state")
        return Vp, Gp

    def step_info(self, i: int, stream=None) -> dict:
        k = self.ks[i]
        alpha = np.zeros(k)
        beta = np.zeros(k)
        coef = np.zeros(4 * k)
        nr = np.zeros(k, dtype=np.int32)
        _check(self._lib.ofm_batch_get_step_info(
            self.handle, int(i), alpha.ctypes.data_as(ctypes.c_void_p),
            beta.ctypes.data_as(ctypes.c_void_p), coef.ctypes.data_as(ctypes.c_void_p),
            nr.ctypes.data_as(ctypes.c_void_p), _stream(stream)), "ofm_batch_get_step_info")
        return {"alpha": alpha, "beta": beta, "coeffs": coef.reshape(k, 4).T.copy(), "nroots": nr}

    def solve(self, Xs, stream=None):
        n = len(self.laps)
        ptrs = self._ptrs(Xs)
        stats = (Stats * n)()
        _check(self._lib.ofm_batch_solve(self.handle, ptrs, _stream(stream), stats),
               "ofm_batch_solve")
        return [s.as_dict() for s in stats]

    def set_schedule(self, tpw: int, workers: int = 128):
        """Fix every group's schedule: tiles per wavefront (2, 4, 8 or 16) and
        blocks per XCD (128, 64 or 8-63); tpw = 0: time the candidates again."""
        _check(self._lib.ofm_batch_set_schedule(self.handle, int(tpw), int(workers)),
               "ofm_batch_set_schedule")

    def set_persistent(self, on: bool = True):
        """Run the lockstep loop as one persistent launch per width group and
        chunk of check_every updates (f1 / tri-f1, FP32, no recurrence, k <= 32)."""
        _check(self._lib.ofm_batch_set_persistent(self.handle, 1 if on else 0),
               "ofm_batch_set_persistent")

    def persist_info(self):
        """(persistent launches of the last solve, fewest workers per XCD used)."""
        n = ctypes.c_int64()
        w = ctypes.c_int()
        _check(self._lib.ofm_batch_persist_info(self.handle, ctypes.byref(n), ctypes.byref(w)),
               "ofm_batch_persist_info")
        return n.value, w.value

    def schedule(self):
        """([{k, tpw, workers, ms[8]} per width group], graphs finished in
        FP64 by the last solve)."""
        ng = ctypes.c_int()
        esc = ctypes.c_int()
        self._lib.ofm_batch_schedule(self.handle, -1, ctypes.byref(ng), None, None, None, None,
                                     ctypes.byref(esc))
        out = []
        for gi in range(ng.value):
            k, tpw, wk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            ms = np.zeros(8)
            _check(self._lib.ofm_batch_schedule(self.handle, gi, None, ctypes.byref(k),
                                                ctypes.byref(tpw), ctypes.byref(wk),
                                                ms.ctypes.data_as(ctypes.c_void_p), None),
                   "ofm_batch_schedule")
            out.append({"k": k.value, "tpw": tpw.value, "workers": wk.value, "ms": ms})
        return out, esc.value

    def phases(self):
        """(lockstep FP32 loop ms, FP64 finishing ms) of the last solve (host
        time); ``self.replays`` gets the graph replays of its lockstep loop."""
        a = ctypes.c_double()
        b = ctypes.c_double()
        r = ctypes.c_int64()
        _check(self._lib.ofm_batch_phases(self.handle, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(r)), "ofm_batch_phases")
        self.replays = r.value
        return a.value, b.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self._lib.ofm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grouped_order(row_ptr, groups):
    """Host-only: (order int32[n], slot_start int64[9]) of the XCD-grouped row
    order that ``Laplacian(..., groups=groups)`` lays out."""
    rp = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int32)
    gr = np.ascontiguousarray(np.asarray(groups), dtype=np.int32)
    n = rp.shape[0] - 1
    if gr.shape != (n,):
        raise ValueError("groups must hold one entry per node")
    order = np.empty(n, dtype=np.int32)
    slots = np.empty(9, dtype=np.int64)
    _check(load().ofm_grouped_order(n, rp.ctypes.data_as(ctypes.c_void_p),
                                    gr.ctypes.data_as(ctypes.c_void_p),
                                    order.ctypes.data_as(ctypes.c_void_p),
                                    slots.ctypes.data_as(ctypes.c_void_p)), "ofm_grouped_order")
    return order, slots


def select_roots(variant, coeffs, stream=None):
    """The device root rules of the line search on given cubics: ``coeffs``
    [count, 4] rows (a3, a2, a1, a0); returns (alpha FP64[count], nroots
    int32[count]) as host arrays (synchronizing)."""
    torch = _torch()
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    co = torch.as_tensor(np.ascontiguousarray(coeffs, dtype=np.float64).reshape(-1, 4)).cuda()
    n = co.shape[0]
    al = torch.empty(n, dtype=torch.float64, device="cuda")
    nr = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(load().ofm_select_roots(v, n, _ptr(co), _ptr(al), _ptr(nr), _stream(stream)),
           "ofm_select_roots")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return al.cpu().numpy(), nr.cpu().numpy()


def gather_rows(idx, Z, S: int, Y=None, stream=None):
    """Memory-system measurement: Y_r = sum of the S rows Z[idx[r S + e]]
    (FP32 rows of 16, 32 or 64 values); idx int32 on the device, values in
    [0, rows of Z)."""
    torch = _torch()
    if idx.dtype != torch.int32 or Z.dtype != torch.float32 or not (idx.is_cuda and Z.is_cuda):
        raise TypeError("idx int32 and Z float32 device tensors")
    nrows = idx.numel() // S
    if Y is None:
        Y = torch.empty((nrows, Z.shape[1]), dtype=torch.float32, device=Z.device)
    _check(load().ofm_gather_rows(nrows, S, Z.shape[1], _ptr(idx), _ptr(Z), Z.shape[0], _ptr(Y),
                                  _stream(stream)), "ofm_gather_rows")
    return Y


def scale(X, s, Y=None, stream=None):
    """Y = s * X with s a one-element FP64 device tensor (no host sync)."""
    torch = _torch()
    if not (X.is_cuda and X.is_contiguous()):
        raise ValueError("expected a contiguous device tensor")
    if s.dtype != torch.float64 or s.numel() != 1 or not s.is_cuda:
        raise ValueError("scale must be one FP64 value on the device")
    if Y is None:
        Y = torch.empty_like(X)
    _check(load().ofm_scale(X.numel(), _prec(X), _ptr(s.contiguous()), _ptr(X), _ptr(Y),
                            _stream(stream)), "ofm_scale")
    return Y


def row_normalize(X, Y=None, stream=None):
    torch = _torch()
    _dev_block(X)
    if Y is None:
        Y = torch.empty_like(X)
    _check(load().ofm_row_normalize(X.shape[0], X.shape[1], _prec(X), _ptr(X), _ptr(Y),
                                    _stream(stream)), "ofm_row_normalize")
    return Y


def kmeans_assign(Y, centroids, want_dist: bool = False, stream=None):
    torch = _torch()
    _dev_block(Y)
    n, dim = Y.shape
    labels = torch.empty(n, dtype=torch.int32, device=Y.device)
    d2 = torch.empty(n, dtype=torch.float32, device=Y.device) if want_dist else None
    _check(load().ofm_kmeans_assign(n, dim, centroids.shape[0], _ptr(Y), _ptr(centroids),
                                    _ptr(labels), _ptr(d2) if d2 is not None else None,
                                    _stream(stream)), "ofm_kmeans_assign")
    return (labels, d2) if want_dist else labels


def kmeans(Y, n_clusters: int, uniforms, max_iter: int = 300, stream=None, labels=None,
           centroids=None, noalloc: bool = False):
    """K-means++ seeded by ``uniforms`` then Lloyd; returns (labels, centroids,
    iters).  ``labels`` / ``centroids``: optional output tensors.  ``noalloc``:
    ofm_kmeans_noalloc (the library allocates nothing; its buffers are a
    fixed device array shared by every call on the device)."""
    torch = _torch()
    _dev_block(Y)
    n, dim = Y.shape
    u = np.ascontiguousarray(uniforms, dtype=np.float64)
    if u.shape[0] < n_clusters:
        raise ValueError("need one uniform per cluster")
    if labels is None:
        labels = torch.empty(n, dtype=torch.int32, device=Y.device)
    if centroids is None:
        centroids = torch.empty((n_clusters, dim), dtype=torch.float32, device=Y.device)
    iters = ctypes.c_int32()
    fn = load().ofm_kmeans_noalloc if noalloc else load().ofm_kmeans
    _check(fn(n, dim, n_clusters, _ptr(Y), u.ctypes.data_as(ctypes.c_void_p), max_iter,
              _ptr(labels), _ptr(centroids), ctypes.byref(iters), _stream(stream)),
           "ofm_kmeans_noalloc" if noalloc else "ofm_kmeans")
    return labels, centroids, iters.value

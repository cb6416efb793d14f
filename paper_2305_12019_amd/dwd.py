"""ctypes binding of libdwd (include/dwd.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module only converts
arrays and parameters to the C structs and back.  It raises ImportError if
the built library is missing: there is no fallback.

Data convention: ``X`` is an array of shape (n, d) whose row i is the sample
x_i, i.e. the d x n matrix of the paper stored column-major.  It may be a
NumPy array (host) or a torch tensor (host or device).  ``y`` holds +-1.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwd.so")

FP64, FP32, BF16 = 0, 1, 2
DENSE, CSR = 0, 1
STATUS = {0: "DWD_OK", 1: "DWD_NOT_CONVERGED", -1: "DWD_E_INVALID", -2: "DWD_E_NOMEM",
          -3: "DWD_E_DEVICE", -4: "DWD_E_NUMERIC", -5: "DWD_E_BUSY"}
_STORAGE = {"f64": FP64, "fp64": FP64, "f32": FP32, "fp32": FP32, "bf16": BF16}
_SOLVER = {"smw": 0, "direct": 1, "auto": 2, "iterative": 3}


class DwdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Matrix(C.Structure):
    _fields_ = [("d", C.c_int64), ("n", C.c_int64), ("dtype", C.c_int32), ("layout", C.c_int32),
                ("values", C.c_void_p), ("indptr", C.c_void_p), ("indices", C.c_void_p),
                ("nnz", C.c_int64), ("on_device", C.c_int32), ("reserved", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("C", C.c_double), ("q", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("storage", C.c_int32), ("tau", C.c_double),
                ("mu", C.c_double), ("sigma0", C.c_double), ("eps_c", C.c_double),
                ("rho_residual", C.c_int32), ("resync", C.c_int32), ("check_every", C.c_int32),
                ("refine", C.c_int32), ("lowp_tol", C.c_double), ("profile", C.c_int32),
                ("batch_fp32", C.c_int32), ("batch_tile", C.c_int32), ("graph", C.c_int32),
                ("sigma_every", C.c_int32), ("representer", C.c_int32),
                ("class_weights", C.c_int32), ("solver", C.c_int32), ("ell", C.c_int32),
                ("e", C.c_void_p), ("psqmr_max", C.c_int32), ("reserved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("beta", C.c_double), ("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("eta_p", C.c_double), ("eta_d", C.c_double), ("eta_c", C.c_double),
                ("eta_gap", C.c_double), ("eta_p_check", C.c_double),
                ("eta_d_check", C.c_double), ("kkt_check", C.c_double), ("sigma", C.c_double),
                ("iters", C.c_int32), ("n_double", C.c_int32), ("newton_max", C.c_int32),
                ("converged", C.c_int32), ("iters_lowp", C.c_int32), ("status", C.c_int32),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("stream_ms", C.c_double),
                ("stream_launches", C.c_int32), ("resumed", C.c_int32),
                ("streamT_ms", C.c_double), ("streamT_launches", C.c_int32),
                ("graph_launches", C.c_int32), ("psqmr_steps", C.c_int32),
                ("psqmr_solves", C.c_int32), ("psqmr_switch", C.c_int32),
                ("representer", C.c_int32)]

    def to_dict(self) -> Dict:
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Request(C.Structure):
    _fields_ = [("X", Matrix), ("y", C.c_void_p), ("params", Params), ("t_arrival", C.c_double)]


class ServeOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_double), ("max_slots", C.c_int32),
                ("iters_per_round", C.c_int32)]


class Response(C.Structure):
    _fields_ = [("w", C.c_void_p), ("info", Info), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("status", C.c_int32), ("reserved", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2305_12019_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    lib.dwd_default_params.argtypes = [C.POINTER(Params)]
    lib.dwd_default_params.restype = None
    lib.dwd_setup.argtypes = [C.POINTER(Matrix), dp, C.POINTER(Params), C.c_void_p,
                              C.POINTER(C.c_void_p)]
    lib.dwd_setup.restype = C.c_int
    lib.dwd_solve.argtypes = [C.c_void_p, C.POINTER(Params), dp, C.POINTER(Info), dp, dp, dp, dp,
                              dp]
    lib.dwd_solve.restype = C.c_int
    lib.dwd_solve_batch.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Params), dp,
                                    C.POINTER(Info)]
    lib.dwd_solve_batch.restype = C.c_int
    lib.dwd_free.argtypes = [C.c_void_p]
    lib.dwd_free.restype = None
    lib.dwd_serve.argtypes = [C.POINTER(Request), C.c_int32, C.POINTER(ServeOpts),
                              C.POINTER(Response)]
    lib.dwd_serve.restype = C.c_int
    lib.dwd_footprint.argtypes = [C.POINTER(Matrix), C.POINTER(Params)]
    lib.dwd_footprint.restype = C.c_int64
    lib.dwd_suggest_C.argtypes = [C.c_void_p, C.c_double, dp]
    lib.dwd_suggest_C.restype = C.c_int
    lib.dwd_suggest_C_noalloc.argtypes = [C.c_void_p, C.c_double, dp]
    lib.dwd_suggest_C_noalloc.restype = C.c_int
    lib.dwd_inspect.argtypes = [C.c_void_p, C.c_char_p, dp, C.c_int64]
    lib.dwd_inspect.restype = C.c_int
    lib.dwd_status_str.argtypes = [C.c_int]
    lib.dwd_status_str.restype = C.c_char_p
    lib.dwd_last_error.argtypes = []
    lib.dwd_last_error.restype = C.c_char_p
    lib.dwd_version.argtypes = []
    lib.dwd_version.restype = C.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def last_error() -> str:
    return _lib.dwd_last_error().decode()


def version() -> str:
    return _lib.dwd_version().decode()


def _check(status: int, allow_not_converged: bool = True) -> int:
    if status < 0 or (status == 1 and not allow_not_converged):
        raise DwdError(status, last_error())
    return status


def params(**kw) -> Params:
    """Default parameters (dwd_default_params) with keyword overrides;
    ``storage`` may be a string ("f64", "f32", "bf16"); ``e`` an array of n
    penalty weights (kept alive as ``p.keep``; a copy of the structure does
    not keep it, so callers that copy hold ``p.keep`` themselves)."""
    p = Params()
    _lib.dwd_default_params(C.byref(p))
    p.keep = None
    for k, v in kw.items():
        if k == "storage" and isinstance(v, str):
            v = _STORAGE[v]
        if k == "solver" and isinstance(v, str):
            v = _SOLVER[v]
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        if k == "e":
            if v is None:
                p.e = None
                continue
            v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            p.keep = v
            p.e = v.ctypes.data
            continue
        setattr(p, k, v)
    return p


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch absent
        pass
    return C.c_void_p(None)


def dense_matrix(X, keep: List) -> Matrix:
    """Describe an (n, d) array as the d x n column-major dwd_matrix."""
    if _is_torch(X):
        import torch
        if X.dim() != 2:
            raise ValueError("X must be 2-D (n, d)")
        if not X.is_contiguous():
            X = X.contiguous()
        if X.dtype not in (torch.float32, torch.float64):
            raise ValueError("X must be float32 or float64")
        keep.append(X)
        return Matrix(d=X.shape[1], n=X.shape[0], dtype=FP64 if X.dtype == torch.float64 else FP32,
                      layout=DENSE, values=X.data_ptr(), indptr=None, indices=None, nnz=0,
                      on_device=1 if X.is_cuda else 0)
    X = np.asarray(X)
    if X.ndim != 2:
        raise ValueError("X must be 2-D (n, d)")
    if X.dtype not in (np.float32, np.float64):
        X = X.astype(np.float64)
    X = np.ascontiguousarray(X)
    keep.append(X)
    return Matrix(d=X.shape[1], n=X.shape[0], dtype=FP64 if X.dtype == np.float64 else FP32,
                  layout=DENSE, values=X.ctypes.data, indptr=None, indices=None, nnz=0,
                  on_device=0)


def csr_matrix(indptr, indices, values, d: int, keep: List) -> Matrix:
    """Describe CSR of X^T (one row per sample) on the host."""
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    values = np.ascontiguousarray(values)
    if values.dtype not in (np.float32, np.float64):
        values = values.astype(np.float64)
    keep.extend([indptr, indices, values])
    return Matrix(d=d, n=len(indptr) - 1, dtype=FP64 if values.dtype == np.float64 else FP32,
                  layout=CSR, values=values.ctypes.data, indptr=indptr.ctypes.data,
                  indices=indices.ctypes.data, nnz=len(values), on_device=0)


def _check_e(e, n: int):
    if e is not None and np.shape(e) != (n,):
        raise ValueError("e must have n entries")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """A set-up problem (dwd_setup); free with close() or by garbage collection."""

    def __init__(self, X=None, y=None, storage="f32", mu: float = 1.0, csr=None, stream=None,
                 solver="smw", ell: int = 0):
        keep: List = []
        if csr is not None:
            indptr, indices, values, d = csr
            m = csr_matrix(indptr, indices, values, d, keep)
        else:
            m = dense_matrix(X, keep)
        self.d, self.n = int(m.d), int(m.n)
        yy = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        if yy.shape != (self.n,):
            raise ValueError("y must have n entries")
        p = params(storage=storage, mu=mu, solver=solver, ell=ell)
        self._h = C.c_void_p()
        st = _current_stream() if stream is None else C.c_void_p(stream)
        _check(_lib.dwd_setup(C.byref(m), _dptr(yy), C.byref(p), st, C.byref(self._h)))
        self.storage = storage
        self.mu = mu

    def solve(self, C_: float = 1.0, q: float = 1.0, tol: float = 1e-5, want_state: bool = True,
              **kw) -> Dict:
        _check_e(kw.get("e"), self.n)
        p = params(C=C_, q=q, tol=tol, storage=self.storage, mu=self.mu, **kw)
        w = np.empty(self.d)
        info = Info()
        if want_state:
            alpha, r, xi = np.empty(self.n), np.empty(self.n), np.empty(self.n)
            u, rho = np.empty(self.d), np.empty(self.d)
            st = _lib.dwd_solve(self._h, C.byref(p), _dptr(w), C.byref(info), _dptr(alpha),
                                _dptr(r), _dptr(xi), _dptr(u), _dptr(rho))
        else:
            nul = C.POINTER(C.c_double)()
            st = _lib.dwd_solve(self._h, C.byref(p), _dptr(w), C.byref(info), nul, nul, nul, nul,
                                nul)
        _check(st)
        out = dict(status=st, w=w, beta=info.beta, info=info.to_dict())
        if want_state:
            out.update(alpha=alpha, r=r, xi=xi, u=u, rho=rho)
        return out

    def solve_batch(self, plist: Sequence[Dict]) -> Dict:
        B = len(plist)
        arr = (Params * B)()
        keep = []
        for j, kw in enumerate(plist):
            kw = dict(kw)
            kw.setdefault("storage", self.storage)
            kw.setdefault("mu", self.mu)
            if "C_" in kw:
                kw["C"] = kw.pop("C_")
            _check_e(kw.get("e"), self.n)
            pj = params(**kw)
            keep.append(pj.keep)
            arr[j] = pj
        W = np.empty((B, self.d))  # row j = w of problem j (d x B column-major)
        infos = (Info * B)()
        st = _check(_lib.dwd_solve_batch(self._h, B, arr, _dptr(W), infos))
        return dict(status=st, W=W, info=[infos[j].to_dict() for j in range(B)])

    def suggest_C(self, q: float = 1.0) -> float:
        """The Section 4.1 choice of C for exponent q (dwd_suggest_C)."""
        out = np.empty(1)
        _check(_lib.dwd_suggest_C(self._h, q, _dptr(out)))
        return float(out[0])

    def suggest_C_noalloc(self, q: float = 1.0) -> float:
        """The same value from the allocation-free entry point
        (dwd_suggest_C_noalloc)."""
        out = np.empty(1)
        _check(_lib.dwd_suggest_C_noalloc(self._h, q, _dptr(out)))
        return float(out[0])

    def inspect(self, what: str) -> np.ndarray:
        """Copy a set-up quantity to the host (dwd_inspect)."""
        if what == "lam":
            m = int(self.inspect("ell")[0])
            out = np.empty(m)
            _check(_lib.dwd_inspect(self._h, b"lam", _dptr(out), m))
            return out
        if what == "psqmr_steps":
            m = int(self.inspect("psqmr_count")[0])
            out = np.empty(m)
            if m:
                _check(_lib.dwd_inspect(self._h, b"psqmr_steps", _dptr(out), m))
            return out.astype(np.int64)
        size = {"zscale": 1, "ymy": 1, "solver": 1, "ell": 1, "psqmr_count": 1,
                "G": self.n * self.n,
                "Minv": self.n * self.n, "my": self.n,
                "Ainv": (self.d + 1) * (self.d + 1)}[what]
        out = np.empty(size)
        _check(_lib.dwd_inspect(self._h, what.encode(), _dptr(out), size))
        if what in ("G", "Minv"):
            return out.reshape(self.n, self.n)
        if what == "Ainv":
            return out.reshape(self.d + 1, self.d + 1)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.dwd_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(X, y, C_: float = 1.0, q: float = 1.0, tol: float = 1e-5, storage="f32", **kw) -> Dict:
    """Set up and solve one problem; returns w (unscaled), beta, state and info."""
    P = Problem(X, y, storage=storage, mu=kw.pop("mu", 1.0), solver=kw.pop("solver", "smw"),
                ell=kw.pop("ell", 0))
    try:
        return P.solve(C_, q, tol, **kw)
    finally:
        P.close()


def footprint(d: int, n: int, storage="f32", layout=DENSE, nnz: int = 0) -> int:
    m = Matrix(d=d, n=n, dtype=FP32, layout=layout, values=None, indptr=None, indices=None,
               nnz=nnz, on_device=0)
    p = params(storage=storage)
    return int(_lib.dwd_footprint(C.byref(m), C.byref(p)))


def serve(requests: Sequence[Dict], hbm_budget_bytes: float = 0.0, max_slots: int = 0,
          iters_per_round: int = 0) -> List[Dict]:
    """Replay a trace with dwd_serve.  Each request is a dict with ``X``
    (or ``csr=(indptr, indices, values, d)``), ``y``, ``t_arrival`` (s) and
    ``params`` (keyword overrides of :func:`params`)."""
    keep: List = []
    nreq = len(requests)
    arr = (Request * max(nreq, 1))()
    resp = (Response * max(nreq, 1))()
    ws = []
    for j, rq in enumerate(requests):
        if "csr" in rq:
            m = csr_matrix(*rq["csr"], keep)
        else:
            m = dense_matrix(rq["X"], keep)
        yy = np.ascontiguousarray(np.asarray(rq["y"], dtype=np.float64))
        keep.append(yy)
        kw = dict(rq.get("params", {}))
        if "C_" in kw:
            kw["C"] = kw.pop("C_")
        arr[j].X = m
        arr[j].y = yy.ctypes.data
        _check_e(kw.get("e"), int(m.n))
        pj = params(**kw)
        keep.append(pj.keep)
        arr[j].params = pj
        arr[j].t_arrival = float(rq.get("t_arrival", 0.0))
        w = np.empty(int(m.d))
        ws.append(w)
        resp[j].w = w.ctypes.data
    opts = ServeOpts(hbm_budget_bytes=hbm_budget_bytes, max_slots=max_slots,
                     iters_per_round=iters_per_round)
    _check(_lib.dwd_serve(arr, nreq, C.byref(opts), resp))
    out = []
    for j in range(nreq):
        r = resp[j]
        out.append(dict(status=int(r.status), w=ws[j], beta=r.info.beta, info=r.info.to_dict(),
                        t_admit=r.t_admit, t_done=r.t_done,
                        latency=r.t_done - float(requests[j].get("t_arrival", 0.0))))
    return out

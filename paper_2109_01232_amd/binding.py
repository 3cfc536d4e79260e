"""ctypes binding of libgmresir (include/gmresir.h): argument marshalling only.

Every function named ``gmresir_*`` here calls the C entry point of the same
name; the classes below only allocate device buffers with PyTorch and pass
raw pointers and the current HIP stream.  All arithmetic of the solver runs
in the library's HIP kernels; if the library is not built, loading fails
loudly (there is no fallback).
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgmresir.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "gmresir.h")

OK, NOT_CONVERGED, STAGNATED, BREAKDOWN = 0, 1, 2, 3
ERR_INVALID_ARG, ERR_HIP, ERR_WORKSPACE, ERR_NUMERIC, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
FP64, FP32, BF16 = 0, 1, 2
NCAT = 7
CATEGORIES = ("spmv_proj", "update_proj", "update_norm", "poly", "refine", "other", "tail")
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16}


class Params(ctypes.Structure):
    _fields_ = [
        ("restart", ctypes.c_int32),
        ("inner_cap", ctypes.c_int32),
        ("max_iters", ctypes.c_int64),
        ("rtol", ctypes.c_double),
        ("inner_prec", ctypes.c_int32),
        ("basis_prec", ctypes.c_int32),
        ("poly_degree", ctypes.c_int32),
        ("check_mode", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("poly_prec", ctypes.c_int32),
        ("bj_block", ctypes.c_int32),
        ("ortho", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("refinements", ctypes.c_int32),
        ("iters", ctypes.c_int64),
        ("cycles", ctypes.c_int64),
        ("rel_resid_true", ctypes.c_double),
        ("rel_resid_implicit", ctypes.c_double),
        ("solve_s", ctypes.c_double),
        ("cat_time_s", ctypes.c_double * NCAT),
        ("cat_bytes", ctypes.c_double * NCAT),
        ("cat_launches", ctypes.c_int64 * NCAT),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_[:7]}
        d["cat_time_s"] = dict(zip(CATEGORIES, list(self.cat_time_s)))
        d["cat_bytes"] = dict(zip(CATEGORIES, list(self.cat_bytes)))
        d["cat_launches"] = dict(zip(CATEGORIES, list(self.cat_launches)))
        return d


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)

_SIGS = {
    "gmresir_abi_version": (_i32, []),
    "gmresir_last_error": (ctypes.c_char_p, []),
    "gmresir_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gmresir_matrix_storage_bytes": (_sz, [_i64, _i64]),
    "gmresir_matrix_create": (ctypes.c_int, [_i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(_vp)]),
    "gmresir_matrix_destroy": (ctypes.c_int, [_vp]),
    "gmresir_matrix_n": (_i64, [_vp]),
    "gmresir_matrix_nnz": (_i64, [_vp]),
    "gmresir_matrix_tiles": (_i64, [_vp]),
    "gmresir_matrix_layout": (_i32, [_vp]),
    "gmresir_spmv": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "gmresir_workspace_bytes": (_sz, [_vp, ctypes.POINTER(Params)]),
    "gmresir_solve": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(Params), _dp, _vp, _sz,
                                     ctypes.POINTER(Result), _dp, _i64, _vp]),
    "gmresir_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(Params), _dp, ctypes.POINTER(Result),
                                             _dp, _i64, _vp]),
    "gmresir_fd_workspace_bytes": (_sz, [_vp, ctypes.POINTER(Params), _i64]),
    "gmresir_solve_fd": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(Params), _i64, _vp, _sz,
                                        ctypes.POINTER(Result), _dp, _i64, _vp]),
    "gmresir_poly_workspace_bytes": (_sz, [_vp, _i32]),
    "gmresir_poly_setup": (ctypes.c_int, [_vp, _i32, _vp, ctypes.c_uint64, _vp, _sz, _dp, _dp, _vp]),
    "gmresir_poly_apply": (ctypes.c_int, [_vp, _i32, _dp, _vp, _vp, _vp, _sz, _vp]),
    "gmresir_features": (ctypes.c_int, [_vp, _vp, _vp, _sz, _fp, _vp]),
    "gmresir_mlp_forward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "gmresir_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "gmresir_mlp_train_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float, _i32,
                                              _vp, _vp]),
    "gmresir_host_hessenberg_eigvals": (ctypes.c_int, [_i32, _dp, _i32, _dp, _dp]),
    "gmresir_host_harmonic_ritz_leja": (ctypes.c_int, [_i32, _dp, _i32, _dp]),
}


def lib() -> ctypes.CDLL:
    """Load libgmresir.so (built in the package directory) once."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2109_01232_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions declared in include/gmresir.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmresir_[a-z0-9_]+)\s*\(", text)))


def last_error() -> str:
    return lib().gmresir_last_error().decode()


def status_string(st: int) -> str:
    return lib().gmresir_status_string(st).decode()


class GmresirError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} returned {status} ({status_string(status)}): {last_error()}")
        self.status = status


def _check(fn, st, ok=(OK,)):
    if st not in ok:
        raise GmresirError(fn, st)
    return st


# ---------------------------------------------------------------------------
# host-only helpers (no GPU)
# ---------------------------------------------------------------------------

def gmresir_host_hessenberg_eigvals(H: np.ndarray) -> np.ndarray:
    H = np.asfortranarray(np.asarray(H, dtype=np.float64))
    n = H.shape[0]
    wr = np.zeros(n)
    wi = np.zeros(n)
    _check("gmresir_host_hessenberg_eigvals",
           lib().gmresir_host_hessenberg_eigvals(n, H.ctypes.data_as(_dp), n, wr.ctypes.data_as(_dp),
                                                 wi.ctypes.data_as(_dp)))
    return wr + 1j * wi


def gmresir_host_harmonic_ritz_leja(Hbar: np.ndarray) -> np.ndarray:
    Hbar = np.asfortranarray(np.asarray(Hbar, dtype=np.float64))
    k = Hbar.shape[1]
    out = np.zeros(2 * k)
    _check("gmresir_host_harmonic_ritz_leja",
           lib().gmresir_host_harmonic_ritz_leja(k, Hbar.ctypes.data_as(_dp), k + 1, out.ctypes.data_as(_dp)))
    return out[0::2] + 1j * out[1::2]


def roots_to_array(roots) -> np.ndarray:
    """(re, im) pairs as the C ABI expects them."""
    roots = np.asarray(roots, dtype=np.complex128)
    out = np.empty(2 * len(roots))
    out[0::2] = roots.real
    out[1::2] = roots.imag
    return out


# ---------------------------------------------------------------------------
# device-side wrappers (PyTorch supplies memory and the stream)
# ---------------------------------------------------------------------------

def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _empty_bytes(nbytes, device):
    torch = _torch()
    # PyTorch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Matrix:
    """CSR matrix on the GPU plus the library handle (fp32 copy, row tiles)."""

    def __init__(self, rowptr, colidx, vals, device="cuda"):
        torch = _torch()
        self.n = int(len(rowptr) - 1)
        self.nnz = int(rowptr[-1])
        self.rowptr = torch.as_tensor(np.asarray(rowptr, dtype=np.int32)).to(device)
        self.colidx = torch.as_tensor(np.asarray(colidx, dtype=np.int32)).to(device)
        self.vals = torch.as_tensor(np.asarray(vals, dtype=np.float64)).to(device)
        self.device = device
        nbytes = lib().gmresir_matrix_storage_bytes(self.n, self.nnz)
        if nbytes == 0:
            raise GmresirError("gmresir_matrix_storage_bytes", ERR_INVALID_ARG)
        self.storage = _empty_bytes(nbytes, device)
        h = _vp()
        _check("gmresir_matrix_create",
               lib().gmresir_matrix_create(self.n, self.nnz, _ptr(self.rowptr), _ptr(self.colidx), _ptr(self.vals),
                                           _ptr(self.storage), nbytes, _stream(), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_csr(cls, A, device="cuda"):
        return cls(A.rowptr, A.colidx, A.vals, device)

    @property
    def tiles(self) -> int:
        return int(lib().gmresir_matrix_tiles(self.handle))

    @property
    def layout(self) -> int:
        """0 = CSR row tiles only, 1 = sliced ELLPACK with 32-bit columns,
        2 = sliced ELLPACK with 16-bit column offsets, 3 = sliced ELLPACK with
        one column-offset list per slice."""
        return int(lib().gmresir_matrix_layout(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().gmresir_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params(restart=50, inner="fp32", basis=None, rtol=1e-10, max_iters=1_000_000, inner_cap=0,
                poly_degree=0, check_mode=1, profile=0, poly_prec=None, bj_block=0, ortho=0) -> Params:
    if basis is None:
        basis = "fp64" if inner == "fp64" else "fp32"
    p = Params()
    p.restart = restart
    p.inner_cap = inner_cap
    p.max_iters = max_iters
    p.rtol = rtol
    p.inner_prec = PREC[inner]
    p.basis_prec = PREC[basis]
    p.poly_degree = poly_degree
    p.check_mode = check_mode
    p.profile = profile
    p.poly_prec = 0 if poly_prec is None else PREC[poly_prec]
    p.bj_block = bj_block
    p.ortho = {"cgs2": 0, "dcgs2": 1}.get(ortho, ortho)
    return p


def gmresir_workspace_bytes(A: Matrix, p: Params) -> int:
    return int(lib().gmresir_workspace_bytes(A.handle, ctypes.byref(p)))


def gmresir_spmv(A: Matrix, x, y, prec="fp64"):
    return _check("gmresir_spmv", lib().gmresir_spmv(A.handle, PREC[prec], _ptr(x), _ptr(y), _stream()))


class Workspace:
    """A reusable device workspace (grows on demand)."""

    def __init__(self, device="cuda"):
        self.buf = None
        self.device = device

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = _empty_bytes(nbytes, self.device)
        return self.buf


def gmresir_solve(A: Matrix, b, x, p: Params, poly_roots=None, ws=None, hist_cap=0):
    """Run gmresir_solve; x (fp64 device tensor) is updated in place.

    Returns (status, result dict, history numpy array).
    """
    need = gmresir_workspace_bytes(A, p)
    if need == 0:
        raise GmresirError("gmresir_workspace_bytes", ERR_INVALID_ARG)
    buf = (ws or Workspace(A.device)).get(need)
    res = Result()
    hist = np.zeros(max(hist_cap, 0))
    roots = None if poly_roots is None else roots_to_array(poly_roots)
    st = lib().gmresir_solve(A.handle, _ptr(b), _ptr(x), ctypes.byref(p),
                             roots.ctypes.data_as(_dp) if roots is not None else None, _ptr(buf), buf.numel(),
                             ctypes.byref(res), hist.ctypes.data_as(_dp) if hist_cap > 0 else None, hist_cap,
                             _stream())
    if st < 0:
        raise GmresirError("gmresir_solve", st)
    d = res.as_dict()
    n_hist = min(hist_cap, d["iters"])
    return st, d, hist[:n_hist]


# GMRESIR_NOALLOC_MAX_BYTES of the header: the static scratch array's size
NOALLOC_MAX_BYTES = 64 << 20


def gmresir_solve_noalloc(A: Matrix, b, x, p: Params, poly_roots=None, hist_cap=0):
    """Run gmresir_solve_noalloc (workspace from the library's static device
    array, nothing allocated); x is updated in place.  Returns (status, result
    dict, history numpy array); raises GmresirError on negative statuses."""
    res = Result()
    hist = np.zeros(max(hist_cap, 0))
    roots = None if poly_roots is None else roots_to_array(poly_roots)
    st = lib().gmresir_solve_noalloc(A.handle, _ptr(b), _ptr(x), ctypes.byref(p),
                                     roots.ctypes.data_as(_dp) if roots is not None else None, ctypes.byref(res),
                                     hist.ctypes.data_as(_dp) if hist_cap > 0 else None, hist_cap, _stream())
    if st < 0:
        raise GmresirError("gmresir_solve_noalloc", st)
    d = res.as_dict()
    return st, d, hist[: min(hist_cap, d["iters"])]


def solve(A: Matrix, b, x0=None, ws=None, hist_cap=0, poly_roots=None, **kw):
    """Convenience: returns (x, result dict, history)."""
    torch = _torch()
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    p = make_params(**kw)
    st, d, h = gmresir_solve(A, b, x, p, poly_roots=poly_roots, ws=ws, hist_cap=hist_cap)
    return x, d, h


def gmresir_fd_workspace_bytes(A: Matrix, p: Params, switch_iters: int) -> int:
    return int(lib().gmresir_fd_workspace_bytes(A.handle, ctypes.byref(p), switch_iters))


def gmresir_solve_fd(A: Matrix, b, x, p: Params, switch_iters: int, ws=None, hist_cap=0):
    """Run gmresir_solve_fd (GMRES-FD); x (fp64 device tensor) is updated in place.

    Returns (status, result dict, history numpy array).
    """
    need = gmresir_fd_workspace_bytes(A, p, switch_iters)
    if need == 0:
        raise GmresirError("gmresir_fd_workspace_bytes", ERR_INVALID_ARG)
    buf = (ws or Workspace(A.device)).get(need)
    res = Result()
    hist = np.zeros(max(hist_cap, 0))
    st = lib().gmresir_solve_fd(A.handle, _ptr(b), _ptr(x), ctypes.byref(p), switch_iters, _ptr(buf), buf.numel(),
                                ctypes.byref(res), hist.ctypes.data_as(_dp) if hist_cap > 0 else None, hist_cap,
                                _stream())
    if st < 0:
        raise GmresirError("gmresir_solve_fd", st)
    d = res.as_dict()
    return st, d, hist[: min(hist_cap, d["iters"])]


def solve_fd(A: Matrix, b, switch_iters: int, x0=None, ws=None, hist_cap=0, **kw):
    """Convenience for GMRES-FD: returns (x, result dict, history)."""
    torch = _torch()
    x = torch.zeros_like(b) if x0 is None else x0.clone()
    p = make_params(inner="fp32", **kw)
    st, d, h = gmresir_solve_fd(A, b, x, p, switch_iters, ws=ws, hist_cap=hist_cap)
    return x, d, h


def gmresir_poly_setup(A: Matrix, degree: int, start=None, seed: int = 0, ws=None, with_hbar=False):
    need = int(lib().gmresir_poly_workspace_bytes(A.handle, degree))
    buf = (ws or Workspace(A.device)).get(need)
    roots = np.zeros(2 * (degree + 1))
    hbar = np.zeros((degree + 2) * (degree + 1)) if with_hbar else None
    st = lib().gmresir_poly_setup(A.handle, degree, _ptr(start), seed, _ptr(buf), buf.numel(),
                                  roots.ctypes.data_as(_dp), hbar.ctypes.data_as(_dp) if with_hbar else None,
                                  _stream())
    if st != OK:
        raise GmresirError("gmresir_poly_setup", st)
    r = roots[0::2] + 1j * roots[1::2]
    if with_hbar:
        return r, hbar.reshape(degree + 1, degree + 2).T
    return r


def gmresir_poly_apply(A: Matrix, roots, v, y, ws=None):
    degree = len(roots) - 1
    need = int(lib().gmresir_poly_workspace_bytes(A.handle, degree))
    buf = (ws or Workspace(A.device)).get(need)
    arr = roots_to_array(roots)
    return _check("gmresir_poly_apply",
                  lib().gmresir_poly_apply(A.handle, degree, arr.ctypes.data_as(_dp), _ptr(v), _ptr(y), _ptr(buf),
                                           buf.numel(), _stream()))


def gmresir_features(A: Matrix, b, ws=None) -> np.ndarray:
    need = int(lib().gmresir_poly_workspace_bytes(A.handle, 10))
    buf = (ws or Workspace(A.device)).get(need)
    f = np.zeros(16, dtype=np.float32)
    _check("gmresir_features",
           lib().gmresir_features(A.handle, _ptr(b), _ptr(buf), buf.numel(), f.ctypes.data_as(_fp), _stream()))
    return f


def gmresir_mlp_forward(params, shift, scale, X, Y):
    return _check("gmresir_mlp_forward",
                  lib().gmresir_mlp_forward(_ptr(params), _ptr(shift), _ptr(scale), _ptr(X), _ptr(Y), X.shape[0],
                                            _stream()))


def gmresir_mlp_loss_grad(params, shift, scale, X, T, grad, loss):
    return _check("gmresir_mlp_loss_grad",
                  lib().gmresir_mlp_loss_grad(_ptr(params), _ptr(shift), _ptr(scale), _ptr(X), _ptr(T), X.shape[0],
                                              _ptr(grad), _ptr(loss), _stream()))


def gmresir_mlp_train_step(params, m, v, shift, scale, X, T, lr, step, loss):
    return _check("gmresir_mlp_train_step",
                  lib().gmresir_mlp_train_step(_ptr(params), _ptr(m), _ptr(v), _ptr(shift), _ptr(scale), _ptr(X),
                                               _ptr(T), X.shape[0], float(lr), int(step), _ptr(loss), _stream()))

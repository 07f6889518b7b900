"""ctypes binding of librbffd.so: argument marshalling only.

Tensors are passed as raw device pointers (``data_ptr()``) and every call is
enqueued on the current torch stream of the tensors' device.  Every step of the
path runs in the HIP library; there is no CPU fallback: if the library is not
built, or a tensor is not on a GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librbffd.so")

OPS = ("lap", "dx", "dy", "dz")
OP_BITS = {"lap": 1, "dx": 2, "dy": 4, "dz": 8}
PREC = {"f64": 0, "f32_ir": 1}

ST_OK, ST_REFINED, ST_FALLBACK, ST_SURROGATE, ST_SURROGATE_REJECTED = 0, 1, 2, 3, 4
ST_SINGULAR, ST_BADSIZE = -1, -2

_lib = None
_lock = threading.Lock()


class RbfError(RuntimeError):
    pass


class rbf_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_refine", ctypes.c_int), ("phs_power", ctypes.c_int),
                ("scale_mode", ctypes.c_int), ("repro_tol", ctypes.c_double), ("refine_tol", ctypes.c_double)]


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_U = ctypes.c_uint
_SZ = ctypes.c_size_t

_SIGS = {
    "rbf_options_default": [ctypes.POINTER(rbf_options)],
    "rbf_status_string": [_I],
    "rbf_ctx_create": [ctypes.POINTER(_P), _I, _P],
    "rbf_ctx_set_stream": [_P, _P],
    "rbf_ctx_destroy": [_P],
    "rbf_select_stencils_workspace": [_I64, _I, _I, ctypes.POINTER(_SZ)],
    "rbf_select_stencils": [_P, _P, _I64, _I, _P, _I, _P, _P, _SZ],
    "rbf_compute_weights": [_P, _P, _I64, _I, _P, _P, _I64, _I, _I, _U, ctypes.POINTER(rbf_options), _P, _P],
    "rbf_assemble_csr": [_P, _I64, _P, _P, _P, _I, _I64, _I, _P, _P, _P],
}


def lib():
    """Load librbffd.so once; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RbfError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_13282_amd.build`")
            L = ctypes.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = ctypes.c_char_p if name == "rbf_status_string" else ctypes.c_int32
            _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().rbf_status_string(rc).decode()
        raise RbfError(f"{what} failed: {msg} ({rc})")


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise RbfError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise RbfError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise RbfError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context bound to one device; every call uses the current torch stream."""

    def __init__(self, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = dev
        h = ctypes.c_void_p()
        _check(lib().rbf_ctx_create(ctypes.byref(h), dev.index or 0, None), "rbf_ctx_create")
        self._h = h

    def _sync_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().rbf_ctx_set_stream(self._h, ctypes.c_void_p(s)), "rbf_ctx_set_stream")
        return self._h

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.rbf_ctx_destroy(self._h)
        except Exception:
            pass


_ctx_cache: dict = {}


def context(device=None) -> Context:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = dev.index or 0
    if key not in _ctx_cache:
        _ctx_cache[key] = Context(dev)
    return _ctx_cache[key]


def options(precision="f64", max_refine=10, phs_power=3, scale_mode=0, repro_tol=1e-8,
            refine_tol=0.0) -> rbf_options:
    o = rbf_options()
    _check(lib().rbf_options_default(ctypes.byref(o)), "rbf_options_default")
    o.precision = PREC[precision]
    o.max_refine = int(max_refine)
    o.phs_power = int(phs_power)
    o.scale_mode = int(scale_mode)
    o.repro_tol = float(repro_tol)
    o.refine_tol = float(refine_tol)
    return o


def op_mask(ops) -> int:
    m = 0
    for o in ops:
        m |= OP_BITS[o]
    return m


# ------------------------------------------------------------------ workspaces
def select_stencils_workspace(N: int, d: int, n_max: int) -> int:
    b = _SZ()
    _check(lib().rbf_select_stencils_workspace(N, d, n_max, ctypes.byref(b)), "rbf_select_stencils_workspace")
    return b.value


# ------------------------------------------------------------------ entry points
def select_stencils(X: torch.Tensor, offsets: torch.Tensor, n_max: int, idx: torch.Tensor | None = None,
                    workspace: torch.Tensor | None = None, ctx: Context | None = None) -> torch.Tensor:
    """Stencils of the n_i closest nodes, self first (int32 [offsets[N]])."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    pX = _dev(X, torch.float64, "X")
    po = _dev(offsets, torch.int64, "offsets")
    if offsets.numel() != N + 1:
        raise RbfError("offsets must have N+1 entries")
    if idx is None:
        idx = torch.empty(int(offsets[-1].item()), dtype=torch.int32, device=X.device)
    pi = _dev(idx, torch.int32, "idx")
    ws_bytes = select_stencils_workspace(N, d, n_max)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    pw = _dev(workspace, torch.uint8, "workspace")
    _check(lib().rbf_select_stencils(ctx._sync_stream(), pX, N, d, po, int(n_max), pi, pw, workspace.numel()),
           "rbf_select_stencils")
    return idx


def compute_weights(X: torch.Tensor, offsets: torch.Tensor, idx: torch.Tensor, n_max: int, degree: int,
                    ops=("lap",), precision="f64", w: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, ctx: Context | None = None, **opt):
    """RBF-FD weights [len(ops), nnz] float64 and per-stencil status int8 [N]."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    nnz = idx.numel()
    ops = tuple(o for o in OPS if o in ops)
    if w is None:
        w = torch.empty((len(ops), nnz), dtype=torch.float64, device=X.device)
    if status is None:
        status = torch.empty(N, dtype=torch.int8, device=X.device)
    o = options(precision=precision, **opt)
    _check(lib().rbf_compute_weights(ctx._sync_stream(), _dev(X, torch.float64, "X"), N, d,
                                     _dev(offsets, torch.int64, "offsets"), _dev(idx, torch.int32, "idx"), nnz,
                                     int(n_max), int(degree), op_mask(ops), ctypes.byref(o),
                                     _dev(w, torch.float64, "w"), _dev(status, torch.int8, "status")),
           "rbf_compute_weights")
    return w, status


def assemble_csr(offsets: torch.Tensor, idx: torch.Tensor, w: torch.Tensor | None, n_max: int,
                 row_ptr=None, col=None, vals=None, ctx: Context | None = None):
    """CSR (row_ptr int64 [N+1], col int32 [nnz], vals float64 [R, nnz])."""
    ctx = ctx or context(offsets.device)
    N = offsets.numel() - 1
    nnz = idx.numel()
    n_ops = 0 if w is None else (w.shape[0] if w.dim() == 2 else 1)
    dev = offsets.device
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=dev) if row_ptr is None else row_ptr
    col = torch.empty(nnz, dtype=torch.int32, device=dev) if col is None else col
    if n_ops:
        vals = torch.empty((n_ops, nnz), dtype=torch.float64, device=dev) if vals is None else vals
    pw = _dev(w, torch.float64, "w") if n_ops else None
    pv = _dev(vals, torch.float64, "vals") if n_ops else None
    _check(lib().rbf_assemble_csr(ctx._sync_stream(), N, _dev(offsets, torch.int64, "offsets"),
                                  _dev(idx, torch.int32, "idx"), pw, n_ops, nnz, int(n_max),
                                  _dev(row_ptr, torch.int64, "row_ptr"), _dev(col, torch.int32, "col"), pv),
           "rbf_assemble_csr")
    return row_ptr, col, vals

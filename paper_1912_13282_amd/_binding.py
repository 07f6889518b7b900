"""ctypes binding of librbffd.so: argument marshalling only.

Tensors are passed as raw device pointers (``data_ptr()``) and every call is
enqueued on the current torch stream of the tensors' device.  Every step of the
path runs in the HIP library; there is no CPU fallback: if the library is not
built, or a tensor is not on a GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
import threading

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librbffd.so")

OPS = ("lap", "dx", "dy", "dz", "dxx", "dxy", "dxz", "dyy", "dyz", "dzz")
OP_BITS = {o: 1 << i for i, o in enumerate(OPS)}
PREC = {"f64": 0, "f32_ir": 1}

ST_OK, ST_REFINED, ST_FALLBACK, ST_SURROGATE, ST_SURROGATE_REJECTED = 0, 1, 2, 3, 4
ST_SINGULAR, ST_BADSIZE = -1, -2

_lib = None
_lock = threading.Lock()


class RbfError(RuntimeError):
    pass


class rbf_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_refine", ctypes.c_int), ("phs_power", ctypes.c_int),
                ("scale_mode", ctypes.c_int), ("repro_tol", ctypes.c_double), ("refine_tol", ctypes.c_double),
                ("surrogate_tol", ctypes.c_double), ("surrogate_corr_tol", ctypes.c_double)]


class rbf_domain_desc(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("N", ctypes.c_int64), ("d", ctypes.c_int), ("offsets", ctypes.c_void_p),
                ("idx", ctypes.c_void_p), ("nnz", ctypes.c_int64), ("degree", ctypes.c_void_p),
                ("degree_uniform", ctypes.c_int), ("n_max", ctypes.c_int), ("op_mask", ctypes.c_uint),
                ("w", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class rbf_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("residual", ctypes.c_double),
                ("true_residual", ctypes.c_double)]


class rbf_plan(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int), ("waves_per_cu", ctypes.c_int), ("ms", ctypes.c_float)]


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
    "rbf_select_stencils_static": [_P, _P, _I64, _I, _P, _I, _P],
    "rbf_compute_weights": [_P, _P, _I64, _I, _P, _P, _I64, _I, _P, _I, _U, ctypes.POINTER(rbf_options), _P, _P],
    "rbf_assemble_csr": [_P, _I64, _P, _P, _P, _I, _I64, _I, _P, _P, _P],
    "rbf_batched_workspace": [ctypes.POINTER(rbf_domain_desc), _I, ctypes.POINTER(_SZ)],
    "rbf_compute_weights_batched": [_P, ctypes.POINTER(rbf_domain_desc), _I, ctypes.POINTER(rbf_options), _P, _SZ],
    "rbf_autotune_batched": [_P, ctypes.POINTER(rbf_domain_desc), _I, ctypes.POINTER(rbf_options), _P, _SZ,
                             ctypes.c_char_p, ctypes.POINTER(rbf_plan)],
    "rbf_set_plan": [_P, ctypes.POINTER(rbf_plan)],
    "rbf_batched_class_size": [_I, ctypes.POINTER(_I)],
    "rbf_mlp_pack": [_P, _P, _P],
    "rbf_mlp_forward": [_P, _P, _P, _P, _I64, _P],
    "rbf_mlp_grad_workspace": [_I64, ctypes.POINTER(_SZ)],
    "rbf_mlp_grad": [_P, _P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, _SZ],
    "rbf_mlp_adam": [_P, _P, _P, _P, _P, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P],
    "rbf_surrogate_dataset": [_P, _P, _I64, _P, _P, _I64, _P, _P, _P, _P],
    "rbf_surrogate_load": [_P, _P],
    "rbf_surrogate_weights": [_P, _P, _I64, _I, _P, _P, _I64, _I, ctypes.POINTER(rbf_options), _P, _P],
    "rbf_get_plan": [_P, ctypes.POINTER(rbf_plan)],
    "rbf_apply_operators": [_P, _I64, _P, _P, _P, _I, _I64, _I, _P, _I64, _P],
    "rbf_combine_operators": [_P, _I64, _P, _I64, _I, _P, _I, _P, _P],
    "rbf_explicit_step": [_P, _I64, _I, _P, _P, _I64, _I, _P, _P, _P, _P, _P, _P, _P, ctypes.c_double, _P],
    "rbf_compute_weights_wls": [_P, _P, _I64, _I, _P, _P, _I64, _I, _I, _U, _I, ctypes.c_double,
                                ctypes.POINTER(rbf_options), _P, _P],
    "rbf_assemble_implicit": [_P, _I64, _I, _P, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P],
    "rbf_bicgstab_workspace": [_I64, _I64, _I, ctypes.POINTER(_SZ)],
    "rbf_bicgstab": [_P, _I64, _P, _P, _P, _I64, _I, _P, _P, ctypes.c_double, _I, _I, _P, _SZ, _P, _SZ,
                     ctypes.POINTER(rbf_solve_info)],
    "rbf_block_jacobi_size": [_I64, _I, ctypes.POINTER(_SZ)],
    "rbf_block_jacobi_setup": [_P, _P, _I64, _I, _P, _P, _P, _I64, _P, _SZ],
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
            refine_tol=0.0, surrogate_tol=1e-6, surrogate_corr_tol=0.25) -> rbf_options:
    o = rbf_options()
    _check(lib().rbf_options_default(ctypes.byref(o)), "rbf_options_default")
    o.precision = PREC[precision]
    o.max_refine = int(max_refine)
    o.phs_power = int(phs_power)
    o.scale_mode = int(scale_mode)
    o.repro_tol = float(repro_tol)
    o.refine_tol = float(refine_tol)
    o.surrogate_tol = float(surrogate_tol)
    o.surrogate_corr_tol = float(surrogate_corr_tol)
    return o


def op_mask(ops) -> int:
    m = 0
    for o in ops:
        if o not in OP_BITS:
            raise RbfError(f"unknown operator {o!r}; known: {OPS}")
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


SELECT_STATIC_BYTES = 64 * 1024 * 1024   # RBF_SELECT_STATIC_BYTES


def select_stencils_static(X: torch.Tensor, offsets: torch.Tensor, n_max: int, idx: torch.Tensor | None = None,
                           ctx: Context | None = None) -> torch.Tensor:
    """select_stencils without a workspace: the library's fixed per-device array
    (RBF_SELECT_STATIC_BYTES) holds the selection buffers; nothing is allocated
    besides idx when it is not given."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    if offsets.numel() != N + 1:
        raise RbfError("offsets must have N+1 entries")
    if idx is None:
        idx = torch.empty(int(offsets[-1].item()), dtype=torch.int32, device=X.device)
    _check(lib().rbf_select_stencils_static(ctx._sync_stream(), _dev(X, torch.float64, "X"), N, d,
                                            _dev(offsets, torch.int64, "offsets"), int(n_max),
                                            _dev(idx, torch.int32, "idx")),
           "rbf_select_stencils_static")
    return idx


def compute_weights(X: torch.Tensor, offsets: torch.Tensor, idx: torch.Tensor, n_max: int, degree,
                    ops=("lap",), precision="f64", w: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, ctx: Context | None = None,
                    degree_max: int | None = None, **opt):
    """RBF-FD weights [len(ops), nnz] float64 and per-stencil status int8 [N].

    degree: an int (every node) or a per-node int8 tensor [N]; with a tensor,
    degree_max bounds its values (default 4)."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    nnz = idx.numel()
    ops = tuple(o for o in OPS if o in ops)
    if w is None:
        w = torch.empty((len(ops), nnz), dtype=torch.float64, device=X.device)
    if status is None:
        status = torch.empty(N, dtype=torch.int8, device=X.device)
    o = options(precision=precision, **opt)
    if isinstance(degree, torch.Tensor):
        pdeg, dmax = _dev(degree, torch.int8, "degree"), (4 if degree_max is None else int(degree_max))
    else:
        pdeg, dmax = None, int(degree)
    _check(lib().rbf_compute_weights(ctx._sync_stream(), _dev(X, torch.float64, "X"), N, d,
                                     _dev(offsets, torch.int64, "offsets"), _dev(idx, torch.int32, "idx"), nnz,
                                     int(n_max), pdeg, dmax, op_mask(ops), ctypes.byref(o),
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


# ------------------------------------------------------------------ GWLS engine
WLS_WEIGHT = {"unit": 0, "gaussian": 1}


def compute_weights_wls(X: torch.Tensor, offsets: torch.Tensor, idx: torch.Tensor, n_max: int, degree: int,
                        ops=("lap",), weight: str = "gaussian", sigma: float = 1.0, w: torch.Tensor | None = None,
                        status: torch.Tensor | None = None, ctx: Context | None = None, **opt):
    """GWLS weights [len(ops), nnz] float64 (monomial basis, Sec. 2.2.1) and status int8 [N]."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    nnz = idx.numel()
    ops = tuple(o for o in OPS if o in ops)
    if weight not in WLS_WEIGHT:
        raise RbfError(f"weight must be one of {sorted(WLS_WEIGHT)}")
    if w is None:
        w = torch.empty((len(ops), nnz), dtype=torch.float64, device=X.device)
    if status is None:
        status = torch.empty(N, dtype=torch.int8, device=X.device)
    o = options(**opt)
    _check(lib().rbf_compute_weights_wls(ctx._sync_stream(), _dev(X, torch.float64, "X"), N, d,
                                         _dev(offsets, torch.int64, "offsets"), _dev(idx, torch.int32, "idx"), nnz,
                                         int(n_max), int(degree), op_mask(ops), WLS_WEIGHT[weight], float(sigma),
                                         ctypes.byref(o), _dev(w, torch.float64, "w"),
                                         _dev(status, torch.int8, "status")),
           "rbf_compute_weights_wls")
    return w, status


# ------------------------------------------------------------------ explicit evaluation
NODE_INTERIOR, NODE_DIRICHLET, NODE_NEUMANN = 0, 1, 2


def apply_operators(offsets: torch.Tensor, idx: torch.Tensor, w: torch.Tensor, n_max: int, u: torch.Tensor,
                    out=None, ctx: Context | None = None) -> torch.Tensor:
    """out [R, N] float64: out[r, i] = sum over stencil i of w[r, p] u[idx[p]] (w [R, nnz] or [nnz])."""
    ctx = ctx or context(offsets.device)
    N = offsets.numel() - 1
    nnz = idx.numel()
    w2 = w if w.dim() == 2 else w.reshape(1, -1)
    R = w2.shape[0]
    if w2.shape[1] != nnz:
        raise RbfError(f"w has {w2.shape[1]} columns, idx {nnz} entries")
    out = torch.empty((R, N), dtype=torch.float64, device=offsets.device) if out is None else out
    if out.shape != (R, N):
        raise RbfError(f"out must be [{R}, {N}], got {tuple(out.shape)}")
    _check(lib().rbf_apply_operators(ctx._sync_stream(), N, _dev(offsets, torch.int64, "offsets"),
                                     _dev(idx, torch.int32, "idx"), _dev(w2, torch.float64, "w"), R, nnz,
                                     int(n_max), _dev(u, torch.float64, "u"), u.numel(),
                                     _dev(out, torch.float64, "out")),
           "rbf_apply_operators")
    return out


def explicit_step(offsets: torch.Tensor, idx: torch.Tensor, n_max: int, w_lap: torch.Tensor, kind: torch.Tensor,
                  u: torch.Tensor, dt: float, w_grad=None, normals=None, g=None, s=None, out=None,
                  ctx: Context | None = None) -> torch.Tensor:
    """One explicit Euler step (kind uint8 [N]: NODE_INTERIOR / NODE_DIRICHLET / NODE_NEUMANN).

    w_grad [d, nnz] and normals [N, d] serve the Neumann nodes; g [N] holds the
    Dirichlet values and Neumann fluxes at the new time; s [N] the source."""
    ctx = ctx or context(offsets.device)
    N = offsets.numel() - 1
    nnz = idx.numel()
    d = normals.shape[1] if normals is not None else (w_grad.shape[0] if w_grad is not None else 2)
    if w_lap.numel() != nnz or kind.numel() != N or u.numel() != N:
        raise RbfError("w_lap must have nnz entries, kind and u N entries")
    if w_grad is not None and tuple(w_grad.shape) != (d, nnz):
        raise RbfError(f"w_grad must be [{d}, {nnz}], got {tuple(w_grad.shape)}")
    if normals is not None and tuple(normals.shape) != (N, d):
        raise RbfError(f"normals must be [{N}, {d}], got {tuple(normals.shape)}")
    for name, t in (("g", g), ("s", s)):
        if t is not None and t.numel() != N:
            raise RbfError(f"{name} must have N entries")
    out = torch.empty(N, dtype=torch.float64, device=offsets.device) if out is None else out
    if out.numel() != N:
        raise RbfError("out must have N entries")
    opt = lambda t, name: None if t is None else _dev(t, torch.float64, name)  # noqa: E731
    _check(lib().rbf_explicit_step(ctx._sync_stream(), N, d, _dev(offsets, torch.int64, "offsets"),
                                   _dev(idx, torch.int32, "idx"), nnz, int(n_max), _dev(w_lap, torch.float64, "w_lap"),
                                   opt(w_grad, "w_grad"), _dev(kind, torch.uint8, "kind"), opt(normals, "normals"),
                                   opt(g, "g"), opt(s, "s"), _dev(u, torch.float64, "u"), float(dt),
                                   _dev(out, torch.float64, "out")),
           "rbf_explicit_step")
    return out


def combine_operators(offsets: torch.Tensor, w: torch.Tensor, n_max: int, coef: torch.Tensor, out=None,
                      ctx: Context | None = None) -> torch.Tensor:
    """Weights of L = sum_k coef[:, k] op_k from stored operator rows w [K, nnz] (eq. gen-op)."""
    ctx = ctx or context(offsets.device)
    N = offsets.numel() - 1
    K, nnz = w.shape
    if tuple(coef.shape) != (N, K):
        raise RbfError(f"coef must be [{N}, {K}], got {tuple(coef.shape)}")
    out = torch.empty(nnz, dtype=torch.float64, device=offsets.device) if out is None else out
    if out.numel() != nnz:
        raise RbfError("out must have nnz entries")
    _check(lib().rbf_combine_operators(ctx._sync_stream(), N, _dev(offsets, torch.int64, "offsets"), nnz,
                                       int(n_max), _dev(w, torch.float64, "w"), K, _dev(coef, torch.float64, "coef"),
                                       _dev(out, torch.float64, "out")),
           "rbf_combine_operators")
    return out


# ------------------------------------------------------------------ implicit solution
SOLVE_CONVERGED, SOLVE_MAXITER, SOLVE_BREAKDOWN, SOLVE_BADDIAG, SOLVE_DIVERGED = 0, 1, 2, 3, 4
PRECOND = {"none": 0, "jacobi": 1, "block_jacobi": 2}


def assemble_implicit(offsets: torch.Tensor, idx: torch.Tensor, w_lap: torch.Tensor, kind: torch.Tensor,
                      w_grad=None, normals=None, f=None, g=None, d: int | None = None, vals=None, rhs=None,
                      ctx: Context | None = None):
    """(vals [nnz], rhs [N]) of the implicit system M u = r in the stencil layout."""
    ctx = ctx or context(offsets.device)
    N = offsets.numel() - 1
    nnz = idx.numel()
    if d is None:
        d = normals.shape[1] if normals is not None else (w_grad.shape[0] if w_grad is not None else 2)
    if w_lap.numel() != nnz or kind.numel() != N:
        raise RbfError("w_lap must have nnz entries and kind N entries")
    if w_grad is not None and tuple(w_grad.shape) != (d, nnz):
        raise RbfError(f"w_grad must be [{d}, {nnz}]")
    if normals is not None and tuple(normals.shape) != (N, d):
        raise RbfError(f"normals must be [{N}, {d}]")
    for name, t in (("f", f), ("g", g)):
        if t is not None and t.numel() != N:
            raise RbfError(f"{name} must have N entries")
    dev = offsets.device
    vals = torch.empty(nnz, dtype=torch.float64, device=dev) if vals is None else vals
    rhs = torch.empty(N, dtype=torch.float64, device=dev) if rhs is None else rhs
    opt = lambda t, name: None if t is None else _dev(t, torch.float64, name)  # noqa: E731
    _check(lib().rbf_assemble_implicit(ctx._sync_stream(), N, int(d), _dev(offsets, torch.int64, "offsets"),
                                       _dev(idx, torch.int32, "idx"), nnz, _dev(w_lap, torch.float64, "w_lap"),
                                       opt(w_grad, "w_grad"), _dev(kind, torch.uint8, "kind"), opt(normals, "normals"),
                                       opt(f, "f"), opt(g, "g"), _dev(vals, torch.float64, "vals"),
                                       _dev(rhs, torch.float64, "rhs")),
           "rbf_assemble_implicit")
    return vals, rhs


def bicgstab_workspace(N: int, nnz: int = 0, precond: str = "jacobi") -> int:
    """Workspace bytes of bicgstab() for N rows, nnz stored entries and the preconditioner."""
    if precond not in PRECOND:
        raise RbfError(f"precond must be one of {sorted(PRECOND)}")
    b = ctypes.c_size_t()
    _check(lib().rbf_bicgstab_workspace(N, nnz, PRECOND[precond], ctypes.byref(b)), "rbf_bicgstab_workspace")
    return b.value


def block_jacobi_size(N: int, d: int) -> int:
    """Bytes of the block-Jacobi preconditioner of an N-node system in d dimensions."""
    b = _SZ()
    _check(lib().rbf_block_jacobi_size(N, d, ctypes.byref(b)), "rbf_block_jacobi_size")
    return b.value


def block_jacobi(X: torch.Tensor, offsets: torch.Tensor, idx: torch.Tensor, vals: torch.Tensor,
                 pc: torch.Tensor | None = None, ctx: Context | None = None) -> torch.Tensor:
    """The block-Jacobi preconditioner of M (uint8 device tensor for bicgstab(pc=...))."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    nb = block_jacobi_size(N, d)
    if pc is None or pc.numel() < nb:
        pc = torch.empty(nb, dtype=torch.uint8, device=X.device)
    _check(lib().rbf_block_jacobi_setup(ctx._sync_stream(), _dev(X, torch.float64, "X"), N, d,
                                        _dev(offsets, torch.int64, "offsets"), _dev(idx, torch.int32, "idx"),
                                        _dev(vals, torch.float64, "vals"), idx.numel(),
                                        _dev(pc, torch.uint8, "pc"), pc.numel()), "rbf_block_jacobi_setup")
    return pc


def bicgstab(offsets: torch.Tensor, idx: torch.Tensor, vals: torch.Tensor, n_max: int, rhs: torch.Tensor,
             x: torch.Tensor | None = None, tol: float = 1e-10, max_iter: int = 10000, precond: str = "jacobi",
             workspace: torch.Tensor | None = None, ctx: Context | None = None, pc: torch.Tensor | None = None):
    """Solve M x = rhs by BiCGStab on the GPU; returns (x, info dict).  x (if given) is the
    initial guess and is overwritten; otherwise the solve starts from zero.  precond
    "block_jacobi" needs pc from block_jacobi() of the same matrix."""
    ctx = ctx or context(offsets.device)
    N = offsets.numel() - 1
    nnz = idx.numel()
    if vals.numel() != nnz or rhs.numel() != N:
        raise RbfError("vals must have nnz entries and rhs N entries")
    if precond not in PRECOND:
        raise RbfError(f"precond must be one of {sorted(PRECOND)}")
    x = torch.zeros(N, dtype=torch.float64, device=offsets.device) if x is None else x
    if x.numel() != N:
        raise RbfError("x must have N entries")
    ws_bytes = bicgstab_workspace(N, nnz, precond)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=offsets.device)
    info = rbf_solve_info()
    _check(lib().rbf_bicgstab(ctx._sync_stream(), N, _dev(offsets, torch.int64, "offsets"),
                              _dev(idx, torch.int32, "idx"), _dev(vals, torch.float64, "vals"), nnz, int(n_max),
                              _dev(rhs, torch.float64, "rhs"), _dev(x, torch.float64, "x"), float(tol),
                              int(max_iter), PRECOND[precond],
                              _dev(pc, torch.uint8, "pc") if pc is not None else None,
                              pc.numel() if pc is not None else 0, _dev(workspace, torch.uint8, "workspace"),
                              workspace.numel(), ctypes.byref(info)),
           "rbf_bicgstab")
    return x, {"status": info.status, "iterations": info.iterations, "residual": info.residual,
               "true_residual": info.true_residual}


# ------------------------------------------------------------------ batched form
class Domain:
    """One node set of a batched call: device tensors and stencil parameters.

    X [N, d] float64, offsets [N+1] int64, idx [nnz] int32, degree [N] int8 (or
    an int for a uniform degree), ops: tuple of operator names.  Outputs w and
    status are allocated on first use.
    """

    def __init__(self, X, offsets, idx, n_max, degree, ops):
        self.X, self.offsets, self.idx, self.n_max = X, offsets, idx, int(n_max)
        self.degree = degree
        self.ops = tuple(o for o in OPS if o in ops)
        self.w = torch.empty((len(self.ops), idx.numel()), dtype=torch.float64, device=X.device)
        self.status = torch.empty(X.shape[0], dtype=torch.int8, device=X.device)

    def desc(self) -> rbf_domain_desc:
        D = rbf_domain_desc()
        D.X = _dev(self.X, torch.float64, "X")
        D.N = self.X.shape[0]
        D.d = self.X.shape[1]
        D.offsets = _dev(self.offsets, torch.int64, "offsets")
        D.idx = _dev(self.idx, torch.int32, "idx")
        D.nnz = self.idx.numel()
        if isinstance(self.degree, torch.Tensor):
            D.degree = _dev(self.degree, torch.int8, "degree")
            D.degree_uniform = 0
        else:
            D.degree = None
            D.degree_uniform = int(self.degree)
        D.n_max = self.n_max
        D.op_mask = op_mask(self.ops)
        D.w = _dev(self.w, torch.float64, "w")
        D.status = _dev(self.status, torch.int8, "status")
        return D


def _descs(domains):
    arr = (rbf_domain_desc * len(domains))()
    for k, d in enumerate(domains):
        arr[k] = d.desc()
    return arr


def batched_workspace(domains) -> int:
    b = _SZ()
    arr = _descs(domains)
    _check(lib().rbf_batched_workspace(arr, len(domains), ctypes.byref(b)), "rbf_batched_workspace")
    return b.value


def compute_weights_batched(domains, precision="f64", workspace=None, ctx: Context | None = None, **opt):
    """Weights of every domain in one persistent launch (per precision); results in domain.w/.status."""
    ctx = ctx or context(domains[0].X.device)
    arr = _descs(domains)
    nb = batched_workspace(domains)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=domains[0].X.device)
    o = options(precision=precision, **opt)
    _check(lib().rbf_compute_weights_batched(ctx._sync_stream(), arr, len(domains), ctypes.byref(o),
                                             _dev(workspace, torch.uint8, "workspace"), workspace.numel()),
           "rbf_compute_weights_batched")
    return domains


BATCHED_CLASSES = 8   # RBF_BATCHED_CLASSES


def batched_class_sizes():
    """Largest n + m of each batched size class."""
    out = []
    for c in range(BATCHED_CLASSES):
        v = ctypes.c_int()
        _check(lib().rbf_batched_class_size(c, ctypes.byref(v)), "rbf_batched_class_size")
        out.append(v.value)
    return out


def _plans(arr):
    return [{"chunk": p.chunk, "waves_per_cu": p.waves_per_cu, "ms": p.ms} for p in arr]


def autotune_batched(domains, precision="f64", cache_path=None, workspace=None, ctx: Context | None = None, **opt):
    """Time the candidate plans on this batch class by class; each class's fastest
    becomes its plan in the context.  Returns one plan per size class."""
    ctx = ctx or context(domains[0].X.device)
    arr = _descs(domains)
    nb = batched_workspace(domains)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=domains[0].X.device)
    o = options(precision=precision, **opt)
    plans = (rbf_plan * BATCHED_CLASSES)()
    cp = cache_path.encode() if cache_path else None
    _check(lib().rbf_autotune_batched(ctx._sync_stream(), arr, len(domains), ctypes.byref(o),
                                      _dev(workspace, torch.uint8, "workspace"), workspace.numel(), cp,
                                      plans), "rbf_autotune_batched")
    return _plans(plans)


def set_plan(plans=None, ctx: Context | None = None, device=None):
    """plans: None (defaults), one (chunk, waves_per_cu) pair for every class, or a
    list of BATCHED_CLASSES dicts / pairs."""
    ctx = ctx or context(device)
    if plans is None:
        _check(lib().rbf_set_plan(ctx._h, None), "rbf_set_plan")
        return
    if isinstance(plans, tuple) and len(plans) == 2 and all(isinstance(v, int) for v in plans):
        plans = [plans] * BATCHED_CLASSES
    if len(plans) != BATCHED_CLASSES:
        raise RbfError(f"set_plan needs {BATCHED_CLASSES} plans")
    arr = (rbf_plan * BATCHED_CLASSES)()
    for c, p in enumerate(plans):
        ch, w = (p["chunk"], p["waves_per_cu"]) if isinstance(p, dict) else p
        arr[c] = rbf_plan(int(ch), int(w), 0.0)
    _check(lib().rbf_set_plan(ctx._h, arr), "rbf_set_plan")


def get_plan(ctx: Context | None = None, device=None):
    ctx = ctx or context(device)
    arr = (rbf_plan * BATCHED_CLASSES)()
    _check(lib().rbf_get_plan(ctx._h, arr), "rbf_get_plan")
    return [{"chunk": p.chunk, "waves_per_cu": p.waves_per_cu} for p in arr]


# ------------------------------------------------------------------ surrogate
MLP_NPARAM = 38927
MLP_PACKED_BYTES = 148 * 1024
MLP_SHAPES = (("W1", (128, 30)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
              ("W3", (128, 128)), ("b3", (128,)), ("W4", (15, 128)), ("b4", (15,)))


def mlp_flatten(params: dict) -> torch.Tensor:
    """Parameter dict (W1..W4 [out, in], b1..b4) -> the flat float32 layout of the library."""
    return torch.cat([torch.as_tensor(params[k]).reshape(-1).to(torch.float32) for k, _ in MLP_SHAPES])


def mlp_unflatten(flat) -> dict:
    flat = torch.as_tensor(flat)
    out, o = {}, 0
    for k, shp in MLP_SHAPES:
        n = math.prod(shp)
        out[k] = flat[o:o + n].reshape(shp)
        o += n
    return out


def _f32(t, name):
    return _dev(t, torch.float32, name)


def mlp_pack(params: torch.Tensor, packed: torch.Tensor | None = None, ctx: Context | None = None):
    ctx = ctx or context(params.device)
    if packed is None:
        packed = torch.empty(MLP_PACKED_BYTES, dtype=torch.uint8, device=params.device)
    _check(lib().rbf_mlp_pack(ctx._sync_stream(), _f32(params, "params"), _dev(packed, torch.uint8, "packed")),
           "rbf_mlp_pack")
    return packed


def mlp_forward(params, packed, x, y=None, ctx: Context | None = None):
    ctx = ctx or context(params.device)
    B = x.shape[0]
    if y is None:
        y = torch.empty((B, 15), dtype=torch.float32, device=x.device)
    _check(lib().rbf_mlp_forward(ctx._sync_stream(), _f32(params, "params"), _dev(packed, torch.uint8, "packed"),
                                 _f32(x, "x"), B, _f32(y, "y")), "rbf_mlp_forward")
    return y


def mlp_grad_workspace(B: int) -> int:
    b = _SZ()
    _check(lib().rbf_mlp_grad_workspace(int(B), ctypes.byref(b)), "rbf_mlp_grad_workspace")
    return b.value


def mlp_grad(params, packed, x, t, sel=None, B=None, grads=None, loss=None, workspace=None, ctx: Context | None = None):
    """Gradients of the mean-squared error over rows sel (or all rows) of x, t."""
    ctx = ctx or context(params.device)
    if x.dim() != 2 or t.dim() != 2 or x.shape[1] != 30 or t.shape[1] != 15 or t.shape[0] != x.shape[0]:
        raise ValueError("x must be [rows, 30] and t [rows, 15]")
    B = int(sel.numel() if sel is not None else (B if B is not None else x.shape[0]))
    if grads is None:
        grads = torch.empty(MLP_NPARAM, dtype=torch.float32, device=params.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
    nb = mlp_grad_workspace(B)
    if workspace is None or workspace.numel() < nb:
        workspace = torch.empty(nb, dtype=torch.uint8, device=params.device)
    _check(lib().rbf_mlp_grad(ctx._sync_stream(), _f32(params, "params"), _dev(packed, torch.uint8, "packed"),
                              _f32(x, "x"), _f32(t, "t"), x.shape[0],
                              _dev(sel, torch.int64, "sel") if sel is not None else None, B,
                              _f32(grads, "grads"), _f32(loss, "loss"), _dev(workspace, torch.uint8, "workspace"),
                              workspace.numel()), "rbf_mlp_grad")
    return grads, loss


def mlp_adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, packed=None, ctx: Context | None = None):
    ctx = ctx or context(params.device)
    _check(lib().rbf_mlp_adam(ctx._sync_stream(), _f32(params, "params"), _f32(grads, "grads"), _f32(m, "m"),
                              _f32(v, "v"), int(step), float(lr), float(beta1), float(beta2), float(eps),
                              _dev(packed, torch.uint8, "packed") if packed is not None else None), "rbf_mlp_adam")


def surrogate_dataset(X, offsets, idx, w_lap=None, ctx: Context | None = None):
    """(features [N,30] f32, targets [N,15] f32 or None, scale [N] f64) of 2D 15-node stencils."""
    ctx = ctx or context(X.device)
    N = X.shape[0]
    feat = torch.empty((N, 30), dtype=torch.float32, device=X.device)
    tgt = torch.empty((N, 15), dtype=torch.float32, device=X.device) if w_lap is not None else None
    scale = torch.empty(N, dtype=torch.float64, device=X.device)
    _check(lib().rbf_surrogate_dataset(ctx._sync_stream(), _dev(X, torch.float64, "X"), N,
                                       _dev(offsets, torch.int64, "offsets"), _dev(idx, torch.int32, "idx"),
                                       idx.numel(),
                                       _dev(w_lap, torch.float64, "w_lap") if w_lap is not None else None,
                                       _f32(feat, "feat"), _f32(tgt, "target") if tgt is not None else None,
                                       _dev(scale, torch.float64, "scale")), "rbf_surrogate_dataset")
    return feat, tgt, scale


def surrogate_load(params, ctx: Context | None = None):
    ctx = ctx or context(params.device)
    _check(lib().rbf_surrogate_load(ctx._sync_stream(), _f32(params, "params")), "rbf_surrogate_load")


def surrogate_weights(X, offsets, idx, n_max, w=None, status=None, ctx: Context | None = None, **opt):
    """Laplacian weights through the loaded network + projection, plain solve where rejected."""
    ctx = ctx or context(X.device)
    N, d = X.shape
    nnz = idx.numel()
    if w is None:
        w = torch.empty(nnz, dtype=torch.float64, device=X.device)
    if status is None:
        status = torch.empty(N, dtype=torch.int8, device=X.device)
    o = options(**opt)
    _check(lib().rbf_surrogate_weights(ctx._sync_stream(), _dev(X, torch.float64, "X"), N, d,
                                       _dev(offsets, torch.int64, "offsets"), _dev(idx, torch.int32, "idx"), nnz,
                                       int(n_max), ctypes.byref(o), _dev(w, torch.float64, "w"),
                                       _dev(status, torch.int8, "status")), "rbf_surrogate_weights")
    return w, status

"""Python binding of libtucker (sparse third-order Tucker decompositions by
HOOI and Multislice Projection on gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library. PyTorch provides device memory and the current stream. The library
must have been built (``python -m paper_0711_2023_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "TuckerError", "lib", "hooi", "mp", "fit", "workspace_bytes", "default_opts",
    "FP64", "FP32", "MIXED_BF16", "INIT_HOSVD", "INIT_GIVEN",
    "Result", "LIB_PATH", "SYMBOLS",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtucker.so")

TK_OK, TK_WARN_NOCONV = 0, 1
TK_ERR_ARG, TK_ERR_INDEX, TK_ERR_VALUE, TK_ERR_EMPTY, TK_ERR_WORKSPACE, TK_ERR_DEVICE = -1, -2, -3, -4, -5, -6
FP64, FP32, MIXED_BF16 = 0, 1, 2
INIT_HOSVD, INIT_GIVEN = 0, 1
ALGO_HOOI, ALGO_MP, ALGO_FIT = 0, 1, 2
_PREC = {"fp64": FP64, "fp32": FP32, "mixed": MIXED_BF16, "bf16": MIXED_BF16}

# every function declared in include/tucker.h
SYMBOLS = ["tucker_default_opts", "tucker_workspace_bytes", "tucker_hooi", "tucker_mp", "tucker_fit",
           "tucker_strerror", "tucker_step_lead_eig_workspace", "tucker_step_lead_eig"]


class tk_coo(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("nnz", ctypes.c_int64), ("dims", ctypes.POINTER(ctypes.c_int64)),
                ("idx", ctypes.c_void_p * 3), ("vals", ctypes.c_void_p)]


class tk_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("init", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("tol", ctypes.c_double), ("eig_max_iters", ctypes.c_int32), ("eig_tol", ctypes.c_double),
                ("timing", ctypes.c_int32)]


class tk_stats(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("init_ms", ctypes.c_double), ("sweeps_ms", ctypes.c_double),
                ("ttmc_ms", ctypes.c_double), ("project_ms", ctypes.c_double), ("project_calls", ctypes.c_int64),
                ("gram_ms", ctypes.c_double), ("gram_calls", ctypes.c_int64), ("eig_ms", ctypes.c_double),
                ("core_ms", ctypes.c_double),
                ("nnz_unique", ctypes.c_int64), ("eig_iters", ctypes.c_int32), ("eig_noconv", ctypes.c_int32),
                ("norm_x", ctypes.c_double)]


class TuckerError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"tucker status {status}: {text}")
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.tucker_default_opts.argtypes = [P(tk_opts)]
        L.tucker_default_opts.restype = None
        L.tucker_workspace_bytes.argtypes = [ctypes.c_int32, P(tk_coo), P(ctypes.c_int32), P(tk_opts),
                                             P(ctypes.c_size_t)]
        L.tucker_workspace_bytes.restype = ctypes.c_int
        sig = [P(tk_coo), P(ctypes.c_int32), P(tk_opts), ctypes.c_void_p, P(ctypes.c_void_p), P(ctypes.c_double),
               P(ctypes.c_int32), P(tk_stats), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        for name in ("tucker_hooi", "tucker_mp"):
            f = getattr(L, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        L.tucker_fit.argtypes = [P(tk_coo), P(ctypes.c_int32), ctypes.c_void_p, P(ctypes.c_void_p),
                                 P(ctypes.c_double), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.tucker_fit.restype = ctypes.c_int
        L.tucker_step_lead_eig_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_size_t)]
        L.tucker_step_lead_eig_workspace.restype = ctypes.c_int
        L.tucker_step_lead_eig.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, P(ctypes.c_int32), ctypes.c_double, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.tucker_step_lead_eig.restype = ctypes.c_int
        L.tucker_strerror.argtypes = [ctypes.c_int]
        L.tucker_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().tucker_strerror(int(status)).decode()


def _check(status: int):
    if status < 0:
        raise TuckerError(status, strerror(status))
    return status


def default_opts() -> tk_opts:
    o = tk_opts()
    lib().tucker_default_opts(ctypes.byref(o))
    return o


def _opts(precision="fp32", init=INIT_HOSVD, max_iters=50, tol=1e-4, eig_max_iters=None, eig_tol=None,
          timing=False) -> tk_opts:
    o = default_opts()
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.init = int(init)
    o.max_iters = int(max_iters)
    o.tol = float(tol)
    if eig_max_iters is not None:
        o.eig_max_iters = int(eig_max_iters)
    if eig_tol is not None:
        o.eig_tol = float(eig_tol)
    o.timing = 1 if timing else 0
    return o


class _Coo:
    """Keeps the ctypes view and the tensors it points to alive together."""

    def __init__(self, idx, vals, dims):
        import torch
        if idx.dtype != torch.int32 or vals.dtype != torch.float64:
            raise TypeError("idx must be int32 [3, nnz], vals float64 [nnz]")
        if not (idx.is_cuda and vals.is_cuda):
            raise TypeError("idx and vals must be on the GPU")
        self.idx = [idx[n].contiguous() for n in range(3)]
        self.vals = vals.contiguous()
        self.dims = (ctypes.c_int64 * 3)(*[int(d) for d in dims])
        self.c = tk_coo()
        self.c.order = 3
        self.c.nnz = int(vals.numel())
        self.c.dims = self.dims
        for n in range(3):
            self.c.idx[n] = self.idx[n].data_ptr()
        self.c.vals = self.vals.data_ptr()


def workspace_bytes(algo: int, idx, vals, dims, core, **opts) -> int:
    coo = _Coo(idx, vals, dims)
    J = (ctypes.c_int32 * 3)(*[int(j) for j in core])
    o = _opts(**opts)
    out = ctypes.c_size_t(0)
    _check(lib().tucker_workspace_bytes(int(algo), ctypes.byref(coo.c), J, ctypes.byref(o), ctypes.byref(out)))
    return int(out.value)


@dataclass
class Result:
    core: "object"
    factors: list
    fits: list
    iters: int
    stats: dict
    status: int


def _stats_dict(s: tk_stats) -> dict:
    return {name: getattr(s, name) for name, _ in s._fields_}


def _run(fn_name: str, algo: int, idx, vals, dims, core_dims, *, precision="fp32", init=INIT_HOSVD,
         max_iters=50, tol=1e-4, eig_max_iters=None, eig_tol=None, timing=False, factors=None, workspace=None,
         stream=None) -> Result:
    import torch
    dev = vals.device
    coo = _Coo(idx, vals, dims)
    o = _opts(precision, init, max_iters, tol, eig_max_iters, eig_tol, timing)
    J = [int(j) for j in core_dims]
    Jc = (ctypes.c_int32 * 3)(*J)
    need = ctypes.c_size_t(0)
    _check(lib().tucker_workspace_bytes(algo, ctypes.byref(coo.c), Jc, ctypes.byref(o), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    G = torch.empty(J, dtype=torch.float64, device=dev)
    if factors is None:
        facs = [torch.empty((int(dims[n]), J[n]), dtype=torch.float64, device=dev) for n in range(3)]
    else:
        facs = [f.to(device=dev, dtype=torch.float64).contiguous().clone() for f in factors]
    fptrs = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in facs])
    hist = (ctypes.c_double * max(1, int(max_iters)))()
    done = ctypes.c_int32(0)
    st = tk_stats()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    status = getattr(lib(), fn_name)(ctypes.byref(coo.c), Jc, ctypes.byref(o), G.data_ptr(), fptrs, hist,
                                     ctypes.byref(done), ctypes.byref(st), workspace.data_ptr(),
                                     int(workspace.numel()), ctypes.c_void_p(s.cuda_stream))
    _check(status)
    return Result(G, facs, [hist[i] for i in range(done.value)], int(done.value), _stats_dict(st), status)


def hooi(idx, vals, dims, core_dims, **kw) -> Result:
    """HOOI (Figure 3). idx: int32 [3, nnz] and vals: float64 [nnz] on the GPU."""
    return _run("tucker_hooi", ALGO_HOOI, idx, vals, dims, core_dims, **kw)


def mp(idx, vals, dims, core_dims, **kw) -> Result:
    """Multislice Projection (Figure 7). Same arguments as ``hooi``."""
    return _run("tucker_mp", ALGO_MP, idx, vals, dims, core_dims, **kw)


def lead_eig(M, J, tol=1e-10, warm=False, workspace=None, stream=None):
    """The J leading eigenvectors and eigenvalues of the symmetric PSD
    matrix M (float64, on the GPU). With warm=True the block left in
    `workspace` by the previous call starts the iteration. Returns
    (F, theta, matvecs, status, workspace)."""
    import torch
    n = int(M.shape[0])
    M = M.to(torch.float64).contiguous()
    need = ctypes.c_size_t(0)
    _check(lib().tucker_step_lead_eig_workspace(n, int(J), ctypes.byref(need)))
    ws = workspace
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(int(need.value), dtype=torch.uint8, device=M.device)
    F = torch.empty((n, int(J)), dtype=torch.float64, device=M.device)
    th = torch.empty(int(J), dtype=torch.float64, device=M.device)
    it = ctypes.c_int32(0)
    s = stream if stream is not None else torch.cuda.current_stream(M.device)
    st = _check(lib().tucker_step_lead_eig(M.data_ptr(), n, int(J), F.data_ptr(), th.data_ptr(), ctypes.byref(it),
                                           float(tol), 1 if warm else 0, ws.data_ptr(), int(ws.numel()),
                                           ctypes.c_void_p(s.cuda_stream)))
    return F, th, int(it.value), st, ws


def fit(idx, vals, dims, core, factors, workspace=None, stream=None) -> float:
    """fit(X, [[G; A1, A2, A3]]) for any core and factors, FP64 on the GPU."""
    import torch
    dev = vals.device
    coo = _Coo(idx, vals, dims)
    J = list(core.shape)
    Jc = (ctypes.c_int32 * 3)(*J)
    o = _opts("fp64")
    need = ctypes.c_size_t(0)
    _check(lib().tucker_workspace_bytes(ALGO_FIT, ctypes.byref(coo.c), Jc, ctypes.byref(o), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    G = core.to(device=dev, dtype=torch.float64).contiguous()
    facs = [f.to(device=dev, dtype=torch.float64).contiguous() for f in factors]
    fptrs = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in facs])
    out = ctypes.c_double(0)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib().tucker_fit(ctypes.byref(coo.c), Jc, G.data_ptr(), fptrs, ctypes.byref(out), workspace.data_ptr(),
                            int(workspace.numel()), ctypes.c_void_p(s.cuda_stream)))
    return float(out.value)

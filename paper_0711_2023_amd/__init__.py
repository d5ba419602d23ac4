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
    "TuckerError", "lib", "hooi", "mp", "sp", "hosvd", "fit", "workspace_bytes", "default_opts",
    "FP64", "FP32", "MIXED_BF16", "MIXED_BF16X3", "INIT_HOSVD", "INIT_GIVEN", "INIT_LEARNED", "INIT_RANDOM",
    "Result", "LIB_PATH", "fit_static", "mp_streamed", "mp_implicit", "SYMBOLS", "lead_eig", "learn_param_count", "learn_sketch", "learn_forward",
    "learn_backward", "learn_align", "learn_adam", "learn_test_width", "batched",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtucker.so")

TK_OK, TK_WARN_NOCONV = 0, 1
TK_ERR_ARG, TK_ERR_INDEX, TK_ERR_VALUE, TK_ERR_EMPTY, TK_ERR_WORKSPACE, TK_ERR_DEVICE = -1, -2, -3, -4, -5, -6
TK_ERR_SIZE = -7
STATIC_SCRATCH_BYTES = 64 << 20  # TK_STATIC_SCRATCH_BYTES of tucker.h
FP64, FP32, MIXED_BF16, MIXED_BF16X3 = 0, 1, 2, 3
INIT_HOSVD, INIT_GIVEN, INIT_LEARNED, INIT_RANDOM = 0, 1, 2, 3
ALGO_HOOI, ALGO_MP, ALGO_FIT, ALGO_SP, ALGO_HOSVD = 0, 1, 2, 3, 4
_PREC = {"fp64": FP64, "fp32": FP32, "mixed": MIXED_BF16, "bf16": MIXED_BF16, "bf16x3": MIXED_BF16X3,
         "mixed3": MIXED_BF16X3}

# every function declared in include/*.h
SYMBOLS = ["tucker_default_opts", "tucker_workspace_bytes", "tucker_hooi", "tucker_mp", "tucker_sp", "tucker_hosvd",
           "tucker_fit", "tucker_fit_static",
           "tucker_strerror", "tucker_step_lead_eig_workspace", "tucker_step_lead_eig",
           "tucker_learn_param_count", "tucker_learn_sketch_workspace", "tucker_learn_sketch",
           "tucker_learn_forward", "tucker_learn_backward_workspace", "tucker_learn_backward",
           "tucker_learn_test_width", "tucker_learn_align_workspace", "tucker_learn_align", "tucker_learn_adam",
           "tucker_batched_workspace_bytes", "tucker_batched", "tucker_mp_streamed_workspace", "tucker_mp_streamed",
           "tucker_mp_implicit_workspace", "tucker_mp_implicit"]


class tk_coo(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("nnz", ctypes.c_int64), ("dims", ctypes.POINTER(ctypes.c_int64)),
                ("idx", ctypes.c_void_p * 4), ("vals", ctypes.c_void_p)]


class tk_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("init", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("tol", ctypes.c_double), ("eig_max_iters", ctypes.c_int32), ("eig_tol", ctypes.c_double),
                ("timing", ctypes.c_int32), ("model", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("tune", ctypes.c_void_p), ("hosvd_fit", ctypes.c_int32), ("trace", ctypes.c_void_p)]


PHASES = ("project", "ttmc2", "gram", "eig", "core")  # TK_PHASE_* in order


class tk_event(ctypes.Structure):
    _fields_ = [("phase", ctypes.c_int32), ("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("sweep", ctypes.c_int32), ("ms", ctypes.c_double)]


class tk_trace(ctypes.Structure):
    _fields_ = [("events", ctypes.c_void_p), ("capacity", ctypes.c_int32), ("count", ctypes.c_int32),
                ("dropped", ctypes.c_int64)]


class tk_tune(ctypes.Structure):
    """Launch choices of the projection and Gram kernels (0 = the default)."""
    _fields_ = [("proj_elems", ctypes.c_int32), ("proj_min_blocks", ctypes.c_int32),
                ("gram_items", ctypes.c_int32), ("gram_min_stages", ctypes.c_int32)]

    def key(self):
        return (self.proj_elems, self.proj_min_blocks, self.gram_items, self.gram_min_stages)


def make_tune(tune) -> tk_tune:
    """A tk_tune from a tk_tune, a dict of its fields or a 4-tuple."""
    if isinstance(tune, tk_tune):
        return tune
    t = tk_tune()
    if isinstance(tune, dict):
        for k, v in tune.items():
            setattr(t, k, int(v))
    else:
        t.proj_elems, t.proj_min_blocks, t.gram_items, t.gram_min_stages = (int(v) for v in tune)
    return t


class tk_stats(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("init_ms", ctypes.c_double), ("sweeps_ms", ctypes.c_double),
                ("ttmc_ms", ctypes.c_double), ("project_ms", ctypes.c_double), ("project_calls", ctypes.c_int64),
                ("gram_ms", ctypes.c_double), ("gram_calls", ctypes.c_int64), ("eig_ms", ctypes.c_double),
                ("core_ms", ctypes.c_double),
                ("nnz_unique", ctypes.c_int64), ("eig_iters", ctypes.c_int32), ("eig_noconv", ctypes.c_int32),
                ("norm_x", ctypes.c_double), ("init_fallbacks", ctypes.c_int32), ("hosvd_fit", ctypes.c_double),
                ("core_norm", ctypes.c_double), ("ttmc_sweep_ms", ctypes.c_double * 64),
                ("streamed_bytes", ctypes.c_int64), ("streamed_slabs", ctypes.c_int64),
                ("product_fibres", ctypes.c_int64), ("product_pairs", ctypes.c_int64)]


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
        for name in ("tucker_hooi", "tucker_mp", "tucker_sp"):
            f = getattr(L, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        L.tucker_hosvd.argtypes = [P(tk_coo), P(ctypes.c_int32), P(tk_opts), ctypes.c_void_p, P(ctypes.c_void_p),
                                   P(ctypes.c_double), P(tk_stats), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.tucker_hosvd.restype = ctypes.c_int
        L.tucker_fit.argtypes = [P(tk_coo), P(ctypes.c_int32), ctypes.c_void_p, P(ctypes.c_void_p),
                                 P(ctypes.c_double), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.tucker_fit.restype = ctypes.c_int
        L.tucker_fit_static.argtypes = [P(tk_coo), P(ctypes.c_int32), ctypes.c_void_p, P(ctypes.c_void_p),
                                        P(ctypes.c_double), ctypes.c_void_p]
        L.tucker_fit_static.restype = ctypes.c_int
        L.tucker_step_lead_eig_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_size_t)]
        L.tucker_step_lead_eig_workspace.restype = ctypes.c_int
        L.tucker_step_lead_eig.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, P(ctypes.c_int32), ctypes.c_double, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.tucker_step_lead_eig.restype = ctypes.c_int
        L.tucker_strerror.argtypes = [ctypes.c_int]
        L.tucker_strerror.restype = ctypes.c_char_p
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        L.tucker_learn_param_count.argtypes = []
        L.tucker_learn_sketch_workspace.argtypes = [P(tk_coo), P(sz)]
        L.tucker_learn_sketch.argtypes = [P(tk_coo), i32, ctypes.c_uint64, vp, vp, vp, sz, vp]
        L.tucker_learn_forward.argtypes = [vp, vp, i64, vp, vp, vp, vp]
        L.tucker_learn_backward_workspace.argtypes = [i64, P(sz)]
        L.tucker_learn_backward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
        L.tucker_learn_test_width.argtypes = [i32]
        L.tucker_learn_align_workspace.argtypes = [i64, i32, i32, P(sz)]
        L.tucker_learn_align.argtypes = [vp, i64, i32, vp, i32, ctypes.c_double, P(ctypes.c_double), vp, vp, sz,
                                         vp]
        L.tucker_learn_adam.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, i32, vp]
        L.tucker_batched_workspace_bytes.argtypes = [i32, i32, P(tk_coo), P(i32), P(tk_opts), P(tk_tune), P(sz)]
        L.tucker_batched.argtypes = [i32, i32, P(tk_coo), P(i32), P(tk_opts), P(vp), P(vp), P(ctypes.c_double),
                                     P(i32), P(i32), P(tk_stats), P(tk_tune), i32, P(vp), sz, P(vp)]
        L.tucker_mp_streamed_workspace.argtypes = [P(tk_coo), P(i32), P(tk_opts), sz, P(sz)]
        L.tucker_mp_streamed.argtypes = [P(tk_coo), P(i32), P(tk_opts), sz, vp, P(vp), P(ctypes.c_double), P(i32),
                                         P(tk_stats), vp, sz, vp]
        L.tucker_mp_implicit_workspace.argtypes = [P(tk_coo), P(i32), P(tk_opts), P(sz)]
        L.tucker_mp_implicit.argtypes = [P(tk_coo), P(i32), P(tk_opts), vp, P(vp), P(ctypes.c_double), P(i32),
                                         P(tk_stats), vp, sz, vp]
        for name in SYMBOLS:
            if name.startswith("tucker_learn") or name.startswith("tucker_batched") or \
                    name.startswith("tucker_mp_streamed") or name.startswith("tucker_mp_implicit"):
                getattr(L, name).restype = ctypes.c_int
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
          timing=False, model=None, seed=None, tune=None, hosvd_fit=False) -> tk_opts:
    o = default_opts()
    o.hosvd_fit = 1 if hosvd_fit else 0
    if model is not None:
        o.model = model.data_ptr()
    if seed is not None:
        o.seed = int(seed)
    if tune is not None:
        o._tune = make_tune(tune)  # kept alive with the options
        o.tune = ctypes.addressof(o._tune)
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
            raise TypeError("idx must be int32 [N, nnz], vals float64 [nnz]")
        if not (idx.is_cuda and vals.is_cuda):
            raise TypeError("idx and vals must be on the GPU")
        self.order = len(dims)
        if self.order not in (3, 4) or idx.shape[0] != self.order:
            raise TypeError("idx must have one row per mode (3 or 4)")
        self.idx = [idx[n].contiguous() for n in range(self.order)]
        self.vals = vals.contiguous()
        self.dims = (ctypes.c_int64 * self.order)(*[int(d) for d in dims])
        self.c = tk_coo()
        self.c.order = self.order
        self.c.nnz = int(vals.numel())
        self.c.dims = self.dims
        for n in range(self.order):
            self.c.idx[n] = self.idx[n].data_ptr()
        self.c.vals = self.vals.data_ptr()


def workspace_bytes(algo: int, idx, vals, dims, core, **opts) -> int:
    coo = _Coo(idx, vals, dims)
    J = (ctypes.c_int32 * len(core))(*[int(j) for j in core])
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
    d = {name: getattr(s, name) for name, _ in s._fields_}
    d["ttmc_sweep_ms"] = list(s.ttmc_sweep_ms)
    return d


def _run(fn_name: str, algo: int, idx, vals, dims, core_dims, *, precision="fp32", init=INIT_HOSVD,
         max_iters=50, tol=1e-4, eig_max_iters=None, eig_tol=None, timing=False, factors=None, workspace=None,
         stream=None, model=None, seed=None, tune=None, hosvd_fit=False, trace=0, ws_query=None) -> Result:
    """`model`: float32 tensor of learn_param_count() parameters on the GPU,
    used with init=INIT_LEARNED. `tune`: launch choices (see make_tune).
    `trace`: room for that many per-launch events (0 = no trace); they are
    returned in Result.stats["trace"] as dicts."""
    import torch
    dev = vals.device
    coo = _Coo(idx, vals, dims)
    if model is not None and (model.dtype != torch.float32 or not model.is_cuda or not model.is_contiguous()):
        raise TypeError("model must be a contiguous float32 tensor on the GPU")
    o = _opts(precision, init, max_iters, tol, eig_max_iters, eig_tol, timing, model, seed, tune, hosvd_fit)
    tr = None
    if trace:
        evs = (tk_event * int(trace))()
        tr = tk_trace()
        tr.events = ctypes.cast(evs, ctypes.c_void_p)
        tr.capacity = int(trace)
        tr._evs = evs  # kept alive with the trace
        o.trace = ctypes.addressof(tr)
    J = [int(j) for j in core_dims]
    N = len(J)
    Jc = (ctypes.c_int32 * N)(*J)
    need = ctypes.c_size_t(0)
    if ws_query is None:
        _check(lib().tucker_workspace_bytes(algo, ctypes.byref(coo.c), Jc, ctypes.byref(o), ctypes.byref(need)))
    else:
        _check(getattr(lib(), ws_query)(ctypes.byref(coo.c), Jc, ctypes.byref(o), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    G = torch.empty(J, dtype=torch.float64, device=dev)
    if factors is None:
        facs = [torch.empty((int(dims[n]), J[n]), dtype=torch.float64, device=dev) for n in range(N)]
    else:
        facs = [f.to(device=dev, dtype=torch.float64).contiguous().clone() for f in factors]
    fptrs = (ctypes.c_void_p * N)(*[f.data_ptr() for f in facs])
    hist = (ctypes.c_double * max(1, int(max_iters)))()
    done = ctypes.c_int32(0)
    st = tk_stats()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    status = getattr(lib(), fn_name)(ctypes.byref(coo.c), Jc, ctypes.byref(o), G.data_ptr(), fptrs, hist,
                                     ctypes.byref(done), ctypes.byref(st), workspace.data_ptr(),
                                     int(workspace.numel()), ctypes.c_void_p(s.cuda_stream))
    _check(status)
    sd = _stats_dict(st)
    if tr is not None:
        sd["trace"] = [{"phase": PHASES[e.phase], "mode": e.mode, "precision": e.precision, "sweep": e.sweep,
                        "ms": e.ms} for e in tr._evs[:tr.count]]
        sd["trace_dropped"] = int(tr.dropped)
    return Result(G, facs, [hist[i] for i in range(done.value)], int(done.value), sd, status)


def hooi(idx, vals, dims, core_dims, **kw) -> Result:
    """HOOI (Figure 3; Figure 4 for a fourth-order tensor). idx: int32
    [N, nnz] (N = 3 or 4) and vals: float64 [nnz] on the GPU."""
    return _run("tucker_hooi", ALGO_HOOI, idx, vals, dims, core_dims, **kw)


def mp(idx, vals, dims, core_dims, **kw) -> Result:
    """Multislice Projection (Figure 7; Figure 8 for a fourth-order tensor).
    Same arguments as ``hooi``."""
    return _run("tucker_mp", ALGO_MP, idx, vals, dims, core_dims, **kw)


def mp_implicit(idx, vals, dims, core_dims, **kw) -> Result:
    """Multislice Projection through implicit Gram products over the
    non-empty fibres (tucker_mp_implicit): the decomposition of ``mp`` for
    tensors much sparser than the squares of their mode sizes. Same
    arguments as ``mp``; starts INIT_RANDOM (the default here) or
    INIT_GIVEN."""
    kw.setdefault("init", INIT_RANDOM)
    return _run("tucker_mp_implicit", ALGO_MP, idx, vals, dims, core_dims, ws_query="tucker_mp_implicit_workspace",
                **kw)


def sp(idx, vals, dims, core_dims, **kw) -> Result:
    """Slice Projection (Figure 5); stops on the core growth Delta_G. The
    paper's random start is init=INIT_RANDOM (the default here)."""
    kw.setdefault("init", INIT_RANDOM)
    return _run("tucker_sp", ALGO_SP, idx, vals, dims, core_dims, **kw)


def hosvd(idx, vals, dims, core_dims, precision="fp64", eig_tol=None, workspace=None, stream=None) -> Result:
    """HO-SVD (Figure 1): every factor from its unfolding Gram, then the
    core; Result.fits holds the one fit."""
    import torch
    dev = vals.device
    coo = _Coo(idx, vals, dims)
    o = _opts(precision, eig_tol=eig_tol)
    J = [int(j) for j in core_dims]
    N = len(J)
    Jc = (ctypes.c_int32 * N)(*J)
    need = ctypes.c_size_t(0)
    _check(lib().tucker_workspace_bytes(ALGO_HOSVD, ctypes.byref(coo.c), Jc, ctypes.byref(o), ctypes.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=dev)
    G = torch.empty(J, dtype=torch.float64, device=dev)
    facs = [torch.empty((int(dims[n]), J[n]), dtype=torch.float64, device=dev) for n in range(N)]
    fptrs = (ctypes.c_void_p * N)(*[f.data_ptr() for f in facs])
    out = ctypes.c_double(0)
    st = tk_stats()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    status = _check(lib().tucker_hosvd(ctypes.byref(coo.c), Jc, ctypes.byref(o), G.data_ptr(), fptrs,
                                       ctypes.byref(out), ctypes.byref(st), workspace.data_ptr(),
                                       int(workspace.numel()), ctypes.c_void_p(s.cuda_stream)))
    return Result(G, facs, [float(out.value)], 0, _stats_dict(st), status)


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


def fit_static(idx, vals, dims, core, factors, stream=None) -> float:
    """``fit`` without a workspace: the library's static device scratch
    (TK_STATIC_SCRATCH_BYTES per device) serves it. Calls that overlap on one
    device race; TuckerError(TK_ERR_SIZE) when the problem does not fit."""
    import torch
    dev = vals.device
    coo = _Coo(idx, vals, dims)
    J = list(core.shape)
    Jc = (ctypes.c_int32 * 3)(*J)
    G = core.to(device=dev, dtype=torch.float64).contiguous()
    facs = [f.to(device=dev, dtype=torch.float64).contiguous() for f in factors]
    fptrs = (ctypes.c_void_p * 3)(*[f.data_ptr() for f in facs])
    out = ctypes.c_double(0)
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    _check(lib().tucker_fit_static(ctypes.byref(coo.c), Jc, G.data_ptr(), fptrs, ctypes.byref(out),
                                   ctypes.c_void_p(s.cuda_stream)))
    return float(out.value)


class _HostCoo:
    """A tk_coo over host arrays (the streamed entry point reads them there)."""

    def __init__(self, idx, vals, dims):
        import numpy as np
        self.idx = [np.ascontiguousarray(idx[n], dtype=np.int32) for n in range(3)]
        self.vals = np.ascontiguousarray(vals, dtype=np.float64)
        self.dims = (ctypes.c_int64 * 3)(*[int(d) for d in dims])
        self.c = tk_coo()
        self.c.order = 3
        self.c.nnz = int(self.vals.size)
        self.c.dims = self.dims
        for n in range(3):
            self.c.idx[n] = self.idx[n].ctypes.data
        self.c.vals = self.vals.ctypes.data


def mp_streamed(idx, vals, dims, core_dims, slab_bytes, precision="fp32", init=INIT_RANDOM, max_iters=50, tol=1e-4,
                eig_max_iters=None, eig_tol=None, seed=None, factors=None, workspace=None, stream=None,
                device="cuda") -> Result:
    """MP of a tensor in HOST memory (numpy int32 [3, nnz] and float64 [nnz]),
    streamed through two device slab buffers of slab_bytes each. Results on
    the device as for ``mp``."""
    import torch
    dev = torch.device(device)
    coo = _HostCoo(idx, vals, dims)
    o = _opts(precision, init, max_iters, tol, eig_max_iters, eig_tol, False, None, seed)
    J = [int(j) for j in core_dims]
    Jc = (ctypes.c_int32 * 3)(*J)
    need = ctypes.c_size_t(0)
    _check(lib().tucker_mp_streamed_workspace(ctypes.byref(coo.c), Jc, ctypes.byref(o), int(slab_bytes),
                                              ctypes.byref(need)))
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
    status = _check(lib().tucker_mp_streamed(ctypes.byref(coo.c), Jc, ctypes.byref(o), int(slab_bytes),
                                             G.data_ptr(), fptrs, hist, ctypes.byref(done), ctypes.byref(st),
                                             workspace.data_ptr(), int(workspace.numel()),
                                             ctypes.c_void_p(s.cuda_stream)))
    return Result(G, facs, [hist[i] for i in range(done.value)], int(done.value), _stats_dict(st), status)


# ---------------------------------------------------------------- learned start
def _stream_ptr(dev, stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    return ctypes.c_void_p(s.cuda_stream)


def learn_param_count() -> int:
    return int(lib().tucker_learn_param_count())


def learn_sketch(idx, vals, dims, mode: int, seed: int, stream=None):
    """Row features (In x 64) and row norms (In) of the mode's sketch."""
    import torch
    coo = _Coo(idx, vals, dims)
    need = ctypes.c_size_t(0)
    _check(lib().tucker_learn_sketch_workspace(ctypes.byref(coo.c), ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=vals.device)
    In = int(dims[mode])
    F = torch.empty((In, 64), dtype=torch.float32, device=vals.device)
    rho = torch.empty(In, dtype=torch.float32, device=vals.device)
    _check(lib().tucker_learn_sketch(ctypes.byref(coo.c), int(mode), ctypes.c_uint64(int(seed)), F.data_ptr(),
                                     rho.data_ptr(), ws.data_ptr(), int(ws.numel()),
                                     _stream_ptr(vals.device, stream)))
    return F, rho


def learn_forward(F, rho, params, want_z1=True, stream=None):
    """Network output R (rows x 128) and the hidden pre-activations."""
    import torch
    rows = int(F.shape[0])
    R = torch.empty((rows, 128), dtype=torch.float32, device=F.device)
    Z1 = torch.empty((rows, 128), dtype=torch.float32, device=F.device) if want_z1 else None
    _check(lib().tucker_learn_forward(F.data_ptr(), rho.data_ptr(), rows, params.data_ptr(), R.data_ptr(),
                                      Z1.data_ptr() if Z1 is not None else None, _stream_ptr(F.device, stream)))
    return R, Z1


def learn_backward(F, rho, params, Z1, dR, stream=None):
    """Gradient of a scalar w.r.t. the parameters given its gradient dR."""
    import torch
    rows = int(F.shape[0])
    need = ctypes.c_size_t(0)
    _check(lib().tucker_learn_backward_workspace(rows, ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=F.device)
    g = torch.empty(learn_param_count(), dtype=torch.float32, device=F.device)
    _check(lib().tucker_learn_backward(F.data_ptr(), rho.data_ptr(), rows, params.data_ptr(), Z1.data_ptr(),
                                       dR.data_ptr(), g.data_ptr(), ws.data_ptr(), int(ws.numel()),
                                       _stream_ptr(F.device, stream)))
    return g


def learn_test_width(J: int) -> int:
    return int(_check(lib().tucker_learn_test_width(int(J))))


def learn_align(R, K: int, A, shift=1e-8, want_grad=True, stream=None):
    """(loss, dL/dR or None): how much of span(A) lies outside the span of
    R's first K columns."""
    import torch
    rows = int(R.shape[0])
    J = int(A.shape[1])
    need = ctypes.c_size_t(0)
    _check(lib().tucker_learn_align_workspace(rows, int(K), J, ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device=R.device)
    A = A.to(torch.float64).contiguous()
    dR = torch.empty((rows, 128), dtype=torch.float32, device=R.device) if want_grad else None
    loss = ctypes.c_double(0)
    _check(lib().tucker_learn_align(R.data_ptr(), rows, int(K), A.data_ptr(), J, float(shift), ctypes.byref(loss),
                                    dR.data_ptr() if dR is not None else None, ws.data_ptr(), int(ws.numel()),
                                    _stream_ptr(R.device, stream)))
    return float(loss.value), dR


def learn_adam(params, grad, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().tucker_learn_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                   int(params.numel()), float(lr), float(beta1), float(beta2), float(eps), int(step),
                                   _stream_ptr(params.device, stream)))


# ---------------------------------------------------------------- many tensors
def batched(algo: int, tensors, cores, nstreams: int = 8, streams=None, workspaces=None, tunes=None, **opts):
    """Decompose many tensors in one call (ALGO_MP or ALGO_HOOI): `tensors` is
    a list of (idx, vals, dims) on the GPU, `cores` the core sizes. Returns
    (list of Result, overall status). The streams (default: `nstreams` new
    ones) and per-stream workspaces can be passed in to reuse them; `tunes`
    (one launch choice per tensor, see make_tune) overrides the shared one."""
    import torch
    count = len(tensors)
    dev = tensors[0][1].device
    coos = [_Coo(i, v, d) for (i, v, d) in tensors]
    carr = (tk_coo * count)(*[c.c for c in coos])
    J = [int(j) for core in cores for j in core]
    Jc = (ctypes.c_int32 * (3 * count))(*J)
    o = _opts(**opts)
    tarr = None
    if tunes is not None:
        if len(tunes) != count:
            raise ValueError("one tune per tensor")
        tarr = (tk_tune * count)(*[make_tune(t) for t in tunes])
    need = ctypes.c_size_t(0)
    _check(lib().tucker_batched_workspace_bytes(int(algo), count, carr, Jc, ctypes.byref(o), tarr,
                                                ctypes.byref(need)))
    if streams is None:
        streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    nstreams = len(streams)
    if workspaces is None or any(w.numel() < need.value for w in workspaces):
        workspaces = [torch.empty(int(need.value), dtype=torch.uint8, device=dev) for _ in range(nstreams)]
    Gs = [torch.empty(tuple(int(x) for x in core), dtype=torch.float64, device=dev) for core in cores]
    facs = [[torch.empty((int(d[n]), int(core[n])), dtype=torch.float64, device=dev) for n in range(3)]
            for (_, _, d), core in zip(tensors, cores)]
    cptr = (ctypes.c_void_p * count)(*[g.data_ptr() for g in Gs])
    fptr = (ctypes.c_void_p * (3 * count))(*[f.data_ptr() for fs in facs for f in fs])
    mi = max(1, int(o.max_iters))
    hist = (ctypes.c_double * (mi * count))()
    done = (ctypes.c_int32 * count)()
    stat = (ctypes.c_int32 * count)()
    sts = (tk_stats * count)()
    wptr = (ctypes.c_void_p * nstreams)(*[w.data_ptr() for w in workspaces])
    sptr = (ctypes.c_void_p * nstreams)(*[s.cuda_stream for s in streams])
    torch.cuda.synchronize(dev)  # inputs are complete before the workers start
    overall = lib().tucker_batched(int(algo), count, carr, Jc, ctypes.byref(o), cptr, fptr, hist, done, stat, sts,
                                   tarr, nstreams, wptr, int(need.value), sptr)
    _check(overall)
    hm = int(o.max_iters)
    res = [Result(Gs[t], facs[t], [hist[hm * t + i] for i in range(done[t])], int(done[t]), _stats_dict(sts[t]),
                  int(stat[t])) for t in range(count)]
    return res, overall

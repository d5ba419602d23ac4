"""Launch-choice tuner of the projection and Gram kernels.

The projection's run length (slots per workgroup) and the Gram's split-K
factor decide how many workgroups a launch has and how much each does. The
best choice depends on the tensor's shape: a small tensor needs short runs to
fill 256 compute units, a large one longer runs to amortise the staging. The
projection's choices change no result bit (each output sums its nonzeros in
the same order); the Gram's change where its FP32 partial sums split the
summed dimension, so results move within rounding but stay deterministic for
a given choice (both checked by the GPU tests). Either way they can be picked
by measurement alone.

The tuner times one short decomposition per candidate with the library's own
HIP-event timers (tk_stats.project_ms and gram_ms), picks the projection
choice first and the Gram choice with it, and caches the winner per shape
bucket (algorithm, precision, nonzeros and largest mode to the nearest power
of two, largest core size to a multiple of 16) in a JSON file. A candidate
replaces the built-in choice only when it is faster by more than `margin`.
"""
from __future__ import annotations

import json
import math
import os

from . import ALGO_HOOI, ALGO_MP, hooi, make_tune, mp, tk_tune

# (proj_elems, proj_min_blocks); (0, 0) is the built-in (32768, 1536)
PROJ_CANDIDATES = ((0, 0), (16384, 1536), (65536, 1536), (32768, 512), (32768, 4096), (8192, 4096), (16384, 4096))
GRAM_ITEMS = (0, 256, 512, 2048, 4096)   # 0 is the built-in 1024
GRAM_STAGES = (0, 2, 8)                  # 0 is the built-in 4

_ALGO_NAME = {ALGO_MP: "mp", ALGO_HOOI: "hooi"}


def bucket(algo: int, precision: str, dims, nnz: int, core) -> str:
    """The cache key of one tensor shape."""
    lg = lambda x: int(round(math.log2(max(1, int(x)))))
    j16 = 16 * math.ceil(max(int(j) for j in core) / 16)
    return f"{_ALGO_NAME[int(algo)]}/{precision}/nnz~2^{lg(nnz)}/I~2^{lg(max(int(d) for d in dims))}/J<={j16}"


class TuneCache:
    """bucket -> launch choice (and the times that chose it), as JSON."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.entries: dict = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, key: str) -> tk_tune | None:
        e = self.entries.get(key)
        return make_tune(e["tune"]) if e else None

    def put(self, key: str, tune: tk_tune, info: dict):
        self.entries[key] = {"tune": list(tune.key()), **info}

    def save(self, path: str | None = None):
        path = path or self.path
        if not path:
            raise ValueError("no cache path")
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, path)


def _time(algo, idx, vals, dims, core, tune, precision, sweeps, reps):
    run = mp if int(algo) == ALGO_MP else hooi
    best_p = best_g = float("inf")
    for _ in range(reps):
        st = run(idx, vals, dims, core, precision=precision, max_iters=sweeps, tol=0.0, timing=True,
                 tune=tune).stats
        best_p = min(best_p, st["project_ms"])
        best_g = min(best_g, st["gram_ms"])
    return best_p, best_g


def tune_tensor(algo: int, idx, vals, dims, core, precision: str = "mixed", cache: TuneCache | None = None,
                sweeps: int = 1, reps: int = 2, margin: float = 0.03, log=None) -> tk_tune:
    """The launch choice for this tensor's bucket: from `cache` if it holds
    one, else measured (and stored in `cache`)."""
    key = bucket(algo, precision, dims, int(vals.numel()), core)
    if cache is not None:
        hit = cache.get(key)
        if hit is not None:
            return hit
    _time(algo, idx, vals, dims, core, None, precision, sweeps, 1)  # first-call costs out of the way
    base_p, base_g = _time(algo, idx, vals, dims, core, None, precision, sweeps, reps)
    pe, pb, best_p = 0, 0, base_p
    for cpe, cpb in PROJ_CANDIDATES[1:]:
        t, _ = _time(algo, idx, vals, dims, core, (cpe, cpb, 0, 0), precision, sweeps, reps)
        if t < best_p * (1.0 - margin) and t < base_p * (1.0 - margin):
            pe, pb, best_p = cpe, cpb, t
    gi, gs, best_g = 0, 0, base_g
    for cgi in GRAM_ITEMS[1:]:
        _, t = _time(algo, idx, vals, dims, core, (pe, pb, cgi, 0), precision, sweeps, reps)
        if t < best_g * (1.0 - margin):
            gi, best_g = cgi, t
    for cgs in GRAM_STAGES[1:]:
        _, t = _time(algo, idx, vals, dims, core, (pe, pb, gi, cgs), precision, sweeps, reps)
        if t < best_g * (1.0 - margin):
            gs, best_g = cgs, t
    tune = make_tune((pe, pb, gi, gs))
    info = {"project_ms": [base_p, best_p], "gram_ms": [base_g, best_g]}
    if log:
        log(f"{key}: tune {tune.key()} projection {base_p:.3f} -> {best_p:.3f} ms, "
            f"Gram {base_g:.3f} -> {best_g:.3f} ms")
    if cache is not None:
        cache.put(key, tune, info)
    return tune


def tune_batch(algo: int, tensors, cores, precision: str = "mixed", cache: TuneCache | None = None,
               **kw) -> list:
    """One launch choice per tensor of a many-tensor call (tensors: list of
    (idx, vals, dims)); each bucket is measured once, on its first tensor."""
    cache = cache if cache is not None else TuneCache()
    return [tune_tensor(algo, i, v, d, J, precision, cache, **kw) for (i, v, d), J in zip(tensors, cores)]

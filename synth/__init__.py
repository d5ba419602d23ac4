"""Seeded synthetic sparse third-order tensors.

This module only draws inputs. It holds none of the decomposition's arithmetic,
and both the FP64 oracle and the GPU library are fed from it. Every generator
returns host arrays:

* ``idx``  int32 array of shape (N, nnz), 0-based coordinates (N = 3, or 4
  for the fourth-order generators and shapes);
* ``vals`` float64 array of shape (nnz,);
* ``dims`` tuple of N ints.

The workload family is the paper's: random sparse third-order tensors whose
nonzero values are uniform on [0, 1) (Section 5, "Varying Tensor Sizes"; the
appendix generator draws a Bernoulli cell mask and uniform values). Here the
number of nonzeros is fixed and coordinates are distinct, sampled uniformly
without replacement with numpy's PCG64 generator.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_sparse",
    "bernoulli_sparse",
    "exact_tucker_block",
    "exact_tucker_block_n",
    "superdiagonal",
    "matrix_as_tensor",
    "planted_tucker",
    "skewed_sparse",
    "batch_configs",
    "with_duplicates",
    "WORKLOADS",
]


def _unravel(lin: np.ndarray, dims) -> np.ndarray:
    return np.stack(np.unravel_index(lin, dims)).astype(np.int32)


def _distinct_linear(total: int, nnz: int, rng: np.random.Generator) -> np.ndarray:
    """nnz distinct integers drawn uniformly from [0, total), in random order."""
    if nnz > total:
        raise ValueError("more nonzeros than cells")
    if total <= 50_000_000 or nnz * 4 > total:
        return rng.choice(total, size=nnz, replace=False).astype(np.int64)
    picked = np.empty(0, dtype=np.int64)
    while picked.size < nnz:
        need = nnz - picked.size
        draw = rng.integers(0, total, size=int(need * 1.05) + 16, dtype=np.int64)
        picked = np.unique(np.concatenate([picked, draw]))
    # unique() sorted them: keep a uniformly random subset, in random order
    return rng.permutation(picked)[:nnz]


def uniform_sparse(dims, nnz: int, seed: int):
    """nnz distinct uniformly random coordinates with U(0,1) values (any
    number of modes: idx has one row per mode)."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    lin = _distinct_linear(int(np.prod(dims, dtype=np.int64)), int(nnz), rng)
    vals = rng.random(lin.size)
    return _unravel(lin, dims), vals, dims


def bernoulli_sparse(dims, density: float, seed: int):
    """Each cell is nonzero with probability ``density``; values U(0,1) (any
    number of modes).

    This is the appendix generator's distribution (a cell mask drawn by
    comparing a uniform number with the density, then a uniform value).
    """
    dims = tuple(int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    total = int(np.prod(dims, dtype=np.int64))
    lins = []
    chunk = 1 << 24
    for start in range(0, total, chunk):
        n = min(chunk, total - start)
        mask = rng.random(n) < density
        lins.append(np.nonzero(mask)[0].astype(np.int64) + start)
    lin = np.concatenate(lins)
    vals = rng.random(lin.size)
    perm = rng.permutation(lin.size)
    return _unravel(lin[perm], dims), vals[perm], dims


def exact_tucker_block_n(dims, block, rank, seed: int):
    """Any order: zero except on a random index block, where it equals a dense
    Tucker tensor of multilinear rank ``rank``."""
    dims = tuple(int(d) for d in dims)
    N = len(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = [np.sort(rng.choice(dims[n], size=block[n], replace=False)) for n in range(N)]
    dense = rng.standard_normal(rank)
    for n in range(N):
        f = _orthonormal(block[n], rank[n], rng)
        dense = np.moveaxis(np.tensordot(f, np.moveaxis(dense, n, 0), axes=(1, 0)), 0, n)
    grids = np.meshgrid(*rows, indexing="ij")
    idx = np.stack([g.ravel() for g in grids]).astype(np.int32)
    vals = dense.ravel().copy()
    perm = rng.permutation(vals.size)
    return idx[:, perm], vals[perm], dims


def _orthonormal(n: int, r: int, rng: np.random.Generator) -> np.ndarray:
    q, rr = np.linalg.qr(rng.standard_normal((n, r)))
    return q * np.sign(np.diag(rr))


def exact_tucker_block(dims, block, rank, seed: int):
    """A tensor that is zero except on a random index block, where it equals
    a dense Tucker tensor of multilinear rank ``rank``. Its exact Tucker rank
    is ``rank``, so a decomposition with core >= rank reproduces it."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = [np.sort(rng.choice(dims[n], size=block[n], replace=False)) for n in range(3)]
    core = rng.standard_normal(rank)
    fac = [_orthonormal(block[n], rank[n], rng) for n in range(3)]
    dense = np.einsum("pqr,ip,jq,kr->ijk", core, fac[0], fac[1], fac[2])
    ii, jj, kk = np.meshgrid(*rows, indexing="ij")
    idx = np.stack([ii.ravel(), jj.ravel(), kk.ravel()]).astype(np.int32)
    vals = dense.ravel().copy()
    perm = rng.permutation(vals.size)
    return idx[:, perm], vals[perm], dims


def superdiagonal(n: int, seed: int):
    """x_iii = d_i with distinct |d_i| in [1, 2), all other cells zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = 1.0 + rng.permutation(n) / n + rng.random(n) * (0.5 / n)
    d *= rng.choice([-1.0, 1.0], size=n)
    i = np.arange(n, dtype=np.int32)
    return np.stack([i, i, i]), d, (n, n, n)


def matrix_as_tensor(rows: int, cols: int, nnz: int, seed: int):
    """A sparse I1 x I2 x 1 tensor: a matrix with one trivial third mode."""
    idx, vals, _ = uniform_sparse((rows, cols, 1), nnz, seed)
    return idx, vals, (rows, cols, 1)


def planted_tucker(dims, core, nnz: int, noise: float, seed: int):
    """Values of a random Tucker model sampled at distinct uniform coordinates.

    Factors are the Q of a QR of a Gaussian matrix, the core is i.i.d. N(0,1).
    The sampled values are scaled to unit RMS, then i.i.d. N(0, noise^2) is
    added. Evaluation groups the coordinates by their first index so that
    each horizontal model slice is formed once.
    """
    dims = tuple(int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    fac = [_orthonormal(dims[n], core[n], rng) for n in range(3)]
    g = rng.standard_normal(tuple(core))
    lin = _distinct_linear(int(np.prod(dims, dtype=np.int64)), int(nnz), rng)
    idx = _unravel(lin, dims)
    vals = np.empty(lin.size)
    order = np.argsort(idx[0], kind="stable")
    starts = np.searchsorted(idx[0][order], np.arange(dims[0] + 1))
    g1 = g.reshape(core[0], -1)
    for i in range(dims[0]):
        sel = order[starts[i]:starts[i + 1]]
        if sel.size == 0:
            continue
        h = (fac[0][i] @ g1).reshape(core[1], core[2])          # core slice for row i
        bj = fac[1][idx[1][sel]]                                # rows of B
        ck = fac[2][idx[2][sel]]                                # rows of C
        vals[sel] = ((bj @ h) * ck).sum(axis=1)                # b_j^T H_i c_k per nonzero
    vals /= np.sqrt(np.mean(vals * vals))
    vals += noise * rng.standard_normal(vals.size)
    return idx, vals, dims


def skewed_sparse(dims, nnz: int, s: float, seed: int):
    """nnz distinct coordinates whose every index follows a truncated Zipf
    law, P(i) proportional to (i + 1)^-s on [0, I_m), drawn independently per
    mode, with U(0,1) values: a few slices and fibres hold most of the
    nonzeros, as in term-frequency tensors, and the fibres near the origin are
    dense. Duplicate draws are dropped and drawing continues until nnz distinct
    cells are found."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    cdf = []
    for d in dims:
        w = (np.arange(1, d + 1, dtype=np.float64)) ** (-float(s))
        c = np.cumsum(w)
        cdf.append(c / c[-1])
    total = int(np.prod(dims, dtype=np.int64))
    if nnz > total // 2:
        raise ValueError("too many nonzeros for a skewed draw")
    picked = np.empty(0, dtype=np.int64)
    for _ in range(200):
        need = nnz - picked.size
        if need <= 0:
            break
        m = int(need * 1.3) + 64
        lin = np.zeros(m, dtype=np.int64)
        for c, d in zip(cdf, dims):
            i = np.minimum(np.searchsorted(c, rng.random(m), side="right"), d - 1)
            lin = lin * d + i
        picked = np.unique(np.concatenate([picked, lin]))
    if picked.size < nnz:
        raise ValueError("skewed draw did not reach nnz distinct cells")
    lin = rng.permutation(picked)[:nnz]
    idx = _unravel(lin, dims)
    vals = rng.random(nnz)
    return idx, vals, dims


def with_duplicates(idx, vals, ndup: int, seed: int):
    """Append ``ndup`` repeated coordinates (with new values), shuffled in."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.integers(0, vals.size, size=ndup)
    idx2 = np.concatenate([idx, idx[:, pick]], axis=1)
    vals2 = np.concatenate([vals, rng.random(ndup)])
    perm = rng.permutation(vals2.size)
    return idx2[:, perm].copy(), vals2[perm].copy()


def batch_configs(count: int = 64, seed_base: int = 3000):
    """Shapes of the batched workload: mode sizes U{200..800}, cores U{10..40},
    density 0.5 %, one seed per tensor."""
    out = []
    for t in range(count):
        rng = np.random.Generator(np.random.PCG64(seed_base + t))
        dims = tuple(int(x) for x in rng.integers(200, 801, size=3))
        core = tuple(int(x) for x in rng.integers(10, 41, size=3))
        nnz = int(round(0.005 * np.prod(dims, dtype=np.int64)))
        out.append({"dims": dims, "core": core, "nnz": nnz, "seed": seed_base + t})
    return out


# Named workloads (sizes of the benchmarked configurations).
WORKLOADS = {
    "cube100_nnz10k": {"dims": (100, 100, 100), "nnz": 10_000, "core": (10, 10, 10), "seed": 5678},
    "cube1000_nnz1m": {"dims": (1000, 1000, 1000), "nnz": 1_000_000, "core": (50, 50, 50), "seed": 1},
    "unbal_2000x1000x500_core100x20x5": {"dims": (2000, 1000, 500), "nnz": 2_000_000, "core": (100, 20, 5), "seed": 2},
    "unbal_2000x1000x500_core10x50x100": {"dims": (2000, 1000, 500), "nnz": 2_000_000, "core": (10, 50, 100), "seed": 2},
    "cube4000_nnz10m_planted": {"dims": (4000, 4000, 4000), "nnz": 10_000_000, "core": (100, 100, 100), "seed": 4},
    # fourth order, the paper's shape (Table 5): 100^4 at 10 % density, cores 10^4 .. 90^4
    "hyper100_nnz10m": {"dims": (100, 100, 100, 100), "nnz": 10_000_000, "core": (50, 50, 50, 50), "seed": 6},
}

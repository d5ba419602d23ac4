"""Parity at the benchmarked sizes, in the configurations the benchmark runs.

At these sizes the oracle's whole decomposition takes minutes, so the checks
are ones the oracle can make one output at a time, and properties that hold
at any size:

* sampled core entries G[p, q, r] = sum x_ijk A[i,p] B[j,q] C[k,r] (the n-mode
  product definition, Section 3) computed by the oracle from the GPU's own
  returned factors, against the GPU core (FP32/BF16 projections feed an FP64
  core: 1e-5 of the core's largest entry);
* the per-sweep fit from the identity against the general fit formula on the
  returned core and factors (FP64, 1e-7);
* orthonormal factors (1e-10) and the fit between 0 and 1.

Workloads: 1000^3 with 1M nonzeros and core 50^3 (the benchmark), 2000 x 1000
x 500 with 2M nonzeros and cores (100, 20, 5) and (10, 50, 100), eight of the
64 tensors of the many-tensor workload (run through the many-tensor call),
and the 4000^3 / 10M / core 100^3 shape with uniform U(0,1) values standing in
for the planted values (the planted generator needs about 1e11 host flops at
that size).
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0711_2023_amd as m
    m.lib()
    return m


def _dev(idx, vals):
    return (torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float64)).cuda())


def _check(tk, X, di, dv, dims, J, res, nsample=24, seed=0):
    G = res.core.cpu().numpy()
    A, B, C = (f.cpu().numpy() for f in res.factors)
    for F in (A, B, C):
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-10
    rng = np.random.default_rng(seed)
    scale = np.abs(G).max()
    picks = [(0, 0, 0)] + [tuple(int(rng.integers(j)) for j in J) for _ in range(nsample)]
    for p, q, r in picks:
        g = O.core_entry(X, A, B, C, p, q, r)
        assert abs(G[p, q, r] - g) <= 1e-5 * scale, ((p, q, r), G[p, q, r], g)
    f_general = tk.fit(di, dv, dims, res.core, res.factors)
    assert abs(f_general - res.fits[-1]) <= 1e-7, (f_general, res.fits[-1])
    assert 0.0 < res.fits[-1] < 1.0


@pytest.fixture(scope="module")
def cube1000():
    w = synth.WORKLOADS["cube1000_nnz1m"]
    idx, vals, dims = synth.uniform_sparse(tuple(w["dims"]), int(w["nnz"]), w["seed"])
    return idx, vals, dims, tuple(w["core"]), O.SparseTensor3(idx, vals, dims)


@pytest.mark.parametrize("algo,prec", [("mp", "mixed"), ("mp", "fp32"), ("hooi", "mixed")])
def test_cube1000(tk, cube1000, algo, prec):
    idx, vals, dims, J, X = cube1000
    _say(f"1000^3 {algo} {prec}")
    di, dv = _dev(idx, vals)
    res = getattr(tk, algo)(di, dv, dims, J, precision=prec, max_iters=3, tol=0.0)
    _check(tk, X, di, dv, dims, J, res)


@pytest.mark.parametrize("name", ["unbal_2000x1000x500_core100x20x5", "unbal_2000x1000x500_core10x50x100"])
@pytest.mark.parametrize("algo", ["mp", "hooi"])
def test_unbalanced(tk, name, algo):
    w = synth.WORKLOADS[name]
    idx, vals, dims = synth.uniform_sparse(tuple(w["dims"]), int(w["nnz"]), w["seed"])
    J = tuple(w["core"])
    _say(f"{name} {algo} mixed")
    X = O.SparseTensor3(idx, vals, dims)
    di, dv = _dev(idx, vals)
    res = getattr(tk, algo)(di, dv, dims, J, precision="mixed", max_iters=2, tol=0.0)
    _check(tk, X, di, dv, dims, J, res)


def test_many_tensor_workload_sample(tk):
    cfgs = synth.batch_configs(64, 3000)[:8]
    tensors, cores, Xs = [], [], []
    for c in cfgs:
        idx, vals, dims = synth.uniform_sparse(c["dims"], c["nnz"], c["seed"])
        tensors.append((*_dev(idx, vals), dims))
        cores.append(c["core"])
        Xs.append(O.SparseTensor3(idx, vals, dims))
    _say("many-tensor workload, first 8 tensors, 4 streams")
    res, st = tk.batched(tk.ALGO_MP, tensors, cores, nstreams=4, precision="mixed", max_iters=3, tol=0.0)
    assert st >= 0
    for (di, dv, dims), J, X, r in zip(tensors, cores, Xs, res):
        _check(tk, X, di, dv, dims, J, r, nsample=8)


def test_cube4000_shape(tk):
    w = synth.WORKLOADS["cube4000_nnz10m_planted"]
    _say("4000^3 / 10M: generating (uniform values)")
    idx, vals, dims = synth.uniform_sparse(tuple(w["dims"]), int(w["nnz"]), w["seed"])
    J = tuple(w["core"])
    di, dv = _dev(idx, vals)
    _say("4000^3 / 10M: MP mixed, one sweep")
    res = tk.mp(di, dv, dims, J, precision="mixed", max_iters=1, tol=0.0)
    _say(f"4000^3 / 10M: fit {res.fits[-1]:.6e}; oracle sampling")
    X = O.SparseTensor3(idx, vals, dims)
    _check(tk, X, di, dv, dims, J, res, nsample=12)

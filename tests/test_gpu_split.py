"""Split-BF16 Grams (TK_MIXED_BF16X3, MP only): each projection stored as a
BF16 pair (rounded value and rounded remainder, from FP32 factor rows), the
Gram as hi hi^T + hi lo^T + lo hi^T on BF16 MFMA with FP32 accumulation.

* Against the FP64 oracle's stored MP run on the small uniform tensor (10
  sweeps from the HO-SVD start, tests/golden/small_reference.npz, pinned to
  the oracle by a CPU test): the fit per sweep within 1e-6 and every factor
  subspace within 1e-3 rad — the tensor on which plain BF16 Grams leave the
  subspace undetermined (its J-th eigenvalue gap is below BF16 rounding).
* At the benchmark size (1000^3, 1M nonzeros, core 50^3): sampled core
  entries G[p,q,r] = sum x_ijk A[i,p] B[j,q] C[k,r] (Section 3) from the
  returned factors, the fit identity against the general fit, orthonormal
  factors.
* HOOI rejects the precision.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def _angle(A, B):
    return O.subspace_angle(A, B)


@pytest.mark.parametrize("case", ["uniform", "planted"])
def test_split_mp_matches_stored_oracle(tk, case):
    ref = np.load(os.path.join(ROOT, "tests", "golden", "small_reference.npz"), allow_pickle=False)
    dims = tuple(int(x) for x in ref[f"{case}_dims"])
    J = tuple(int(x) for x in ref[f"{case}_core"])
    nnz, seed = int(ref[f"{case}_nnz"]), int(ref[f"{case}_seed"])
    if case == "uniform":
        idx, vals, dims = synth.uniform_sparse(dims, nnz, seed)
    else:
        idx, vals, dims = synth.planted_tucker(dims, J, nnz, float(ref["planted_noise"]), seed)
    di = torch.from_numpy(idx.astype(np.int32)).cuda()
    dv = torch.from_numpy(vals).cuda()
    fo = ref[f"{case}_mp_fits"]
    _say(f"split-BF16 MP on the small {case} tensor")
    r = tk.mp(di, dv, dims, J, precision="bf16x3", max_iters=len(fo), tol=0.0)
    assert np.abs(np.array(r.fits) - fo).max() <= 1e-6, (r.fits, fo)
    for k, F in zip("ABC", r.factors):
        Fn = F.cpu().numpy()
        assert np.abs(Fn.T @ Fn - np.eye(Fn.shape[1])).max() < 1e-10
        assert _angle(ref[f"{case}_mp_{k}"], Fn) <= 1e-3, k


def test_split_mp_full_size(tk):
    w = synth.WORKLOADS["cube1000_nnz1m"]
    idx, vals, dims = synth.uniform_sparse(tuple(w["dims"]), int(w["nnz"]), w["seed"])
    J = tuple(w["core"])
    di = torch.from_numpy(idx.astype(np.int32)).cuda()
    dv = torch.from_numpy(vals).cuda()
    _say("split-BF16 MP at 1000^3 / 1M, 2 sweeps")
    res = tk.mp(di, dv, dims, J, precision="bf16x3", max_iters=2, tol=0.0)
    X = O.SparseTensor3(idx, vals, dims)
    G = res.core.cpu().numpy()
    A, B, C = (f.cpu().numpy() for f in res.factors)
    for F in (A, B, C):
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-10
    scale = np.abs(G).max()
    rng = np.random.default_rng(3)
    for p, q, r in [(0, 0, 0)] + [tuple(int(rng.integers(j)) for j in J) for _ in range(8)]:
        assert abs(G[p, q, r] - O.core_entry(X, A, B, C, p, q, r)) <= 1e-5 * scale
    assert abs(tk.fit(di, dv, dims, res.core, res.factors) - res.fits[-1]) <= 1e-7


def test_hooi_rejects_split(tk):
    idx, vals, dims = synth.uniform_sparse((30, 20, 10), 600, 1)
    di = torch.from_numpy(idx.astype(np.int32)).cuda()
    dv = torch.from_numpy(vals).cuda()
    with pytest.raises(tk.TuckerError) as e:
        tk.hooi(di, dv, dims, (3, 3, 3), precision="bf16x3", max_iters=2)
    assert e.value.status == tk.TK_ERR_ARG

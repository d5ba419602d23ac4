"""Skewed tensors: every index drawn from a truncated Zipf law (synth.skewed_sparse),
so a few fibres hold hundreds of nonzeros while most hold one or two, as in
term-frequency data. Fibres with more than 12 (BF16 rows) or 8 (FP32 and FP64
rows) nonzeros are projected by one workgroup each, in the same launch as the
rest (k_project_fused: nonzeros dealt round robin to thread groups, partial
rows summed in a fixed order); the rest go to the
per-thread walk, which skips the long ones.

* MP (Figure 7, pseudo HO-SVD start of Section 4.4) in FP64 against the FP64
  oracle's trajectory on the same tensor: fits per sweep, the oracle's
  slice-wise fit of the returned core and factors, factor subspaces.
* The reduced forms (FP32, mixed BF16 with the dual mode-3 projection,
  split-BF16) against the same oracle trajectory at their tolerances.
* Run to run: the mixed decomposition twice, bitwise equal.
* SP (Figure 5, shared random start) and HOOI (Figure 3, whose projections
  write every slot: long slots get the same treatment) against the oracle.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS, NNZ, ZIPF, SEED, CORE = (200, 180, 160), 200_000, 1.0, 21, (8, 8, 8)


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


@pytest.fixture(scope="module")
def skewed():
    idx, vals, dims = synth.skewed_sparse(DIMS, NNZ, ZIPF, SEED)
    X = O.SparseTensor3(idx, vals, dims)
    # the case must hold long fibres in every ordering
    for m in range(3):
        a, b = [n for n in range(3) if n != m]
        _, cnt = np.unique(idx[a].astype(np.int64) * dims[b] + idx[b], return_counts=True)
        assert (cnt > 32).sum() > 100 and cnt.max() > 100
    ref = O.mp(X, CORE, 3, 0.0, fit="identity")
    di = torch.from_numpy(idx.astype(np.int32)).cuda()
    dv = torch.from_numpy(vals).cuda()
    return dims, X, ref, di, dv


def test_skewed_mp_fp64_matches_oracle(tk, skewed):
    dims, X, ref, di, dv = skewed
    _say(f"skewed {dims} {NNZ} zipf {ZIPF}: mp fp64")
    r = tk.mp(di, dv, dims, CORE, precision="fp64", max_iters=3, tol=0.0, eig_tol=1e-14)
    np.testing.assert_allclose(r.fits, ref.fits, rtol=0, atol=1e-10)
    # the core's norm does not depend on the basis chosen inside each
    # subspace (nearly equal eigenvalues inside the leading eight leave the
    # individual eigenvectors, and so the core's entries, less determined
    # than the subspaces and the fit)
    g = r.core.cpu().numpy()
    assert abs(np.linalg.norm(g) - np.linalg.norm(ref.core)) <= 1e-10 * np.linalg.norm(ref.core)
    f_or = O.fit_slicewise(X, g, *[f.cpu().numpy() for f in r.factors])
    assert abs(f_or - r.fits[-1]) < 1e-10
    for n in range(3):
        # eigenvalue ratio lambda_8 / lambda_9 is about 1.1 in every mode
        assert O.subspace_angle(r.factors[n].cpu().numpy(), ref.factors[n]) < 1e-5


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("mixed", 1e-4), ("bf16x3", 1e-6)])
def test_skewed_mp_reduced_precision(tk, skewed, prec, tol):
    dims, X, ref, di, dv = skewed
    _say(f"skewed {dims}: mp {prec}")
    r = tk.mp(di, dv, dims, CORE, precision=prec, max_iters=3, tol=0.0)
    assert max(abs(a - b) for a, b in zip(r.fits, ref.fits)) <= tol


def test_skewed_mp_run_to_run(tk, skewed):
    dims, X, ref, di, dv = skewed
    _say(f"skewed {dims}: mp mixed twice")
    r1 = tk.mp(di, dv, dims, CORE, precision="mixed", max_iters=3, tol=0.0)
    r2 = tk.mp(di, dv, dims, CORE, precision="mixed", max_iters=3, tol=0.0)
    assert r1.fits == r2.fits
    for a, b in zip(r1.factors, r2.factors):
        assert torch.equal(a, b)
    assert torch.equal(r1.core, r2.core)


def test_skewed_sp_fp64_matches_oracle(tk, skewed):
    # Slice Projection (Figure 5) from the SplitMix64 random start both sides
    # draw (seed 0x5EED): its three projections take the same long-fibre path
    dims, X, ref, di, dv = skewed
    _say(f"skewed {dims}: sp fp64")
    C0 = O.random_start(dims[2], CORE[2], 2, 0x5EED)
    ref_sp = O.sp_algorithm(X, CORE, C0, 3, 0.0, fit="identity")
    r = tk.sp(di, dv, dims, CORE, precision="fp64", max_iters=3, tol=0.0, seed=0x5EED, eig_tol=1e-14)
    np.testing.assert_allclose(r.fits, ref_sp.fits, rtol=0, atol=1e-10)
    g = r.core.cpu().numpy()
    assert abs(np.linalg.norm(g) - np.linalg.norm(ref_sp.core)) <= 1e-10 * np.linalg.norm(ref_sp.core)


@pytest.fixture(scope="module")
def skewed_hooi(skewed):
    dims, X, ref, di, dv = skewed
    return O.hooi(X, CORE, 3, 0.0, fit="identity")


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-6), ("mixed", 1e-4)])
def test_skewed_hooi_matches_oracle(tk, skewed, skewed_hooi, prec, tol):
    # HOOI (Figure 3) projects into every slot: its slots of more than 8
    # nonzeros get one workgroup each in the same launch
    dims, X, ref, di, dv = skewed
    _say(f"skewed {dims}: hooi {prec}")
    kw = {"eig_tol": 1e-14} if prec == "fp64" else {}
    r = tk.hooi(di, dv, dims, CORE, precision=prec, max_iters=3, tol=0.0, **kw)
    assert max(abs(a - b) for a, b in zip(r.fits, skewed_hooi.fits)) <= tol

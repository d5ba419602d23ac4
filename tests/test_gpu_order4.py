"""Fourth-order HO-SVD, HOOI and MP on the GPU (tk_coo.order = 4) against
the order-N FP64 oracle (oracle/tucker_n.py: Figures 2, 4 and 8).

* FP64 trajectories (fit after every sweep) within 1e-9 of the oracle's on
  ragged shapes with unequal cores, HO-SVD's fit within 1e-10; FP32 within
  1e-6 and mixed (BF16 Grams / products) within 1e-4;
* exact Tucker rank gives fit 1; a trivial fourth mode (I4 = J4 = 1)
  reproduces the third-order GPU results; duplicates are summed; the order
  of distinct nonzeros changes no bit;
* the paper's shape: 60^4 at 10 % density with core 20^4, HOOI and MP
  against the oracle;
* the HO-SVD start Grams come from the dense unfolding where at least one
  cell in sixteen holds a nonzero (the ragged tensor: 9000 nonzeros in
  96,577 cells, and every other tensor above) and from the sparse walk
  below that (31 x 27 x 19 x 23 with 6000 nonzeros in 365,769 cells): both
  forms are checked against the oracle.
"""
import sys

import numpy as np
import pytest

from oracle import tucker_n as ON
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


@pytest.fixture(scope="module")
def ragged():
    idx, vals, dims = synth.uniform_sparse((23, 19, 17, 13), 9000, 404)
    return idx, vals, dims, (5, 4, 6, 3), ON.SparseTensorN(idx, vals, dims)


@pytest.mark.parametrize("algo", ["mp", "hooi"])
def test_fp64_trajectory_matches_oracle(tk, ragged, algo):
    idx, vals, dims, J, X = ragged
    _say(f"order 4 {algo} fp64 {dims} core {J}")
    ref = getattr(ON, algo)(X, J, 6, 0.0)
    di, dv = _dev(idx, vals)
    r = getattr(tk, algo)(di, dv, dims, J, precision="fp64", max_iters=6, tol=0.0)
    d = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
    _say(f"  gpu {r.fits[-1]:.9f} oracle {ref.fits[-1]:.9f} max|d| {d:.2e}")
    assert d < 1e-9
    G = r.core.cpu().numpy()
    assert G.shape == J
    facs = [f.cpu().numpy() for f in r.factors]
    for F in facs:
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-10
    # the core is [[X; A^T ...]] of the returned factors (row-major J1 x J2 x J3 x J4)
    np.testing.assert_allclose(G, ON.core(X, facs), rtol=0, atol=1e-10 * np.abs(G).max())


@pytest.mark.parametrize("algo,prec,tol", [("mp", "fp32", 1e-6), ("mp", "mixed", 1e-4), ("hooi", "fp32", 1e-6),
                                           ("hooi", "mixed", 1e-4)])
def test_reduced_precision_fits(tk, ragged, algo, prec, tol):
    idx, vals, dims, J, X = ragged
    ref = getattr(ON, algo)(X, J, 6, 0.0)
    di, dv = _dev(idx, vals)
    r = getattr(tk, algo)(di, dv, dims, J, precision=prec, max_iters=6, tol=0.0)
    d = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
    _say(f"order 4 {algo} {prec}: max|dfit| {d:.2e}")
    assert d < tol


def test_hosvd_matches_oracle(tk, ragged):
    idx, vals, dims, J, X = ragged
    ref = ON.hosvd(X, J)
    di, dv = _dev(idx, vals)
    r = tk.hosvd(di, dv, dims, J)
    _say(f"order 4 hosvd: gpu {r.fits[0]:.12f} oracle {ref.fits[0]:.12f}")
    assert abs(r.fits[0] - ref.fits[0]) < 1e-10
    np.testing.assert_allclose(r.core.cpu().numpy(), ref.core, rtol=0, atol=1e-9 * np.abs(ref.core).max())


@pytest.mark.parametrize("algo", ["mp", "hooi", "hosvd"])
def test_sparse_start_matches_oracle(tk, algo):
    idx, vals, dims = synth.uniform_sparse((31, 27, 19, 23), 6000, 405)
    assert 16 * len(vals) < int(np.prod(dims))  # below the dense-start density
    J = (4, 5, 3, 4)
    X = ON.SparseTensorN(idx, vals, dims)
    di, dv = _dev(idx, vals)
    _say(f"order 4 sparse start {algo} fp64 {dims} core {J}")
    if algo == "hosvd":
        ref = ON.hosvd(X, J)
        r = tk.hosvd(di, dv, dims, J)
        assert abs(r.fits[0] - ref.fits[0]) < 1e-10
        np.testing.assert_allclose(r.core.cpu().numpy(), ref.core, rtol=0, atol=1e-9 * np.abs(ref.core).max())
    else:
        ref = getattr(ON, algo)(X, J, 4, 0.0)
        r = getattr(tk, algo)(di, dv, dims, J, precision="fp64", max_iters=4, tol=0.0)
        d = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
        _say(f"  gpu {r.fits[-1]:.9f} oracle {ref.fits[-1]:.9f} max|d| {d:.2e}")
        assert d < 1e-9


@pytest.mark.parametrize("algo", ["mp", "hooi", "hosvd"])
def test_exact_tucker_rank_fit_one(tk, algo):
    idx, vals, dims = synth.exact_tucker_block_n((14, 12, 11, 9), (8, 7, 6, 5), (3, 2, 3, 2), 77)
    di, dv = _dev(idx, vals)
    J = (3, 2, 3, 2)
    if algo == "hosvd":
        f = tk.hosvd(di, dv, dims, J).fits[-1]
    else:
        f = getattr(tk, algo)(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0).fits[-1]
    _say(f"order 4 exact rank {algo}: fit {f:.12f}")
    assert f > 1 - 1e-7


def test_trivial_fourth_mode_equals_third_order(tk):
    """I4 = J4 = 1: HOOI and HO-SVD of the fourth-order tensor reproduce the
    third-order GPU results on the squeezed tensor."""
    idx, vals, dims = synth.uniform_sparse((40, 35, 30), 6000, 12)
    idx4 = np.vstack([idx, np.zeros((1, idx.shape[1]), dtype=np.int32)])
    J = (6, 5, 4)
    d3, v3 = _dev(idx, vals)
    d4, v4 = _dev(idx4, vals)
    r3 = tk.hooi(d3, v3, dims, J, precision="fp64", max_iters=5, tol=0.0)
    r4 = tk.hooi(d4, v4, dims + (1,), J + (1,), precision="fp64", max_iters=5, tol=0.0)
    _say(f"trivial 4th mode hooi: {r3.fits[-1]:.12f} vs {r4.fits[-1]:.12f}")
    np.testing.assert_allclose(r4.fits, r3.fits, rtol=0, atol=1e-10)
    h3 = tk.hosvd(d3, v3, dims, J).fits[0]
    h4 = tk.hosvd(d4, v4, dims + (1,), J + (1,)).fits[0]
    assert abs(h3 - h4) < 1e-10


def test_duplicates_summed_and_order_invariant(tk, ragged):
    idx, vals, dims, J, X = ragged
    idx2, vals2 = synth.with_duplicates(idx, vals, 500, 3)
    # the same tensor: duplicates' values folded into the originals
    ref = ON.mp(ON.SparseTensorN(idx2, vals2, dims), J, 3, 0.0)
    di, dv = _dev(idx2, vals2)
    r = tk.mp(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0)
    assert np.max(np.abs(np.array(r.fits) - np.array(ref.fits))) < 1e-9
    # distinct coordinates: the orderings sort by the full coordinate, so the
    # input order changes no bit (repeated coordinates are summed in input
    # order, which rounds differently)
    d0, v0 = _dev(idx, vals)
    r0 = tk.mp(d0, v0, dims, J, precision="fp64", max_iters=3, tol=0.0)
    perm = np.random.default_rng(0).permutation(vals.size)
    dp, vp = _dev(idx[:, perm], vals[perm])
    r2 = tk.mp(dp, vp, dims, J, precision="fp64", max_iters=3, tol=0.0)
    assert r2.fits == r0.fits
    assert torch.equal(r2.core, r0.core)


@pytest.mark.parametrize("algo", ["hooi", "mp"])
def test_paper_shape_small(tk, algo):
    """60^4 at 10 % density (1.3M nonzeros), core 20^4: the shape of the
    paper's fourth-order experiments scaled down so that the oracle finishes
    in seconds; FP64 within 1e-9 of its fit after each of 3 sweeps, mixed
    within 1e-4."""
    idx, vals, dims = synth.uniform_sparse((60, 60, 60, 60), 1_296_000, 61)
    J = (20, 20, 20, 20)
    X = ON.SparseTensorN(idx, vals, dims)
    _say(f"order 4 paper shape {algo}: oracle")
    ref = ON.hooi(X, J, 3, 0.0) if algo == "hooi" else None
    di, dv = _dev(idx, vals)
    r = getattr(tk, algo)(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0)
    rm = getattr(tk, algo)(di, dv, dims, J, precision="mixed", max_iters=3, tol=0.0)
    if ref is None:  # MP's literal slice sums are slow at this size: check the fit of the returned factors
        G = ON.core(X, [f.cpu().numpy() for f in r.factors])
        f_or = ON.fit_identity(X.norm2(), G)
        _say(f"  mp gpu {r.fits[-1]:.9f} oracle fit of its factors {f_or:.9f} mixed {rm.fits[-1]:.9f}")
        assert abs(r.fits[-1] - f_or) < 1e-9
        assert abs(rm.fits[-1] - r.fits[-1]) < 1e-4
    else:
        d = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
        dm = np.max(np.abs(np.array(rm.fits) - np.array(ref.fits)))
        _say(f"  hooi gpu {r.fits[-1]:.9f} oracle {ref.fits[-1]:.9f} max|d| fp64 {d:.2e} mixed {dm:.2e}")
        assert d < 1e-9 and dm < 1e-4

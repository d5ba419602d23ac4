"""Parity of Slice Projection (Section 4.3, Figure 5), HO-SVD (Section 4.1,
Figure 1), the random start and the HO-SVD fit report with the FP64 oracle,
through the C ABI.

SP starts from the SplitMix64 draw that both sides implement from its
published definition (oracle.random_start, the library's TK_INIT_RANDOM),
so the GPU and the oracle follow the same trajectory. Tolerances as the MP
and HOOI parity tests: FP64 fits to 1e-9, FP32 to 1e-6, BF16 Grams to the
1e-4 bar; subspaces only where the eigengap makes them unique.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 0x5EED


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


def _np(r):
    return [f.cpu().numpy() for f in r.factors]


@pytest.fixture(scope="module")
def cube100():
    w = synth.WORKLOADS["cube100_nnz10k"]
    idx, vals, dims = synth.uniform_sparse(w["dims"], w["nnz"], w["seed"])
    return idx, vals, dims, O.SparseTensor3(idx, vals, dims), w["core"]


@pytest.fixture(scope="module")
def planted():
    idx, vals, dims = synth.planted_tucker((120, 110, 100), (8, 7, 6), 120_000, 0.1, 9200)
    return idx, vals, dims, O.SparseTensor3(idx, vals, dims), (8, 7, 6)


def test_sp_fp64_trajectory_matches_oracle(tk, cube100):
    idx, vals, dims, X, J = cube100
    _say("sp cube100 fp64")
    C0 = O.random_start(dims[2], J[2], 2, SEED)
    ref = O.sp_algorithm(X, J, C0, 10, 0.0, fit="identity")
    di, dv = _dev(idx, vals)
    r = tk.sp(di, dv, dims, J, precision="fp64", max_iters=10, tol=0.0, seed=SEED, eig_tol=1e-14)
    assert r.iters == 10
    np.testing.assert_allclose(r.fits, ref.fits, rtol=0, atol=1e-9)
    np.testing.assert_allclose(r.core.cpu().numpy(), ref.core, atol=1e-9 * np.abs(ref.core).max())
    for F in _np(r):
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-12


def test_sp_stops_on_core_growth_like_oracle(tk, planted):
    idx, vals, dims, X, J = planted
    _say("sp planted fp64, Delta_G stop")
    C0 = O.random_start(dims[2], J[2], 2, SEED)
    ref = O.sp_algorithm(X, J, C0, 50, 1e-4, fit="identity")
    di, dv = _dev(idx, vals)
    r = tk.sp(di, dv, dims, J, precision="fp64", max_iters=50, tol=1e-4, seed=SEED)
    assert r.iters == ref.iters
    np.testing.assert_allclose(r.fits, ref.fits, rtol=0, atol=1e-9)
    # the stop itself: Delta_G from the returned fits (||G||^2 = ||X||^2 (1 - (1 - fit)^2))
    nx = r.stats["norm_x"]
    gn = [nx * math.sqrt(1 - (1 - f) ** 2) for f in r.fits]
    dG = [1 - (gn[t - 1] if t else 0.0) / gn[t] for t in range(len(gn))]
    np.testing.assert_allclose(dG, ref.extra["core_growth"], rtol=0, atol=1e-9)
    assert dG[-1] < 1e-4 and all(d >= 1e-4 for d in dG[:-1])
    assert abs(r.stats["core_norm"] - math.sqrt(np.sum(ref.core ** 2))) < 1e-9 * nx
    # gapped planted model: the subspaces are unique
    for a, b in zip(ref.factors, _np(r)):
        assert O.subspace_angle(a, b) < 1e-8


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("mixed", 1e-4), ("bf16x3", 1e-6)])
def test_sp_reduced_precision(tk, cube100, prec, tol):
    idx, vals, dims, X, J = cube100
    _say(f"sp cube100 {prec}")
    C0 = O.random_start(dims[2], J[2], 2, SEED)
    ref = O.sp_algorithm(X, J, C0, 6, 0.0, fit="identity")
    di, dv = _dev(idx, vals)
    r = tk.sp(di, dv, dims, J, precision=prec, max_iters=6, tol=0.0, seed=SEED)
    assert max(abs(a - b) for a, b in zip(r.fits, ref.fits)) <= tol


def test_sp_ragged_modes_and_given_start(tk):
    """Modes of different sizes past one tile (iterative eigensolver, ragged
    Gram tiles), and a given unnormalised start whose columns the library
    normalises as Figure 5 does."""
    _say("sp 301x257x190 fp64, given start")
    idx, vals, dims = synth.uniform_sparse((301, 257, 190), 60_000, 21)
    X = O.SparseTensor3(idx, vals, dims)
    J = (23, 17, 9)
    rng = np.random.default_rng(4)
    C0 = rng.random((dims[2], J[2]))
    ref = O.sp_algorithm(X, J, C0, 4, 0.0, fit="identity")
    di, dv = _dev(idx, vals)
    start = [torch.zeros((dims[0], J[0]), dtype=torch.float64), torch.zeros((dims[1], J[1]), dtype=torch.float64),
             torch.from_numpy(C0)]
    r = tk.sp(di, dv, dims, J, precision="fp64", max_iters=4, tol=0.0, init=tk.INIT_GIVEN, factors=start,
              eig_tol=1e-13)
    np.testing.assert_allclose(r.fits, ref.fits, rtol=0, atol=1e-7)
    f_or = O.fit_slicewise(X, r.core.cpu().numpy(), *_np(r))
    assert abs(f_or - r.fits[-1]) < 1e-9


def test_sp_size_one_mode_is_truncated_svd(tk):
    _say("sp size-one mode")
    idx, vals, dims = synth.matrix_as_tensor(180, 150, 3000, 7)
    M = np.zeros((180, 150))
    np.add.at(M, (idx[0], idx[1]), vals)
    s = np.linalg.svd(M, compute_uv=False)
    J = (12, 9, 1)
    di, dv = _dev(idx, vals)
    r = tk.sp(di, dv, dims, J, precision="fp64", max_iters=4, tol=0.0, eig_tol=1e-14)
    rk = min(J[0], J[1])
    expected = 1 - math.sqrt(np.sum(s[rk:] ** 2)) / math.sqrt(np.sum(s ** 2))
    assert abs(r.fits[-1] - expected) < 1e-10


def test_sp_superdiagonal(tk):
    _say("sp superdiagonal")
    idx, vals, dims = synth.superdiagonal(150, 10)
    J = (6, 6, 6)
    a = np.sort(np.abs(vals))[::-1]
    expected = 1 - math.sqrt(np.sum(a[6:] ** 2)) / math.sqrt(np.sum(a ** 2))
    di, dv = _dev(idx, vals)
    # from the HO-SVD start C spans the coordinate axes of the six largest
    # |d_k|, and each Gram of Figure 5 is then diagonal on those same axes
    # (from a random start SP keeps whichever axes d_k^2 |c_k|^2 ranks first:
    # a fixed point of its own, not the closed form)
    r = tk.sp(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0, init=tk.INIT_HOSVD)
    assert abs(r.fits[-1] - expected) < 1e-10
    C0 = O.random_start(150, 6, 2, SEED)
    ref = O.sp_algorithm(O.SparseTensor3(idx, vals, dims), J, C0, 3, 0.0, fit="identity")
    r = tk.sp(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0, seed=SEED)
    np.testing.assert_allclose(r.fits, ref.fits, rtol=0, atol=1e-10)


@pytest.mark.parametrize("algo", ["mp", "hooi"])
def test_random_start_mp_hooi_match_oracle(tk, cube100, algo):
    idx, vals, dims, X, J = cube100
    _say(f"random start {algo}")
    B0 = O.random_start(dims[1], J[1], 1, SEED)
    C0 = O.random_start(dims[2], J[2], 2, SEED)
    ref = (O.mp if algo == "mp" else O.hooi)(X, J, 5, 0.0, init=(None, B0, C0), fit="identity")
    di, dv = _dev(idx, vals)
    r = getattr(tk, algo)(di, dv, dims, J, precision="fp64", max_iters=5, tol=0.0, init=tk.INIT_RANDOM, seed=SEED,
                          eig_tol=1e-14)
    np.testing.assert_allclose(r.fits, ref.fits, rtol=0, atol=1e-9)


def test_hosvd_matches_oracle(tk, cube100, planted):
    for name, (idx, vals, dims, X, J) in (("cube100", cube100), ("planted", planted)):
        _say(f"hosvd {name}")
        ref = O.hosvd(X, J, fit="identity")
        di, dv = _dev(idx, vals)
        r = tk.hosvd(di, dv, dims, J, precision="fp64", eig_tol=1e-14)
        assert abs(r.fits[0] - ref.fits[0]) < 1e-10
        assert abs(O.fit_slicewise(X, r.core.cpu().numpy(), *_np(r)) - r.fits[0]) < 1e-10
        if name == "planted":
            for a, b in zip(ref.factors, _np(r)):
                assert O.subspace_angle(a, b) < 1e-8


@pytest.mark.parametrize("algo,init", [("mp", "hosvd"), ("hooi", "hosvd"), ("sp", "hosvd"), ("sp", "random"),
                                       ("mp", "random")])
def test_hosvd_fit_report(tk, cube100, algo, init):
    """stats.hosvd_fit is the oracle's HO-SVD fit, and asking for it leaves
    the decomposition bit for bit unchanged."""
    idx, vals, dims, X, J = cube100
    _say(f"hosvd_fit report {algo} {init}")
    ref = O.hosvd(X, J, fit="identity").fits[0]
    di, dv = _dev(idx, vals)
    fn = getattr(tk, algo)
    iv = tk.INIT_HOSVD if init == "hosvd" else tk.INIT_RANDOM
    a = fn(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0, init=iv, hosvd_fit=True, eig_tol=1e-14)
    b = fn(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0, init=iv, eig_tol=1e-14)
    assert abs(a.stats["hosvd_fit"] - ref) < 1e-10
    assert b.stats["hosvd_fit"] == 0.0
    assert a.fits == b.fits
    assert torch.equal(a.core, b.core)
    for fa, fb in zip(a.factors, b.factors):
        assert torch.equal(fa, fb)

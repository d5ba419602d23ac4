"""Pins of the order-N oracle (oracle/tucker_n.py) against what the paper and
the mathematics fix, without a GPU: einsum written out on the densified
tensor for the products, unfoldings and Grams; the pseudo HO-SVD matrix of
MP against (N - 1) X_(n) X_(n)^T; agreement with the third-order oracle on
third-order input; a trivial fourth mode reducing HO-SVD and HOOI to their
third-order results; exact Tucker rank, full cores and superdiagonals
(closed forms); HOOI's monotone fit; brute force on 2x2x2x2; and the fit the
paper prints for HO-SVD on 100^4 tensors of 10 % density (Table 6, core
50^4: 6.988 %), reproduced within the sampling band."""

import numpy as np
import pytest

import oracle as O3
from oracle import tucker_n as ON
import synth


def _rand4(dims=(6, 5, 4, 3), nnz=150, seed=7):
    rng = np.random.default_rng(seed)
    total = int(np.prod(dims))
    lin = rng.choice(total, size=nnz, replace=False)
    idx = np.stack(np.unravel_index(lin, dims))
    return ON.SparseTensorN(idx, rng.random(nnz), dims)


def _orth(n, r, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, r)))
    return q


def test_duplicates_summed_and_dense():
    idx = np.array([[0, 0, 1], [1, 1, 0], [2, 2, 2], [0, 0, 1]])
    X = ON.SparseTensorN(idx, np.array([1.0, 2.0, 5.0]), (2, 2, 3, 2))
    D = X.dense()
    assert X.nnz == 2 and D[0, 1, 2, 0] == 3.0 and D[1, 0, 2, 1] == 5.0


def test_unfolding_and_gram_match_einsum():
    X = _rand4()
    D = X.dense()
    subs = {0: "iabc,jabc->ij", 1: "aibc,ajbc->ij", 2: "abic,abjc->ij", 3: "abci,abcj->ij"}
    for n in range(4):
        np.testing.assert_allclose(ON.unfolding_gram(X, n), np.einsum(subs[n], D, D), rtol=1e-13, atol=1e-13)
    # column order: the lower remaining mode varies fastest (Section 3)
    U = X.unfolding(1).toarray()
    i0, i2, i3 = 3, 2, 1
    col = i0 + 6 * (i2 + 4 * i3)
    np.testing.assert_array_equal(U[:, col], D[i0, :, i2, i3])


def test_projection_matches_einsum():
    X = _rand4()
    D = X.dense()
    letters = "abcd"
    for m in range(4):
        A = _orth(X.dims[m], 2, m)
        out = letters[:m] + "r" + letters[m + 1:]
        want = np.einsum(f"abcd,{letters[m]}r->{out}", D, A)
        np.testing.assert_allclose(ON.project(X, A, m), want, rtol=1e-13, atol=1e-14)
    facs = [_orth(X.dims[n], 2, 10 + n) for n in range(4)]
    np.testing.assert_allclose(ON.core(X, facs), np.einsum("abcd,ap,bq,cr,ds->pqrs", D, *facs), rtol=1e-12,
                               atol=1e-13)
    Z = ON.multi_project(X, facs, skip=2)
    np.testing.assert_allclose(Z, np.einsum("abcd,ap,bq,ds->pqcs", D, facs[0], facs[1], facs[3]), rtol=1e-12,
                               atol=1e-13)


def test_mp_gram_is_the_sum_of_projected_unfolding_grams():
    """Figure 8's slice sums regrouped: for each other mode m the slices with
    free modes (n, m), projected by A(m), sum to T(m)_(n) T(m)_(n)^T with
    T(m) = X x_m A(m)^T (einsum here)."""
    X = _rand4()
    D = X.dense()
    facs = [_orth(X.dims[n], 2 + (n % 2), 20 + n) for n in range(4)]
    letters = "abcd"
    for n in range(4):
        want = np.zeros((X.dims[n], X.dims[n]))
        for m in range(4):
            if m == n:
                continue
            out = letters[:m] + "r" + letters[m + 1:]
            T = np.einsum(f"abcd,{letters[m]}r->{out}", D, facs[m])
            Tn = np.moveaxis(T, n, 0).reshape(X.dims[n], -1)
            want += Tn @ Tn.T
        np.testing.assert_allclose(ON.mp_gram(X, n, facs), want, rtol=1e-12, atol=1e-13)


def test_mp_start_gram_is_n_minus_one_unfolding_grams():
    X = _rand4()
    for n in range(4):
        np.testing.assert_allclose(ON.mp_init_gram(X, n), 3.0 * ON.unfolding_gram(X, n), rtol=1e-13, atol=1e-13)


def test_third_order_input_agrees_with_the_third_order_oracle():
    idx, vals, dims = synth.uniform_sparse((12, 10, 9), 300, 5)
    X3 = O3.SparseTensor3(idx, vals, dims)
    XN = ON.SparseTensorN(idx, vals, dims)
    J = (3, 4, 2)
    np.testing.assert_allclose(ON.hosvd(XN, J).fits, O3.hosvd(X3, J, fit="identity").fits, rtol=0, atol=1e-12)
    np.testing.assert_allclose(ON.hooi(XN, J, 5, 0.0).fits, O3.hooi(X3, J, 5, 0.0, fit="identity").fits, rtol=0,
                               atol=1e-12)
    np.testing.assert_allclose(ON.mp(XN, J, 5, 0.0).fits, O3.mp(X3, J, 5, 0.0, fit="identity").fits, rtol=0,
                               atol=1e-12)


def test_trivial_fourth_mode_reduces_to_third_order():
    """I4 = J4 = 1: the fourth factor is [1] and HO-SVD and HOOI of order
    four equal the third-order ones on the squeezed tensor."""
    idx, vals, dims = synth.uniform_sparse((11, 9, 8), 250, 9)
    X3 = O3.SparseTensor3(idx, vals, dims)
    X4 = ON.SparseTensorN(np.vstack([idx, np.zeros((1, idx.shape[1]), dtype=idx.dtype)]), vals, dims + (1,))
    J = (3, 3, 2)
    np.testing.assert_allclose(ON.hosvd(X4, J + (1,)).fits, O3.hosvd(X3, J, fit="identity").fits, rtol=0,
                               atol=1e-12)
    np.testing.assert_allclose(ON.hooi(X4, J + (1,), 6, 0.0).fits, O3.hooi(X3, J, 6, 0.0, fit="identity").fits,
                               rtol=0, atol=1e-12)


def _exact4(dims=(7, 6, 5, 4), rank=(2, 3, 2, 2), seed=3):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal(rank)
    facs = [np.linalg.qr(rng.standard_normal((dims[n], rank[n])))[0] for n in range(4)]
    D = np.einsum("pqrs,ap,bq,cr,ds->abcd", G, *facs)
    idx = np.stack(np.unravel_index(np.arange(D.size), dims))
    return ON.SparseTensorN(idx, D.ravel(), dims)


@pytest.mark.parametrize("algo", ["hosvd", "hooi", "mp"])
def test_exact_tucker_rank_gives_fit_one(algo):
    X = _exact4()
    J = (2, 3, 2, 2)
    d = ON.hosvd(X, J) if algo == "hosvd" else getattr(ON, algo)(X, J, 3, 0.0)
    assert d.fits[-1] > 1 - 1e-7
    np.testing.assert_allclose(ON.fit_dense(X.dense(), d.core, d.factors), d.fits[-1], atol=1e-9)


def test_full_core_gives_fit_one():
    """J = I: the factors are square orthogonal and the fit is 1 (the
    identity's sqrt(||X||^2 - ||G||^2) resolves it to about sqrt(eps))."""
    X = _rand4(dims=(4, 3, 3, 2), nnz=40)
    d = ON.hooi(X, X.dims, 2, 0.0)
    assert d.fits[-1] > 1 - 1e-7
    assert ON.fit_dense(X.dense(), d.core, d.factors) > 1 - 1e-12


def test_superdiagonal_closed_form():
    """x_iiii = d_i with distinct |d_i|: every method keeps the coordinate
    vectors of the J largest |d_i|; fit = 1 - sqrt(sum of the other d^2) /
    sqrt(sum d^2)."""
    n, J = 9, 4
    d = 1.0 + np.arange(n)[::-1] / n
    idx = np.stack([np.arange(n)] * 4)
    X = ON.SparseTensorN(idx, d, (n,) * 4)
    want = 1.0 - np.sqrt(np.sum(d[J:] ** 2)) / np.sqrt(np.sum(d ** 2))
    for res in (ON.hosvd(X, (J,) * 4), ON.hooi(X, (J,) * 4, 3, 0.0), ON.mp(X, (J,) * 4, 3, 0.0)):
        assert abs(res.fits[-1] - want) < 1e-12


def test_hooi_monotone_and_above_hosvd():
    X = _rand4(dims=(8, 7, 6, 5), nnz=400, seed=11)
    J = (3, 3, 2, 2)
    h = ON.hosvd(X, J).fits[0]
    f = ON.hooi(X, J, 8, 0.0).fits
    assert f[0] >= h - 1e-12
    assert all(b >= a - 1e-12 for a, b in zip(f, f[1:]))
    d = ON.hooi(X, J, 3, 0.0)
    np.testing.assert_allclose(ON.fit_dense(X.dense(), d.core, d.factors), d.fits[-1], atol=1e-12)


def test_brute_force_rank_one_on_2x2x2x2():
    """The best rank-(1,1,1,1) fit over a grid of unit vectors (angles in
    [0, pi)) bounds HOOI's fit from above up to the grid's resolution, and
    HOOI comes within it."""
    rng = np.random.default_rng(5)
    D = rng.random((2, 2, 2, 2))
    idx = np.stack(np.unravel_index(np.arange(16), (2,) * 4))
    X = ON.SparseTensorN(idx, D.ravel(), (2,) * 4)
    th = np.linspace(0, np.pi, 60, endpoint=False)
    U = np.stack([np.cos(th), np.sin(th)], axis=1)                     # 60 x 2
    g = np.einsum("abcd,pa,qb,rc,sd->pqrs", D, U, U, U, U)
    best = 1.0 - np.sqrt(max(0.0, (D * D).sum() - (g * g).max())) / np.sqrt((D * D).sum())
    f = ON.hooi(X, (1, 1, 1, 1), 30, 0.0).fits[-1]
    assert f >= best - 1e-12
    assert f - best < 2e-3


@pytest.mark.slow
def test_paper_hosvd_fit_100_to_the_fourth():
    """Table 6: HO-SVD on random 100^4 tensors of 10 % density with U(0,1)
    values and core 50^4 fits 6.988 %. One draw of the appendix generator's
    distribution must land within +-0.03 percentage points (the spread of
    such draws is far smaller at 10M nonzeros)."""
    idx, vals, dims = _bernoulli4((100, 100, 100, 100), 0.1, 4)
    X = ON.SparseTensorN(idx, vals, dims)
    f = 100.0 * ON.hosvd(X, (50, 50, 50, 50)).fits[0]
    assert abs(f - 6.988) <= 0.03, f


def _bernoulli4(dims, density, seed):
    """Each cell nonzero with probability `density`, values U(0,1) (the
    appendix generator's distribution), for a fourth-order shape."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = int(np.prod(dims))
    lins = []
    chunk = 1 << 24
    for start in range(0, total, chunk):
        n = min(chunk, total - start)
        lins.append(np.nonzero(rng.random(n) < density)[0].astype(np.int64) + start)
    lin = np.concatenate(lins)
    vals = rng.random(lin.size)
    return np.stack(np.unravel_index(lin, dims)), vals, dims

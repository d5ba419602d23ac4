"""Pins of the FP64 oracle against things other than itself: library routines
(einsum, SVD), closed forms, invariants, brute force and the fits the paper
prints. A plausible slip in the oracle (a transposed slice, a dropped Gram
term, a wrong factor in a product, a sign) fails at least one of these."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth


def _tiny(dims=(7, 6, 5), nnz=60, seed=3):
    idx, vals, dims = synth.uniform_sparse(dims, nnz, seed)
    return O.SparseTensor3(idx, vals, dims)


def _orth(n, r, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, r)))
    return q


# ---------------------------------------------------------------- Section 3
def test_mode_product_matches_einsum():
    X = np.random.default_rng(0).standard_normal((4, 5, 6))
    for n, sub in enumerate(["ai,ijk->ajk", "aj,ijk->iak", "ak,ijk->ija"]):
        A = np.random.default_rng(n + 1).standard_normal((3, X.shape[n]))
        np.testing.assert_allclose(O.mode_product_dense(X, A, n), np.einsum(sub, A, X), rtol=1e-13, atol=1e-13)


def test_matricization_definition_and_product_relation():
    X = np.random.default_rng(1).standard_normal((3, 4, 5))
    X1 = O.unfold_dense(X, 0)
    # X_(1) = [X_::1 X_::2 ... X_::I3] (frontal slices side by side)
    np.testing.assert_array_equal(X1, np.concatenate([X[:, :, k] for k in range(5)], axis=1))
    # X_(2) = [X_::1^T X_::2^T ...]
    np.testing.assert_array_equal(O.unfold_dense(X, 1), np.concatenate([X[:, :, k].T for k in range(5)], axis=1))
    for n in range(3):
        A = np.random.default_rng(9 + n).standard_normal((2, X.shape[n]))
        Y = O.mode_product_dense(X, A, n)
        np.testing.assert_allclose(O.unfold_dense(Y, n), A @ O.unfold_dense(X, n), rtol=1e-13, atol=1e-13)


def test_sparse_unfolding_matches_dense():
    X = _tiny()
    D = X.dense()
    for n in range(3):
        np.testing.assert_array_equal(X.unfolding(n).toarray(), O.unfold_dense(D, n))


def test_slices_orientation():
    X = _tiny()
    D = X.dense()
    np.testing.assert_array_equal(X.horizontal(2).toarray(), D[2, :, :])
    np.testing.assert_array_equal(X.lateral(3).toarray(), D[:, 3, :])
    np.testing.assert_array_equal(X.frontal(4).toarray(), D[:, :, 4])


def test_duplicates_are_summed():
    idx, vals, dims = synth.uniform_sparse((6, 5, 4), 40, 5)
    idx2, vals2 = synth.with_duplicates(idx, vals, 15, 6)
    X2 = O.SparseTensor3(idx2, vals2, dims)
    D = np.zeros(dims)
    np.add.at(D, (idx2[0], idx2[1], idx2[2]), vals2)
    np.testing.assert_allclose(X2.dense(), D, rtol=1e-15)
    assert math.isclose(X2.norm2(), float(np.sum(D * D)), rel_tol=1e-14)


# ---------------------------------------------------------------- Grams
def test_unfolding_gram_matches_einsum():
    X = _tiny()
    D = X.dense()
    refs = [np.einsum("ijk,ljk->il", D, D), np.einsum("ijk,ilk->jl", D, D), np.einsum("ijk,ijl->kl", D, D)]
    for n in range(3):
        np.testing.assert_allclose(O.unfolding_gram(X, n), refs[n], rtol=1e-13, atol=1e-13)


def test_mp_init_is_twice_the_hosvd_gram():
    X = _tiny()
    D = X.dense()
    M2, M3 = O.mp_init_grams(X)
    np.testing.assert_allclose(M2, 2 * np.einsum("ijk,ilk->jl", D, D), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(M3, 2 * np.einsum("ijk,ijl->kl", D, D), rtol=1e-13, atol=1e-13)


def test_mp_gram_is_sum_of_single_mode_projection_grams():
    X = _tiny()
    D = X.dense()
    A, B, C = _orth(7, 3, 1), _orth(6, 2, 2), _orth(5, 4, 3)
    T_B = np.einsum("ijk,jq->iqk", D, B)
    T_C = np.einsum("ijk,kr->ijr", D, C)
    T_A = np.einsum("ijk,ip->pjk", D, A)
    ref1 = np.einsum("iqk,lqk->il", T_B, T_B) + np.einsum("ijr,ljr->il", T_C, T_C)
    ref2 = np.einsum("pjk,plk->jl", T_A, T_A) + np.einsum("ijr,ilr->jl", T_C, T_C)
    ref3 = np.einsum("pjk,pjl->kl", T_A, T_A) + np.einsum("iqk,iql->kl", T_B, T_B)
    np.testing.assert_allclose(O.mp_gram(X, 0, None, B, C), ref1, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.mp_gram(X, 1, A, None, C), ref2, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.mp_gram(X, 2, A, B, None), ref3, rtol=1e-12, atol=1e-13)


def test_sp_gram_uses_one_factor():
    X = _tiny()
    D = X.dense()
    A, B, C = _orth(7, 3, 1), _orth(6, 2, 2), _orth(5, 4, 3)
    T_C = np.einsum("ijk,kr->ijr", D, C)
    T_A = np.einsum("ijk,ip->pjk", D, A)
    T_B = np.einsum("ijk,jq->iqk", D, B)
    np.testing.assert_allclose(O.sp_gram(X, 0, C), np.einsum("ijr,ljr->il", T_C, T_C), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.sp_gram(X, 1, A), np.einsum("pjk,plk->jl", T_A, T_A), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.sp_gram(X, 2, B), np.einsum("iqk,iql->kl", T_B, T_B), rtol=1e-12, atol=1e-13)


def test_hooi_gram_matches_einsum():
    X = _tiny()
    D = X.dense()
    A, B, C = _orth(7, 3, 1), _orth(6, 2, 2), _orth(5, 4, 3)
    U = np.einsum("ijk,jq,kr->iqr", D, B, C)
    V = np.einsum("ijk,ip,kr->pjr", D, A, C)
    W = np.einsum("ijk,ip,jq->pqk", D, A, B)
    np.testing.assert_allclose(O.hooi_gram(X, 0, None, B, C), np.einsum("iqr,lqr->il", U, U), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.hooi_gram(X, 1, A, None, C), np.einsum("pjr,plr->jl", V, V), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.hooi_gram(X, 2, A, B, None), np.einsum("pqk,pql->kl", W, W), rtol=1e-12, atol=1e-13)


def test_project_dense_layout():
    D = _tiny().dense()
    C = _orth(5, 4, 3)
    T = O.project_dense(D, C, 2)
    np.testing.assert_allclose(T, np.einsum("ijk,kr->ijr", D, C), rtol=1e-13, atol=1e-14)
    A = _orth(7, 3, 1)
    np.testing.assert_allclose(O.project_dense(D, A, 0), np.einsum("ijk,ip->jkp", D, A), rtol=1e-13, atol=1e-14)


def test_project_sparse_matches_the_definition():
    """The sparse projection against the n-mode product written out as
    einsum on the densified tensor, every mode, ragged sizes (a transposed
    fold or a swapped pair of other modes would fail here)."""
    X = _tiny()
    D = X.dense()
    subs = {0: "ijk,ip->jkp", 1: "ijk,jq->ikq", 2: "ijk,kr->ijr"}
    for m in range(3):
        A = _orth(D.shape[m], 3, 10 + m)
        np.testing.assert_allclose(O.project_sparse(X, A, m), np.einsum(subs[m], D, A), rtol=1e-13, atol=1e-14)


# ---------------------------------------------------------------- core / fit
def test_core_matches_einsum():
    X = _tiny()
    D = X.dense()
    A, B, C = _orth(7, 3, 1), _orth(6, 2, 2), _orth(5, 4, 3)
    np.testing.assert_allclose(O.core_from_slices(X, A, B, C), np.einsum("ijk,ip,jq,kr->pqr", D, A, B, C),
                               rtol=1e-12, atol=1e-13)


def test_fit_three_ways_agree():
    X = _tiny()
    D = X.dense()
    A, B, C = _orth(7, 3, 1), _orth(6, 2, 2), _orth(5, 4, 3)
    G = O.core_from_slices(X, A, B, C)
    f_dense = O.fit_dense(D, G, [A, B, C])
    assert abs(O.fit_slicewise(X, G, A, B, C) - f_dense) < 1e-13
    assert abs(O.fit_identity(X.norm2(), G) - f_dense) < 1e-12
    # a non-optimal core: the identity no longer holds, the explicit forms agree
    G2 = G + 0.1
    assert abs(O.fit_slicewise(X, G2, A, B, C) - O.fit_dense(D, G2, [A, B, C])) < 1e-13


def test_tucker_operator_reconstructs_svd():
    M = np.random.default_rng(4).standard_normal((6, 4))
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    G = np.diag(s)[:, :, None]
    R = O.tucker_dense(G, [U, Vt.T, np.ones((1, 1))])
    np.testing.assert_allclose(R[:, :, 0], M, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- eigenvectors
def test_lead_eigvecs_residual_and_order():
    R = np.random.default_rng(5).standard_normal((30, 50))
    M = R @ R.T
    V, w = O.lead_eigvecs(M, 7)
    assert np.all(np.diff(w) <= 0)
    np.testing.assert_allclose(M @ V, V * w, atol=1e-11 * np.abs(w).max())
    np.testing.assert_allclose(V.T @ V, np.eye(7), atol=1e-13)
    for c in range(7):
        assert V[np.argmax(np.abs(V[:, c])), c] > 0


def test_eigvecs_of_MMt_equal_eigvecs_of_psd_M():
    R = np.random.default_rng(6).standard_normal((25, 40))
    M = R @ R.T
    V1, w1 = O.lead_eigvecs(M, 6)
    V2, w2 = O.lead_eigvecs_of_MMt(M, 6)
    np.testing.assert_allclose(w2, w1 ** 2, rtol=1e-10)
    assert O.subspace_angle(V1, V2) < 1e-8


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("algo", ["hosvd", "hooi", "mp", "sp"])
def test_one_mode_of_size_one_is_truncated_svd(algo):
    idx, vals, dims = synth.matrix_as_tensor(20, 15, 120, 7)
    X = O.SparseTensor3(idx, vals, dims)
    M = X.dense()[:, :, 0]
    U, s, Vt = np.linalg.svd(M)
    J = (4, 3, 1)
    if algo == "hosvd":
        d = O.hosvd(X, J)
    elif algo == "hooi":
        d = O.hooi(X, J, 5, 0.0)
    elif algo == "mp":
        d = O.mp(X, J, 5, 0.0)
    else:
        d = O.sp_algorithm(X, J, np.random.default_rng(1).random((1, 1)), 5, 0.0)
    r = min(J[0], J[1])
    expected = 1 - math.sqrt(np.sum(s[r:] ** 2)) / math.sqrt(np.sum(s ** 2))
    assert abs(d.fits[-1] - expected) < 1e-10
    # the leading columns span the leading singular subspaces; HOOI's
    # columns beyond rank(U_(1)) = J2 J3 = r are any orthonormal completion
    assert O.subspace_angle(U[:, :r], d.factors[0][:, :r]) < 1e-8
    assert O.subspace_angle(Vt[:r].T, d.factors[1][:, :r]) < 1e-8


@pytest.mark.parametrize("algo", ["hosvd", "hooi", "mp"])
def test_exact_tucker_rank_gives_fit_one(algo):
    idx, vals, dims = synth.exact_tucker_block((30, 25, 20), (12, 10, 9), (3, 2, 4), 8)
    X = O.SparseTensor3(idx, vals, dims)
    J = (3, 2, 4)
    d = {"hosvd": lambda: O.hosvd(X, J), "hooi": lambda: O.hooi(X, J, 3, 0.0),
         "mp": lambda: O.mp(X, J, 3, 0.0)}[algo]()
    assert d.fits[-1] > 1 - 1e-7


def test_full_core_gives_fit_one():
    X = _tiny((6, 5, 4), 50, 9)
    for d in (O.hosvd(X, (6, 5, 4)), O.hooi(X, (6, 5, 4), 2, 0.0), O.mp(X, (6, 5, 4), 2, 0.0)):
        assert d.fits[-1] > 1 - 1e-7


@pytest.mark.parametrize("algo", ["hosvd", "hooi", "mp"])
def test_superdiagonal_closed_form(algo):
    idx, vals, dims = synth.superdiagonal(12, 10)
    X = O.SparseTensor3(idx, vals, dims)
    J = (4, 4, 4)
    d = {"hosvd": lambda: O.hosvd(X, J), "hooi": lambda: O.hooi(X, J, 3, 0.0),
         "mp": lambda: O.mp(X, J, 3, 0.0)}[algo]()
    a = np.sort(np.abs(vals))[::-1]
    expected = 1 - math.sqrt(np.sum(a[4:] ** 2)) / math.sqrt(np.sum(a ** 2))
    assert abs(d.fits[-1] - expected) < 1e-12
    top = np.argsort(-np.abs(vals))[:4]
    E = np.zeros((12, 4))
    E[top, np.arange(4)] = 1
    for F in d.factors:
        assert O.subspace_angle(E, F) < 1e-10


# ---------------------------------------------------------------- invariants
def test_hooi_fit_monotone_and_above_hosvd():
    idx, vals, dims = synth.uniform_sparse((40, 35, 30), 3000, 11)
    X = O.SparseTensor3(idx, vals, dims)
    J = (5, 4, 6)
    h = O.hosvd(X, J)
    d = O.hooi(X, J, 8, 0.0)
    assert d.fits[0] >= h.fits[0] - 1e-12
    assert all(b >= a - 1e-12 for a, b in zip(d.fits, d.fits[1:]))


def test_scale_and_permutation_invariance():
    idx, vals, dims = synth.uniform_sparse((20, 18, 16), 600, 12)
    X = O.SparseTensor3(idx, vals, dims)
    J = (3, 3, 3)
    d = O.mp(X, J, 4, 0.0)
    Xs = O.SparseTensor3(idx, 3.5 * vals, dims)
    ds = O.mp(Xs, J, 4, 0.0)
    np.testing.assert_allclose(ds.fits, d.fits, rtol=1e-9)
    np.testing.assert_allclose(ds.core, 3.5 * d.core, rtol=1e-7, atol=1e-9)
    perm = np.random.default_rng(2).permutation(20)
    idx_p = idx.copy()
    idx_p[0] = perm[idx[0]]
    dp = O.mp(O.SparseTensor3(idx_p, vals, dims), J, 4, 0.0)
    np.testing.assert_allclose(dp.fits, d.fits, rtol=1e-9)
    A_back = np.empty_like(dp.factors[0])
    A_back[:] = dp.factors[0][perm]
    assert O.subspace_angle(d.factors[0], A_back) < 1e-7


def test_nonzero_order_is_irrelevant():
    idx, vals, dims = synth.uniform_sparse((15, 14, 13), 400, 13)
    perm = np.random.default_rng(3).permutation(400)
    a = O.hooi(O.SparseTensor3(idx, vals, dims), (3, 3, 3), 3, 0.0)
    b = O.hooi(O.SparseTensor3(idx[:, perm], vals[perm], dims), (3, 3, 3), 3, 0.0)
    np.testing.assert_allclose(a.fits, b.fits, rtol=1e-12)


def test_brute_force_rank_one_on_2x2x2():
    rng = np.random.default_rng(14)
    for trial in range(5):
        D = rng.random((2, 2, 2))
        idx = np.array(np.nonzero(np.ones((2, 2, 2))), dtype=np.int32)
        X = O.SparseTensor3(idx, D[idx[0], idx[1], idx[2]], (2, 2, 2))
        d = O.hooi(X, (1, 1, 1), 30, 0.0)
        # grid search over unit vectors (cos t, sin t) for each mode
        ts = np.linspace(0, np.pi, 181)
        U = np.stack([np.cos(ts), np.sin(ts)])
        g = np.einsum("ijk,ia,jb,kc->abc", D, U, U, U)
        best = np.max(g * g)
        best_fit = 1 - math.sqrt(max(0.0, np.sum(D * D) - best)) / math.sqrt(np.sum(D * D))
        assert d.fits[-1] >= best_fit - 1e-6
        assert d.fits[-1] <= best_fit + 2e-3


def test_exact_rank_factors_span_the_unfolding_column_spaces():
    idx, vals, dims = synth.exact_tucker_block((30, 25, 20), (12, 10, 9), (3, 2, 4), 16)
    X = O.SparseTensor3(idx, vals, dims)
    D = X.dense()
    J = (3, 2, 4)
    for d in (O.hosvd(X, J), O.hooi(X, J, 3, 0.0), O.mp(X, J, 3, 0.0)):
        for n in range(3):
            U, s, _ = np.linalg.svd(O.unfold_dense(D, n), full_matrices=False)
            assert O.subspace_angle(U[:, :J[n]], d.factors[n]) < 1e-9


# ---------------------------------------------------------------- the paper's numbers
@pytest.mark.slow
def test_paper_fits_250cube(golden_dir):
    with open(os.path.join(golden_dir, "paper_fits_250cube.json")) as f:
        g = json.load(f)
    dims = tuple(g["tensor"]["dims"])
    idx, vals, dims = synth.bernoulli_sparse(dims, g["tensor"]["density"], 11)
    X = O.SparseTensor3(idx, vals, dims)
    J = tuple(g["core"])
    tol, it = g["stopping"]["threshold"], g["stopping"]["max_iters"]
    got = {
        "HO-SVD": O.hosvd(X, J, fit="identity").fits[-1],
        "HOOI": O.hooi(X, J, it, tol, fit="identity").fits[-1],
        "MP": O.mp(X, J, it, tol, fit="identity").fits[-1],
        "SP": O.sp_algorithm(X, J, np.random.default_rng(7).random((dims[2], J[2])), it, tol,
                             fit="identity").fits[-1],
    }
    band = g["band_percent_points"]
    for name, pct in g["fit_percent"].items():
        assert abs(100 * got[name] - pct) <= band, (name, 100 * got[name], pct)


def test_core_entry_definition_matches_slicewise_core():
    idx, vals, dims = synth.uniform_sparse((13, 11, 9), 300, 77)
    idx2, vals2 = synth.with_duplicates(idx, vals, 40, 3)
    X = O.SparseTensor3(idx2, vals2, dims)
    rng = np.random.default_rng(5)
    A, B, C = (np.linalg.qr(rng.standard_normal((d, j)))[0] for d, j in zip(dims, (4, 3, 5)))
    G = O.core_from_slices(X, A, B, C)
    for p, q, r in [(0, 0, 0), (3, 2, 4), (1, 2, 3), (2, 0, 1)]:
        assert abs(O.core_entry(X, A, B, C, p, q, r) - G[p, q, r]) <= 1e-12 * max(1.0, np.abs(G).max())


def test_small_reference_is_the_oracles():
    """tests/golden/small_reference.npz (the benchmark's parity reference) is
    what the oracle computes now."""
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("msr", os.path.join(here, "golden", "make_small_reference.py"))
    msr = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(msr)
    now = msr.compute()
    stored = np.load(os.path.join(here, "golden", "small_reference.npz"), allow_pickle=False)
    assert sorted(now) == sorted(stored.files)
    for k in now:
        np.testing.assert_allclose(stored[k], now[k], rtol=0, atol=1e-12, err_msg=k)


def _rot(n, pairs, thetas):
    """Orthonormal columns: column c is cos(t) e_a + sin(t) e_b for
    (a, b), t in zip(pairs, thetas)."""
    B = np.zeros((n, len(pairs)))
    for c, ((a, b), t) in enumerate(zip(pairs, thetas)):
        B[a, c] = np.cos(t)
        B[b, c] = np.sin(t)
    return B


@pytest.mark.parametrize("theta", [0.0, 1e-12, 1e-9, 1e-6, 1e-3, 0.1, 0.7, 1.2, np.pi / 2])
def test_subspace_angle_known_angles(theta):
    """span{e1} against span{cos(t) e1 + sin(t) e2} is at angle t exactly,
    including the small-angle regime where arccos of the cosine loses it."""
    n = 7
    A = np.eye(n)[:, :1]
    B = _rot(n, [(0, 1)], [theta])
    got = O.subspace_angle(A, B)
    assert abs(got - theta) <= 1e-15 + 1e-12 * theta, (got, theta)
    # the largest of several principal angles, whatever the column order
    A3 = np.eye(n)[:, :3]
    B3 = _rot(n, [(0, 3), (1, 4), (2, 5)], [theta / 3, theta, theta / 2])
    assert abs(O.subspace_angle(A3, B3) - theta) <= 1e-15 + 1e-12 * theta
    assert abs(O.subspace_angle(A3, B3[:, ::-1]) - theta) <= 1e-15 + 1e-12 * theta


def test_subspace_angle_basis_invariance_and_symmetry():
    """The angle depends on the spans only: any orthonormal basis of either
    gives the same value, and for equal dimensions it is symmetric."""
    rng = np.random.default_rng(3)
    n, k = 40, 5
    A = np.linalg.qr(rng.standard_normal((n, k)))[0]
    B = np.linalg.qr(A + 0.05 * rng.standard_normal((n, k)))[0]
    a = O.subspace_angle(A, B)
    assert a > 1e-3
    Q = np.linalg.qr(rng.standard_normal((k, k)))[0]
    assert abs(O.subspace_angle(A @ Q, B) - a) < 1e-13
    assert abs(O.subspace_angle(A, B @ Q) - a) < 1e-13
    assert abs(O.subspace_angle(B, A) - a) < 1e-13
    # against the principal angles from the singular values of A^T B
    # (Bjorck and Golub), accurate at this size
    s = np.linalg.svd(A.T @ B, compute_uv=False)
    assert abs(np.arccos(np.clip(s.min(), -1, 1)) - a) < 1e-8
    # a span and itself
    assert O.subspace_angle(A, A @ Q) < 1e-14


def test_bench_angle_is_the_oracles():
    """The benchmark's own copy of the comparison (it may not import the
    oracle outside its CPU-baseline leg) equals the oracle's function."""
    import bench
    rng = np.random.default_rng(5)
    for k in (1, 4, 9):
        A = np.linalg.qr(rng.standard_normal((30, k)))[0]
        B = np.linalg.qr(A + 0.1 * rng.standard_normal((30, k)))[0]
        assert bench.subspace_angle(A, B) == O.subspace_angle(A, B)


def test_random_start_columns():
    """SP's start (Figure 5): entries uniform on [0, 1) from SplitMix64
    before normalisation (mean 1/2, second moment 1/3), unit columns, and the
    draw of entry (i, r) fixed by (mode, i, r, seed) alone."""
    from oracle.learn import splitmix64_at
    C = O.random_start(300, 4, 2, 77)
    assert np.allclose(np.linalg.norm(C, axis=0), 1.0, atol=1e-15)
    raw = np.array([[(splitmix64_at(77, (2 << 40) + i * 4 + r) >> 11) * 2.0 ** -53 for r in range(4)]
                    for i in range(300)])
    assert raw.min() >= 0.0 and raw.max() < 1.0
    assert abs(raw.mean() - 0.5) < 0.03 and abs((raw ** 2).mean() - 1 / 3) < 0.03
    assert np.allclose(C * np.linalg.norm(raw, axis=0), raw, rtol=1e-15, atol=0)
    assert not np.allclose(O.random_start(300, 4, 1, 77), C)

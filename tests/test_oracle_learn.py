"""Pins of the learned-start oracle (no GPU): the counter-based generator
against its published test vectors, the Gaussian transform against its
moments, the sketch against a dense brute-force product, and both hand-written
gradients (perceptron backward pass, alignment loss) against central finite
differences."""
import json
import os

import numpy as np
import pytest

from oracle import learn as L

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.json")


def test_splitmix64_published_vectors():
    d = json.load(open(GOLD))
    for v in d["vectors"]:
        want = [int(h, 16) for h in v["outputs_hex"]] if "outputs_hex" in v else v["outputs"]
        assert L.splitmix64(v["seed"], len(want)) == want
        assert [L.splitmix64_at(v["seed"], k) for k in range(len(want))] == want


def test_box_muller_moments():
    rows = np.stack([L.sketch_omega(99, 1, lin) for lin in range(400)])  # 25,600 draws
    x = rows.ravel()
    assert abs(x.mean()) < 0.03
    assert abs(x.var() - 1.0) < 0.04
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(rows[:, 0::2].ravel(), rows[:, 1::2].ravel())[0, 1]) < 0.03
    # fourth moment of a standard normal is 3
    assert abs((x ** 4).mean() - 3.0) < 0.3


def _tiny(seed=3):
    rng = np.random.default_rng(seed)
    dims = (5, 4, 3)
    lin = rng.choice(60, 25, replace=False)
    i, r = np.divmod(lin, 12)
    j, k = np.divmod(r, 3)
    idx = np.stack([i, j, k]).astype(np.int32)
    vals = rng.uniform(0, 1, 25)
    return idx, vals, dims


@pytest.mark.parametrize("n", [0, 1, 2])
def test_sketch_equals_dense_unfolding_times_omega(n):
    idx, vals, dims = _tiny()
    a, b = (n + 1) % 3, (n + 2) % 3
    Xn = np.zeros((dims[n], dims[a] * dims[b]))
    for p in range(len(vals)):
        Xn[idx[n][p], idx[a][p] * dims[b] + idx[b][p]] += vals[p]
    Om = L.sketch_dense_omega(7, n, dims)
    np.testing.assert_allclose(L.sketch(idx, vals, dims, n, 7), Xn @ Om, rtol=1e-13, atol=1e-13)
    # other seeds and other modes give other matrices
    assert not np.allclose(Om, L.sketch_dense_omega(8, n, dims))


def test_row_features():
    S = np.array([[3.0, 4.0], [0.0, 0.0]])
    F, rho = L.row_features(S)
    np.testing.assert_allclose(rho, [5.0, 0.0])
    np.testing.assert_allclose(F, [[0.6, 0.8], [0.0, 0.0]])


def _mlp_case(seed=0, rows=9):
    rng = np.random.default_rng(seed)
    theta = 0.2 * rng.standard_normal(L.param_count())
    F = rng.standard_normal((rows, L.N_IN))
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    rho = rng.uniform(0.5, 2.0, rows)
    return theta, F, rho


def test_mlp_forward_matches_layer_definition():
    theta, F, rho = _mlp_case()
    W1, b1, W2, b2 = L.unpack(theta)
    R, Z1 = L.mlp_forward(F, rho, theta)
    for i in range(F.shape[0]):  # one row at a time, written out
        h = np.array([max(0.0, sum(F[i, k] * W1[k, u] for k in range(L.N_IN)) + b1[u]) for u in range(L.N_HID)])
        r = rho[i] * (h @ W2 + b2)
        np.testing.assert_allclose(R[i], r, rtol=1e-12, atol=1e-12)


def test_mlp_backward_against_central_differences():
    theta, F, rho = _mlp_case(1)
    rng = np.random.default_rng(5)
    G = rng.standard_normal((F.shape[0], L.N_OUT))   # scalar = <R, G>, so dR = G

    def f(t):
        return float((L.mlp_forward(F, rho, t)[0] * G).sum())

    R, Z1 = L.mlp_forward(F, rho, theta)
    g = L.mlp_backward(F, rho, theta, Z1, G)
    h = 1e-6
    picks = np.concatenate([rng.choice(L.param_count(), 60, replace=False),
                            [0, L.N_IN * L.N_HID, L.param_count() - 1]])
    for p in picks:
        e = np.zeros_like(theta)
        e[p] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(fd)), (p, fd, g[p])
    # a random direction through all parameters at once
    d = rng.standard_normal(theta.size)
    fd = (f(theta + h * d) - f(theta - h * d)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd))


def _orth(rng, n, J):
    return np.linalg.qr(rng.standard_normal((n, J)))[0]


def test_align_loss_values_and_invariance():
    rng = np.random.default_rng(2)
    n, J, K = 40, 6, 9
    A = _orth(rng, n, J)
    M = rng.standard_normal((K, K)) + 3 * np.eye(K)
    # span(Rk) contains span(A): loss 0
    Rk = np.concatenate([A, rng.standard_normal((n, K - J))], axis=1) @ M
    R = np.concatenate([Rk, rng.standard_normal((n, 3))], axis=1)
    assert abs(L.align_loss(R, K, A, 0.0)[0]) < 1e-12
    Rp = _orth(rng, n, K)
    l1 = L.align_loss(Rp, K, A, 0.0)[0]
    assert 0.0 <= l1 <= 1.0
    # column mixing of Rk leaves the loss unchanged
    assert abs(L.align_loss(Rp @ M, K, A, 0.0)[0] - l1) < 1e-12
    # mean squared sine of the principal angles (textbook definition via SVD)
    s = np.linalg.svd(A.T @ Rp, compute_uv=False)
    assert abs(l1 - (1.0 - np.sum(s ** 2) / J)) < 1e-12
    # orthogonal complement: loss 1
    Q = np.linalg.qr(np.concatenate([A, rng.standard_normal((n, K))], axis=1))[0][:, J:]
    assert abs(L.align_loss(Q, K, A, 0.0)[0] - 1.0) < 1e-12


def test_align_loss_gradient_against_central_differences():
    rng = np.random.default_rng(4)
    n, J, K, W = 30, 5, 7, 10
    A = _orth(rng, n, J)
    R = rng.standard_normal((n, W))
    lam = 1e-3
    Lv, dR = L.align_loss(R, K, A, lam)
    h = 1e-6
    for _ in range(40):
        i, c = rng.integers(n), rng.integers(W)
        E = np.zeros_like(R)
        E[i, c] = h
        fd = (L.align_loss(R + E, K, A, lam)[0] - L.align_loss(R - E, K, A, lam)[0]) / (2 * h)
        assert abs(fd - dR[i, c]) <= 1e-7 * max(1.0, abs(fd)), (i, c, fd, dR[i, c])
    assert np.all(dR[:, K:] == 0)


def test_start_factor_is_rayleigh_ritz_on_the_test_span():
    rng = np.random.default_rng(6)
    n, J = 60, 5
    K = L.test_width(J)
    assert K == 10 and L.test_width(100) == 128
    Y = rng.standard_normal((n, 3 * n))
    H = Y @ Y.T
    R = rng.standard_normal((n, 16))
    U, th, g = L.start_factor(R, H, J)
    assert np.abs(U.T @ U - np.eye(J)).max() < 1e-12
    P = np.linalg.qr(R[:, :K])[0]
    assert np.abs(P @ (P.T @ U) - U).max() < 1e-10            # inside span(R[:, :K])
    np.testing.assert_allclose(np.diag(U.T @ H @ U), th, rtol=1e-10)
    # the best J-dimensional subspace of H within the span (Courant-Fischer)
    w = np.linalg.eigvalsh(P.T @ H @ P)[::-1][:J]
    np.testing.assert_allclose(th, w, rtol=1e-10)
    # when the span contains H's leading eigenvectors, they are recovered
    E = np.linalg.eigh(H)[1][:, ::-1][:, :J]
    R2 = np.concatenate([E, rng.standard_normal((n, K - J))], axis=1) @ rng.standard_normal((K, K))
    U2 = L.start_factor(R2, H, J)[0]
    assert np.abs(U2 @ U2.T - E @ E.T).max() < 1e-9


def test_bf16_round_values():
    # exactly representable values stay, ties go to the even significand
    x = np.array([1.0, -2.5, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, 65504.0, 0.0], dtype=np.float32)
    want = [1.0, -2.5, 1.0, 1.0 + 4 * 2.0 ** -8, 1.0, 65536.0, 0.0]
    np.testing.assert_array_equal(L.bf16_round(x), want)
    # relative rounding error at most 2^-8 (half a unit in the 8-bit significand)
    r = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    rel = np.abs(L.bf16_round(r) - r) / np.abs(r)
    assert rel.max() <= 2.0 ** -8 * (1 + 1e-6)

"""Step-level parity on the GPU: the leading-eigenvector solver against LAPACK
(numpy.linalg.eigh) on the Grams the oracle builds for HOOI and MP, and on
synthetic matrices with known spectra (gapped, one dominant eigenvalue over a
clustered bulk, rank-deficient), at the oracle-level tolerance and at the looser
ones of the reduced-precision forms."""
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


def _check(tk, M, J, tol=1e-14, angle=None, warm=False, ws=None):
    F, th, it, st, _ = tk.lead_eig(torch.from_numpy(M).cuda(), J, tol=tol, warm=warm, workspace=ws)
    F = F.cpu().numpy()
    th = th.cpu().numpy()
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(th))
    assert np.abs(F.T @ F - np.eye(J)).max() < 1e-12
    w, V = np.linalg.eigh(0.5 * (M + M.T))
    w, V = w[::-1], V[:, ::-1]
    e_ref = w[:J].sum()
    e_got = np.trace(F.T @ M @ F)
    scale = max(abs(w[0]), 1e-300)
    assert abs(e_got - e_ref) <= 1e-11 * scale * J, (e_got, e_ref)
    assert np.all(np.diff(th) <= 1e-12 * scale)
    np.testing.assert_allclose(th, w[:J], rtol=0, atol=1e-9 * scale)
    if angle is not None:
        assert O.subspace_angle(V[:, :J], F) < angle
    for c in range(J):
        assert F[np.argmax(np.abs(F[:, c])), c] > 0
    return it


@pytest.fixture(scope="module")
def mid_grams():
    idx, vals, dims = synth.uniform_sparse((301, 257, 190), 60_000, 21)
    X = O.SparseTensor3(idx, vals, dims)
    J = (23, 17, 9)
    h = O.hosvd(X, J)
    A, B, C = h.factors
    return {
        "hooi0": (O.hooi_gram(X, 0, None, B, C), J[0]),
        "hooi1": (O.hooi_gram(X, 1, A, None, C), J[1]),
        "hooi2": (O.hooi_gram(X, 2, A, B, None), J[2]),
        "mp0": (O.mp_gram(X, 0, None, B, C), J[0]),
        "hosvd1": (O.unfolding_gram(X, 1), J[1]),
    }


@pytest.mark.parametrize("name", ["hooi0", "hooi1", "hooi2", "mp0", "hosvd1"])
def test_lead_eig_on_method_grams(tk, mid_grams, name):
    _say(f"lead_eig {name}")
    M, J = mid_grams[name]
    _check(tk, M, J)


def test_lead_eig_gapped_subspace(tk):
    _say("lead_eig gapped")
    rng = np.random.default_rng(1)
    n, J = 400, 30
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.concatenate([np.linspace(100, 50, J), np.linspace(20, 0.1, n - J)])
    M = (Q * lam) @ Q.T
    _check(tk, M, J, angle=1e-9)


def test_lead_eig_spike_over_clustered_bulk(tk):
    _say("lead_eig spike")
    rng = np.random.default_rng(2)
    n, J = 600, 50
    R = rng.standard_normal((n, 20 * n)) / np.sqrt(20 * n)
    M = R @ R.T
    u = np.ones(n) / np.sqrt(n)
    M += 500.0 * np.outer(u, u)
    _check(tk, M, J)


def test_lead_eig_flat_spectrum_cold_start(tk):
    """A few leading eigenvalues over a long flat bulk (the spectrum of MP's
    Grams on very sparse uniform tensors: 1M nonzeros in 10000^3). The Ritz
    values of a random start block sit near the bulk's middle, far below the
    top; the first filters must take their degree from an upper bound of the
    whole spectrum, or the leading directions are amplified past what the
    block's orthonormalisation resolves (non-finite output)."""
    _say("lead_eig flat spectrum, cold start")
    rng = np.random.default_rng(4)
    n, J = 3000, 50
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    top = np.array([1.67, 1.39, 1.05, 0.91, 0.83])
    shelf = np.linspace(0.80, 0.62, 60)
    bulk = np.linspace(0.60, 0.16, n - top.size - shelf.size)
    lam = np.concatenate([top, shelf, bulk])
    M = (Q * lam) @ Q.T
    _check(tk, M, J, tol=1e-12)


def test_lead_eig_rank_deficient(tk):
    _say("lead_eig rank deficient")
    rng = np.random.default_rng(3)
    n, r, J = 350, 12, 20
    Y = rng.standard_normal((n, r))
    M = Y @ Y.T
    F, th, it, st, _ = tk.lead_eig(torch.from_numpy(M).cuda(), J, tol=1e-14)
    F = F.cpu().numpy()
    assert np.all(np.isfinite(F))
    assert np.abs(F.T @ F - np.eye(J)).max() < 1e-12
    U = np.linalg.svd(Y, full_matrices=False)[0]
    assert O.subspace_angle(U, F[:, :r]) < 1e-8


@pytest.mark.parametrize("n,J", [(100, 10), (140, 40), (33, 33), (7, 1)])
def test_lead_eig_direct_sizes(tk, n, J):
    _say(f"lead_eig direct {n} {J}")
    rng = np.random.default_rng(n)
    R = rng.standard_normal((n, 3 * n))
    M = R @ R.T
    _check(tk, M, J, angle=1e-8 if J < n else None)


def test_lead_eig_warm_start_sequence(tk):
    """The sweep order of HOOI: a cold solve of the HO-SVD Gram of mode 3,
    then a warm solve of HOOI's mode-3 Gram from the block it left."""
    _say("lead_eig warm sequence")
    idx, vals, dims = synth.uniform_sparse((301, 257, 190), 60_000, 21)
    X = O.SparseTensor3(idx, vals, dims)
    J = (23, 17, 9)
    d = O.hooi(X, J, 1, 0.0)
    A, B, _ = d.factors
    H2 = O.unfolding_gram(X, 2)
    M2 = O.hooi_gram(X, 2, A, B, None)
    n = dims[2]
    need = tk.lib  # keep flake quiet
    F, th, it, st, ws = tk.lead_eig(torch.from_numpy(H2).cuda(), J[2], tol=1e-13)
    _check(tk, M2, J[2], tol=1e-13, warm=True, ws=ws)


@pytest.mark.parametrize("n,J", [(150, 128), (300, 120), (1200, 60)])
def test_lead_eig_wide_subspace_and_k_split(tk, n, J):
    """J at the API cap (128) and near it, where the block (at most 140
    columns) has few extra columns, and a larger n (1200: one-pass products
    over 75 row strips), on a gapped spectrum."""
    _say(f"lead_eig wide {n} {J}")
    rng = np.random.default_rng(n + J)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.concatenate([np.linspace(200, 100, J), np.linspace(30, 0.01, n - J)])
    M = (Q * lam) @ Q.T
    _check(tk, M, J, angle=1e-8)


def test_lead_eig_split_k_products(tk):
    """n = 2500 > 2048: the eigensolver's products over n use split-K partial
    strips summed in a fixed order by a second kernel."""
    _say("lead_eig split-K 2500")
    rng = np.random.default_rng(7)
    n, J = 2500, 20
    Y = rng.standard_normal((n, 60))
    lam = np.concatenate([np.linspace(10, 5, J), np.linspace(1, 0.1, 40)])
    M = (Y * lam) @ Y.T / n + 1e-3 * np.eye(n)
    _check(tk, M, J, angle=1e-7)


@pytest.mark.parametrize("tol", [1e-4, 1e-8])
@pytest.mark.parametrize("case", ["gapped", "mp0"])
def test_lead_eig_loose_tolerance(tk, mid_grams, case, tol):
    """The tolerances of the reduced-precision forms (1e-4 mixed, 1e-8 FP32):
    the sum E of the J leading Ritz values within tol * E of LAPACK's (the
    stop rule), each returned value the diagonal entry of F^T M F, and the
    closing Rayleigh-Ritz step's Jacobi stopped at an off-diagonal norm of
    at most 1e-4 tol relative to the whole of F^T M F; F orthonormal with
    the sign convention at any tolerance."""
    _say(f"lead_eig loose {case} {tol}")
    if case == "gapped":
        rng = np.random.default_rng(11)
        n, J = 400, 30
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        lam = np.concatenate([np.linspace(100, 50, J), np.linspace(20, 0.1, n - J)])
        M = (Q * lam) @ Q.T
    else:
        M, J = mid_grams["mp0"]
    F, th, it, st, _ = tk.lead_eig(torch.from_numpy(M).cuda(), J, tol=tol)
    F = F.cpu().numpy()
    th = th.cpu().numpy()
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(th))
    assert np.abs(F.T @ F - np.eye(J)).max() < 1e-12
    w = np.linalg.eigvalsh(0.5 * (M + M.T))[::-1]
    scale = abs(w[0])
    e_ref = w[:J].sum()
    H = F.T @ M @ F
    assert abs(np.trace(H) - e_ref) <= tol * abs(e_ref), (np.trace(H), e_ref)
    np.testing.assert_allclose(th, np.diag(H), rtol=0, atol=1e-11 * scale)
    assert np.all(np.diff(th) <= 1e-12 * scale)
    assert np.all(th <= w[:J] + 1e-11 * scale)  # Ritz values never exceed the eigenvalues
    # locked columns (residual at most 1e-11 of the top value) couple to the
    # rest at that level, outside the closing step's block
    off = np.linalg.norm(H - np.diag(np.diag(H)))  # directly: a difference of squared sums cancels
    assert off <= 2e-4 * tol * np.linalg.norm(H) + 1e-9 * scale, off
    for c in range(J):
        assert F[np.argmax(np.abs(F[:, c])), c] > 0

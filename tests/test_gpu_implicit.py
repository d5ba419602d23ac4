"""Multislice Projection through implicit Gram products (tucker_mp_implicit)
against the FP64 oracle's MP (Figure 7) and the GPU's dense tucker_mp.

* Ragged low-occupancy tensors (a planted Tucker model sampled at uniform
  coordinates, whose leading eigenvalues are well separated; uniform values
  at a tighter eigensolver tolerance) with one mode small enough (<= 140) for M_n
  to be formed from products with the identity and two modes solved through
  the operator: FP64 fit after every sweep within 1e-9 of the oracle's, core
  and orthonormal factors, the same random start as the oracle's;
* FP64 within 1e-10 of the dense GPU path, FP32 within 1e-6 and mixed
  (BF16 projections) within 1e-4 of the dense path at the same precision,
  both within 1e-4 of the oracle on uniform values;
* a given start with the paper's stopping rule stops after the same sweep as
  the dense path; duplicates are summed; the order of distinct nonzeros
  changes no bit; exact Tucker rank gives fit 1;
* 4000 x 3000 x 2000 with 300,000 planted-model nonzeros (occupancy of the
  fibres below 0.05): against the dense path in FP64 and mixed, every product kernel
  launch traced;
* 20000^3 with 1,000,000 nonzeros, where the dense projections would take
  tens of GB: orthonormal factors, core entries sampled against the oracle's
  definition (one entry at a time over the nonzeros), fit from the identity.
"""
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


@pytest.fixture(scope="module")
def ragged():
    # slots per ordering 230*170 .. 170*90: about 15 % of the fibres
    # non-empty. A planted Tucker model (core 7 x 5 x 4, 10 % noise) sampled
    # at uniform coordinates: its leading eigenvalues stand apart from the
    # rest, so two correct solvers agree on the subspaces to rounding and the
    # fits to 1e-10 (on pure noise near-ties of the J-th eigenvalue let the
    # fits of correct solves differ by about 1e-9).
    idx, vals, dims = synth.planted_tucker((230, 170, 90), (7, 5, 4), 6000, 0.1, 311)
    return idx, vals, dims, (7, 5, 4)


def _oracle_mp(idx, vals, dims, J, sweeps, tol=0.0, B0=None, C0=None):
    X = O.SparseTensor3(idx, vals, dims)
    if B0 is None:
        B0 = O.random_start(dims[1], J[1], 1, SEED)
        C0 = O.random_start(dims[2], J[2], 2, SEED)
    return X, O.mp(X, J, sweeps, tol, init=(None, B0, C0), fit="identity")


def test_fp64_matches_oracle(tk, ragged):
    idx, vals, dims, J = ragged
    _say(f"implicit mp fp64 {dims} core {J}")
    X, ref = _oracle_mp(idx, vals, dims, J, 5)
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, J, precision="fp64", max_iters=5, tol=0.0, seed=SEED)
    d = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
    _say(f"  gpu {r.fits[-1]:.10f} oracle {ref.fits[-1]:.10f} max|d| {d:.2e}")
    assert r.iters == 5 and d < 1e-9
    facs = [f.cpu().numpy() for f in r.factors]
    for F in facs:
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-10
    G = r.core.cpu().numpy()
    np.testing.assert_allclose(G, O.core_from_slices(X, *facs), rtol=0, atol=1e-10 * np.abs(G).max())
    # the factors span the oracle's subspaces
    for n in range(3):
        assert O.subspace_angle(facs[n], ref.factors[n]) < 1e-6


def test_uniform_noise_matches_dense_path(tk):
    """Uniform U(0,1) values (the paper's random tensors): near-tied
    eigenvalues, so the implicit and dense paths are compared at a tighter
    eigensolver tolerance, fits within 1e-9."""
    idx, vals, dims = synth.uniform_sparse((230, 170, 90), 6000, 311)
    J = (7, 5, 4)
    di, dv = _dev(idx, vals)
    kw = dict(precision="fp64", max_iters=5, tol=0.0, init=tk.INIT_RANDOM, seed=SEED, eig_tol=1e-15)
    r = tk.mp_implicit(di, dv, dims, J, **kw)
    c = tk.mp(di, dv, dims, J, **kw)
    d = np.max(np.abs(np.array(r.fits) - np.array(c.fits)))
    _say(f"implicit vs dense, uniform values: fit {r.fits[-1]:.10f} max|d| {d:.2e}")
    assert d < 1e-9


def test_fp64_matches_dense_path(tk, ragged):
    idx, vals, dims, J = ragged
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, J, precision="fp64", max_iters=4, tol=0.0, seed=SEED)
    c = tk.mp(di, dv, dims, J, precision="fp64", max_iters=4, tol=0.0, init=tk.INIT_RANDOM, seed=SEED)
    d = np.max(np.abs(np.array(r.fits) - np.array(c.fits)))
    _say(f"implicit vs dense fp64: max|d| {d:.2e}")
    assert d < 1e-10
    Gi, Gc = r.core.cpu().numpy(), c.core.cpu().numpy()
    assert np.abs(np.abs(Gi) - np.abs(Gc)).max() < 1e-8 * np.abs(Gc).max()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("mixed", 1e-4)])
def test_reduced_precision(tk, ragged, prec, tol):
    """Against the dense path at the same precision (the same operator up to
    the products' rounding). On this noisy model the reduced-precision
    rounding itself moves both paths' fits away from FP64 alike (FP32 by
    about 4e-6, BF16 by about 1e-3), so the oracle bar is checked on uniform
    values below."""
    idx, vals, dims, J = ragged
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, J, precision=prec, max_iters=5, tol=0.0, seed=SEED)
    c = tk.mp(di, dv, dims, J, precision=prec, max_iters=5, tol=0.0, init=tk.INIT_RANDOM, seed=SEED)
    d = np.max(np.abs(np.array(r.fits) - np.array(c.fits)))
    _say(f"implicit {prec}: |d| dense {d:.2e}")
    assert d < tol


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
def test_reduced_precision_uniform_values_vs_oracle(tk, prec):
    """Uniform U(0,1) values, the paper's random tensors: within 1e-4 of the
    FP64 oracle's fit after every sweep."""
    idx, vals, dims = synth.uniform_sparse((230, 170, 90), 6000, 311)
    J = (7, 5, 4)
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, J, precision=prec, max_iters=5, tol=0.0, seed=SEED)
    _, ref = _oracle_mp(idx, vals, dims, J, 5)
    do = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
    _say(f"implicit {prec}, uniform values: |d| oracle {do:.2e}")
    assert do < 1e-4


def test_given_start_stopping_rule_and_duplicates(tk, ragged):
    idx, vals, dims, J = ragged
    idx2, vals2 = synth.with_duplicates(idx, vals, 800, 21)
    rng = np.random.default_rng(5)
    facs = [torch.zeros((dims[0], J[0]), dtype=torch.float64)] + [
        torch.from_numpy(np.linalg.qr(rng.standard_normal((dims[n], J[n])))[0]) for n in (1, 2)]
    di, dv = _dev(idx2, vals2)
    r = tk.mp_implicit(di, dv, dims, J, precision="fp64", max_iters=30, tol=1e-4, init=tk.INIT_GIVEN, factors=facs)
    c = tk.mp(di, dv, dims, J, precision="fp64", max_iters=30, tol=1e-4, init=tk.INIT_GIVEN, factors=facs)
    _say(f"implicit given start: sweeps {r.iters} vs {c.iters}, fit {r.fits[-1]:.9f} vs {c.fits[-1]:.9f}")
    assert r.iters == c.iters
    assert np.max(np.abs(np.array(r.fits) - np.array(c.fits))) < 1e-10
    assert r.stats["nnz_unique"] == c.stats["nnz_unique"] < vals2.size
    _, ref = _oracle_mp(idx2, vals2, dims, J, r.iters, 0.0, facs[1].numpy(), facs[2].numpy())
    assert np.max(np.abs(np.array(r.fits) - np.array(ref.fits))) < 1e-9


def test_input_order_changes_no_bit(tk, ragged):
    idx, vals, dims, J = ragged
    d0, v0 = _dev(idx, vals)
    r0 = tk.mp_implicit(d0, v0, dims, J, precision="fp64", max_iters=3, tol=0.0, seed=SEED)
    perm = np.random.default_rng(1).permutation(vals.size)
    dp, vp = _dev(idx[:, perm], vals[perm])
    r1 = tk.mp_implicit(dp, vp, dims, J, precision="fp64", max_iters=3, tol=0.0, seed=SEED)
    assert r1.fits == r0.fits
    assert torch.equal(r1.core, r0.core)


def test_exact_tucker_rank_fit_one(tk):
    idx, vals, dims = synth.exact_tucker_block((400, 300, 100), (160, 150, 12), (3, 2, 3), 8)
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, (3, 2, 3), precision="fp64", max_iters=3, tol=0.0, seed=SEED)
    _say(f"implicit exact rank: fit {r.fits[-1]:.12f}")
    assert r.fits[-1] > 1 - 1e-7


def test_mid_size_against_dense(tk):
    """4000 x 3000 x 2000, 300,000 nonzeros of a planted model with core
    16 x 12 x 8 (10 % noise): the dense path still fits (projections of
    6e6 - 1.2e7 slots) and agrees."""
    idx, vals, dims = synth.planted_tucker((4000, 3000, 2000), (16, 12, 8), 300_000, 0.1, 4242)
    J = (16, 12, 8)
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0, seed=SEED, timing=True, trace=4096)
    c = tk.mp(di, dv, dims, J, precision="fp64", max_iters=3, tol=0.0, init=tk.INIT_RANDOM, seed=SEED)
    d = np.max(np.abs(np.array(r.fits) - np.array(c.fits)))
    nprod = sum(1 for e in r.stats["trace"] if e["phase"] == "gram")
    _say(f"implicit 4000x3000x2000 fp64: fit {r.fits[-1]:.10f} dense {c.fits[-1]:.10f} |d| {d:.2e}; "
         f"sweeps {r.stats['sweeps_ms']:.1f} ms vs dense {c.stats['sweeps_ms']:.1f} ms; {nprod} product kernels, "
         f"{r.stats['gram_ms']:.1f} ms")
    assert d < 1e-10
    assert r.stats["trace_dropped"] == 0 and nprod == r.stats["gram_calls"] > 0
    rm = tk.mp_implicit(di, dv, dims, J, precision="mixed", max_iters=3, tol=0.0, seed=SEED)
    dm = np.max(np.abs(np.array(rm.fits) - np.array(c.fits)))
    _say(f"  mixed: fit {rm.fits[-1]:.8f} |d| vs dense fp64 {dm:.2e}")
    assert dm < 1e-4


def test_20000_cube_one_million(tk):
    """20000^3 with 1,000,000 uniform nonzeros, core 20^3, FP64, 2 sweeps."""
    idx, vals, dims = synth.uniform_sparse((20000, 20000, 20000), 1_000_000, 2007)
    J = (20, 20, 20)
    di, dv = _dev(idx, vals)
    r = tk.mp_implicit(di, dv, dims, J, precision="fp64", max_iters=2, tol=0.0, seed=SEED)
    facs = [f.cpu().numpy() for f in r.factors]
    for F in facs:
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-10
    X = O.SparseTensor3(idx, vals, dims)
    G = r.core.cpu().numpy()
    rng = np.random.default_rng(0)
    worst = 0.0
    for _ in range(12):
        p, q, s = (int(rng.integers(0, j)) for j in J)
        worst = max(worst, abs(O.core_entry(X, *facs, p, q, s) - G[p, q, s]))
    f_or = O.fit_identity(X.norm2(), G)
    _say(f"implicit 20000^3 1M fp64: fit {r.fits[-1]:.10f} (oracle identity {f_or:.10f}), core sample "
         f"|d| {worst:.2e}, sweeps {r.stats['sweeps_ms']:.1f} ms, prep {r.stats['prep_ms']:.1f} ms")
    assert worst < 1e-10 * np.abs(G).max()
    assert abs(r.fits[-1] - f_or) < 1e-12

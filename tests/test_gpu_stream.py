"""Multislice Projection streamed from host memory (tucker_mp_streamed)
against the in-core tucker_mp and the FP64 oracle.

The same random start (Figure 5's, TK_INIT_RANDOM) on both: the streamed
form sums each Gram over slabs of the major index instead of over the whole
projection, so FP64 trajectories agree with the in-core ones to rounding
(1e-10) and with the oracle's (1e-9); FP32 within 1e-6 and mixed within
1e-4 of the in-core runs. Slab sizes from one slab per Gram term down to
one slice per slab (hundreds of uploads per sweep); duplicates summed on
the host; a given start; the second call reuses the workspace.
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


@pytest.fixture(scope="module")
def tensor():
    idx, vals, dims = synth.uniform_sparse((210, 150, 97), 60_000, 77)
    return idx, vals, dims, (9, 7, 6)


def _incore(tk, idx, vals, dims, J, prec, sweeps):
    di = torch.from_numpy(idx).cuda()
    dv = torch.from_numpy(vals).cuda()
    return tk.mp(di, dv, dims, J, precision=prec, max_iters=sweeps, tol=0.0, init=tk.INIT_RANDOM, seed=SEED)


# 13568 bytes: the smallest slab (a multiple of 256) that holds one slice of
# the widest projection here (210 rows of 8 FP64 columns): one or two slices
# per slab
@pytest.mark.parametrize("slab_bytes", [1 << 26, 1 << 16, 13_568])
def test_fp64_matches_incore_and_oracle(tk, tensor, slab_bytes):
    idx, vals, dims, J = tensor
    _say(f"streamed mp fp64 slab {slab_bytes}")
    r = tk.mp_streamed(idx, vals, dims, J, slab_bytes, precision="fp64", max_iters=5, tol=0.0, seed=SEED)
    c = _incore(tk, idx, vals, dims, J, "fp64", 5)
    X = O.SparseTensor3(idx, vals, dims)
    B0 = O.random_start(dims[1], J[1], 1, SEED)
    C0 = O.random_start(dims[2], J[2], 2, SEED)
    ref = O.mp(X, J, 5, 0.0, init=(None, B0, C0), fit="identity")
    d_in = np.max(np.abs(np.array(r.fits) - np.array(c.fits)))
    d_or = np.max(np.abs(np.array(r.fits) - np.array(ref.fits)))
    _say(f"  slabs {r.stats['streamed_slabs']} bytes {r.stats['streamed_bytes']}: |d| in-core {d_in:.2e} "
         f"oracle {d_or:.2e}")
    assert d_in < 1e-10 and d_or < 1e-9
    # the cores: norms within 1e-8 (the eigensolver tolerance); entries within 1e-6 (near-tied
    # trailing eigenvalues leave their eigenvectors free to rotate by about
    # the rounding of M over the gap, which the fit does not see)
    G, Gc = r.core.cpu().numpy(), c.core.cpu().numpy()
    assert abs(np.linalg.norm(G) - np.linalg.norm(Gc)) < 1e-8 * np.linalg.norm(Gc)
    assert np.abs(G - Gc).max() < 1e-6 * np.abs(Gc).max()
    for F in r.factors:
        F = F.cpu().numpy()
        assert np.abs(F.T @ F - np.eye(F.shape[1])).max() < 1e-10
    # every sweep uploads each ordering once per Gram term plus the core's
    assert r.stats["streamed_slabs"] >= 5 * 7


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("mixed", 1e-4)])
def test_reduced_precision_matches_incore(tk, tensor, prec, tol):
    idx, vals, dims, J = tensor
    r = tk.mp_streamed(idx, vals, dims, J, 1 << 16, precision=prec, max_iters=5, tol=0.0, seed=SEED)
    c = _incore(tk, idx, vals, dims, J, prec, 5)
    d = np.max(np.abs(np.array(r.fits) - np.array(c.fits)))
    _say(f"streamed mp {prec}: |d| in-core {d:.2e}")
    assert d < tol


def test_duplicates_given_start_and_stopping_rule(tk, tensor):
    idx, vals, dims, J = tensor
    idx2, vals2 = synth.with_duplicates(idx, vals, 3000, 5)
    rng = np.random.default_rng(3)
    facs = [torch.zeros((dims[0], J[0]), dtype=torch.float64)] + [
        torch.from_numpy(np.linalg.qr(rng.standard_normal((dims[n], J[n])))[0]) for n in (1, 2)]
    r = tk.mp_streamed(idx2, vals2, dims, J, 1 << 16, precision="fp64", max_iters=30, tol=1e-4,
                       init=tk.INIT_GIVEN, factors=facs)
    di = torch.from_numpy(idx2).cuda()
    dv = torch.from_numpy(vals2).cuda()
    c = tk.mp(di, dv, dims, J, precision="fp64", max_iters=30, tol=1e-4, init=tk.INIT_GIVEN, factors=facs)
    _say(f"streamed given start: sweeps {r.iters} vs {c.iters}, fit {r.fits[-1]:.9f} vs {c.fits[-1]:.9f}")
    assert r.iters == c.iters
    assert np.max(np.abs(np.array(r.fits) - np.array(c.fits))) < 1e-10
    assert r.stats["nnz_unique"] == c.stats["nnz_unique"]


def test_workspace_reuse_and_a_larger_tensor(tk):
    """1000 x 800 x 600 with 1M nonzeros streamed through 4 MiB slabs, twice
    in a row on one workspace: bitwise equal runs, in-core fits within
    1e-10 (FP64)."""
    idx, vals, dims = synth.uniform_sparse((1000, 800, 600), 1_000_000, 9)
    J = (20, 16, 12)
    r1 = tk.mp_streamed(idx, vals, dims, J, 4 << 20, precision="fp64", max_iters=3, tol=0.0, seed=SEED)
    import ctypes
    coo = tk._HostCoo(idx, vals, dims)
    Jc = (ctypes.c_int32 * 3)(*J)
    o = tk._opts("fp64", init=tk.INIT_RANDOM, seed=SEED, max_iters=3, tol=0.0)
    out = ctypes.c_size_t(0)
    assert tk.lib().tucker_mp_streamed_workspace(ctypes.byref(coo.c), Jc, ctypes.byref(o), 4 << 20,
                                                 ctypes.byref(out)) == 0
    need = out.value
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    ra = tk.mp_streamed(idx, vals, dims, J, 4 << 20, precision="fp64", max_iters=3, tol=0.0, seed=SEED, workspace=ws)
    rb = tk.mp_streamed(idx, vals, dims, J, 4 << 20, precision="fp64", max_iters=3, tol=0.0, seed=SEED, workspace=ws)
    assert ra.fits == rb.fits == r1.fits
    assert torch.equal(ra.core, rb.core)
    c = _incore(tk, idx, vals, dims, J, "fp64", 3)
    _say(f"streamed 1M: slabs {ra.stats['streamed_slabs']} fits {ra.fits[-1]:.9f} in-core {c.fits[-1]:.9f}")
    assert np.max(np.abs(np.array(ra.fits) - np.array(c.fits))) < 1e-10

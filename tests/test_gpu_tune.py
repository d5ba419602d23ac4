"""Launch choices (tk_tune) and the tuner on the GPU.

* The projection's choices (run length and the workgroup count it aims for)
  change no result bit: each output sums the nonzeros of its slot in order.
* The Gram's choices move its split over the summed dimension, so results may
  move within rounding: each choice is deterministic (two runs, same bits),
  the fit agrees with the built-in choice's, and the core still matches the
  oracle's n-mode product (Section 3) of the returned factors.
* The many-tensor call with one choice per tensor equals the single calls
  made with those choices, bit for bit.
* The tuner returns a choice in range, stores it per shape bucket and reads
  it back from its JSON cache.
"""
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


@pytest.fixture(scope="module")
def planted():
    dims, core = (300, 250, 200), (20, 15, 10)
    idx, vals, dims = synth.planted_tucker(dims, core, 120_000, 0.05, 4242)
    di = torch.from_numpy(idx.astype(np.int32)).cuda()
    dv = torch.from_numpy(vals).cuda()
    return di, dv, dims, core, O.SparseTensor3(idx, vals, dims)


def _same(a, b):
    assert a.fits == b.fits
    assert torch.equal(a.core, b.core)
    for n in range(3):
        assert torch.equal(a.factors[n], b.factors[n])


PROJ_TUNES = [(1024, 64, 0, 0), (65536, 16384, 0, 0), (8192, 4096, 0, 0), (2048, 512, 0, 0)]


@pytest.mark.parametrize("algo,prec", [("mp", "mixed"), ("mp", "fp32"), ("hooi", "fp64")])
def test_projection_choices_change_no_bit(tk, planted, algo, prec):
    di, dv, dims, core, _ = planted
    fn = getattr(tk, algo)
    _say(f"projection tunes {algo} {prec}")
    ref = fn(di, dv, dims, core, precision=prec, max_iters=3, tol=0.0)
    for t in PROJ_TUNES:
        _same(fn(di, dv, dims, core, precision=prec, max_iters=3, tol=0.0, tune=t), ref)


GRAM_TUNES = [(0, 0, 64, 1), (0, 0, 16384, 1), (0, 0, 256, 64), (16384, 4096, 4096, 2)]
# Relative fit change allowed between two Gram splits. The split moves the
# rounding of the partial sums by at most K u (summed length K up to 6e4,
# u = 2^-24 for FP32 accumulators, 2^-53 for FP64), amplified by the small
# eigengaps of a sparsely sampled tensor (fit about 0.4 %): 1e-3 for the
# FP32 Grams, 1e-9 for FP64. The mixed solves stop at a 1e-4 relative
# resolution of the Ritz sums, and three sweeps compound the different
# stopping points: 5e-3 (2e-5 of fit here, a fifth of the 1e-4 bar).
FIT_RTOL = {"mixed": 5e-3, "fp32": 1e-3, "fp64": 1e-9}


@pytest.mark.parametrize("prec", ["mixed", "fp32", "fp64"])
def test_gram_choices_deterministic_and_within_rounding(tk, planted, prec):
    di, dv, dims, core, X = planted
    _say(f"Gram tunes mp {prec}")
    ref = tk.mp(di, dv, dims, core, precision=prec, max_iters=3, tol=0.0)
    for t in GRAM_TUNES:
        a = tk.mp(di, dv, dims, core, precision=prec, max_iters=3, tol=0.0, tune=t)
        b = tk.mp(di, dv, dims, core, precision=prec, max_iters=3, tol=0.0, tune=t)
        _same(a, b)
        assert abs(a.fits[-1] - ref.fits[-1]) <= FIT_RTOL[prec] * ref.fits[-1], (t, a.fits[-1], ref.fits[-1])
        G = a.core.cpu().numpy()
        A, B, C = (f.cpu().numpy() for f in a.factors)
        scale = np.abs(G).max()
        for p, q, r in [(0, 0, 0), (3, 7, 2), (19, 14, 9), (11, 0, 5)]:
            assert abs(G[p, q, r] - O.core_entry(X, A, B, C, p, q, r)) <= 1e-5 * scale


def test_batched_per_tensor_choices(tk):
    cfgs = synth.batch_configs(5, 3100)
    tensors, cores = [], []
    for c in cfgs:
        dims = tuple(max(20, d // 3) for d in c["dims"])
        core = tuple(min(j // 2, d) for j, d in zip(c["core"], dims))
        idx, vals, dims = synth.uniform_sparse(dims, int(round(0.005 * np.prod(dims))), c["seed"])
        tensors.append((torch.from_numpy(idx.astype(np.int32)).cuda(), torch.from_numpy(vals).cuda(), dims))
        cores.append(core)
    tunes = [(1024, 64, 64, 1), (0, 0, 0, 0), (65536, 16384, 16384, 64), (8192, 4096, 512, 2), (0, 0, 2048, 8)]
    _say("batched, 5 tensors, 2 streams, one tune each")
    res, st = tk.batched(tk.ALGO_MP, tensors, cores, nstreams=2, tunes=tunes, precision="mixed", max_iters=3,
                         tol=0.0)
    assert st >= 0
    for (i, v, d), core, t, r in zip(tensors, cores, tunes, res):
        _same(r, tk.mp(i, v, d, core, precision="mixed", max_iters=3, tol=0.0, tune=t))


def test_tuner_caches_per_bucket(tk, planted, tmp_path):
    from paper_0711_2023_amd import autotune as at
    di, dv, dims, core, _ = planted
    path = str(tmp_path / "tunes.json")
    cache = at.TuneCache(path)
    _say("tuner on the planted 300x250x200 tensor")
    t = at.tune_tensor(tk.ALGO_MP, di, dv, dims, core, "mixed", cache, reps=1)
    key = at.bucket(tk.ALGO_MP, "mixed", dims, dv.numel(), core)
    assert key in cache.entries and cache.get(key).key() == t.key()
    assert t.key()[0] in (0,) + tuple(p[0] for p in at.PROJ_CANDIDATES)
    cache.save()
    again = at.TuneCache(path)
    assert again.get(key).key() == t.key()
    # a cache hit measures nothing and returns the stored choice
    assert at.tune_tensor(tk.ALGO_MP, di, dv, dims, core, "mixed", again).key() == t.key()
    res = tk.mp(di, dv, dims, core, precision="mixed", max_iters=2, tol=0.0, tune=t)
    assert 0.0 < res.fits[-1] < 1.0

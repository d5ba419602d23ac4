"""Many tensors in one call: every tensor's result equals (bit for bit) the
result of its own tucker_mp / tucker_hooi call, whatever stream and worker
took it; a bad tensor in the batch reports its own status."""
import sys

import numpy as np
import pytest

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


def _batch(count=7):
    out = []
    for c in synth.batch_configs(count, 3000):
        dims = tuple(max(20, d // 3) for d in c["dims"])
        core = tuple(min(j // 2, d) for j, d in zip(c["core"], dims))
        nnz = int(round(0.005 * np.prod(dims)))
        idx, vals, dims = synth.uniform_sparse(dims, nnz, c["seed"])
        out.append((idx, vals, dims, core))
    return out


@pytest.mark.parametrize("algo,prec", [("mp", "mixed"), ("hooi", "fp32")])
def test_batched_equals_individual_calls(tk, algo, prec):
    data = _batch()
    dev = [(torch.from_numpy(i.astype(np.int32)).cuda(), torch.from_numpy(v).cuda(), d) for i, v, d, _ in data]
    cores = [c for *_, c in data]
    _say(f"batched {algo} {prec} {len(data)} tensors, 3 streams")
    res, st = tk.batched(tk.ALGO_MP if algo == "mp" else tk.ALGO_HOOI, dev, cores, nstreams=3, precision=prec,
                         max_iters=4, tol=0.0)
    assert st >= 0
    fn = getattr(tk, algo)
    for (i, v, d), core, r in zip(dev, cores, res):
        one = fn(i, v, d, core, precision=prec, max_iters=4, tol=0.0)
        assert r.status == one.status
        assert r.fits == one.fits
        for n in range(3):
            assert torch.equal(r.factors[n], one.factors[n])
        assert torch.equal(r.core, one.core)


def test_batched_reports_per_tensor_status(tk):
    data = _batch(4)
    dev = [(torch.from_numpy(i.astype(np.int32)).cuda(), torch.from_numpy(v).cuda(), d) for i, v, d, _ in data]
    # tensor 2 gets an out-of-range coordinate: only it fails
    bad = dev[2][0].clone()
    bad[0, 0] = int(dev[2][2][0]) + 5
    dev[2] = (bad, dev[2][1], dev[2][2])
    cores = [c for *_, c in data]
    _say("batched with one bad tensor")
    import ctypes  # noqa: F401
    with pytest.raises(tk.TuckerError) as e:
        tk.batched(tk.ALGO_MP, dev, cores, nstreams=2, precision="fp32", max_iters=2, tol=0.0)
    assert e.value.status == -2  # TK_ERR_INDEX

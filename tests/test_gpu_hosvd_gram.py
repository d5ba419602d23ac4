"""HO-SVD (Figure 1) on a tensor whose unfolding Grams are diagonal, so that
the factors and the core are known in closed form.

Every mode-1 index i holds one nonzero, at (i, i mod 100, i div 100) of an
8000 x 100 x 100 tensor: no two nonzeros share a fibre of any mode, hence
X_(n) X_(n)^T is diagonal for every n, with the sums of the squared values
of each index on the diagonal. Five rows carry planted values 10, 9, 8, 7, 6
at distinct mode-2 and mode-3 indices, the rest U(0.1, 1); the planted
indices then lead every mode's diagonal by a wide margin, so the J = 5
leading eigenvectors are the unit vectors of those indices in that order
(sign: largest entry positive), and the core is superdiagonal with the
planted values. Mode 1's Gram has order 8000: its workgroup holds one
partial row of 8000 doubles and a tag table, more LDS than the default
64 KB limit of a launch; modes 2 and 3 (order 100) take sixteen waves per
row with partial rows summed in wave order.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS = (8000, 100, 100)
PLANT_J = [3, 10, 17, 24, 31]
PLANT_K = [5, 16, 27, 38, 49]
PLANT_V = [10.0, 9.0, 8.0, 7.0, 6.0]


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


def _tensor(seed=8128):
    rng = np.random.default_rng(seed)
    i = np.arange(DIMS[0], dtype=np.int64)
    idx = np.stack([i, i % 100, i // 100]).astype(np.int32)  # one row per mode
    vals = rng.uniform(0.1, 1.0, DIMS[0])
    rows = [k * 100 + j for j, k in zip(PLANT_J, PLANT_K)]
    vals[rows] = PLANT_V
    return idx, vals, rows


def test_hosvd_on_diagonal_grams_closed_form(tk):
    idx, vals, rows = _tensor()
    # the planted indices lead each mode's diagonal (checked on the input)
    for n, lead in ((0, rows), (1, PLANT_J), (2, PLANT_K)):
        d = np.bincount(idx[n], weights=vals ** 2, minlength=DIMS[n])
        assert list(np.argsort(-d, kind="stable")[:5]) == list(lead)
        assert d[lead[-1]] > 1.2 * np.sort(d)[-6]
    di = torch.from_numpy(idx).cuda()
    dv = torch.from_numpy(vals).cuda()
    _say(f"hosvd closed form: {DIMS}, {len(vals)} nonzeros, core 5^3, FP64")
    r = tk.hosvd(di, dv, DIMS, (5, 5, 5), precision="fp64", eig_tol=1e-14)
    torch.cuda.synchronize()
    for n, lead in ((0, rows), (1, PLANT_J), (2, PLANT_K)):
        F = r.factors[n].cpu().numpy()
        E = np.zeros_like(F)
        E[lead, np.arange(5)] = 1.0
        err = float(np.max(np.abs(F - E)))
        _say(f"mode {n + 1}: max |F - E| = {err:.3e}")
        assert err <= 1e-9, (n, err)
    G = r.core.cpu().numpy()
    Ge = np.zeros((5, 5, 5))
    Ge[np.arange(5), np.arange(5), np.arange(5)] = PLANT_V
    assert float(np.max(np.abs(G - Ge))) <= 1e-9
    fit = O.fit_identity(float(np.sum(vals ** 2)), Ge)
    assert abs(r.fits[0] - fit) <= 1e-12, (r.fits[0], fit)

"""BF16 Grams of order >= 768 take the 256-row-tile kernel whose operand
stages go straight into an LDS ring (k_gram_dl). This shape runs it on mode
1's Gram (order 800: a last row tile of 32 rows) with Gram terms whose K
(61 x 16 and 47 x 16 columns) ends inside a 32-deep stage, so the zero fill
past a split's end, past the last row and past the term is exercised; modes
2 and 3 (61, 47) take the 128-row kernel.

The MP trajectory (Figure 7, HO-SVD start of Section 4.4) in mixed precision
and with split-BF16 Grams is compared with the FP64 path on the same planted
tensor (Section 3's model sampled at 44 % of its cells with 10 % noise, whose
leading subspaces are well separated): per-sweep fits and the final factor subspaces. A Gram wrong in a
tile or a stage would move both far beyond the tolerances, which are those of
the reduced forms against FP64 elsewhere in the suite.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DIMS, CORE, NNZ, NOISE, SEED = (800, 61, 47), (10, 10, 10), 1_000_000, 0.1, 877


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
def runs(tk):
    idx, vals, dims = synth.planted_tucker(DIMS, CORE, NNZ, NOISE, SEED)
    di = torch.from_numpy(idx.astype(np.int32)).cuda()
    dv = torch.from_numpy(vals).cuda()
    out = {}
    for prec in ("fp64", "mixed", "bf16x3"):
        _say(f"gram tiles: MP {prec} on {dims}, {NNZ} nonzeros, core {CORE}")
        out[prec] = tk.mp(di, dv, dims, CORE, precision=prec, max_iters=6, tol=0.0)
    return out


@pytest.mark.parametrize("prec, fit_tol, angle_tol", [("mixed", 1e-4, 1e-2), ("bf16x3", 1e-6, 1e-3)])
def test_wide_tile_gram_trajectory_matches_fp64(runs, prec, fit_tol, angle_tol):
    ref, got = runs["fp64"], runs[prec]
    assert got.iters == ref.iters == 6
    f64, fr = np.asarray(ref.fits), np.asarray(got.fits)
    assert np.all(np.isfinite(fr))
    assert ref.fits[-1] > 0.0
    ang = [O.subspace_angle(got.factors[n].cpu().numpy(), ref.factors[n].cpu().numpy()) for n in range(3)]
    _say(f"{prec}: fits {fr.tolist()}, max |dfit| {np.max(np.abs(fr - f64)):.3e}, angles {ang}")
    assert np.max(np.abs(fr - f64)) <= fit_tol, (prec, fr - f64)
    assert max(ang) <= angle_tol, (prec, ang)

"""Writes tests/golden/learn_targets.npz: training and held-out targets of the
learned warm start, computed by the FP64 oracle only.

Each tensor comes from the seeded generators (planted Tucker models at a
density where their structure is visible, and uniform random tensors as in
the paper's experiments, Section 5); its target factors are the mode-2 and
mode-3 factors of the oracle's HOOI (Figure 3) after 30 sweeps. The file holds
numeric arrays only: `recipes` (one row per tensor: kind 0 planted / 1
uniform, I1, I2, I3, J1, J2, J3, nnz, seed, noise, held_out), and `t{k}_m1`,
`t{k}_m2` (the factors), `fits` (final HOOI fit).

Run from the repository root: python tests/golden/make_learn_targets.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

RECIPES = [
    # kind, dims, core, nnz, seed, noise, held_out
    (0, (100, 90, 80), (6, 6, 6), 86_000, 700, 0.1, 0),
    (0, (120, 100, 90), (8, 8, 8), 130_000, 701, 0.1, 0),
    (0, (90, 110, 100), (10, 10, 10), 119_000, 702, 0.1, 0),
    (0, (110, 95, 105), (7, 9, 8), 110_000, 703, 0.1, 0),
    (0, (80, 120, 100), (12, 10, 8), 115_000, 704, 0.1, 0),
    (0, (100, 100, 120), (9, 12, 10), 120_000, 705, 0.1, 0),
    (1, (120, 120, 120), (8, 8, 8), 40_000, 710, 0.0, 0),
    (1, (150, 130, 110), (12, 12, 12), 50_000, 711, 0.0, 0),
    (1, (110, 140, 130), (10, 6, 14), 45_000, 712, 0.0, 0),
    (1, (130, 110, 140), (6, 14, 10), 45_000, 713, 0.0, 0),
    # held out
    (0, (100, 100, 100), (8, 8, 8), 100_000, 720, 0.1, 1),
    (1, (140, 140, 140), (10, 10, 10), 50_000, 721, 0.0, 1),
]


def make(kind, dims, core, nnz, seed, noise):
    if kind == 0:
        return synth.planted_tucker(dims, core, nnz, noise, seed)
    return synth.uniform_sparse(dims, nnz, seed)


def main():
    out = {}
    rec = []
    fits = []
    for k, (kind, dims, core, nnz, seed, noise, held) in enumerate(RECIPES):
        idx, vals, dims = make(kind, dims, core, nnz, seed, noise)
        X = O.SparseTensor3(idx, vals, dims)
        d = O.hooi(X, core, 30, 0.0)
        out[f"t{k}_m1"] = d.factors[1]
        out[f"t{k}_m2"] = d.factors[2]
        fits.append(d.fits[-1])
        rec.append([kind, *dims, *core, nnz, seed, noise, held])
        print(k, dims, core, "fit", d.fits[-1], flush=True)
    out["recipes"] = np.array(rec, dtype=np.float64)
    out["fits"] = np.array(fits)
    np.savez_compressed(os.path.join(os.path.dirname(os.path.abspath(__file__)), "learn_targets.npz"), **out)


if __name__ == "__main__":
    main()

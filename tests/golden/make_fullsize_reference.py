"""Writes tests/golden/fullsize_reference.json: the FP64 oracle's per-sweep
fits at the benchmarked sizes, so that the GPU decompositions there can be
compared with the oracle's without re-running it.

Tensors (seeded, from ``synth``):
* 1000 x 1000 x 1000, 1,000,000 uniform distinct nonzeros, U(0,1) values,
  core 50 x 50 x 50 (seed 1);
* 2000 x 1000 x 500, 2,000,000 uniform distinct nonzeros, U(0,1) values,
  cores 100 x 20 x 5 and 10 x 50 x 100 (seed 2).

For each: the HO-SVD fit (Figure 1); HOOI (Figure 3) and MP (Figure 7) from
their HO-SVD / pseudo HO-SVD starts, exactly SWEEPS sweeps each (threshold
0), fit after every sweep by the identity ||X||^2 = ||G||^2 + ||X - Xhat||^2
(the oracle pins it against the slice-wise and dense fits); on the cube, SP
(Figure 5) from the SplitMix64 random start ``oracle.random_start(I3, J3, 2,
SP_SEED)``, SWEEPS sweeps, with its fits and core growth Delta_G per sweep.

Run from the repository root (about 25 minutes on 8 cores):
    python tests/golden/make_fullsize_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

SWEEPS = 10
SP_SEED = 0x5EED
CASES = ["cube1000_nnz1m", "unbal_2000x1000x500_core100x20x5", "unbal_2000x1000x500_core10x50x100"]


def compute(cases=CASES, sweeps=SWEEPS):
    out = {"sweeps": sweeps, "sp_seed": SP_SEED, "fit": "identity", "cases": {}}
    for name in cases:
        w = synth.WORKLOADS[name]
        idx, vals, dims = synth.uniform_sparse(tuple(w["dims"]), int(w["nnz"]), w["seed"])
        J = tuple(w["core"])
        X = O.SparseTensor3(idx, vals, dims)
        rec = {"dims": list(dims), "core": list(J), "nnz": int(w["nnz"]), "seed": int(w["seed"])}
        t = time.time()
        rec["hosvd_fit"] = O.hosvd(X, J, fit="identity").fits[0]
        print(f"{name}: HO-SVD fit {rec['hosvd_fit']:.9e} ({time.time() - t:.0f} s)", flush=True)
        for algo, fn in (("hooi", O.hooi), ("mp", O.mp)):
            t = time.time()
            d = fn(X, J, sweeps, 0.0, fit="identity")
            rec[f"{algo}_fits"] = [float(f) for f in d.fits]
            print(f"{name}: {algo} fits {d.fits} ({time.time() - t:.0f} s)", flush=True)
        if name == "cube1000_nnz1m":
            t = time.time()
            C0 = O.random_start(dims[2], J[2], 2, SP_SEED)
            d = O.sp_algorithm(X, J, C0, sweeps, 0.0, fit="identity")
            rec["sp_fits"] = [float(f) for f in d.fits]
            rec["sp_core_growth"] = [float(g) for g in d.extra["core_growth"]]
            print(f"{name}: sp fits {d.fits} ({time.time() - t:.0f} s)", flush=True)
        out["cases"][name] = rec
    return out


if __name__ == "__main__":
    res = compute()
    with open(os.path.join(ROOT, "tests", "golden", "fullsize_reference.json"), "w") as f:
        json.dump(res, f, indent=1)
    print("written")

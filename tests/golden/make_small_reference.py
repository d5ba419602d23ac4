"""Writes tests/golden/small_reference.npz: the FP64 oracle's MP (Figure 7)
and HOOI (Figure 3), HO-SVD start, exactly 10 sweeps, on two small seeded
tensors: the uniform workload (100 x 100 x 100, 10,000 distinct nonzeros,
U(0,1) values, core 10 x 10 x 10) and a planted Tucker model of the same
shape and core (100,000 sampled entries, noise 0.1), whose leading subspaces
are well separated. The benchmark compares every precision form of the GPU
path with these numbers (fit per sweep, factor subspaces) without running the
oracle itself.

Arrays, for case in uniform, planted and algo in mp, hooi:
`{case}_{algo}_fits` (10 fits), `{case}_{algo}_A|B|C` (final factors);
`{case}_dims`, `{case}_core`, `{case}_nnz`, `{case}_seed`, and
`planted_noise`.

Run from the repository root: python tests/golden/make_small_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

WORKLOAD = "cube100_nnz10k"
SWEEPS = 10


PLANTED = {"dims": (100, 100, 100), "core": (10, 10, 10), "nnz": 100_000, "noise": 0.1, "seed": 9100}


def compute():
    w = synth.WORKLOADS[WORKLOAD]
    cases = {
        "uniform": (synth.uniform_sparse(tuple(w["dims"]), int(w["nnz"]), w["seed"]), tuple(w["core"]),
                    int(w["nnz"]), int(w["seed"])),
        "planted": (synth.planted_tucker(PLANTED["dims"], PLANTED["core"], PLANTED["nnz"], PLANTED["noise"],
                                         PLANTED["seed"]), PLANTED["core"], PLANTED["nnz"], PLANTED["seed"]),
    }
    out = {"planted_noise": np.array(PLANTED["noise"])}
    for case, ((idx, vals, dims), J, nnz, seed) in cases.items():
        X = O.SparseTensor3(idx, vals, dims)
        out.update({f"{case}_dims": np.array(dims), f"{case}_core": np.array(J), f"{case}_nnz": np.array(nnz),
                    f"{case}_seed": np.array(seed)})
        for name, fn in (("mp", O.mp), ("hooi", O.hooi)):
            d = fn(X, J, SWEEPS, 0.0)
            out[f"{case}_{name}_fits"] = np.array(d.fits)
            for k, F in zip("ABC", d.factors):
                out[f"{case}_{name}_{k}"] = np.asarray(F)
    return out


if __name__ == "__main__":
    np.savez(os.path.join(ROOT, "tests", "golden", "small_reference.npz"), **compute())
    print("written")

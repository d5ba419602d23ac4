"""The skewed input generator (synth.skewed_sparse) draws what its
docstring states: distinct in-range coordinates, seeded, with index
frequencies falling off as a Zipf law, so that some fibres are long."""
import numpy as np

import synth


def test_skewed_sparse_distinct_seeded_and_skewed():
    dims, nnz = (120, 90, 70), 40_000
    idx, vals, d = synth.skewed_sparse(dims, nnz, 1.0, 5)
    assert d == dims and idx.shape == (3, nnz) and vals.shape == (nnz,)
    assert idx.dtype == np.int32
    for m in range(3):
        assert idx[m].min() >= 0 and idx[m].max() < dims[m]
    lin = (idx[0].astype(np.int64) * dims[1] + idx[1]) * dims[2] + idx[2]
    assert np.unique(lin).size == nnz
    assert np.all((vals >= 0.0) & (vals < 1.0))
    idx2, vals2, _ = synth.skewed_sparse(dims, nnz, 1.0, 5)
    assert np.array_equal(idx, idx2) and np.array_equal(vals, vals2)
    # index 0 is far more frequent than the last index, and some mode-1
    # fibres (fixed second and third index) are long
    for m in range(3):
        cnt = np.bincount(idx[m], minlength=dims[m])
        assert cnt[0] > 10 * max(cnt[-1], 1)
    _, fib = np.unique(idx[1].astype(np.int64) * dims[2] + idx[2], return_counts=True)
    assert fib.max() > 32

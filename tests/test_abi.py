"""The C ABI without a GPU: the library loads, exports every function that
include/tucker.h declares, and rejects invalid arguments on the host (status
codes) before touching the device."""
import ctypes
import os
import re

import pytest

import paper_0711_2023_amd as tk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = ""
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            with open(os.path.join(ROOT, "include", h)) as f:
                text += f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tucker_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_symbol_list():
    assert _declared_functions() == sorted(tk.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = tk.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_default_opts_are_the_papers():
    o = tk.default_opts()
    assert o.max_iters == 50 and abs(o.tol - 1e-4) < 1e-18
    assert o.precision == tk.FP32 and o.init == tk.INIT_HOSVD and o.timing == 0


def test_strerror_texts():
    for st in (0, 1, -1, -2, -3, -4, -5, -6):
        assert len(tk.strerror(st)) > 0
    assert "unknown" in tk.strerror(99)


def _coo(dims=(10, 9, 8), nnz=5, order=3, null_idx=False):
    c = tk.tk_coo()
    c.order = order
    c.nnz = nnz
    d = (ctypes.c_int64 * 3)(*dims)
    c.dims = d
    for n in range(3):
        c.idx[n] = None if null_idx else 0x1000  # never dereferenced: validation fails first
    c.vals = None if null_idx else 0x2000
    return c, d


def _ws(c, J, opts=None, algo=tk.ALGO_MP):
    Jc = (ctypes.c_int32 * 3)(*J)
    out = ctypes.c_size_t(0)
    o = opts or tk.default_opts()
    st = tk.lib().tucker_workspace_bytes(algo, ctypes.byref(c), Jc, ctypes.byref(o), ctypes.byref(out))
    return st, out.value


def test_workspace_query_positive_and_grows_with_nnz():
    c, d = _coo(nnz=10)
    st, b1 = _ws(c, (3, 3, 3))
    assert st == 0 and b1 > 0
    c2, d2 = _coo(nnz=10000)
    st, b2 = _ws(c2, (3, 3, 3))
    assert st == 0 and b2 > b1
    for algo in (tk.ALGO_HOOI, tk.ALGO_FIT):
        st, b = _ws(c, (3, 3, 3), algo=algo)
        assert st == 0 and b > 0


@pytest.mark.parametrize("case", ["order", "neg_nnz", "J_gt_I", "J_zero", "dim_zero", "null_idx", "bad_prec",
                                  "bad_iters", "bad_algo"])
def test_invalid_arguments_rejected_on_host(case):
    dims, J, order, nnz, null_idx, algo = (10, 9, 8), (3, 3, 3), 3, 5, False, tk.ALGO_MP
    o = tk.default_opts()
    if case == "order":
        order = 4
    elif case == "neg_nnz":
        nnz = -1
    elif case == "J_gt_I":
        J = (3, 10, 3)
    elif case == "J_zero":
        J = (0, 3, 3)
    elif case == "dim_zero":
        dims = (10, 0, 8)
    elif case == "null_idx":
        null_idx = True
    elif case == "bad_prec":
        o.precision = 7
    elif case == "bad_iters":
        o.max_iters = -2
    elif case == "bad_algo":
        algo = 9
    c, d = _coo(dims, nnz, order, null_idx)
    st, _ = _ws(c, J, o, algo)
    assert st == tk.TK_ERR_ARG


def test_entry_points_reject_before_device_work():
    L = tk.lib()
    c, d = _coo()
    J = (ctypes.c_int32 * 3)(3, 10, 3)  # J2 > I2
    o = tk.default_opts()
    facs = (ctypes.c_void_p * 3)(0x10, 0x20, 0x30)
    hist = (ctypes.c_double * 50)()
    done = ctypes.c_int32(0)
    for fn in (L.tucker_hooi, L.tucker_mp):
        st = fn(ctypes.byref(c), J, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50, 1 << 30,
                None)
        assert st == tk.TK_ERR_ARG
    out = ctypes.c_double(0)
    assert L.tucker_fit(ctypes.byref(c), J, 0x40, facs, ctypes.byref(out), 0x50, 1 << 30, None) == tk.TK_ERR_ARG
    # null outputs
    J2 = (ctypes.c_int32 * 3)(3, 3, 3)
    st = L.tucker_mp(ctypes.byref(c), J2, ctypes.byref(o), None, facs, hist, ctypes.byref(done), None, 0x50, 1 << 30,
                     None)
    assert st == tk.TK_ERR_ARG
    # workspace too small is reported before any device work
    st = L.tucker_mp(ctypes.byref(c), J2, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50, 16, None)
    assert st == tk.TK_ERR_WORKSPACE
    # an empty tensor has no fit
    c0, d0 = _coo(nnz=0)
    st = L.tucker_mp(ctypes.byref(c0), J2, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50,
                     1 << 30, None)
    assert st == tk.TK_ERR_EMPTY

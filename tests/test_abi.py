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
    for st in (0, 1, -1, -2, -3, -4, -5, -6, -7):
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
        order = 5
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


def test_learn_param_count_and_queries():
    L = tk.lib()
    assert L.tucker_learn_param_count() == 64 * 128 + 128 + 128 * 128 + 128
    out = ctypes.c_size_t(0)
    assert L.tucker_learn_backward_workspace(1000, ctypes.byref(out)) == 0 and out.value > 0
    assert L.tucker_learn_backward_workspace(-1, ctypes.byref(out)) == tk.TK_ERR_ARG
    assert L.tucker_learn_align_workspace(500, 100, 50, ctypes.byref(out)) == 0 and out.value > 500 * 150 * 8
    for rows, K, J in ((0, 3, 3), (10, 3, 0), (10, 129, 3), (10, 0, 3), (5, 3, 6)):
        assert L.tucker_learn_align_workspace(rows, K, J, ctypes.byref(out)) == tk.TK_ERR_ARG
    assert L.tucker_learn_test_width(5) == 10 and L.tucker_learn_test_width(100) == 128
    assert L.tucker_learn_test_width(0) == tk.TK_ERR_ARG and L.tucker_learn_test_width(129) == tk.TK_ERR_ARG
    c, d = _coo(nnz=100)
    assert L.tucker_learn_sketch_workspace(ctypes.byref(c), ctypes.byref(out)) == 0 and out.value > 0


def test_learn_entry_points_reject_before_device_work():
    L = tk.lib()
    c, d = _coo(nnz=5)
    assert L.tucker_learn_sketch(ctypes.byref(c), 3, 1, 0x10, 0x20, 0x30, 1 << 30, None) == tk.TK_ERR_ARG
    assert L.tucker_learn_sketch(ctypes.byref(c), 0, 1, None, 0x20, 0x30, 1 << 30, None) == tk.TK_ERR_ARG
    assert L.tucker_learn_sketch(ctypes.byref(c), 0, 1, 0x10, 0x20, 0x30, 8, None) == tk.TK_ERR_WORKSPACE
    c0, d0 = _coo(nnz=0)
    assert L.tucker_learn_sketch(ctypes.byref(c0), 0, 1, 0x10, 0x20, 0x30, 1 << 30, None) == tk.TK_ERR_EMPTY
    assert L.tucker_learn_forward(None, 0x10, 4, 0x20, 0x30, None, None) == tk.TK_ERR_ARG
    assert L.tucker_learn_forward(0x10, 0x10, -1, 0x20, 0x30, None, None) == tk.TK_ERR_ARG
    assert L.tucker_learn_backward(0x10, 0x10, 4, 0x20, None, 0x30, 0x40, 0x50, 1 << 30, None) == tk.TK_ERR_ARG
    assert L.tucker_learn_backward(0x10, 0x10, 4, 0x20, 0x28, 0x30, 0x40, 0x50, 8, None) == tk.TK_ERR_WORKSPACE
    loss = ctypes.c_double(0)
    assert L.tucker_learn_align(0x10, 10, 6, 0x20, 11, 0.0, ctypes.byref(loss), None, 0x30, 1 << 30,
                                None) == tk.TK_ERR_ARG
    assert L.tucker_learn_align(0x10, 10, 6, 0x20, 3, -1.0, ctypes.byref(loss), None, 0x30, 1 << 30,
                                None) == tk.TK_ERR_ARG
    assert L.tucker_learn_align(0x10, 10, 6, 0x20, 3, 0.0, ctypes.byref(loss), None, 0x30, 8, None) == \
        tk.TK_ERR_WORKSPACE
    f = ctypes.c_float
    assert L.tucker_learn_adam(0x10, 0x20, 0x30, 0x40, 10, f(1e-3), f(0.9), f(0.999), f(1e-8), 0, None) == \
        tk.TK_ERR_ARG
    assert L.tucker_learn_adam(0x10, 0x20, 0x30, 0x40, 10, f(1e-3), f(1.0), f(0.999), f(1e-8), 1, None) == \
        tk.TK_ERR_ARG


def test_learned_init_requires_a_model():
    c, d = _coo(nnz=10)
    o = tk.default_opts()
    o.init = tk.INIT_LEARNED
    st, _ = _ws(c, (3, 3, 3), o)
    assert st == tk.TK_ERR_ARG
    o.model = 0x1000
    st, b = _ws(c, (3, 3, 3), o)
    assert st == 0
    o.init = tk.INIT_HOSVD
    st, b0 = _ws(c, (3, 3, 3), o)
    assert st == 0 and b > b0  # the learned start's buffers


def test_batched_rejects_bad_arguments_on_host():
    L = tk.lib()
    c1, d1 = _coo(nnz=10)
    c2, d2 = _coo(dims=(12, 11, 10), nnz=20)
    arr = (tk.tk_coo * 2)(c1, c2)
    J = (ctypes.c_int32 * 6)(3, 3, 3, 4, 4, 4)
    o = tk.default_opts()
    out = ctypes.c_size_t(0)
    assert L.tucker_batched_workspace_bytes(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), None, ctypes.byref(out)) == 0
    b2 = _ws(c2, (4, 4, 4), o)[1]
    assert out.value == max(_ws(c1, (3, 3, 3), o)[1], b2)
    assert L.tucker_batched_workspace_bytes(tk.ALGO_FIT, 2, arr, J, ctypes.byref(o), None, ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    assert L.tucker_batched_workspace_bytes(tk.ALGO_MP, 0, arr, J, ctypes.byref(o), None, ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    Jbad = (ctypes.c_int32 * 6)(3, 3, 3, 4, 40, 4)
    assert L.tucker_batched_workspace_bytes(tk.ALGO_MP, 2, arr, Jbad, ctypes.byref(o), None, ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    # per-tensor launch choices: checked per tensor
    tunes = (tk.tk_tune * 2)(tk.make_tune((4096, 256, 128, 2)), tk.make_tune((0, 0, 0, 0)))
    assert L.tucker_batched_workspace_bytes(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), tunes, ctypes.byref(out)) == 0
    tunes[1].gram_items = 5
    assert L.tucker_batched_workspace_bytes(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), tunes, ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    vp = ctypes.c_void_p
    cores = (vp * 2)(0x10, 0x20)
    facs = (vp * 6)(*[0x30] * 6)
    hist = (ctypes.c_double * 100)()
    done = (ctypes.c_int32 * 2)()
    stat = (ctypes.c_int32 * 2)()
    ws = (vp * 2)(0x40, 0x50)
    st = (vp * 2)(None, None)
    for n in (0, 65):
        assert L.tucker_batched(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), cores, facs, hist, done, stat, None, None, n, ws,
                                1 << 30, st) == tk.TK_ERR_ARG
    assert L.tucker_batched(tk.ALGO_MP, 2, arr, Jbad, ctypes.byref(o), cores, facs, hist, done, stat, None, None,
                            2, ws, 1 << 30, st) == tk.TK_ERR_ARG
    assert L.tucker_batched(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), cores, facs, hist, done, stat, None, None, 2,
                            ws, 16, st) == tk.TK_ERR_WORKSPACE
    assert L.tucker_batched(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), None, facs, hist, done, stat, None, None, 2, ws,
                            1 << 30, st) == tk.TK_ERR_ARG
    assert L.tucker_batched(tk.ALGO_MP, 2, arr, J, ctypes.byref(o), cores, facs, hist, done, stat, None, tunes, 2,
                            ws, 1 << 30, st) == tk.TK_ERR_ARG


@pytest.mark.parametrize("field,bad,good", [("proj_elems", 512, 1024), ("proj_elems", 70000, 65536),
                                            ("proj_min_blocks", 32, 64), ("proj_min_blocks", 20000, 16384),
                                            ("gram_items", 63, 64), ("gram_items", 16385, 16384),
                                            ("gram_min_stages", 65, 64), ("gram_min_stages", -1, 1)])
def test_tune_ranges_checked_on_host(field, bad, good):
    c, d = _coo()
    for v, want in ((bad, tk.TK_ERR_ARG), (good, 0), (0, 0)):
        o = tk._opts(tune={field: v})
        st, b = _ws(c, (3, 3, 3), o)
        assert st == want, (field, v, st)


def test_tune_changes_no_workspace_rule():
    """A launch choice may change the Gram's split scratch, never the
    validation: every tune in range gives a positive workspace."""
    c, d = _coo(dims=(300, 200, 100), nnz=5000)
    for t in [(1024, 64, 64, 1), (65536, 16384, 16384, 64), (8192, 768, 512, 8)]:
        st, b = _ws(c, (20, 10, 5), tk._opts(tune=t))
        assert st == 0 and b > 0


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and field offsets of the option and statistics structs as a C
    compiler lays them out, against the binding's ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"tk_opts": tk.tk_opts, "tk_stats": tk.tk_stats, "tk_tune": tk.tk_tune, "tk_coo": tk.tk_coo,
               "tk_event": tk.tk_event, "tk_trace": tk.tk_trace}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tucker.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)


def test_split_bf16_precision_is_mp_only():
    c, d = _coo(dims=(40, 30, 20), nnz=500)
    o = tk.default_opts()
    o.precision = tk.MIXED_BF16X3
    st, b3 = _ws(c, (5, 4, 3), o, tk.ALGO_MP)
    assert st == 0
    o.precision = tk.MIXED_BF16
    st, b2 = _ws(c, (5, 4, 3), o, tk.ALGO_MP)
    assert st == 0 and b3 > b2  # lo parts, FP32 factor rows, six-term Gram splits
    o.precision = tk.MIXED_BF16X3
    st, _ = _ws(c, (5, 4, 3), o, tk.ALGO_HOOI)
    assert st == tk.TK_ERR_ARG
    o.precision = 4
    st, _ = _ws(c, (5, 4, 3), o, tk.ALGO_MP)
    assert st == tk.TK_ERR_ARG


def test_sp_and_hosvd_entry_points_reject_before_device_work():
    L = tk.lib()
    c, d = _coo()
    facs = (ctypes.c_void_p * 3)(0x10, 0x20, 0x30)
    hist = (ctypes.c_double * 50)()
    done = ctypes.c_int32(0)
    out = ctypes.c_double(0)
    o = tk.default_opts()
    o.init = tk.INIT_RANDOM
    bad = (ctypes.c_int32 * 3)(3, 10, 3)  # J2 > I2
    assert L.tucker_sp(ctypes.byref(c), bad, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50,
                       1 << 30, None) == tk.TK_ERR_ARG
    assert L.tucker_hosvd(ctypes.byref(c), bad, ctypes.byref(o), 0x40, facs, ctypes.byref(out), None, 0x50, 1 << 30,
                          None) == tk.TK_ERR_ARG
    J = (ctypes.c_int32 * 3)(3, 3, 3)
    assert L.tucker_sp(ctypes.byref(c), J, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50, 16,
                       None) == tk.TK_ERR_WORKSPACE
    assert L.tucker_hosvd(ctypes.byref(c), J, ctypes.byref(o), 0x40, facs, ctypes.byref(out), None, 0x50, 16,
                          None) == tk.TK_ERR_WORKSPACE
    assert L.tucker_hosvd(ctypes.byref(c), J, ctypes.byref(o), 0x40, facs, None, None, 0x50, 1 << 30,
                          None) == tk.TK_ERR_ARG
    # SP has no learned start
    o.init = tk.INIT_LEARNED
    o.model = 0x60
    assert L.tucker_sp(ctypes.byref(c), J, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50,
                       1 << 30, None) == tk.TK_ERR_ARG
    c0, d0 = _coo(nnz=0)
    o = tk.default_opts()
    o.init = tk.INIT_RANDOM
    assert L.tucker_sp(ctypes.byref(c0), J, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50,
                       1 << 30, None) == tk.TK_ERR_EMPTY


def test_random_start_and_hosvd_fit_options():
    c, d = _coo(dims=(40, 30, 20), nnz=500)
    for algo in (tk.ALGO_HOOI, tk.ALGO_MP, tk.ALGO_SP):
        o = tk.default_opts()
        o.init = tk.INIT_RANDOM
        st, b0 = _ws(c, (5, 4, 3), o, algo)
        assert st == 0 and b0 > 0
        o.hosvd_fit = 1  # one more FP64 projection buffer
        st, b1 = _ws(c, (5, 4, 3), o, algo)
        assert st == 0 and b1 > b0
        o.init = tk.INIT_GIVEN  # the report needs the factor buffers as scratch
        assert _ws(c, (5, 4, 3), o, algo)[0] == tk.TK_ERR_ARG
        o.init = tk.INIT_HOSVD
        o.hosvd_fit = 2
        assert _ws(c, (5, 4, 3), o, algo)[0] == tk.TK_ERR_ARG
        o.init = 4
        o.hosvd_fit = 0
        assert _ws(c, (5, 4, 3), o, algo)[0] == tk.TK_ERR_ARG
    st, b = _ws(c, (5, 4, 3), tk.default_opts(), tk.ALGO_HOSVD)
    assert st == 0 and b > 0
    assert _ws(c, (5, 4, 3), tk.default_opts(), 5)[0] == tk.TK_ERR_ARG


@pytest.mark.parametrize("case", ["J_over_128", "hosvd_dim", "slot_product"])
def test_documented_limits(case):
    """The limits listed in tucker.h, each at its edge: accepted on one side,
    TK_ERR_ARG on the other."""
    o = tk.default_opts()
    if case == "J_over_128":
        c, d = _coo(dims=(300, 200, 200), nnz=100)
        assert _ws(c, (128, 5, 5), o)[0] == 0
        assert _ws(c, (129, 5, 5), o)[0] == tk.TK_ERR_ARG
    elif case == "hosvd_dim":
        # modes 2 and 3 need their start Gram with an HO-SVD start; mode 1 does not
        c, d = _coo(dims=(9000, 10, 8192), nnz=100)
        assert _ws(c, (3, 3, 3), o)[0] == 0
        c, d = _coo(dims=(10, 8193, 10), nnz=100)
        assert _ws(c, (3, 3, 3), o)[0] == tk.TK_ERR_ARG
        for init in (tk.INIT_GIVEN, tk.INIT_RANDOM):
            o.init = init
            assert _ws(c, (3, 3, 3), o)[0] == 0
        o.init = tk.INIT_RANDOM
        o.hosvd_fit = 1
        assert _ws(c, (3, 3, 3), o)[0] == tk.TK_ERR_ARG
        o.hosvd_fit = 0
        c, d = _coo(dims=(8193, 10, 10), nnz=100)
        assert _ws(c, (3, 3, 3), tk.default_opts(), tk.ALGO_HOSVD)[0] == tk.TK_ERR_ARG
    else:
        # I_a * I_b < 2^31 for every pair of modes
        o.init = tk.INIT_GIVEN
        c, d = _coo(dims=(46340, 46340, 2), nnz=10)
        assert _ws(c, (1, 1, 1), o)[0] == 0
        c, d = _coo(dims=(46341, 46341, 2), nnz=10)
        assert _ws(c, (1, 1, 1), o)[0] == tk.TK_ERR_ARG


def test_fit_static_rejects_before_device_work():
    """The workspace-free fit checks its arguments and its size limit on the
    host, before it looks up the static scratch on a device."""
    L = tk.lib()
    facs = (ctypes.c_void_p * 3)(0x10, 0x20, 0x30)
    out = ctypes.c_double(0)
    c, d = _coo()
    bad = (ctypes.c_int32 * 3)(3, 10, 3)  # J2 > I2
    assert L.tucker_fit_static(ctypes.byref(c), bad, 0x40, facs, ctypes.byref(out), None) == tk.TK_ERR_ARG
    J = (ctypes.c_int32 * 3)(3, 3, 3)
    assert L.tucker_fit_static(ctypes.byref(c), J, None, facs, ctypes.byref(out), None) == tk.TK_ERR_ARG
    assert L.tucker_fit_static(ctypes.byref(c), J, 0x40, facs, None, None) == tk.TK_ERR_ARG
    # 2000 x 2000 x 100 with J3 = 50: the FP64 projection alone is 1.6 GB
    big, dbig = _coo(dims=(2000, 2000, 100), nnz=1000)
    J50 = (ctypes.c_int32 * 3)(50, 50, 50)
    st, need = _ws(big, (50, 50, 50), algo=tk.ALGO_FIT)
    assert st == 0 and need > tk.STATIC_SCRATCH_BYTES
    assert L.tucker_fit_static(ctypes.byref(big), J50, 0x40, facs, ctypes.byref(out), None) == tk.TK_ERR_SIZE
    assert "static" in tk.strerror(tk.TK_ERR_SIZE)
    # a small problem fits the static scratch
    st, need = _ws(c, (3, 3, 3), algo=tk.ALGO_FIT)
    assert st == 0 and need <= tk.STATIC_SCRATCH_BYTES


def _coo4(dims=(10, 9, 8, 7), nnz=5):
    c = tk.tk_coo()
    c.order = 4
    c.nnz = nnz
    d = (ctypes.c_int64 * 4)(*dims)
    c.dims = d
    for n in range(4):
        c.idx[n] = 0x1000
    c.vals = 0x2000
    return c, d


def test_fourth_order_options_checked_on_host():
    """Order 4 is accepted by HOOI, MP and HO-SVD (workspace query) and
    rejected by SP and the general fit; within MP and HOOI the options the
    fourth-order path does not offer are rejected before any device work."""
    c, d = _coo4()
    J = (ctypes.c_int32 * 4)(3, 3, 2, 2)
    out = ctypes.c_size_t(0)
    L = tk.lib()
    for algo in (tk.ALGO_HOOI, tk.ALGO_MP, tk.ALGO_HOSVD):
        o = tk.default_opts()
        assert L.tucker_workspace_bytes(algo, ctypes.byref(c), J, ctypes.byref(o), ctypes.byref(out)) == 0
        assert out.value > 0
    for algo in (tk.ALGO_SP, tk.ALGO_FIT):
        o = tk.default_opts()
        assert L.tucker_workspace_bytes(algo, ctypes.byref(c), J, ctypes.byref(o), ctypes.byref(out)) == tk.TK_ERR_ARG
    bad = []
    for field, value in (("precision", tk.MIXED_BF16X3), ("init", tk.INIT_LEARNED), ("init", tk.INIT_RANDOM),
                         ("max_iters", 0), ("hosvd_fit", 1)):
        o = tk.default_opts()
        setattr(o, field, value)
        bad.append(L.tucker_workspace_bytes(tk.ALGO_MP, ctypes.byref(c), J, ctypes.byref(o), ctypes.byref(out)))
    assert all(b == tk.TK_ERR_ARG for b in bad), bad
    # J > I, J > 128, slots beyond 32 bits
    o = tk.default_opts()
    Jbad = (ctypes.c_int32 * 4)(3, 3, 9, 2)
    assert L.tucker_workspace_bytes(tk.ALGO_MP, ctypes.byref(c), Jbad, ctypes.byref(o), ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    cb, db = _coo4(dims=(2000, 2000, 1000, 10))
    assert L.tucker_workspace_bytes(tk.ALGO_MP, ctypes.byref(cb), J, ctypes.byref(o), ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    # the drivers reject before device work too (null core)
    facs = (ctypes.c_void_p * 4)(0x10, 0x20, 0x30, 0x40)
    hist = (ctypes.c_double * 50)()
    done = ctypes.c_int32(0)
    assert L.tucker_mp(ctypes.byref(c), J, ctypes.byref(o), None, facs, hist, ctypes.byref(done), None, 0x50,
                       1 << 30, None) == tk.TK_ERR_ARG
    assert L.tucker_hooi(ctypes.byref(c), J, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None, 0x50, 16,
                         None) == tk.TK_ERR_WORKSPACE


def test_streamed_mp_checks_on_host():
    """The streamed MP reads host arrays: its arguments, slab size and the
    data's index and value checks all run on the host, before device work."""
    import numpy as np
    L = tk.lib()
    idx = np.array([[0, 1, 2, 3], [0, 1, 2, 0], [1, 1, 1, 1]], dtype=np.int32)
    vals = np.array([1.0, 2.0, 3.0, 4.0])
    coo = tk._HostCoo(idx, vals, (4, 3, 2))
    J = (ctypes.c_int32 * 3)(2, 2, 1)
    o = tk._opts("fp64", init=tk.INIT_RANDOM)
    out = ctypes.c_size_t(0)
    assert L.tucker_mp_streamed_workspace(ctypes.byref(coo.c), J, ctypes.byref(o), 1 << 16, ctypes.byref(out)) == 0
    ws_small = out.value
    assert L.tucker_mp_streamed_workspace(ctypes.byref(coo.c), J, ctypes.byref(o), 1 << 20, ctypes.byref(out)) == 0
    assert out.value > ws_small
    # a slab that cannot hold one slice of a projection (400 rows of 16 bytes
    # against the smallest slab of 256 bytes)
    wide = tk._HostCoo(idx, vals, (400, 3, 2))
    assert L.tucker_mp_streamed_workspace(ctypes.byref(wide.c), J, ctypes.byref(o), 8, ctypes.byref(out)) == \
        tk.TK_ERR_ARG
    for field, value in (("init", tk.INIT_HOSVD), ("precision", tk.MIXED_BF16X3), ("max_iters", 0)):
        ob = tk._opts("fp64", init=tk.INIT_RANDOM)
        setattr(ob, field, value)
        assert L.tucker_mp_streamed_workspace(ctypes.byref(coo.c), J, ctypes.byref(ob), 1 << 16,
                                              ctypes.byref(out)) == tk.TK_ERR_ARG
    facs = (ctypes.c_void_p * 3)(0x10, 0x20, 0x30)
    hist = (ctypes.c_double * 50)()
    done = ctypes.c_int32(0)
    assert L.tucker_mp_streamed_workspace(ctypes.byref(coo.c), J, ctypes.byref(o), 1 << 16, ctypes.byref(out)) == 0
    need = out.value
    # workspace too small, then index and value errors found on the host
    assert L.tucker_mp_streamed(ctypes.byref(coo.c), J, ctypes.byref(o), 1 << 16, 0x40, facs, hist,
                                ctypes.byref(done), None, 0x50, 16, None) == tk.TK_ERR_WORKSPACE
    bad = idx.copy()
    bad[1, 2] = 7
    cb = tk._HostCoo(bad, vals, (4, 3, 2))
    assert L.tucker_mp_streamed(ctypes.byref(cb.c), J, ctypes.byref(o), 1 << 16, 0x40, facs, hist,
                                ctypes.byref(done), None, 0x50, need, None) == tk.TK_ERR_INDEX
    vb = vals.copy()
    vb[3] = np.nan
    cv = tk._HostCoo(idx, vb, (4, 3, 2))
    assert L.tucker_mp_streamed(ctypes.byref(cv.c), J, ctypes.byref(o), 1 << 16, 0x40, facs, hist,
                                ctypes.byref(done), None, 0x50, need, None) == tk.TK_ERR_VALUE


def test_implicit_mp_checks_on_host():
    """tucker_mp_implicit rejects bad problems and options before device
    work; its workspace bound grows with the nonzeros (fibres), not with the
    mode sizes squared."""
    L = tk.lib()
    J = (ctypes.c_int32 * 3)(4, 3, 2)
    out = ctypes.c_size_t(0)
    o = tk._opts("fp64", init=tk.INIT_RANDOM)
    c, _d = _coo((20000, 20000, 20000), nnz=1000)
    assert L.tucker_mp_implicit_workspace(ctypes.byref(c), J, ctypes.byref(o), ctypes.byref(out)) == 0
    small = out.value
    c2, _d2 = _coo((20000, 20000, 20000), nnz=100_000)
    assert L.tucker_mp_implicit_workspace(ctypes.byref(c2), J, ctypes.byref(o), ctypes.byref(out)) == 0
    big = out.value
    # the dense slot pointers (three orderings of 20000^2 slots) are the same
    # in both; the difference is per nonzero / fibre
    per_nz = (big - small) / 99_000
    assert 100 < per_nz < 4000
    for field, value in (("init", tk.INIT_HOSVD), ("init", tk.INIT_LEARNED), ("precision", tk.MIXED_BF16X3),
                         ("max_iters", 0), ("hosvd_fit", 1), ("eig_max_iters", 0)):
        ob = tk._opts("fp64", init=tk.INIT_RANDOM)
        setattr(ob, field, value)
        assert L.tucker_mp_implicit_workspace(ctypes.byref(c), J, ctypes.byref(ob), ctypes.byref(out)) == \
            tk.TK_ERR_ARG, (field, value)
    # core larger than 128, core larger than the mode, a pair of modes with
    # 2^31 slots, order 4
    for dims, core in (((300, 300, 300), (129, 3, 2)), ((3, 300, 300), (4, 3, 2)),
                       ((50000, 50000, 10), (4, 3, 2))):
        cc, _dd = _coo(dims, nnz=10)
        Jc = (ctypes.c_int32 * 3)(*core)
        assert L.tucker_mp_implicit_workspace(ctypes.byref(cc), Jc, ctypes.byref(o), ctypes.byref(out)) == \
            tk.TK_ERR_ARG, dims
    c4, _d4 = _coo((10, 9, 8), nnz=5, order=4)
    assert L.tucker_mp_implicit_workspace(ctypes.byref(c4), J, ctypes.byref(o), ctypes.byref(out)) == tk.TK_ERR_ARG
    facs = (ctypes.c_void_p * 3)(0x10, 0x20, 0x30)
    hist = (ctypes.c_double * 50)()
    done = ctypes.c_int32(0)
    c3, _d3 = _coo((10, 9, 8), nnz=5)
    assert L.tucker_mp_implicit(ctypes.byref(c3), J, ctypes.byref(o), None, facs, hist, ctypes.byref(done), None,
                                0x50, 1 << 30, None) == tk.TK_ERR_ARG
    assert L.tucker_mp_implicit(ctypes.byref(c3), J, ctypes.byref(o), 0x40, facs, hist, ctypes.byref(done), None,
                                0x50, 16, None) == tk.TK_ERR_WORKSPACE

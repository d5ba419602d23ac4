"""The tuner's host side: shape buckets and the JSON cache (no GPU)."""
import paper_0711_2023_amd as tk
from paper_0711_2023_amd import autotune as at


def test_bucket_rounds_shapes():
    a = at.bucket(tk.ALGO_MP, "mixed", (1000, 1000, 1000), 1_000_000, (50, 50, 50))
    assert a == "mp/mixed/nnz~2^20/I~2^10/J<=64"
    # nearby shapes share a bucket, other algorithms and precisions do not
    assert at.bucket(tk.ALGO_MP, "mixed", (1100, 900, 1000), 1_100_000, (60, 40, 50)) == a
    assert at.bucket(tk.ALGO_HOOI, "mixed", (1000, 1000, 1000), 1_000_000, (50, 50, 50)) != a
    assert at.bucket(tk.ALGO_MP, "fp32", (1000, 1000, 1000), 1_000_000, (50, 50, 50)) != a
    assert at.bucket(tk.ALGO_MP, "mixed", (1000, 1000, 1000), 4_000_000, (50, 50, 50)) != a


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    c = at.TuneCache(path)
    assert c.get("x") is None
    c.put("x", tk.make_tune((4096, 512, 256, 2)), {"project_ms": [1.0, 0.5]})
    c.save()
    d = at.TuneCache(path)
    assert d.get("x").key() == (4096, 512, 256, 2)
    assert d.entries["x"]["project_ms"] == [1.0, 0.5]


def test_make_tune_forms():
    assert tk.make_tune({"gram_items": 128}).key() == (0, 0, 128, 0)
    assert tk.make_tune((1, 2, 3, 4)).key() == (1, 2, 3, 4)
    t = tk.make_tune((5, 6, 7, 8))
    assert tk.make_tune(t) is t


def test_candidates_within_the_header_ranges():
    for pe, pb in at.PROJ_CANDIDATES:
        assert pe == 0 or 1024 <= pe <= 65536
        assert pb == 0 or 64 <= pb <= 16384
    assert all(g == 0 or 64 <= g <= 16384 for g in at.GRAM_ITEMS)
    assert all(s == 0 or 1 <= s <= 64 for s in at.GRAM_STAGES)

"""bench.py's host-side pieces (CPU): the reader of committed profile
summaries takes numbers only while the kernel sources match the digest
recorded with them, and the roofline object follows from the headline's
counts and durations as its keys say."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _summary(tmp_path, digest, **kv):
    p = tmp_path / "summary.txt"
    lines = ["# a summary", "  indented command lines are not keys: x"]
    lines += [f"source_digest: {digest}"] + [f"{k}: {v}" for k, v in kv.items()]
    p.write_text("\n".join(lines) + "\n")
    return str(p)


def test_summary_reader_follows_the_digest(tmp_path, monkeypatch):
    import bench
    import paper_2403_15435_amd.build as b
    monkeypatch.setattr(b, "source_digest", lambda: "a" * 64)
    kv = bench.read_summary(_summary(tmp_path, "a" * 64, step_kernel_avg_us="812.5"))
    assert kv is not None and bench._num(kv, "step_kernel_avg_us") == 812.5
    assert "indented command lines are not keys" not in kv
    assert bench.read_summary(_summary(tmp_path, "b" * 64, step_kernel_avg_us="812.5")) is None
    assert bench.read_summary(str(tmp_path / "missing.txt")) is None


def test_roofline_object(tmp_path, monkeypatch):
    import bench
    import paper_2403_15435_amd.build as b
    monkeypatch.setattr(b, "source_digest", lambda: "c" * 64)
    # 400 launches of 800 us, 20000 patches of 1024 cells updated per launch
    v32 = {"step_kernel_launches": 400, "step_kernel_avg_us": 800.0, "patches_full_update": 400 * 20000,
           "cell_updates": 400 * 25000 * 1024, "accepted_steps": 400, "rejected": 0, "step_threads": 512,
           "step_pad": 0}
    probe = {"best_GBps": 6000.0}
    monkeypatch.setattr(bench, "VALLEY_COUNTERS", _summary(tmp_path, "c" * 64, valu_lane_ops_per_launch=2.0e10,
                                                           fetch_kib_per_launch=500000.0, fetch_scale=2.0,
                                                           write_kib_per_launch=250000.0, write_scale=1.0,
                                                           kernel_shape="512,0"))
    monkeypatch.setattr(bench, "VALLEY_STATS", str(tmp_path / "none.txt"))
    r = bench.roofline(v32, probe)
    cells = 20000 * 1024.0
    t = 800e-6
    assert r["cells_updated_per_launch"] == cells
    assert r["achieved"] == pytest.approx(500.0 * cells / t / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / (256 * 4 * 16 * 2.4))
    assert r["hbm"]["achieved"] == pytest.approx(28.0 * cells / t / 1e9)
    assert r["hbm"]["dense_equivalent_frac"] == pytest.approx(28.0 * 25000 * 1024 / t / 1e9 / 8000.0)
    assert r["traffic"] == pytest.approx(1024.0 * (500000.0 * 2.0 + 250000.0))
    # issued VALU 2e10 / 800 us = 25 Tops/s of 39.3: above the traffic's 1.28 TB/s of 8
    assert r["bound"] == "alu" and r["bound_from"] == "counters"
    assert r["issued_valu_ops_per_cell"] == pytest.approx(2.0e10 / cells)
    # counters of another shape (LDS row padding 1) do not count
    r3 = bench.roofline(dict(v32, step_pad=1), probe)
    assert r3["traffic"] is None and r3["issued_valu_frac"] is None
    monkeypatch.setattr(bench, "VALLEY_COUNTERS", str(tmp_path / "none.txt"))
    r2 = bench.roofline(v32, None)
    assert r2["traffic"] is None and r2["issued_valu_frac"] is None and r2["bound"] == "alu"

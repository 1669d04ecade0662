"""bench.py's readers of the committed profiles (CPU): the HBM traffic and
the kernel durations come back as numbers while the kernel sources match the
digest recorded with them, and as None otherwise."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _digest_matches():
    from paper_2403_15435_amd.build import source_digest
    path = os.path.join(ROOT, "profiles", "step_fp32_reservoir2048_hbm_traffic.txt")
    return os.path.exists(path) and source_digest() in open(path).read()


def test_profile_readers():
    import bench
    if not _digest_matches():
        pytest.skip("profiles were taken on other kernel sources; run the profiles again")
    traffic = bench.measured_traffic()
    assert traffic is not None and 1e6 < traffic < 1e9
    kv = {}
    for line in open(bench.TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    want = (float(kv["fetch_kib_per_step"]) * float(kv["fetch_scale"])
            + float(kv["write_kib_per_step"]) * float(kv["write_scale"])) * 1024.0
    assert traffic == want
    us = bench.profiled_kernel_us()
    assert us is not None and set(us) == {"dry_kernel_us", "step_kernel_us"}
    assert 0.0 < us["dry_kernel_us"] < us["step_kernel_us"] < 1000.0


def test_readers_refuse_other_sources(monkeypatch):
    import bench
    import paper_2403_15435_amd.build as b
    monkeypatch.setattr(b, "source_digest", lambda: "0" * 64)
    assert bench.measured_traffic() is None
    assert bench.profiled_kernel_us() is None

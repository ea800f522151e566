"""The benchmark's byte accounting and its guards, on the host: the
per-unit figures each kernel is charged, the touched-byte figures, the
counter values used only while the kernel source they were taken on is
unchanged, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

TOT = {"frames": 10, "frame_blocks": 1000, "dirty_blocks": 1200, "vertex_blocks": 1300,
       "new_vertices": 5000, "updated_vertices": 20000, "freed_vertices": 4000,
       "moved_vertices": 18000, "new_triangles": 9000, "dropped_triangles": 8000}
NPIX = 640 * 480


def test_method_bytes_per_kernel():
    k, step = bench.algorithmic_bytes(TOT, NPIX)
    assert k == {"collect": 4 * NPIX * 10, "fuse": 8192 * 1000, "classify": 5120 * 1200,
                 "vertices": 20 * 25000 + 8 * 4000}
    assert step == sum(k.values()) + 12 * 9000 + 8 * (9000 + 8000)


def test_refinement_pass_takes_half_the_dirty_total():
    k, step = bench.algorithmic_bytes(TOT, NPIX, refine=True)
    assert k["classify"] == 5120 * 600 and k["refine"] == 3072 * 600
    t = bench.touched_bytes(TOT, NPIX, refine=True)
    assert t["classify"] == 5632 * 600 and t["refine"] == 3648 * 600


def test_touched_bytes_per_kernel():
    t = bench.touched_bytes(TOT, NPIX)
    assert t["fuse"] == 4 * NPIX * 10 + 8192 * 1000
    assert t["vertices"] == 2816 * 1300 + 4 * 18000 + 16 * 5000 + 12 * 4000
    assert "refine" not in t


def test_counted_traffic_only_for_the_source_it_was_taken_on(monkeypatch):
    for k in ("collect", "fuse", "classify", "vertices"):
        assert len(bench.kernel_source_sha1(k)) == 12
    m = dict(bench.MEASURED_TRAFFIC)
    m["vertices"] = dict(m["vertices"], source_sha1=bench.kernel_source_sha1("vertices"))
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", m)
    want = int(1024 * (m["vertices"]["fetch_kib"] * bench.COUNTER_SCALE["fetch"]
                       + m["vertices"]["write_kib"] * bench.COUNTER_SCALE["write"]))
    assert bench.measured_traffic("vertices") == want
    m["vertices"] = dict(m["vertices"], source_sha1="000000000000")
    assert bench.measured_traffic("vertices") is None
    assert bench.measured_traffic("dirty") is None


def test_roofline_fraction():
    # 8 GB in 1 ms is the 8 TB/s peak
    assert bench.frac(8e9, 1.0) == pytest.approx(1.0)
    assert bench.frac(2e9, 1.0) == pytest.approx(0.25)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""

"""Host logic of the throughput measurement (no GPU): the committed HBM
counter figures are used only while the kernel sources are unchanged, and a
multi-GPU request is refused before anything touches a device."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sources_sha():
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2009_03254_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def test_sources_hash_matches_bench():
    assert bench.sources_sha256() == _sources_sha()


def test_traffic_only_for_current_sources(tmp_path, monkeypatch):
    f = tmp_path / "counters.md"
    f.write_text("text\n```\n"
                 f"traffic k_mc_emit bytes_per_dispatch=123456 sources_sha256={_sources_sha()}\n"
                 f"traffic k_cull bytes_per_dispatch=99 sources_sha256={'0' * 64}\n```\n")
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(f))
    assert bench.measured_traffic("k_mc_emit") == 123456
    assert bench.measured_traffic("k_cull") is None           # taken on other sources
    assert bench.measured_traffic("k_masks") is None          # not listed
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("k_mc_emit") is None


def test_committed_counters_name_the_roofline_kernels():
    for f in (bench.COUNTERS_FILE, bench.COUNTERS_FILE_512):
        text = open(f).read()
        for k in bench.kernel_defs(2):
            assert f"traffic {k} bytes_per_dispatch=" in text, (f, k)


def test_kernel_bytes_per_unit():
    """Algorithmic bytes: 8R + 256 per decoded block; 256 per occupied block
    plus 8 per vertex (24 per triangle) for the emission, no bookkeeping."""
    st = {"n_new": 10, "n_occupied": 3, "n_triangles": 7, "n_active": 99}
    kd = bench.kernel_defs(2)
    assert kd["k_assign_decode"][1](st) == 10 * (16 + 256)
    assert kd["k_mc_emit"][1](st) == 3 * 256 + 7 * 24


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""

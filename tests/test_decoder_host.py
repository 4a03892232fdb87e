"""The library's ZFP block decoders (device code, compiled here for the
host) against the oracle's decoder, bit for bit, on random block bits at
rates 1..32: long zero runs, budgets that end inside a group test, the
implied last coefficient.  Covers the plane-by-plane decoder and the
two-pass decoder the staged kernels run, both precisions.  No GPU needed;
skipped when hipcc is absent."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_host_decoders_match_oracle(orc):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = os.path.join(ROOT, "tests", "host", "decoder_check.hip")
    libdir = os.path.join(ROOT, "oracle")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "decoder_check")
        cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", exe, src, "-L", libdir, "-loracle", f"-Wl,-rpath,{libdir}"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-3000:]
        assert "mismatching values 0" in r.stdout

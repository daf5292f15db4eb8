"""The tile orders of the stencil kernels (plain and time series, plain and
XCD-aware), checked on the host: tests/tilemap_check.hip includes the
library's tile-map header, builds the maps for 2880 grid / tile shapes (four plain maps and one time-series map each) and
checks that block slots map one to one onto tiles that cover every plane of
every column exactly once, time-series chunks never straddling a step."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not installed")
def test_tile_orders_cover_every_plane_once(tmp_path):
    exe = tmp_path / "tilemap_check"
    src = os.path.join(ROOT, "tests", "tilemap_check.hip")
    cmd = [HIPCC if os.path.exists(HIPCC) else "hipcc", "-O1", "-std=c++17",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2509_26213_amd", "csrc"), src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout[-2000:]
    last = r.stdout.strip().splitlines()[-1]
    cases, bad = (int(v) for v in last.replace("cases", "").replace("bad", "").split())
    assert cases > 10000 and bad == 0, last

"""Host logic of bench.py: the tile key the traffic profiles are matched on,
reading a traffic summary (quoted only for the kernel source and tile it
was measured on), and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_tile_key_names_pass2_tiles_only_when_they_differ():
    t = dict(vx=2, by=8, zc=64, xcd=0)
    assert bench.tile_key(t) == "vx=2 by=8 zc=64 xcd=0"
    assert bench.tile_key(dict(t, by2=8, zc2=64)) == "vx=2 by=8 zc=64 xcd=0"
    assert bench.tile_key(dict(t, by2=4, zc2=32)) == "vx=2 by=8 zc=64 xcd=0 pass2 by=4 zc=32"


def test_traffic_summary_is_quoted_for_its_source_and_tile_only(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    tile = dict(vx=1, by=8, zc=64, xcd=0)
    text = ["# summary", "", "- kernel: k_cg_pass2", "- workload: demo",
            f"- kernel_source_sha256: {bench.kernel_source_hash()}",
            "- traffic_over_algorithmic: 1.2500", f"- tile: {bench.tile_key(tile)}", ""]
    (tmp_path / "profiles" / "k_cg_pass2_demo_traffic.md").write_text("\n".join(text))
    sha = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha)
    assert bench.measured_traffic("k_cg_pass2", "demo", tile) == 1.25
    assert bench.traffic(1.25, 8.0e9) == 1.0e10
    assert bench.measured_traffic("k_cg_pass2", "demo", dict(tile, by=4)) is None
    assert bench.measured_traffic("k_cg_pass2", "other", tile) is None
    stale = [ln.replace(sha, "0" * 64) for ln in text]
    (tmp_path / "profiles" / "k_cg_pass2_demo_traffic.md").write_text("\n".join(stale))
    assert bench.measured_traffic("k_cg_pass2", "demo", tile) is None
    assert bench.traffic(None, 8.0e9) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]

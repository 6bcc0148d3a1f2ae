"""Host-side behaviour of bench.py that needs no GPU: the one-GPU guard and the
rule that counter traffic is reported only for the kernel sources it was
measured on."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _copy_tree(dst):
    os.makedirs(os.path.join(dst, "profiles"))
    shutil.copy(os.path.join(ROOT, "profiles", "traffic.json"), os.path.join(dst, "profiles"))
    shutil.copytree(os.path.join(ROOT, "paper_2409_02482_amd", "csrc"),
                    os.path.join(dst, "paper_2409_02482_amd", "csrc"))


def test_counter_traffic_follows_the_sources(tmp_path, monkeypatch):
    import bench
    recs = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    key = "metric/shade_bwd"
    assert key in recs and recs[key]["bytes_per_launch"] > 0
    _copy_tree(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # same sources as recorded: the recorded bytes; an unknown kernel: none
    if bench.counter_traffic("metric", "shade_bwd") is None:
        pytest.skip("kernel sources changed since the counters were taken (the bench reports null traffic)")
    assert bench.counter_traffic("metric", "shade_bwd") == recs[key]["bytes_per_launch"]
    assert bench.counter_traffic("metric", "no_such_kernel") is None
    # any change to a kernel source voids every record
    src = tmp_path / "paper_2409_02482_amd" / "csrc" / "vs_shade.h"
    src.write_text(src.read_text() + "\n// edited\n")
    assert bench.counter_traffic("metric", "shade_bwd") is None
    assert bench.counter_traffic("ksdf", "ksdf_render") is None
    # no summary file: none
    os.remove(tmp_path / "profiles" / "traffic.json")
    assert bench.counter_traffic("metric", "shade_bwd") is None

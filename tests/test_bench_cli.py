"""bench.py's host-side contract, without a GPU: it refuses more than one
GPU, and its measured-traffic lookup accepts only a profile of the same sweep
code and launch shape."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_measured_traffic_matches_code_and_shape(tmp_path, monkeypatch):
    import bench
    from paper_0911_5692_amd import workloads as W
    from paper_0911_5692_amd.profile_sweep import sweep_source_hash

    w = W.CFG3
    shape = dict(W.BENCH_SHAPES[w.name])
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"sweep_source_hash": sweep_source_hash(w.stencil), "launch_shape": shape,
           "hbm_bytes_per_launch": 123.0}
    (prof / f"sweep_traffic_{w.name}.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(w.name, w.stencil, shape) == 123.0
    assert bench.measured_traffic(w.name, w.stencil, dict(shape, zchunk=64)) is None
    rec["sweep_source_hash"] = "0" * 16
    (prof / f"sweep_traffic_{w.name}.json").write_text(json.dumps(rec))
    assert bench.measured_traffic(w.name, w.stencil, shape) is None
    assert bench.measured_traffic("no_such_workload", 7, {}) is None


def test_source_hash_ignores_comments_and_spacing():
    from paper_0911_5692_amd.profile_sweep import _code_only
    a = "int x = 1; // one\n/* block\n comment */  int  y=2;\n"
    b = "int x = 1;\nint y=2; // two\n"
    assert _code_only(a) == _code_only(b) == "int x = 1; int y=2;"
    assert _code_only("int x = 1;") != _code_only("int x = 2;")

"""bench.py's command line on a machine without a GPU: the one-GPU rule and
the argument surface (no kernel runs here)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("single", "scan", "learned", "precision", "paper", "--autotune", "--tile-y", "--fused-plaquette"):
        assert w in r.stdout


def test_one_core_oracle_rate_runs_single_threaded():
    sys.path.insert(0, ROOT)
    import bench
    rate, threads, seconds = bench.oracle_one_core_rate((4, 4, 4, 4), 6.0, 1234, 1)
    assert threads == 1 and rate > 0 and seconds > 0


def test_stored_traffic_lookup_matches_walk_and_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    line = ("traffic: kernel=overrelax_kernel prec=f32 shape=8,8,8,8 walk=2,1 bytes_per_launch=1234 "
            f"csrc_sha256={bench.csrc_sha256()}\n")
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "x.md").write_text("# t\n" + line)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "csrc_sha256", lambda: line.split("csrc_sha256=")[1].strip())
    assert bench.profiled_traffic("overrelax_kernel", "f32", "8,8,8,8", (2, 1)) == 1234.0
    assert bench.profiled_traffic("overrelax_kernel", "f32", "8,8,8,8", (2, 2)) is None
    assert bench.profiled_traffic("heatbath_kernel", "f32", "8,8,8,8", (2, 1)) is None
    monkeypatch.setattr(bench, "csrc_sha256", lambda: "0" * 64)
    assert bench.profiled_traffic("overrelax_kernel", "f32", "8,8,8,8", (2, 1)) is None


def test_shipped_walks_are_valid_candidates():
    import json
    path = os.path.join(ROOT, "paper_1104_5432_amd", "tuned_walks.json")
    with open(path) as f:
        table = json.load(f)
    assert table
    for key, v in table.items():
        arch, cus, shape, prec = key.split("|")
        n = tuple(int(x) for x in shape.split("x"))
        assert arch.startswith("gfx") and cus.endswith("cu") and prec in ("f32", "f64")
        assert v["tile"] == -1 or n[2] % v["tile"] == 0
        assert v["tile_y"] == 0 or n[1] % v["tile_y"] == 0

"""bench.py's output line on the GPU: one JSON object with the fields the
measurement contract fixes (throughput, roofline of the dominant kernel,
timed oracle sample), at a small lattice so it runs in seconds."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


def _bench(*args):
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                       text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0])


def test_single_workload_line():
    rec = _bench("--shape", "16,16,16,8", "--steps", "3", "--warmup", "1", "--no-autotune",
                 "--cpu-shape", "4,4,4,4", "--cpu-seconds", "0.5")
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in rec, key
    assert rec["n_gpus"] == 1 and rec["steps"] == 3 and rec["warmup"] == 1
    assert rec["value"] > 0 and rec["ms_per_step"] > 0 and rec["higher_is_better"] is True
    assert rec["unit"] == "link updates/s" and rec["dtype"] == "f32" and rec["vs_baseline"] is None
    # value is the step's link updates over its time
    per_step = 16 * 16 * 16 * 8 * 4 * (1 + 4)
    assert abs(rec["value"] * rec["ms_per_step"] * 1e-3 / per_step - 1) < 1e-6
    assert "workload" in rec["config"]
    roof = rec["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["achieved"] > 0 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    assert roof["traffic"] is None          # no stored counters for this lattice and walk
    cpu = rec["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1 and cpu["sample"]
    assert "cpu" in cpu                     # the host CPU model (None where unreadable)


"""bench.py's output contract: one JSON line with the fields the harness
reads (metric, value, unit, step counts, roofline, CPU baseline), and a clean
refusal of more than one GPU (before any GPU call)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.gpu
def test_one_json_line_with_the_contract_fields():
    """A short run (256^2 grid, 2 timed steps, a 1 s CPU sample); the
    fields, not the numbers, are checked."""
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "256", "--steps", "2", "--warmup", "1",
           "--batch-steps", "0", "--serve-jobs", "0", "--boundaries", "0", "--shard-parts", "0",
           "--cpu-seconds", "1"]
    print("\n[bench] " + " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["value"] > 0
    assert d["higher_is_better"] is True and d["vs_baseline"] is None and "workload" in d["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in d["roofline"], k
    assert 0 < d["roofline"]["frac"] < 1
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]

"""The benchmark's command-line contract where no GPU is needed: more than
one GPU is refused with a message, and without a visible GPU the run fails
loudly (no host fallback) and leaves no oracle timing process behind."""
import json
import os
import re
import subprocess
import sys
import time

import pytest
import torch

ROOT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..")
BENCH = os.path.join(ROOT, "bench.py")


def run(*argv):
    r = subprocess.run([sys.executable, BENCH, *argv], capture_output=True, text=True, timeout=300, cwd=ROOT)
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    return r, (json.loads(lines[-1]) if lines else None)


def test_several_gpus_refused():
    r, out = run("--gpus", "2")
    assert r.returncode == 2
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the behaviour without a GPU")
@pytest.mark.parametrize("workload", ["chamber", "kernels", "serve"])
def test_no_gpu_fails_loudly(workload):
    r, out = run("--workload", workload)
    assert r.returncode == 1 and out == {"error": "no GPU visible"}, (r.returncode, r.stdout, r.stderr[-2000:])
    m = re.search(r"oracle timing started in process (\d+)", r.stderr)
    assert (m is not None) == (workload == "chamber")
    if m:   # the oracle's timing child was stopped and collected with the run
        pid = int(m.group(1))
        time.sleep(0.2)
        assert not os.path.exists(f"/proc/{pid}"), f"oracle timing process {pid} outlived the benchmark"

"""bench.py's command line on the host: with fewer than 16 hardware queues in
its environment (or none) it runs itself as a child process with 16 and exits
with the child's status, and a larger setting is kept; more than one GPU is
refused (no GPU is touched)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(queues):
    env = {k: v for k, v in os.environ.items()
           if k not in ("GPU_MAX_HW_QUEUES", "FACO_BENCH_CHILD")}
    if queues is not None:
        env["GPU_MAX_HW_QUEUES"] = queues
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                          env=env, capture_output=True, text=True, timeout=120)


@pytest.mark.parametrize("queues,seen", [(None, "16"), ("4", "16"), ("16", "16"), ("24", "24")])
def test_hardware_queues_and_status(queues, seen):
    r = _run(queues)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert f"GPU_MAX_HW_QUEUES={seen}" in r.stderr

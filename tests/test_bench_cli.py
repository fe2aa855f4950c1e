"""bench.py measures one GPU: asked for more (by flag or by a launcher's WORLD_SIZE) it exits
with status 2 and says so, before touching any device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=e,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_a_multi_rank_launch_is_refused():
    r = _run(["--gpus", "1"], env={"WORLD_SIZE": "2", "RANK": "1"})
    assert r.returncode == 2
    assert "one GPU" in r.stderr

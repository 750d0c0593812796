"""bench.py's command line on the CPU: a request for more than one GPU (or a
multi-rank launch) is refused with a message before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ, **(env_extra or {}))
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=60, env=env)


def test_more_than_one_gpu_is_refused():
    for n in ("2", "8"):
        r = _run(["--gpus", n, "--steps", "1", "--warmup", "0"])
        assert r.returncode == 2 and r.stdout == ""
        assert "one GPU only" in r.stderr


def test_multi_rank_launch_is_refused():
    r = _run(["--gpus", "1"], {"WORLD_SIZE": "2"})
    assert r.returncode == 2 and "one GPU only" in r.stderr

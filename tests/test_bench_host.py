"""Host-side contract of bench.py (no GPU needed): it runs on one GPU and
refuses any request for more, by argument or by a multi-process launcher's
environment, with a message and exit status 2 before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          env=env, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run(["--gpus", "2", "--steps", "1", "--warmup", "0"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_multi_process_launch_is_refused():
    r = run(["--steps", "1", "--warmup", "0"], {"WORLD_SIZE": "4", "RANK": "0"})
    assert r.returncode == 2
    assert "WORLD_SIZE 4" in r.stderr and r.stdout == ""

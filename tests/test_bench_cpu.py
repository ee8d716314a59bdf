"""bench.py's command-line contract on a host without a GPU: more than one
GPU is refused with a message, and without a device it fails loudly instead
of timing anything on the host."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    r = run_bench(env_extra={"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert r.stdout == ""


def test_no_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        return   # the GPU suite covers the timed path
    r = run_bench("--steps", "1", "--warmup", "0")
    assert r.returncode == 1
    assert "needs a GPU" in r.stderr
    assert r.stdout == ""

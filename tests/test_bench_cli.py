"""bench.py's one-GPU contract, checked on the host: asked for several GPUs
(by flag or by a launcher's WORLD_SIZE) it stops before touching a device,
with a message, and its workloads have the sizes their descriptions state."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=300)


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], None), (["--gpus", "8"], None),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = _run(args, env)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_workload_sizes():
    sys.path.insert(0, ROOT)
    import bench

    desc, bits, jobs = bench.workload("ragged64")
    assert bits == 8 and len(jobs) == 64
    for (_, n, i, h, w, b, ceil) in jobs:
        assert 480 <= h <= 3000 and 640 <= w <= 4000 and b == 8 and 0.03 <= ceil <= 0.4
    desc, bits, jobs = bench.workload("uhd16")
    assert bits == 10 and sorted((h, w) for (_, _, _, h, w, _, _) in jobs) == [(2160, 3840)] * 8 + [(4320, 7680)] * 8
    desc, bits, jobs = bench.workload("single")
    assert bits == 8 and [(h, w) for (_, _, _, h, w, _, _) in jobs] == [(664, 1000)]

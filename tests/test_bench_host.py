"""Host-side behaviour of bench.py that needs no GPU: the one-GPU refusal and the
counter table's references."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run_bench(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line for a refused run


def test_world_size_above_one_is_refused():
    r = run_bench([], {"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_counter_table_points_at_committed_profiles():
    sys.path.insert(0, ROOT)
    import bench
    for (workload, kernel), (nbytes, files, digest, src, busy) in bench.TRAFFIC.items():
        assert nbytes > 0 and 0.0 < busy < 1.0 and len(digest) == 16
        for f in files:
            assert os.path.exists(os.path.join(ROOT, "paper_2004_10811_amd", "csrc", f))
        text = open(os.path.join(ROOT, src)).read()
        assert kernel in text and workload in text
        # the figure is reported only while the kernel's sources are unchanged
        got = bench.measured_traffic(workload, kernel)
        assert got == (None, None, None) or got == (nbytes, src, busy)

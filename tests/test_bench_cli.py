"""bench.py's command-line contract on the host: one GPU only, and the
defaults that the benchmark line is quoted with."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_defaults():
    sys.path.insert(0, ROOT)
    import bench
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert (a.gpus, a.steps, a.warmup, a.mc_per_step, a.workload, a.autotune) == \
        (1, 30, 2, 1000, "cfg2", False)
    assert bench.OPS_PER_WORD_UPDATE == {1: 129, 2: 131, 3: 135, 4: 139}
    # the default line runs the library's default shape, per-phase launches, no skipping
    assert (a.teams, a.tile_cols, a.phase_max, a.persistent, a.skip_empty, a.graph) == \
        (0, 0, 0, False, False, False)

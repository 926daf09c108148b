"""Host-side parts of bench.py that need no GPU: the one-GPU guard of every
mode and the algorithmic byte and operation counts its roofline uses."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1501_05630_amd import inputs  # noqa: E402


@pytest.mark.parametrize("mode", [[], ["--serve", "4"], ["--thermalization", "8"], ["--table1", "8"],
                                  ["--percolation", "8"], ["--anneal", "8"]])
def test_more_than_one_gpu_is_refused(mode):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", *mode],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, r.stderr
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_algorithmic_counts_of_the_bench_workload():
    spec = inputs.WORKLOADS["3d_L8_gauss_1024inst"]
    N = inputs.n_sites(spec["topology"], spec["L"])
    S = spec["n_temps"] * spec["n_replicas"]
    # int8 spin read + write per attempt, the 1536 float couplings once
    b = bench.algorithmic_bytes_per_sweep(spec, N, 3 * N, 4)
    assert b == 2 * 80 * 512 + 1536 * 4 == 88064
    assert abs(b / (S * N) - 2.15) < 1e-3
    # a quarter Philox block (10), six extract + multiply-add (12), the
    # acceptance (5 float, 3 integer), the flip (1)
    assert bench.algorithmic_ops_per_attempt(6, "gauss") == 28
    assert bench.algorithmic_ops_per_attempt(6, "int3") == 26
    assert bench.algorithmic_ops_per_move(512) == 1024
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_launch_threads_follows_the_size_classes():
    # icm_run_config.threads applies to units of up to 512 sites; the classes
    # above take at least 512 (<= 1024 sites) and 1024 threads
    from paper_1501_05630_amd import icm
    assert icm.launch_threads(512, 256) == 256
    assert icm.launch_threads(513, 256) == 512
    assert icm.launch_threads(1024, 256) == 512
    assert icm.launch_threads(1024, 1024) == 1024
    assert icm.launch_threads(1152, 256) == 1024
    assert icm.launch_threads(4096, 512) == 1024
    assert icm.launch_threads(64, 512) == 512

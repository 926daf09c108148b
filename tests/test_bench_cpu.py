"""Host-side parts of bench.py that need no GPU: the one-GPU guard of every
mode, the algorithmic byte counts of its roofline, the step's launch shape and
the rule that measured counters apply only to the kernel they were taken on."""
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
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_default_step_is_several_graph_replayed_launches():
    # a step of the headline line covers four launches of the fused kernel,
    # so the captured graph is replayed inside the timed region, and the 20
    # driver steps cover more than the workload's 2^14 sweeps
    spl = bench.DEFAULT_LAUNCH["sweeps_per_launch"]
    assert bench.SWEEPS_PER_STEP % spl == 0 and bench.SWEEPS_PER_STEP // spl == 4
    assert bench.DEFAULT_LAUNCH["use_graph"] == 1
    assert 20 * bench.SWEEPS_PER_STEP >= inputs.WORKLOADS["3d_L8_gauss_1024inst"]["n_sweeps"]


def test_profiled_counters_apply_only_to_their_kernel_and_shape():
    cfg = dict(bench.DEFAULT_LAUNCH)
    tag = bench.launch_tag(cfg)
    assert tag == "t256_s16_spl256"
    saved = dict(bench.PROFILED)
    try:
        bench.PROFILED["w"] = {"kernel": bench.kernel_source_digest(), "launch": tag,
                               "hbm_bytes_per_launch": 1, "valu_insts_per_launch": 2}
        assert bench.profiled("w", cfg)["valu_insts_per_launch"] == 2
        assert bench.profiled("w", dict(cfg, icm_slots=8)) is None
        bench.PROFILED["w"]["kernel"] = "0" * 16
        assert bench.profiled("w", cfg) is None
        assert bench.profiled("other", cfg) is None
    finally:
        bench.PROFILED.clear()
        bench.PROFILED.update(saved)


def test_launch_threads_follows_the_configured_count_or_the_size_classes():
    # an explicit icm_run_config.threads applies to every size class; 0 / -1
    # pick per class: 256 up to 512 sites, 512 up to 1024, 1024 above
    from paper_1501_05630_amd import icm
    assert icm.launch_threads(512, 256) == 256
    assert icm.launch_threads(1152, 256) == 256
    assert icm.launch_threads(4096, 512) == 512
    assert icm.launch_threads(64, 1024) == 1024
    for auto in (0, -1):
        assert icm.launch_threads(512, auto) == 256
        assert icm.launch_threads(513, auto) == 512
        assert icm.launch_threads(1024, auto) == 512
        assert icm.launch_threads(1152, auto) == 1024
        assert icm.launch_threads(4096, auto) == 1024

"""GPU parity at the headline workload (1024 instances of the 3D L=8 Gaussian
lattice, 20 temperatures x 4 replicas, cluster moves at the 14 coldest):

- the benchmark's own launch (its default shape, its steps of four 256-sweep
  launches replayed from a captured graph, two steps) on couplings moved to
  the library's grid, sampled instances against the oracle element by element;
- the raw float32 couplings of the workload (which the library rounds to its
  2^-20 grid and the oracle does not) against the oracle in distribution:
  per-temperature mean energy per spin over sweeps [2048, 4096) of 64
  instances within 1e-3 absolute and within 3 standard errors of the paired
  difference;
- the launch shape the autotuner picks, against the oracle.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import bench
import gridded
import oracle as orc
from paper_1501_05630_amd import autotune, icm, inputs

pytestmark = pytest.mark.gpu
SEED = inputs.MASTER_SEED
NAME = "3d_L8_gauss_1024inst"
STAT_KEYS = ["metro_accepts", "icm_moves", "icm_nontrivial", "icm_cluster_sites", "icm_2a_flips",
             "pt_attempts", "pt_accepts"]
WORKERS = min(16, os.cpu_count() or 1)


def oracle_run(b, sweeps, grid=True, flags=orc.FLAG_2A | orc.FLAG_PT):
    J, temps, kc, spec = (gridded.workload_instance if grid else inputs.workload_instance)(NAME, b)
    o = orc.Sim(spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc, flags=flags, seed=SEED,
                instance_key=b)
    o.init_hot()
    o.run(sweeps)
    return o


def add_batch(ctx, n, grid=True, flags=icm.FLAG_2A | icm.FLAG_PT):
    hs = []
    for b in range(n):
        J, temps, kc, spec = (gridded.workload_instance if grid else inputs.workload_instance)(NAME, b)
        hs.append(ctx.icm_add_instance(spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc,
                                       flags=flags, instance_key=b))
        ctx.icm_init_states(hs[-1])
    return hs


def compare(ctx, h, o, what):
    st = ctx.icm_read_states(h)
    ref = o.states()
    assert np.array_equal(st, ref), f"{what}: {int(np.sum(st != ref))} spins differ"
    assert np.array_equal(ctx.icm_read_energies(h)[0], o.energies_raw()), f"{what}: energies"
    assert np.array_equal(ctx.icm_read_walkers(h), o.walkers()), f"{what}: PT labels"
    gs, os_ = ctx.icm_read_stats(h), o.stats()
    for k in STAT_KEYS:
        assert gs[k] == os_[k], f"{what}: {k}"


def test_benchmark_launch_sampled_bit_exact():
    ctx = icm.Context(arena_bytes=1 << 30, seed=SEED)
    try:
        hs = add_batch(ctx, 1024)
        ctx.icm_set_run_config(**bench.DEFAULT_LAUNCH)
        steps = 2
        for _ in range(steps):                       # the first captures, both replay
            ctx.icm_run(hs, bench.SWEEPS_PER_STEP)
        ctx.icm_sync()
        sweeps = steps * bench.SWEEPS_PER_STEP
        sample = [0, 341, 682, 1023]
        with cf.ThreadPoolExecutor(WORKERS) as ex:
            refs = list(ex.map(lambda b: oracle_run(b, sweeps), sample))
        for b, o in zip(sample, refs):
            compare(ctx, hs[b], o, f"instance {b}")
            assert ctx.icm_sweep_index(hs[b]) == sweeps
        # at any size: every reported energy is the energy of the reported state
        for b in range(0, 1024, 16):
            J, temps, kc, spec = gridded.workload_instance(NAME, b)
            o = orc.Sim(spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc, seed=SEED)
            st = ctx.icm_read_states(hs[b])
            raw, _ = ctx.icm_read_energies(hs[b])
            for k in range(st.shape[0]):
                for r in range(st.shape[1]):
                    assert raw[k, r] == o.energy_raw(st[k, r]), (b, k, r)
    finally:
        ctx.close()


def test_raw_gaussian_couplings_energy_per_temperature():
    n_inst, sweeps = 64, 4096
    window = 11                                      # time bin t in [2048, 4096)
    N, R = 512, 4
    ctx = icm.Context(arena_bytes=512 << 20, seed=SEED)
    try:
        hs = add_batch(ctx, n_inst, grid=False, flags=icm.FLAG_2A | icm.FLAG_PT | icm.FLAG_MEASURE)
        ctx.icm_set_run_config(**bench.DEFAULT_LAUNCH)
        ctx.icm_run(hs, sweeps)
        ctx.icm_sync()
        gpu = []
        for h in hs:
            sums, counts = ctx.icm_read_observables(h)
            assert counts[window] == 2048
            gpu.append(sums[window, :, :, 0].sum(axis=1) * 2.0 ** -20 / (counts[window] * R * N))
    finally:
        ctx.close()

    def orc_e(b):
        o = oracle_run(b, sweeps, grid=False, flags=orc.FLAG_2A | orc.FLAG_PT | orc.FLAG_MEASURE)
        sums, counts = o.observables()
        return sums[window, :, :, 0].sum(axis=1) * 2.0 ** -20 / (counts[window] * R * N)

    with cf.ThreadPoolExecutor(WORKERS) as ex:
        ref = list(ex.map(orc_e, range(n_inst)))
    d = np.array(gpu) - np.array(ref)                # [instance][temperature]
    mean = d.mean(axis=0)
    se = d.std(axis=0, ddof=1) / np.sqrt(n_inst)
    # the rounding changes the chain: most instances' trajectories part
    assert np.mean(np.any(d != 0, axis=1)) > 0.5
    assert np.all(np.abs(mean) <= 1e-3), mean
    assert np.all(np.abs(mean) <= 3 * se), (mean, se)


def test_autotuned_launch_shape_bit_exact():
    ctx = icm.Context(arena_bytes=512 << 20, seed=SEED)
    try:
        hs = add_batch(ctx, 128)
        best, info = autotune.tune(ctx, hs, cache_path=None)
        assert info["source"] == "search"
        for h in hs:
            ctx.icm_init_states(h)
        ctx.icm_set_run_config(**best)
        ctx.icm_run(hs, 2 * best["sweeps_per_launch"])
        ctx.icm_sync()
        sample = [0, 77, 127]
        with cf.ThreadPoolExecutor(WORKERS) as ex:
            refs = list(ex.map(lambda b: oracle_run(b, 2 * best["sweeps_per_launch"]), sample))
        for b, o in zip(sample, refs):
            compare(ctx, hs[b], o, f"tuned {best} instance {b}")
    finally:
        ctx.close()

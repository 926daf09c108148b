"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Integer couplings: whole trajectories bit-exact (spins, temperature labels,
energies, statistics, ICM labels).  Float couplings: the library simulates the
couplings rounded to a 2^-e grid (e = 20 for Gaussian draws), the oracle the
float32 values as given; the bit-exact tests therefore feed couplings already
on that grid (tests/gridded.py), where the two chains are the same chain, and
the raw float32 draws of the headline workload are compared statistically
(per-temperature mean energy per spin within 1e-3 absolute and 3 standard
errors over 64 instances).
"""
import numpy as np
import pytest

import gridded
import oracle as orc
from paper_1501_05630_amd import icm, inputs

pytestmark = pytest.mark.gpu
SEED = inputs.MASTER_SEED
ORACLE_FLAGS = icm.FLAG_2A | icm.FLAG_PT | icm.FLAG_SKIP_METRO


@pytest.fixture(scope="module")
def ctx():
    c = icm.Context(arena_bytes=1 << 30, seed=SEED)
    yield c
    c.close()


def make_pair(ctx, top, L, J, temps, R, Kc, flags, key=0, j_scale=1):
    h = ctx.icm_add_instance(top, L, J, temps, R, Kc, flags=flags, instance_key=key, j_scale=j_scale)
    o = orc.Sim(top, L, J, temps, R, Kc, flags=flags & ORACLE_FLAGS, seed=SEED, instance_key=key,
                j_scale=j_scale)
    return h, o


STAT_KEYS = ["metro_accepts", "icm_moves", "icm_nontrivial", "icm_cluster_sites", "icm_2a_flips",
             "pt_attempts", "pt_accepts"]


def assert_same(ctx, h, o, what=""):
    st = ctx.icm_read_states(h)
    ref = o.states()
    if not np.array_equal(st, ref):
        bad = np.argwhere(st != ref)
        raise AssertionError(f"{what}: {len(bad)} spins differ, first at {bad[:3].tolist()}")
    raw, _ = ctx.icm_read_energies(h)
    assert np.array_equal(raw, o.energies_raw()), f"{what}: energies differ"
    assert np.array_equal(ctx.icm_read_walkers(h), o.walkers()), f"{what}: PT labels differ"
    gs, os_ = ctx.icm_read_stats(h), o.stats()
    for k in STAT_KEYS:
        assert gs[k] == os_[k], f"{what}: stat {k} {gs[k]} != {os_[k]}"
    assert ctx.icm_sweep_index(h) == o.sweep()


def run_both(ctx, h, o, chunks, what):
    for n in chunks:
        ctx.icm_run([h], n)
        o.run(n)
        ctx.icm_sync()
        assert_same(ctx, h, o, f"{what} after +{n}")


# ------------------------------------------------------------------ trajectories
def test_2d_pmJ_L8_trajectory_bit_exact(ctx):
    J, temps, kc, spec = gridded.workload_instance("2d_L8_pmJ_1inst", 0)
    h, o = make_pair(ctx, spec["topology"], 8, J, temps, 2, kc, icm.FLAG_2A | icm.FLAG_PT)
    ctx.icm_init_states(h)
    o.init_hot()
    assert_same(ctx, h, o, "hot start")
    run_both(ctx, h, o, [1, 3, 60, 200], "2d pmJ")
    ctx.icm_remove_instance(h)


def test_metropolis_only_bit_exact(ctx):
    rng = inputs.make_rng(70, 0)
    for top, L, kind, sc in [(inputs.SQUARE2D, 8, "pmJ", 1), (inputs.CUBIC3D, 4, "gauss", 1),
                             (inputs.CHIMERA, 2, "int3", 3)]:
        J = gridded.make_couplings(kind, top, L, rng)
        h, o = make_pair(ctx, top, L, J, inputs.geometric_temps(0.3, 2.0, 6), 2, 0, 0, j_scale=sc)
        ctx.icm_init_states(h)
        o.init_hot()
        run_both(ctx, h, o, [1, 20], f"metropolis {kind}")
        ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,kind,sc", [(inputs.SQUARE2D, 8, "pmJ", 1), (inputs.CUBIC3D, 6, "gauss", 1),
                                           (inputs.CHIMERA, 4, "int3", 3), (inputs.SQUARE2D, 2, "pmJ", 1),
                                           (inputs.CUBIC3D, 2, "gauss", 1), (inputs.CHIMERA, 1, "int3", 3)])
@pytest.mark.parametrize("two_a", [True, False])
def test_icm_only_labels_and_flips_bit_exact(ctx, top, L, kind, sc, two_a):
    rng = inputs.make_rng(71, L * 10 + top)
    J = gridded.make_couplings(kind, top, L, rng)
    temps = inputs.geometric_temps(0.3, 1.5, 4)
    flags = icm.FLAG_SKIP_METRO | icm.FLAG_RECORD_LABELS | (icm.FLAG_2A if two_a else 0)
    h, o = make_pair(ctx, top, L, J, temps, 4, 4, flags, key=5, j_scale=sc)
    N = o.N
    for trial, frac in enumerate([0.05, 0.3, 0.45, 0.55, 0.8, 0.0, 1.0]):
        st = np.where(rng.random((4, 4, N)) < 0.5, 1, -1).astype(np.int8)
        for k in range(4):
            for r in (1, 3):
                st[k, r] = np.where(rng.random(N) < frac, -st[k, r - 1], st[k, r - 1])
        ctx.icm_set_states(h, st, sweep0=trial * 7)
        o.set_states(st, sweep0=trial * 7)
        ctx.icm_run([h], 1)
        o.run(1)
        ctx.icm_sync()
        for k in range(4):
            for p in range(2):
                lab, seed, nm = ctx.icm_read_labels(h, k, p)
                rl, rs, rn = o.labels(k, p)
                assert nm == rn and seed == rs, (trial, k, p, nm, rn, seed, rs)
                assert np.array_equal(lab, rl), (trial, k, p)
        assert np.array_equal(ctx.icm_read_states(h), o.states()), trial
        assert np.array_equal(ctx.icm_read_energies(h)[0], o.energies_raw()), trial
    ctx.icm_remove_instance(h)


def test_3d_gauss_L8_trajectory_bit_exact(ctx):
    J, temps, kc, spec = gridded.workload_instance("3d_L8_gauss_1024inst", 3)
    h, o = make_pair(ctx, spec["topology"], 8, J, temps, 4, kc, icm.FLAG_2A | icm.FLAG_PT, key=3)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 40, 100], "3d gauss")
    ctx.icm_remove_instance(h)


def test_chimera_C12_trajectory_bit_exact(ctx):
    J, temps, kc, spec = gridded.workload_instance("chimera_C12_int3_512inst", 7)
    h, o = make_pair(ctx, spec["topology"], 12, J, temps, 2, kc, icm.FLAG_2A | icm.FLAG_PT,
                     key=7, j_scale=3)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 30], "chimera C12")
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("case", [
    dict(top=inputs.CUBIC3D, L=2, kind="gauss", K=3, R=2, Kc=3),      # N=8 multigraph, W%4=2
    dict(top=inputs.CHIMERA, L=1, kind="int3", K=5, R=2, Kc=5),       # single cell, open edges
    dict(top=inputs.SQUARE2D, L=4, kind="pmJ", K=1, R=2, Kc=1),       # one temperature, no PT pair
    dict(top=inputs.SQUARE2D, L=6, kind="pmJ", K=7, R=6, Kc=7),       # R=6, ragged quads
    dict(top=inputs.CUBIC3D, L=4, kind="pmJ", K=9, R=2, Kc=0),        # ICM off
    dict(top=inputs.SQUARE2D, L=64, kind="pmJ", K=4, R=2, Kc=4),      # N=4096 (largest resident)
    dict(top=inputs.CHIMERA, L=5, kind="gauss", K=5, R=4, Kc=2),      # float chimera
])
def test_edge_cases_bit_exact(ctx, case):
    rng = inputs.make_rng(72, case["L"] * 100 + case["K"])
    J = gridded.make_couplings(case["kind"], case["top"], case["L"], rng)
    sc = 3 if case["kind"] == "int3" else 1
    temps = inputs.geometric_temps(0.25, 1.8, case["K"]) if case["K"] > 1 else np.array([0.6])
    h, o = make_pair(ctx, case["top"], case["L"], J, temps, case["R"], case["Kc"],
                     icm.FLAG_2A | icm.FLAG_PT, key=11, j_scale=sc)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 25], str(case))
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("K,R,kind", [(21, 2, "pmJ"), (22, 2, "pmJ"), (22, 4, "gauss"), (33, 2, "gauss"),
                                      (33, 16, "pmJ"), (34, 2, "gauss")])
def test_pt_ladder_lengths_bit_exact(ctx, K, R, kind):
    # ladders just below, at and above the range whose swaps are decided up
    # front (22 to 33 temperatures), with up to 16 chains; PT at every sweep
    rng = inputs.make_rng(73, K * 100 + R)
    J = gridded.make_couplings(kind, inputs.SQUARE2D, 8, rng)
    temps = inputs.geometric_temps(0.3, 2.5, K)
    h, o = make_pair(ctx, inputs.SQUARE2D, 8, J, temps, R, 3, icm.FLAG_2A | icm.FLAG_PT, key=13)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 30], f"K={K} R={R} {kind}")
    assert ctx.icm_read_stats(h)["pt_accepts"] > 0
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,kind,K,R", [
    (inputs.CHIMERA, 16, "int3", 6, 2),     # 64 words: one word per lane, full wave
    (inputs.CHIMERA, 17, "gauss", 4, 2),    # 73 words: LDS shift program, chimera terms
    (inputs.CHIMERA, 7, "int3", 6, 4),      # 13 words, rows not word-aligned (C % 4 = 3)
    (inputs.CUBIC3D, 12, "gauss", 5, 4),    # 54 words, x-rows straddle words
    (inputs.CUBIC3D, 10, "pmJ", 6, 2),      # 32 words: two moves per wave
    (inputs.SQUARE2D, 32, "pmJ", 6, 2),     # 32 words
    (inputs.SQUARE2D, 40, "gauss", 5, 2),   # 50 words
    (inputs.SQUARE2D, 48, "pmJ", 5, 2),     # 72 words: LDS shift program, lattice terms
])
def test_each_cluster_search_layout_bit_exact(ctx, top, L, kind, K, R):
    # every layout the cluster search uses (register words, two words per lane,
    # LDS shift program) against the oracle, with cold temperatures so that
    # clusters are large
    rng = inputs.make_rng(76, L * 10 + top)
    J = gridded.make_couplings(kind, top, L, rng)
    sc = 3 if kind == "int3" else 1
    temps = inputs.geometric_temps(0.2, 1.0, K)
    h, o = make_pair(ctx, top, L, J, temps, R, K, icm.FLAG_2A | icm.FLAG_PT, key=13, j_scale=sc)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 12], f"layout top={top} L={L}")
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,jlo,jhi,scale", [
    (inputs.CHIMERA, 6, -128, 127, 64),   # full int8 range: eight bit planes
    (inputs.CUBIC3D, 8, -16, 15, 8),      # five planes, the 8^3 register layout
    (inputs.SQUARE2D, 12, -100, 37, 32),  # asymmetric range: eight planes
])
def test_wide_integer_couplings_bit_exact(ctx, top, L, jlo, jhi, scale):
    # integer couplings beyond +-3: the cluster moves' boundary sums take the
    # couplings as two's-complement bit planes (as many as their width), so
    # wide and asymmetric ranges, with both extremes present, must agree too
    rng = inputs.make_rng(79, L * 10 + top)
    J = gridded.make_couplings("int3", top, L, rng)
    nz = J != 0
    J = np.where(nz, rng.integers(jlo, jhi + 1, size=J.shape), 0).astype(np.int8)
    flat = np.flatnonzero(nz)
    J.flat[flat[0]], J.flat[flat[1]] = jlo, jhi
    temps = inputs.geometric_temps(0.3, 2.0, 6)
    h, o = make_pair(ctx, top, L, J, temps, 4, 4, icm.FLAG_2A | icm.FLAG_PT, key=17, j_scale=scale)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 10], f"wide J top={top} L={L} [{jlo}, {jhi}]")
    ctx.icm_remove_instance(h)


def test_batched_per_instance_and_graph_agree(ctx):
    rng = inputs.make_rng(73, 0)
    specs = [(inputs.SQUARE2D, 8, "pmJ", 1, 16, 2), (inputs.CUBIC3D, 4, "gauss", 1, 10, 4),
             (inputs.CHIMERA, 3, "int3", 3, 12, 2), (inputs.CUBIC3D, 6, "gauss", 1, 8, 4)]
    made = []
    for x, (top, L, kind, sc, K, R) in enumerate(specs * 2):
        J = gridded.make_couplings(kind, top, L, rng)
        temps = inputs.geometric_temps(0.2, 2.0, K)
        made.append((top, L, J, temps, R, inputs.icm_cutoff(temps), sc, x))

    def run(mode):
        hs = []
        for (top, L, J, temps, R, kc, sc, x) in made:
            h = ctx.icm_add_instance(top, L, J, temps, R, kc, instance_key=x, j_scale=sc)
            ctx.icm_init_states(h)
            hs.append(h)
        if mode == "batched":
            ctx.icm_set_run_config(sweeps_per_launch=16, use_graph=0)
            ctx.icm_run(hs, 80)
        elif mode == "graph":
            ctx.icm_set_run_config(sweeps_per_launch=16, use_graph=1)
            ctx.icm_run(hs, 48)
            ctx.icm_run(hs, 32)
        else:
            ctx.icm_set_run_config(sweeps_per_launch=16, use_graph=0)
            ctx.icm_run_per_instance(hs, 80)
        ctx.icm_sync()
        out = [(ctx.icm_read_states(h), ctx.icm_read_energies(h)[0]) for h in hs]
        for h in hs:
            ctx.icm_remove_instance(h)
        return out

    a, b, c = run("batched"), run("per_instance"), run("graph")
    ctx.icm_set_run_config(sweeps_per_launch=256, use_graph=0)
    for x in range(len(made)):
        for y in (b, c):
            assert np.array_equal(a[x][0], y[x][0]) and np.array_equal(a[x][1], y[x][1]), x


@pytest.mark.parametrize("threads,slots,tables", [(256, 1, 1), (512, 3, 2), (1024, 8, 1),
                                                  (1024, 16, 2), (512, 8, 2), (512, 32, 1), (256, 16, 2), (512, 20, 1)])
@pytest.mark.parametrize("name", ["3d_L8_gauss_1024inst", "chimera_C12_int3_512inst"])
def test_launch_shape_does_not_change_results(ctx, threads, slots, tables, name):
    J, temps, kc, spec = gridded.workload_instance(name, 1)
    h, o = make_pair(ctx, spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc,
                     icm.FLAG_2A | icm.FLAG_PT, key=1, j_scale=spec["j_scale"])
    ctx.icm_set_run_config(threads=threads, icm_slots=slots, sweeps_per_launch=7,
                           table_placement=tables)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [20], f"threads={threads} slots={slots} tables={tables}")
    ctx.icm_set_run_config(threads=512, icm_slots=8, sweeps_per_launch=256, table_placement=0)
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("threads,slots", [(64, 4), (128, 8), (128, 3)])
@pytest.mark.parametrize("name,L", [("table1_3d_gauss", 4), ("table1_chimera_gauss", 4), ("table1_2d_gauss", 16),
                                    ("3d_L8_gauss_1024inst", 8)])
def test_small_workgroups_bit_exact(ctx, threads, slots, name, L):
    # one or two waves per instance (several instances share a CU): the whole
    # sweep -- Metropolis tasks, every cluster move of the unit and the PT scan
    # -- runs on those waves
    J, temps, kc, spec = gridded.workload_instance(name, 5, L=L)
    h, o = make_pair(ctx, spec["topology"], L, J, temps, spec["n_replicas"], kc,
                     icm.FLAG_2A | icm.FLAG_PT, key=5, j_scale=spec["j_scale"])
    ctx.icm_set_run_config(threads=threads, icm_slots=slots, sweeps_per_launch=9, table_placement=0)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 20], f"{name} L={L} threads={threads} slots={slots}")
    ctx.icm_set_run_config(threads=512, icm_slots=8, sweeps_per_launch=256, table_placement=0)
    ctx.icm_remove_instance(h)


def test_per_class_thread_counts_bit_exact(ctx):
    # one batch of units from three size classes (3D L = 4, 6; 10; 12), each
    # class launched with its own thread count
    name = "3d_uneven_gauss_1536inst"
    pairs = []
    for b in (0, 300, 800, 1100):
        J, temps, kc, spec = gridded.workload_instance(name, b)
        h, o = make_pair(ctx, spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc,
                         icm.FLAG_2A | icm.FLAG_PT, key=b)
        ctx.icm_init_states(h)
        o.init_hot()
        pairs.append((h, o, spec["L"]))
    ctx.icm_set_run_config(threads=256, icm_slots=8, sweeps_per_launch=7, class_threads=(64, 1024, 512, -1))
    assert ctx.icm_get_run_config()["class_threads"] == [64, 1024, 512, 0]
    for n in (3, 12):
        ctx.icm_run([h for h, _, _ in pairs], n)
        ctx.icm_sync()
        for h, o, L in pairs:
            o.run(n)
            assert_same(ctx, h, o, f"L={L} after +{n}")
    ctx.icm_set_run_config(threads=512, icm_slots=8, sweeps_per_launch=256, class_threads=(-1, -1, -1, -1))
    assert ctx.icm_get_run_config()["class_threads"] == [0, 0, 0, 0]
    for h, _, _ in pairs:
        ctx.icm_remove_instance(h)


def test_large_3d_L16_runs_with_tables_in_global_memory(ctx):
    # 4096 sites x 96 walkers: the spins fit LDS bit-packed, the tables do not.
    J = gridded.gaussian_couplings(inputs.CUBIC3D, 16, inputs.make_rng(75, 0))
    temps = inputs.geometric_temps(0.2, 2.0, 24)
    h, o = make_pair(ctx, inputs.CUBIC3D, 16, J, temps, 4, inputs.icm_cutoff(temps),
                     icm.FLAG_2A | icm.FLAG_PT, key=2)
    ctx.icm_init_states(h)
    o.init_hot()
    run_both(ctx, h, o, [1, 4], "3d L16")
    ctx.icm_remove_instance(h)


# ---------------------------------------------------------- full-size workloads
def _full_size(ctx, name, n_inst, sweeps, sample, threads=512):
    hs = []
    for b in range(n_inst):
        J, temps, kc, spec = gridded.workload_instance(name, b)
        hs.append(ctx.icm_add_instance(spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc,
                                       instance_key=b, j_scale=spec["j_scale"]))
        ctx.icm_init_states(hs[-1])
    ctx.icm_set_run_config(threads=threads, sweeps_per_launch=sweeps)
    ctx.icm_run(hs, sweeps)
    ctx.icm_sync()
    for b in sample:
        J, temps, kc, spec = gridded.workload_instance(name, b)
        o = orc.Sim(spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc,
                    flags=orc.FLAG_2A | orc.FLAG_PT, seed=SEED, instance_key=b, j_scale=spec["j_scale"])
        o.init_hot()
        o.run(sweeps)
        assert_same(ctx, hs[b], o, f"{name} instance {b}")
    # property at any size: every reported energy equals the energy of the state
    for b in range(0, n_inst, max(1, n_inst // 64)):
        J, temps, kc, spec = gridded.workload_instance(name, b)
        o = orc.Sim(spec["topology"], spec["L"], J, temps, spec["n_replicas"], kc,
                    seed=SEED, j_scale=spec["j_scale"])
        st = ctx.icm_read_states(hs[b])
        raw, _ = ctx.icm_read_energies(hs[b])
        for k in range(st.shape[0]):
            for r in range(st.shape[1]):
                assert raw[k, r] == o.energy_raw(st[k, r]), (b, k, r)
    for h in hs:
        ctx.icm_remove_instance(h)
    ctx.icm_set_run_config(sweeps_per_launch=256)


def test_full_size_3d_gauss_1024_instances_sampled(ctx):
    _full_size(ctx, "3d_L8_gauss_1024inst", 1024, 12, [0, 341, 1023])


def test_full_size_chimera_512_instances_sampled(ctx):
    _full_size(ctx, "chimera_C12_int3_512inst", 512, 6, [0, 511])


def test_full_size_uneven_3d_batch_sampled():
    # 256 instances each of L = 4, 6, 8, 10, 12, 16 in one run (one launch per
    # size class); one instance of every side checked against the oracle.
    c = icm.Context(arena_bytes=3 << 30, seed=SEED)
    try:
        _full_size(c, "3d_uneven_gauss_1536inst", 1536, 4,
                   [0, 256 + 5, 512 + 77, 768 + 130, 1024 + 201, 1280 + 255], threads=256)
    finally:
        c.close()


@pytest.mark.parametrize("top,L,kind,K,R", [
    (inputs.SQUARE2D, 8, "pmJ", 6, 2),
    (inputs.CUBIC3D, 8, "gauss", 5, 4),
    (inputs.CHIMERA, 12, "int3", 6, 2),
    (inputs.CUBIC3D, 6, "gauss", 4, 6),
    (inputs.SQUARE2D, 64, "pmJ", 3, 2),
])
def test_observables_bit_exact(ctx, top, L, kind, K, R):
    # energies, link overlap and spin overlap per logarithmic time bin, summed
    # on the device after every step, equal the oracle's sums
    rng = inputs.make_rng(77, L * 10 + top)
    J = gridded.make_couplings(kind, top, L, rng)
    sc = 3 if kind == "int3" else 1
    temps = inputs.geometric_temps(0.3, 1.8, K)
    flags = icm.FLAG_2A | icm.FLAG_PT | icm.FLAG_MEASURE
    h = ctx.icm_add_instance(top, L, J, temps, R, inputs.icm_cutoff(temps), flags=flags, instance_key=21,
                             j_scale=sc)
    o = orc.Sim(top, L, J, temps, R, inputs.icm_cutoff(temps), flags=orc.FLAG_2A | orc.FLAG_PT | orc.FLAG_MEASURE,
                seed=SEED, instance_key=21, j_scale=sc)
    ctx.icm_init_states(h)
    o.init_hot()
    for n in (1, 6, 40, 90):
        ctx.icm_run([h], n)
        o.run(n)
        ctx.icm_sync()
        gs, gc = ctx.icm_read_observables(h)
        os_, oc = o.observables()
        assert np.array_equal(gc, oc), (n, gc[:8], oc[:8])
        assert np.array_equal(gs, os_), (n, np.argwhere(gs != os_)[:4].tolist())
    assert_same(ctx, h, o, "with observables")
    ctx.icm_remove_instance(h)


def test_observables_reset_by_set_states_and_absent_without_flag(ctx):
    J = inputs.pm_j_couplings(inputs.SQUARE2D, 8, inputs.make_rng(78, 0))
    temps = inputs.geometric_temps(0.4, 1.4, 3)
    h = ctx.icm_add_instance(inputs.SQUARE2D, 8, J, temps, 2, 2, flags=icm.FLAG_MEASURE | icm.FLAG_PT)
    ctx.icm_init_states(h)
    ctx.icm_run([h], 20)
    st = ctx.icm_read_states(h)
    ctx.icm_set_states(h, st, sweep0=100)
    ctx.icm_run([h], 3)
    ctx.icm_sync()
    _, counts = ctx.icm_read_observables(h)
    assert counts.sum() == 3 and counts[6] == 3           # t = 101..103 -> bin 6
    ctx.icm_remove_instance(h)
    h2 = ctx.icm_add_instance(inputs.SQUARE2D, 8, J, temps, 2, 2, flags=icm.FLAG_PT)
    with pytest.raises(icm.IcmError):
        ctx.icm_read_observables(h2)
    ctx.icm_remove_instance(h2)


@pytest.mark.parametrize("metro", [False, True])
def test_step_2a_is_strict_at_exactly_half(ctx, metro):
    # ferromagnet, replica a all up, replica b down on two of four rows: the
    # replicas differ on exactly N/2 sites, which is not more than half, so
    # step 2a must not reverse b; at T = 0.05 no Metropolis flip of this state
    # is accepted, so the full step reaches the tie too
    L, N = 4, 16
    J = np.ones((N, 2), dtype=np.int8)
    flags = icm.FLAG_2A | icm.FLAG_RECORD_LABELS | (0 if metro else icm.FLAG_SKIP_METRO)
    a = np.ones(N, dtype=np.int8)
    b = a.copy()
    b[:2 * L] = -1
    for extra in (False, True):
        # a fresh pair per case: the statistics compared below count from it
        h, o = make_pair(ctx, inputs.SQUARE2D, L, J, [0.05], 2, 1, flags, key=23)
        bb = b.copy()
        if extra and not metro:
            bb[N - 1] = -1             # one site more: now 2 n_minus > N
        st = np.stack([a, bb])[None]
        ctx.icm_set_states(h, st, sweep0=3)
        o.set_states(st, sweep0=3)
        ctx.icm_run([h], 1)
        o.run(1)
        ctx.icm_sync()
        lab, seed, nm = ctx.icm_read_labels(h, 0, 0)
        rl, rs, rn = o.labels(0, 0)
        assert (nm, seed) == (rn, rs) and np.array_equal(lab, rl)
        assert_same(ctx, h, o, f"2a tie extra={extra}")
        if extra and not metro:
            assert nm == N // 2 - 1 and ctx.icm_read_stats(h)["icm_2a_flips"] == 1
        else:
            assert nm == N // 2 and ctx.icm_read_stats(h)["icm_2a_flips"] == 0
            out = ctx.icm_read_states(h)[0]
            assert np.array_equal(out[0], b) and np.array_equal(out[1], a)
        ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,kind,K,R", [
    (inputs.SQUARE2D, 8, "pmJ", 6, 2),
    (inputs.CUBIC3D, 6, "gauss", 5, 4),
    (inputs.CHIMERA, 4, "int3", 6, 2),
    (inputs.CUBIC3D, 2, "gauss", 3, 2),      # multigraph: both bonds of a pair counted
    (inputs.CHIMERA, 12, "int3", 4, 2),
])
def test_overlaps_readout(ctx, top, L, kind, K, R):
    # spin overlap sum_i q_i and link-overlap numerator sum over bonds of q_i q_j
    # (Eq. 1) per temperature and pair, formed on the device, against the
    # oracle's states of the same trajectory (with step 2a on, so that some
    # stored replicas are reversed)
    rng = inputs.make_rng(120, L * 10 + top)
    J = gridded.make_couplings(kind, top, L, rng)
    sc = 3 if kind == "int3" else 1
    temps = inputs.geometric_temps(0.2, 1.6, K)
    h, o = make_pair(ctx, top, L, J, temps, R, K, icm.FLAG_2A | icm.FLAG_PT, key=29, j_scale=sc)
    ctx.icm_init_states(h)
    o.init_hot()
    ij, _ = o.bonds()
    for n in (0, 7, 40):
        ctx.icm_run([h], n)
        o.run(n)
        ctx.icm_sync()
        q, ql = ctx.icm_read_overlaps(h)
        st = o.states().astype(np.int64)
        assert np.array_equal(ctx.icm_read_states(h), o.states())
        for k in range(K):
            for p in range(R // 2):
                qi = st[k, 2 * p] * st[k, 2 * p + 1]
                assert q[k, p] == qi.sum(), (n, k, p)
                assert ql[k, p] == int(np.sum(qi[ij[:, 0]] * qi[ij[:, 1]])), (n, k, p)
    assert ctx.icm_read_stats(h)["icm_2a_flips"] > 0
    ctx.icm_remove_instance(h)

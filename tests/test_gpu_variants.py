"""GPU parity of the method's variants (through the C-ABI) against the CPU
oracle, bit-exact: simulated annealing with cluster moves at every
temperature step (icm_set_temperatures between runs), a PT ladder replaced
mid-run, zero-temperature dynamics with cluster moves (energies never rise),
and HCA mode (no step 2a, cluster moves at every temperature)."""
import numpy as np
import pytest

import gridded
import oracle as orc
from paper_1501_05630_amd import icm, inputs

pytestmark = pytest.mark.gpu
SEED = inputs.MASTER_SEED


@pytest.fixture(scope="module")
def ctx():
    c = icm.Context(arena_bytes=256 << 20, seed=SEED)
    yield c
    c.close()


def pair(ctx, top, L, J, temps, R, Kc, flags, key, scale):
    h = ctx.icm_add_instance(top, L, J, temps, R, Kc, flags=flags, instance_key=key, j_scale=scale)
    o = orc.Sim(top, L, J, temps, R, Kc, flags=flags & (icm.FLAG_2A | icm.FLAG_PT), seed=SEED, instance_key=key,
                j_scale=scale)
    return h, o


def same(ctx, h, o, what):
    assert np.array_equal(ctx.icm_read_states(h), o.states()), what
    assert np.array_equal(ctx.icm_read_energies(h)[0], o.energies_raw()), what
    assert np.array_equal(ctx.icm_read_walkers(h), o.walkers()), what
    gs, os_ = ctx.icm_read_stats(h), o.stats()
    for k in ("metro_accepts", "icm_moves", "icm_nontrivial", "icm_cluster_sites", "icm_2a_flips", "pt_accepts"):
        assert gs[k] == os_[k], (what, k, gs[k], os_[k])


CASES = [(inputs.SQUARE2D, 16, "pmJ", 1), (inputs.CUBIC3D, 6, "gauss", 1), (inputs.CHIMERA, 4, "int3", 3),
         (inputs.CHIMERA, 7, "gauss", 1)]


@pytest.mark.parametrize("top,L,kind,scale", CASES)
def test_annealing_with_cluster_moves_bit_exact(ctx, top, L, kind, scale):
    J = gridded.make_couplings(kind, top, L, inputs.make_rng(110, L))
    h, o = pair(ctx, top, L, J, [3.0], 8, 1, icm.FLAG_2A, 21, scale)
    ctx.icm_init_states(h)
    o.init_hot()
    for step, T in enumerate(np.geomspace(3.0, 0.1, 12)):
        ctx.icm_set_temperatures(h, [T])
        o.set_temperatures([T])
        ctx.icm_run([h], 5)
        o.run(5)
        ctx.icm_sync()
        same(ctx, h, o, f"step {step} T={T}")
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,kind,scale", CASES[:3])
def test_pt_ladder_replaced_mid_run_bit_exact(ctx, top, L, kind, scale):
    J = gridded.make_couplings(kind, top, L, inputs.make_rng(111, L))
    temps = inputs.geometric_temps(0.5, 2.0, 5)
    h, o = pair(ctx, top, L, J, temps, 2, 3, icm.FLAG_2A | icm.FLAG_PT, 22, scale)
    ctx.icm_init_states(h)
    o.init_hot()
    ctx.icm_run([h], 10)
    o.run(10)
    new = temps * 0.8              # same spacing ratios: the PT table still fits
    ctx.icm_set_temperatures(h, new)
    o.set_temperatures(new)
    ctx.icm_run([h], 17)
    o.run(17)
    ctx.icm_sync()
    same(ctx, h, o, "after the new ladder")
    if kind != "gauss":
        # a much closer pair needs a longer integer PT table than was built
        close = np.array(new)
        close[1] = close[0] * (1 + 1e-6)
        with pytest.raises(icm.IcmError):
            ctx.icm_set_temperatures(h, close)
    with pytest.raises(icm.IcmError):
        ctx.icm_set_temperatures(h, new[::-1].copy())
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,kind,scale", [(inputs.SQUARE2D, 16, "pmJ", 1), (inputs.CHIMERA, 4, "int3", 3)])
def test_zero_temperature_cluster_hopping_bit_exact(ctx, top, L, kind, scale):
    # anneal, then at a temperature where no uphill flip is accepted the energy
    # of each replica pair never rises (a cluster move keeps E_a + E_b and moves
    # energy between the two) while the cluster moves keep changing the states
    J = gridded.make_couplings(kind, top, L, inputs.make_rng(112, L))
    R = 8
    h, o = pair(ctx, top, L, J, [2.0], R, 1, icm.FLAG_2A, 23, scale)
    ctx.icm_init_states(h)
    o.init_hot()
    for T in np.geomspace(2.0, 0.2, 10):
        ctx.icm_set_temperatures(h, [T])
        o.set_temperatures([T])
        ctx.icm_run([h], 10)
        o.run(10)
    ctx.icm_set_temperatures(h, [1e-3])
    o.set_temperatures([1e-3])
    ctx.icm_sync()
    prev = ctx.icm_read_energies(h)[0].reshape(-1, 2).sum(axis=1)
    moved = 0
    for _ in range(20):
        before = ctx.icm_read_states(h)
        ctx.icm_run([h], 1)
        o.run(1)
        ctx.icm_sync()
        e = ctx.icm_read_energies(h)[0].reshape(-1, 2).sum(axis=1)
        assert np.all(e <= prev), (prev, e)
        prev = e
        moved += int(np.sum(np.any(ctx.icm_read_states(h) != before, axis=2)))
        same(ctx, h, o, "zero temperature")
    assert moved > 0
    assert ctx.icm_read_stats(h)["icm_nontrivial"] > 0
    ctx.icm_remove_instance(h)


@pytest.mark.parametrize("top,L,kind,scale", [(inputs.SQUARE2D, 8, "pmJ", 1), (inputs.CUBIC3D, 4, "gauss", 1),
                                              (inputs.CHIMERA, 3, "int3", 3)])
def test_hca_mode_trajectory_bit_exact(ctx, top, L, kind, scale):
    J = gridded.make_couplings(kind, top, L, inputs.make_rng(113, L))
    temps = inputs.geometric_temps(0.4, 2.5, 6)
    h, o = pair(ctx, top, L, J, temps, 4, len(temps), icm.FLAG_PT, 24, scale)
    ctx.icm_init_states(h)
    o.init_hot()
    for n in (1, 30, 64):
        ctx.icm_run([h], n)
        o.run(n)
        ctx.icm_sync()
        same(ctx, h, o, f"+{n}")
    assert ctx.icm_read_stats(h)["icm_2a_flips"] == 0
    ctx.icm_remove_instance(h)

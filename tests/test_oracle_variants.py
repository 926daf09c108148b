"""Pins of the method's variants that reuse the same step (the introduction's
simulated annealing with cluster moves at every temperature step, the
zero-temperature ground-state hopping of the discussion of Fig. 1, and the
Houdayer algorithm without step 2a).

- changing the temperatures of a running simulation continues exactly as a
  simulation created at the new temperatures from the same states and sweep
  count (one temperature slot, so walker and slot indices coincide);
- at a temperature where no uphill flip can be accepted, replicas started in
  exact ground states (enumeration) stay at the ground-state energy at every
  step and visit several distinct ground states, the cluster moves among
  them;
- HCA mode (no 2a, cluster moves at every temperature) still samples the
  exact thermal energy.
"""
import numpy as np
import pytest

import oracle as orc
from paper_1501_05630_amd import inputs

import exact


@pytest.mark.parametrize("kind,top,L,scale", [("pmJ", inputs.SQUARE2D, 6, 1), ("gauss", inputs.CUBIC3D, 4, 1),
                                              ("int3", inputs.CHIMERA, 2, 3)])
def test_set_temperatures_equals_fresh_start(kind, top, L, scale):
    J = inputs.make_couplings(kind, top, L, inputs.make_rng(97, L))
    R = 8
    a = orc.Sim(top, L, J, [2.0], R, 1, flags=orc.FLAG_2A, seed=9, instance_key=4, j_scale=scale)
    a.init_hot()
    a.run(30)
    st, t = a.states(), a.sweep()
    a.set_temperatures([0.45])
    a.run(40)
    b = orc.Sim(top, L, J, [0.45], R, 1, flags=orc.FLAG_2A, seed=9, instance_key=4, j_scale=scale)
    b.set_states(st, sweep0=t)
    b.run(40)
    assert np.array_equal(a.states(), b.states())
    assert np.array_equal(a.energies_raw(), b.energies_raw())
    sa, sb = a.stats(), b.stats()
    # the second run's statistics: a's include its first 30 sweeps
    assert sa["icm_moves"] == sb["icm_moves"] + 30 * (R // 2)
    with pytest.raises(ValueError):
        a.set_temperatures([0.0])


def ground_states_2d(L, J):
    N = L * L
    bonds = exact.bond_list(inputs.SQUARE2D, L, J)
    E = exact.all_energies(N, bonds)
    S = exact.all_states(N)
    gs = S[np.abs(E - E.min()) < 1e-9]
    return gs, float(E.min()), bonds


def test_zero_temperature_hopping_stays_in_the_ground_state_manifold():
    L = 4
    for b in range(50):                          # the first instance with a degenerate manifold
        J = inputs.pm_j_couplings(inputs.SQUARE2D, L, inputs.make_rng(98, b))
        gs, e0, bonds = ground_states_2d(L, J)
        if len(gs) >= 8:
            break
    assert len(gs) >= 8
    rng = np.random.default_rng(3)
    R = 8
    visited = {}
    for icm_on in (0, 1):
        s = orc.Sim(inputs.SQUARE2D, L, J, [1e-3], R, icm_on, flags=orc.FLAG_2A, seed=9, instance_key=5)
        s.set_states(gs[rng.integers(0, len(gs), size=R)].reshape(1, R, L * L), sweep0=0)
        seen = set()
        for _ in range(100):
            tr = s.run_trace(1)
            assert np.all(tr == round(e0)), tr             # every step stays at E_0
            for x in s.states()[0]:
                assert abs(exact.energy(inputs.SQUARE2D, L, J, x) - e0) < 1e-9
                seen.add(x.tobytes() if x[0] > 0 else (-x).tobytes())
        visited[icm_on] = len(seen)
    assert visited[1] > 1, visited
    if icm_on:
        assert s.stats()["icm_nontrivial"] > 0


def test_hca_mode_samples_the_exact_energy():
    top, L = inputs.SQUARE2D, 4
    J = inputs.pm_j_couplings(top, L, inputs.make_rng(99, 0))
    temps = inputs.geometric_temps(0.8, 2.0, 4)
    bonds = exact.bond_list(top, L, np.asarray(J, np.float64))
    ref = exact.thermal_mean_energy(exact.all_energies(L * L, bonds), temps)
    s = orc.Sim(top, L, J, temps, 2, len(temps), flags=orc.FLAG_PT, seed=9, instance_key=6)
    s.init_hot()
    s.run(500)
    tr = s.run_trace(16384).astype(np.float64)          # [t][K][R]
    for k in range(len(temps)):
        m, se = exact.binned_mean_se(tr[:, k, :].mean(axis=1))
        assert abs(m - ref[k]) < 4 * se + 1e-9, (k, m, ref[k], se)
    assert s.stats()["icm_2a_flips"] == 0

"""Oracle pins for the simulation step: Metropolis (step 1), ICM (steps 2a/2b),
parallel tempering (step 3) and the whole chain against exact enumeration."""
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import exact
import oracle as orc
from paper_1501_05630_amd import inputs

getcontext().prec = 60


def sim(top, L, J, temps, R=2, Kc=0, flags=0, **kw):
    return orc.Sim(top, L, J, temps, R, Kc, flags=flags, **kw)


# ----------------------------------------------------------------- Metropolis
@pytest.mark.parametrize("scale", [1, 3])
def test_integer_thresholds_match_high_precision_exp(scale):
    # Acceptance count for dE > 0 is floor(2^32 exp(-beta dE / scale)).
    temps = inputs.geometric_temps(0.2, 3.0, 7)
    J = np.ones((16, 2), dtype=np.int8)
    s = sim(inputs.SQUARE2D, 4, J, temps, j_scale=scale)
    for k, T in enumerate(temps):
        for dE in range(1, 40):
            x = (-(Decimal(1) / Decimal(float(T))) * dE / scale).exp() * (Decimal(2) ** 32)
            ref = int(x)  # floor, x > 0
            assert s.metro_accept_count(k, dE) == min(ref, 2 ** 32 - 1)
            frac = x - int(x)
            assert min(frac, 1 - frac) > Decimal("1e-7") or ref == 0
        assert s.metro_accept_count(k, 0) == 2 ** 32
        assert s.metro_accept_count(k, -4) == 2 ** 32


def test_gaussian_acceptance_matches_high_precision_exp():
    temps = inputs.geometric_temps(0.2, 2.0, 5)
    s = sim(inputs.SQUARE2D, 4, np.ones((16, 2), np.float32), temps)
    rng = np.random.default_rng(3)
    for k, T in enumerate(temps):
        for dE in rng.random(50) * 6:
            raw = int(round(dE * 2 ** 40))
            x = (-(Decimal(1) / Decimal(float(T))) * (Decimal(raw) / Decimal(2) ** 40)).exp() * Decimal(2) ** 32
            assert abs(s.metro_accept_count(k, raw) - x) <= 1.000001


def test_first_half_sweep_flip_frequencies():
    # Colour-0 sites are updated once, from the initial state, in the first half
    # of the sweep: each flips with probability min(1, exp(-beta dE_i)).
    top, L, T = inputs.SQUARE2D, 4, 1.3
    rng = inputs.make_rng(50, 0)
    J = inputs.pm_j_couplings(top, L, rng)
    s0 = np.where(rng.random((1, 2, 16)) < 0.5, 1, -1).astype(np.int8)
    bonds = exact.bond_list(top, L, J)
    nbr = [[] for _ in range(16)]
    for i, j, Jij in bonds:
        nbr[i].append((j, int(Jij))); nbr[j].append((i, int(Jij)))

    def dE(state, i):
        return 2 * state[i] * sum(Jij * state[j] for j, Jij in nbr[i])

    colour = np.array([((i % L) + i // L) & 1 for i in range(16)])
    trials = 3000
    flips = np.zeros((2, 16))
    resid, var = 0.0, 0.0
    for key in range(trials):
        s = sim(top, L, J, [T], instance_key=key)
        s.set_states(s0)
        s.run(1)
        out = s.states()[0]
        for r in range(2):
            mid = s0[0, r].copy()
            mid[colour == 0] = out[r][colour == 0]
            flips[r] += out[r] != s0[0, r]
            for j in np.where(colour == 1)[0]:
                p = min(1.0, np.exp(-dE(mid, j) / T))
                resid += float(out[r][j] != mid[j]) - p
                var += p * (1 - p)
    for r in range(2):
        for i in np.where(colour == 0)[0]:
            p = min(1.0, np.exp(-dE(s0[0, r], i) / T))
            sd = np.sqrt(max(p * (1 - p), 1e-12) / trials)
            assert abs(flips[r, i] / trials - p) < 5 * sd + 1e-9
    assert abs(resid) < 5 * np.sqrt(var) + 1e-9


@pytest.mark.parametrize("top,L", [(inputs.CHIMERA, 1), (inputs.CUBIC3D, 2)])
def test_checkerboard_sweep_is_stationary(top, L):
    # Exact transition matrix of one sweep (colour 0 then colour 1) built from
    # the oracle's acceptance counts; the Boltzmann weight must be invariant.
    rng = inputs.make_rng(51, L)
    J = inputs.int_couplings(top, L, rng)
    T = 0.9
    s = sim(top, L, J, [T], j_scale=3)
    N = s.N
    states = exact.all_states(N)
    E = np.array([s.energy_raw(x) for x in states], dtype=np.int64)
    pi = np.exp(-(E - E.min()) / 3.0 / T)
    pi /= pi.sum()
    acc = {}
    P = np.eye(len(states))
    for c in (0, 1):
        Pc = np.zeros_like(P)
        sites = [i for i in range(N) if s.colour(i) == c]
        for a, x in enumerate(states):
            probs = {a: 1.0}
            for i in sites:  # same-colour sites are independent
                y = x.copy(); y[i] = -y[i]
                d = int(s.energy_raw(y) - E[a])
                if (d, 0) not in acc:
                    acc[(d, 0)] = s.metro_accept_count(0, d) / 2.0 ** 32
                pa = acc[(d, 0)]
                bit = 1 << i
                new = {}
                for idx, pr in probs.items():
                    new[idx ^ bit] = new.get(idx ^ bit, 0.0) + pr * pa
                    new[idx] = new.get(idx, 0.0) + pr * (1 - pa)
                probs = new
            for idx, pr in probs.items():
                Pc[a, idx] += pr
        P = P @ Pc
    assert np.max(np.abs(pi @ P - pi)) < 1e-9


def test_zero_temperature_never_raises_energy():
    top, L = inputs.CUBIC3D, 4
    J = inputs.gaussian_couplings(top, L, inputs.make_rng(52, 0))
    s = sim(top, L, J, [1e-3, 2e-3])
    s.init_hot()
    tr = s.run_trace(50)
    assert np.all(np.diff(tr, axis=0) <= 0)


# ------------------------------------------------------------------------ ICM
def _components(N, bonds, mask):
    rows = [i for i, j, _ in bonds if mask[i] and mask[j]]
    cols = [j for i, j, _ in bonds if mask[i] and mask[j]]
    g = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))
    _, lab = connected_components(g, directed=False)
    out = np.full(N, -1)
    for c in np.unique(lab[mask]):
        members = np.where((lab == c) & mask)[0]
        out[members] = members.min()
    return out


@pytest.mark.parametrize("top,L,kind", [(inputs.SQUARE2D, 8, "pmJ"), (inputs.CUBIC3D, 4, "gauss"),
                                        (inputs.CHIMERA, 3, "int3"), (inputs.SQUARE2D, 2, "pmJ")])
@pytest.mark.parametrize("flags", [orc.FLAG_2A, 0])
def test_icm_move_labels_flips_and_invariants(top, L, kind, flags):
    rng = inputs.make_rng(53, L)
    J = inputs.make_couplings(kind, top, L, rng)
    temps = inputs.geometric_temps(0.3, 1.5, 4)
    scale = 3 if kind == "int3" else 1
    bonds = exact.bond_list(top, L, J)
    for trial in range(6):
        s = sim(top, L, J, temps, R=4, Kc=4, flags=flags | orc.FLAG_SKIP_METRO, j_scale=scale)
        N = s.N
        fracs = [0.1, 0.4, 0.6, 0.9][trial % 4]
        before = np.where(rng.random((4, 4, N)) < 0.5, 1, -1).astype(np.int8)
        for k in range(4):
            for r in (1, 3):
                flip = rng.random(N) < fracs
                before[k, r] = np.where(flip, -before[k, r - 1], before[k, r - 1])
        s.set_states(before, sweep0=trial)
        e0 = s.energies_raw()
        s.run(1)
        after, e1 = s.states(), s.energies_raw()
        for k in range(4):
            for p in range(2):
                a, b = 2 * p, 2 * p + 1
                lab, seed, nm = s.labels(k, p)
                xa, xb = before[k, a].copy(), before[k, b].copy()
                mask = xa != xb
                if (flags & orc.FLAG_2A) and 2 * mask.sum() > N:
                    xb = -xb
                    mask = ~mask
                assert nm == mask.sum()
                if flags & orc.FLAG_2A:
                    assert 2 * nm <= N
                assert e1[k, a] + e1[k, b] == e0[k, a] + e0[k, b]       # isoenergetic
                if nm == 0:
                    assert seed == -1 and np.all(lab == -1)
                    assert np.array_equal(after[k, a], xa) and np.array_equal(after[k, b], xb)
                    continue
                assert np.array_equal(lab, _components(N, bonds, mask))
                assert mask[seed]
                cl = lab == lab[seed]
                assert np.array_equal(after[k, a], np.where(cl, -xa, xa))
                assert np.array_equal(after[k, b], np.where(cl, -xb, xb))
                assert np.array_equal(after[k, a] != after[k, b], mask)  # q unchanged
                assert s.energy_raw(after[k, a]) == e1[k, a]


def test_icm_seed_is_uniform_over_mask_sites():
    top, L = inputs.SQUARE2D, 6
    J = inputs.pm_j_couplings(top, L, inputs.make_rng(54, 0))
    rng = np.random.default_rng(1)
    st = np.where(rng.random((1, 2, 36)) < 0.5, 1, -1).astype(np.int8)
    st[0, 1] = st[0, 0]
    idx = rng.choice(36, size=11, replace=False)
    st[0, 1, idx] *= -1
    counts = np.zeros(36)
    trials = 4400
    s = sim(top, L, J, [0.5], Kc=1, flags=orc.FLAG_SKIP_METRO)
    for t in range(trials):
        s.set_states(st, sweep0=t)
        s.run(1)
        _, seed, nm = s.labels(0, 0)
        assert nm == 11
        counts[seed] += 1
    assert set(np.nonzero(counts)[0]) == set(idx)
    exp = trials / 11
    chi2 = np.sum((counts[idx] - exp) ** 2 / exp)
    assert chi2 < 35  # 10 dof


def test_icm_detailed_balance_on_a_cycle():
    # 6-cycle, one pair: from (x, y) the move reaches (x', y') with probability
    # |C|/n, and the reverse move has the same mask, clusters and probability.
    N = 6
    edges = [(i, (i + 1) % N) for i in range(N)]
    colours = [i & 1 for i in range(N)]
    J = np.array([1, -1, 1, 1, -1, 1], dtype=np.int8)
    x = np.array([1, 1, -1, 1, -1, -1], dtype=np.int8)
    y = x.copy(); y[[0, 1, 3]] *= -1          # mask {0,1,3}: clusters {0,1} and {3}
    st = np.stack([x, y])[None]
    outcomes = {}
    trials = 3000
    s = orc.Sim(orc.EXPLICIT, 0, J, [0.7], 2, 1, flags=orc.FLAG_SKIP_METRO,
                edges=edges, colours=colours)
    for t in range(trials):
        s.set_states(st, sweep0=t)
        s.run(1)
        key = s.states().tobytes()
        outcomes[key] = outcomes.get(key, 0) + 1
    assert len(outcomes) == 2
    freq = sorted(v / trials for v in outcomes.values())
    assert abs(freq[0] - 1 / 3) < 5 * np.sqrt(2 / 9 / trials)
    assert abs(freq[1] - 2 / 3) < 5 * np.sqrt(2 / 9 / trials)


# ------------------------------------------------------------------------- PT
def test_pt_equal_energies_always_swap():
    top, L = inputs.SQUARE2D, 4
    J = inputs.pm_j_couplings(top, L, inputs.make_rng(55, 0))
    K = 5
    s = sim(top, L, J, inputs.geometric_temps(0.5, 2, K), R=2,
            flags=orc.FLAG_PT | orc.FLAG_SKIP_METRO)
    st = np.ones((K, 2, 16), dtype=np.int8)
    s.set_states(st)
    w0 = s.walkers()
    s.run(1)
    w1 = s.walkers()
    # every ascending swap is accepted: the coldest walker bubbles to the top
    assert np.array_equal(w1[:-1], w0[1:]) and np.array_equal(w1[-1], w0[0])
    assert s.stats()["pt_accepts"] == 2 * (K - 1)


def test_pt_two_temperature_occupation_is_boltzmann():
    top, L = inputs.SQUARE2D, 4
    J = inputs.gaussian_couplings(top, L, inputs.make_rng(56, 0))
    temps = [0.8, 1.1]
    s = sim(top, L, J, temps, R=2, flags=orc.FLAG_PT | orc.FLAG_SKIP_METRO)
    rng = np.random.default_rng(5)
    st = np.where(rng.random((2, 2, 16)) < 0.5, 1, -1).astype(np.int8)
    s.set_states(st)
    E = s.energies().copy()                     # walker (k, r) energies at t = 0
    w_init = s.walkers().copy()
    tr_w = []
    for _ in range(6000):
        s.run(1)
        tr_w.append(s.walkers()[0].copy())
    tr_w = np.array(tr_w)
    states_before = sorted(map(bytes, st.reshape(4, 16)))
    states_after = sorted(map(bytes, s.states().reshape(4, 16)))
    assert states_before == states_after                   # multiset preserved
    for r in range(2):
        wa, wb = w_init[0, r], w_init[1, r]
        Ea, Eb = E[0, r], E[1, r]
        # stationary probability that walker wa sits at the cold temperature:
        # pi(wb cold) / pi(wa cold) = exp((beta_0 - beta_1) (Ea - Eb))
        ratio = np.exp((1 / temps[0] - 1 / temps[1]) * (Ea - Eb))
        p_cold = 1 / (1 + ratio)
        frac = np.mean(tr_w[:, r] == wa)
        assert abs(frac - p_cold) < 0.03
        assert set(np.unique(tr_w[:, r])) <= {wa, wb}


# ----------------------------------------------------------- whole PT + ICM
CHAIN_CASES = [
    ("2d4_pmJ", inputs.SQUARE2D, 4, "pmJ", 1),
    ("2d4_gauss", inputs.SQUARE2D, 4, "gauss", 1),
    ("3d2_gauss", inputs.CUBIC3D, 2, "gauss", 1),
    ("chimera1_int3", inputs.CHIMERA, 1, "int3", 3),
]


@pytest.mark.parametrize("name,top,L,kind,scale", CHAIN_CASES)
def test_chain_energy_matches_exact_enumeration(name, top, L, kind, scale):
    rng = inputs.make_rng(57, sum(map(ord, name)))
    J = inputs.make_couplings(kind, top, L, rng)
    temps = inputs.geometric_temps(0.3, 1.6, 5)
    s = sim(top, L, J, temps, R=2, Kc=3, flags=orc.FLAG_2A | orc.FLAG_PT, j_scale=scale,
            seed=11, instance_key=3)
    N = s.N
    E_all = exact.all_energies(N, exact.bond_list(top, L, np.asarray(J, np.float64) / scale))
    ref = exact.thermal_mean_energy(E_all, temps)
    s.init_hot()
    s.run(2000)
    tr = s.run_trace(60000) * s.energy_unit()     # [t][k][r]
    for k in range(len(temps)):
        m, se = exact.binned_mean_se(tr[:, k, :].mean(axis=1), 40)
        assert abs(m - ref[k]) < 4 * se + 1e-9, (k, m, ref[k], se)
    assert abs(tr[:, 0, :].min() - E_all.min()) < 1e-6   # ground state visited


def test_chain_without_icm_also_matches_and_icm_changes_the_trajectory():
    top, L = inputs.SQUARE2D, 4
    J = inputs.pm_j_couplings(top, L, inputs.make_rng(58, 0))
    temps = inputs.geometric_temps(0.3, 1.6, 4)
    a = sim(top, L, J, temps, R=2, Kc=0, flags=orc.FLAG_PT)
    b = sim(top, L, J, temps, R=2, Kc=4, flags=orc.FLAG_PT | orc.FLAG_2A)
    for x in (a, b):
        x.init_hot()
        x.run(50)
    assert a.stats()["icm_moves"] == 0 and b.stats()["icm_moves"] == 50 * 4
    assert not np.array_equal(a.states(), b.states())

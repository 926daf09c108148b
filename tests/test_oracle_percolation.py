"""Pins of the oracle's site percolation (Supplemental Material: the largest
cluster of randomly occupied sites and its Binder ratio).

- p = 0 gives no cluster and p = 1 the whole (connected) graph;
- per sample, the largest cluster equals the one found by scipy's connected
  components on the subgraph induced by the occupied sites, the graph built
  from the coupling layout independently of the oracle (exact.bond_list);
- on graphs small enough to enumerate every occupation pattern, the sample
  moments <s_max>, <s_max^2>, <s_max^4> agree with the exact ones within 4
  standard errors at two occupation probabilities;
- the Binder ratio helper is 1 for a constant s_max and matches its formula
  on a two-point distribution.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle as orc
from paper_1501_05630_amd import analysis, inputs

import exact


def sim(top, L, key=0):
    J = inputs.make_couplings("pmJ" if top != inputs.CHIMERA else "int3", top, L, inputs.make_rng(95, L))
    return orc.Sim(top, L, J, [1.0], 2, 0, flags=0, seed=11, instance_key=key,
                   j_scale=1 if top != inputs.CHIMERA else 3), J


def largest(N, bonds, occ):
    idx = np.flatnonzero(occ)
    if len(idx) == 0:
        return 0
    pos = -np.ones(N, dtype=np.int64)
    pos[idx] = np.arange(len(idx))
    e = [(pos[i], pos[j]) for i, j, _ in bonds if occ[i] and occ[j]]
    n = len(idx)
    if e:
        r, c = np.array(e).T
        g = coo_matrix((np.ones(len(e)), (r, c)), shape=(n, n))
    else:
        g = coo_matrix((n, n))
    _, lab = connected_components(g, directed=False)
    return int(np.bincount(lab).max())


CASES = [(inputs.SQUARE2D, 4), (inputs.CUBIC3D, 4), (inputs.CHIMERA, 3), (inputs.CHIMERA, 1),
         (inputs.CUBIC3D, 2)]


@pytest.mark.parametrize("top,L", CASES)
def test_empty_and_full(top, L):
    s, _ = sim(top, L)
    assert np.all(s.percolation_smax(0.0, 50) == 0)
    assert np.all(s.percolation_smax(1.0, 50) == s.N)


@pytest.mark.parametrize("top,L", CASES)
def test_each_sample_matches_connected_components(top, L):
    s, J = sim(top, L, key=3)
    N = s.N
    bonds = exact.bond_list(top, L, J)
    for p in (0.25, 0.45, 0.7):
        got = s.percolation_smax(p, 40, sample0=1000)
        thr = int(np.floor(p * 2.0 ** 32))
        for n in range(40):
            occ = np.zeros(N, dtype=bool)
            for q in range((N + 3) // 4):
                w = orc.philox4x32_10([1000 + n, q, 0, 4], [11, 3])
                for b in range(4):
                    if 4 * q + b < N:
                        occ[4 * q + b] = w[b] < thr
            assert got[n] == largest(N, bonds, occ), (p, n)


def exact_moments(top, L, J, ps):
    N = inputs.n_sites(top, L)
    bonds = exact.bond_list(top, L, J)
    S = exact.all_states(N) < 0                      # every occupation pattern
    sm = np.array([largest(N, bonds, occ) for occ in S], dtype=np.float64)
    k = S.sum(axis=1)
    out = []
    for p in ps:
        w = p ** k * (1 - p) ** (N - k)
        out.append([float(np.sum(w * sm ** m)) for m in (1, 2, 4)])
    return out


@pytest.mark.parametrize("top,L", [(inputs.SQUARE2D, 4), (inputs.CHIMERA, 1), (inputs.CUBIC3D, 2)])
def test_moments_match_exact_enumeration(top, L):
    s, J = sim(top, L, key=5)
    ps = (0.35, 0.6)
    for p, ref in zip(ps, exact_moments(top, L, J, ps)):
        x = s.percolation_smax(p, 20000).astype(np.float64)
        for m, r in zip((1, 2, 4), ref):
            v = x ** m
            se = v.std(ddof=1) / np.sqrt(len(v))
            assert abs(v.mean() - r) < 4 * se, (p, m, v.mean(), r, se)


def test_binder_ratio_helper():
    assert analysis.binder_ratio(np.full(10, 7)) == 1.0
    # s in {1, 3} with equal weight: <s^2> = 5, <s^4> = 41
    assert abs(analysis.binder_ratio([1, 3] * 50) - 0.5 * (3 - 41 / 25)) < 1e-12


def test_binder_collapse_recovers_a_known_scaling_form():
    # g(p, N) = G[N^(1/(2 nu)) (1/p - 1/p_c)] with a cubic G, small noise
    pc, nu = 0.3866, 1.39
    ps = np.linspace(0.36, 0.41, 11)
    sizes = [512, 1152, 2048, 3872]
    rng = np.random.default_rng(0)
    g, se = [], []
    for n in sizes:
        x = n ** (0.5 / nu) * (1 / ps - 1 / pc)
        g.append(0.72 - 0.08 * x + 0.004 * x ** 2 + 0.001 * x ** 3 + rng.normal(0, 1e-4, len(ps)))
        se.append(np.full(len(ps), 1e-4))
    p_fit, nu_fit, chi = analysis.binder_collapse(ps, sizes, g, se, 0.38, 1.2, degree=3)
    assert abs(p_fit - pc) < 2e-4 and abs(nu_fit - nu) < 0.03 and chi < 3.0, (p_fit, nu_fit, chi)

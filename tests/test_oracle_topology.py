"""Oracle pins: graphs, couplings and the Hamiltonian (model paragraph)."""
from fractions import Fraction

import numpy as np
import pytest

import exact
import oracle as orc
from paper_1501_05630_amd import inputs

CASES = [(inputs.SQUARE2D, 2), (inputs.SQUARE2D, 4), (inputs.SQUARE2D, 6), (inputs.CUBIC3D, 2),
         (inputs.CUBIC3D, 4), (inputs.CHIMERA, 1), (inputs.CHIMERA, 3)]


def make(top, L, J, **kw):
    temps = kw.pop("temps", [1.0])
    return orc.Sim(top, L, J, temps, kw.pop("R", 2), kw.pop("Kc", 0), flags=kw.pop("flags", 0), **kw)


def ones(top, L, value=1):
    J = np.full(inputs.coupling_shape(top, L), value, dtype=np.int8)
    if top == inputs.CHIMERA:
        J *= inputs.chimera_edge_mask(L)
    return J


@pytest.mark.parametrize("top,L", CASES)
def test_bond_count_closed_form(top, L):
    s = make(top, L, ones(top, L))
    N = inputs.n_sites(top, L)
    expect = {inputs.SQUARE2D: 2 * N, inputs.CUBIC3D: 3 * N,
              inputs.CHIMERA: 16 * L * L + 8 * L * (L - 1)}[top]
    assert s.N == N and s.n_bonds == expect


@pytest.mark.parametrize("top,L", CASES)
def test_ferromagnet_and_antiferromagnet_ground_states(top, L):
    # All J = +1: every bond satisfied by the uniform state, E = -N_b.  All
    # J = -1 on a bipartite graph: the checkerboard state satisfies every bond.
    s = make(top, L, ones(top, L))
    up = np.ones(s.N, dtype=np.int8)
    assert s.energy_raw(up) == -s.n_bonds
    assert s.energy_raw(-up) == -s.n_bonds
    af = make(top, L, ones(top, L, -1))
    cb = np.array([1 - 2 * af.colour(i) for i in range(af.N)], dtype=np.int8)
    assert af.energy_raw(cb) == -af.n_bonds
    assert af.energy_raw(up) == af.n_bonds


@pytest.mark.parametrize("top,L", CASES)
def test_energy_matches_layout_formula_and_spin_reversal(top, L):
    rng = inputs.make_rng(99, L + 10 * top)
    for kind in ("pmJ", "int3", "gauss"):
        J = inputs.make_couplings(kind, top, L, rng)
        s = make(top, L, J, j_scale=3 if kind == "int3" else 1)
        for _ in range(5):
            spins = np.where(rng.random(s.N) < 0.5, 1, -1).astype(np.int8)
            raw = s.energy_raw(spins)
            assert raw == s.energy_raw(-spins)
            ref = exact.energy(top, L, J, spins)
            if kind == "gauss":
                # float couplings are kept exactly, as multiples of 2^-40: the
                # raw energy is the formula's value on the float32 couplings
                # themselves (at these sizes the float64 sum is exact too)
                assert raw * 2.0 ** -40 == ref
            else:
                assert raw == round(ref)


@pytest.mark.parametrize("top,L", CASES)
def test_neighbours_symmetric_and_colouring_proper(top, L):
    s = make(top, L, ones(top, L))
    deg = []
    for i in range(s.N):
        nb = s.neighbours(i)
        deg.append(len(nb))
        for j in nb:
            assert s.colour(j) != s.colour(i)
            assert np.count_nonzero(s.neighbours(j) == i) == np.count_nonzero(nb == j)
    deg = np.array(deg)
    if top == inputs.SQUARE2D:
        assert np.all(deg == 4)
    elif top == inputs.CUBIC3D:
        assert np.all(deg == 6)
    else:
        assert deg.max() <= 6 and deg.min() >= 4 + (1 if L > 1 else 0)
        assert deg.sum() == 2 * s.n_bonds


def test_chimera_cells_are_k44_and_inter_cell_wiring():
    C = 3
    s = make(inputs.CHIMERA, C, ones(inputs.CHIMERA, C))
    ij, _ = s.bonds()
    bonds = {tuple(sorted(map(int, b))) for b in ij}
    for cell in range(C * C):
        b = 8 * cell
        for u in range(4):
            for v in range(4, 8):
                assert (b + u, b + v) in bonds
        for u in range(4):
            for v in range(4):
                assert (b + min(u, v), b + max(u, v)) not in bonds or u == v
    # u<4 couple vertically (same u, next row); u>=4 horizontally (next column).
    for row in range(C):
        for col in range(C):
            b = 8 * (row * C + col)
            for u in range(4):
                assert ((b + u, 8 * ((row + 1) * C + col) + u) in bonds) == (row + 1 < C)
            for u in range(4, 8):
                assert ((b + u, 8 * (row * C + col + 1) + u) in bonds) == (col + 1 < C)


def test_chimera_rejects_couplings_off_the_grid():
    J = np.ones((4, 24), dtype=np.int8)  # C=2 without the boundary mask
    with pytest.raises(ValueError):
        make(inputs.CHIMERA, 2, J)


def test_gaussian_couplings_are_kept_exactly():
    # the model's Gaussian J reach the oracle as float32 values and are used
    # as given: every bond's raw coupling is J 2^40 with no rounding (float32
    # with |J| >= 2^-17 are multiples of 2^-40), including values near the
    # bound |J| <= 64 and values far from any coarse grid
    rng = inputs.make_rng(98, 0)
    J = inputs.gaussian_couplings(inputs.SQUARE2D, 4, rng)
    J[0, 0] = np.float32(63.99999)
    J[1, 1] = np.float32(-40.0)
    J[2, 0] = np.float32(1.0 + 2.0 ** -23)          # the last mantissa bit of a unit value
    J[3, 1] = np.float32(3.0 * 2.0 ** -17)          # the smallest binade that is exact
    s = make(inputs.SQUARE2D, 4, J)
    _, raw = s.bonds()
    ref = [b[2] for b in exact.bond_list(inputs.SQUARE2D, 4, J)]
    for r, j in zip(raw, ref):
        assert Fraction(int(r), 1 << 40) == Fraction(float(j))
    assert int(raw[0]) == int(Fraction(float(np.float32(63.99999))) * (1 << 40))


def test_tiny_gaussian_couplings_round_to_the_nearest_2_pow_minus_40():
    # below 2^-17 a float32 has bits finer than 2^-40: the nearest multiple
    J = np.ones((16, 2), dtype=np.float32)
    J[5, 0] = np.float32(1.2345678e-7)
    s = make(inputs.SQUARE2D, 4, J)
    ij, raw = s.bonds()
    x = [int(r) for (i, j), r in zip(ij, raw) if (i, j) == (5, 6)][0]
    exact_scaled = Fraction(float(J[5, 0])) * (1 << 40)
    assert abs(Fraction(x) - exact_scaled) <= Fraction(1, 2)


def test_float_energy_change_is_exact_and_symmetric():
    # the energies of a state and of its single-spin flips differ by exactly
    # 2 s_i h_i on the raw couplings (integer sums in units of 2^-40)
    rng = inputs.make_rng(98, 2)
    J = inputs.gaussian_couplings(inputs.CUBIC3D, 4, rng)
    s = make(inputs.CUBIC3D, 4, J)
    ij, raw = s.bonds()
    spins = np.where(rng.random(s.N) < 0.5, 1, -1).astype(np.int8)
    E0 = s.energy_raw(spins)
    for i in range(0, s.N, 7):
        h = 0
        for (a, b), r in zip(ij, raw):
            if a == i:
                h += int(r) * int(spins[b])
            elif b == i:
                h += int(r) * int(spins[a])
        y = spins.copy()
        y[i] = -y[i]
        assert s.energy_raw(y) - E0 == 2 * int(spins[i]) * h

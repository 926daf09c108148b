"""Brute-force helpers for pinning the oracle on tiny systems.

These restate the model from the coupling layouts directly (array shifts for
the lattices, slot loops for chimera) rather than from the oracle's adjacency
lists, and enumerate all 2^N states for exact thermal averages.
"""
import numpy as np

from paper_1501_05630_amd import inputs


def lattice_energy(topology, L, J, s):
    """H = -sum_bonds J s_i s_j for periodic lattices, from the [N][d] layout."""
    J = np.asarray(J, dtype=np.float64)
    if topology == inputs.SQUARE2D:
        g = s.reshape(L, L)              # [y][x]
        Jx = J[:, 0].reshape(L, L)
        Jy = J[:, 1].reshape(L, L)
        return -(np.sum(Jx * g * np.roll(g, -1, axis=1)) + np.sum(Jy * g * np.roll(g, -1, axis=0)))
    if topology == inputs.CUBIC3D:
        g = s.reshape(L, L, L)           # [z][y][x]
        E = 0.0
        for d, ax in ((0, 2), (1, 1), (2, 0)):
            E += np.sum(J[:, d].reshape(L, L, L) * g * np.roll(g, -1, axis=ax))
        return -E
    raise ValueError(topology)


def chimera_energy(C, J, s):
    """H for chimera from the [C*C][24] layout, looping over cells and slots."""
    J = np.asarray(J, dtype=np.float64)
    E = 0.0
    for row in range(C):
        for col in range(C):
            cell = row * C + col
            b = 8 * cell
            for u in range(4):
                for v in range(4, 8):
                    E += J[cell, u * 4 + v - 4] * s[b + u] * s[b + v]
            if row + 1 < C:
                for u in range(4):
                    E += J[cell, 16 + u] * s[b + u] * s[8 * ((row + 1) * C + col) + u]
            if col + 1 < C:
                for u in range(4, 8):
                    E += J[cell, 20 + u - 4] * s[b + u] * s[8 * (row * C + col + 1) + u]
    return -E


def energy(topology, L, J, s):
    s = np.asarray(s, dtype=np.float64)
    if topology == inputs.CHIMERA:
        return chimera_energy(L, J, s)
    return lattice_energy(topology, L, J, s)


def all_states(N):
    """All 2^N spin configurations as an int8 array [2^N][N] (bit i of the index -> site i)."""
    idx = np.arange(1 << N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N)) & 1
    return (1 - 2 * bits).astype(np.int8)


def bond_list(topology, L, J):
    """Bonds (i, j, J) from the canonical layout (independent of the oracle)."""
    J = np.asarray(J)
    out = []
    if topology in (inputs.SQUARE2D, inputs.CUBIC3D):
        dim = 2 if topology == inputs.SQUARE2D else 3
        N = L ** dim
        for i in range(N):
            x, y, z = i % L, (i // L) % L, i // (L * L)
            fwd = [((x + 1) % L) + L * y + L * L * z, x + L * ((y + 1) % L) + L * L * z,
                   x + L * y + L * L * ((z + 1) % L)]
            for d in range(dim):
                out.append((i, fwd[d], J[i, d]))
        return out
    C = L
    for row in range(C):
        for col in range(C):
            cell = row * C + col
            b = 8 * cell
            for u in range(4):
                for v in range(4, 8):
                    out.append((b + u, b + v, J[cell, u * 4 + v - 4]))
            if row + 1 < C:
                for u in range(4):
                    out.append((b + u, 8 * ((row + 1) * C + col) + u, J[cell, 16 + u]))
            if col + 1 < C:
                for u in range(4, 8):
                    out.append((b + u, 8 * (row * C + col + 1) + u, J[cell, 20 + u - 4]))
    return out


def all_energies(N, bonds):
    """Energies of all 2^N states, vectorised over states."""
    S = all_states(N).astype(np.float64)
    E = np.zeros(S.shape[0])
    for i, j, Jij in bonds:
        E -= float(Jij) * S[:, i] * S[:, j]
    return E


def thermal_mean_energy(E_all, temps):
    """Exact <H>_T by enumeration for each temperature."""
    out = []
    for T in temps:
        x = -(E_all - E_all.min()) / T
        w = np.exp(x)
        out.append(float(np.sum(w * E_all) / np.sum(w)))
    return np.array(out)


def binned_mean_se(x, n_bins=32):
    """Mean and standard error from n_bins contiguous bins of a time series."""
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // n_bins
    b = x[: m * n_bins].reshape(n_bins, m).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / np.sqrt(n_bins))


def walsh_hadamard(v):
    """Unnormalised fast Walsh-Hadamard transform of a length-2^N vector."""
    a = np.array(v, dtype=np.float64)
    h = 1
    while h < len(a):
        a = a.reshape(-1, 2, h)
        a = np.stack((a[:, 0] + a[:, 1], a[:, 0] - a[:, 1]), axis=1).reshape(-1)
        h *= 2
    return a


def pair_difference_distribution(w):
    """For two independent replicas with state weights w (indexed as all_states),
    the probability of each difference pattern d (bit i set <=> the replicas
    differ at site i): sum_x w(x) w(x xor d), an xor autocorrelation computed
    through the Walsh-Hadamard transform."""
    f = walsh_hadamard(w)
    return walsh_hadamard(f * f) / len(f)

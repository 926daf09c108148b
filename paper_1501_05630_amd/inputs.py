"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle runs.

This module holds no part of the simulation method: it only draws disorder
(couplings) and lays out temperature ladders, so that the HIP path and the CPU
oracle see identical inputs.  The couplings follow the model paragraph of the
paper (Gaussian J with zero mean and unit variance) plus the bimodal and
chimera-integer variants of the benchmark workloads.

Coupling layouts (canonical, per instance):
  square2d  [N][2]   bond from site i to its +x, +y neighbour (periodic)
  cubic3d   [N][3]   bond from site i to its +x, +y, +z neighbour (periodic)
  chimera   [C*C][24] 16 in-cell bonds (u, v) at u*4+(v-4), u<4<=v; 4 bonds to the
                      cell below (16+u, u<4); 4 bonds to the cell on the right
                      (20+u-4, u>=4).  Bonds that would leave the grid are 0.
"""
import numpy as np

SQUARE2D, CUBIC3D, CHIMERA = 0, 1, 2
TOPOLOGY_NAMES = {SQUARE2D: "square2d", CUBIC3D: "cubic3d", CHIMERA: "chimera"}
MASTER_SEED = 150105630


def make_rng(config_index, instance_index):
    """numpy PCG64 stream for (config, instance)."""
    return np.random.Generator(np.random.PCG64([MASTER_SEED, int(config_index), int(instance_index)]))


def n_sites(topology, L):
    if topology == SQUARE2D:
        return L * L
    if topology == CUBIC3D:
        return L ** 3
    if topology == CHIMERA:
        return 8 * L * L
    raise ValueError(topology)


def coupling_shape(topology, L):
    if topology == SQUARE2D:
        return (L * L, 2)
    if topology == CUBIC3D:
        return (L ** 3, 3)
    if topology == CHIMERA:
        return (L * L, 24)
    raise ValueError(topology)


def chimera_edge_mask(C):
    """1 where a chimera coupling slot is a real bond, 0 where it leaves the grid."""
    m = np.ones((C * C, 24), dtype=np.int8)
    for row in range(C):
        for col in range(C):
            cell = row * C + col
            if row == C - 1:
                m[cell, 16:20] = 0
            if col == C - 1:
                m[cell, 20:24] = 0
    return m


def _mask(topology, L, shape):
    if topology == CHIMERA:
        return chimera_edge_mask(L)
    return np.ones(shape, dtype=np.int8)


def gaussian_couplings(topology, L, rng):
    """J ~ N(0, 1) drawn in float64 and rounded to float32."""
    shape = coupling_shape(topology, L)
    J = rng.standard_normal(shape).astype(np.float32)
    return (J * _mask(topology, L, shape)).astype(np.float32)


def pm_j_couplings(topology, L, rng):
    """Bimodal J = +-1 with probability 1/2 each (int8, scale 1)."""
    shape = coupling_shape(topology, L)
    J = np.where(rng.random(shape) < 0.5, 1, -1).astype(np.int8)
    return (J * _mask(topology, L, shape)).astype(np.int8)


def int_couplings(topology, L, rng, values=(-3, -2, -1, 1, 2, 3)):
    """Integer couplings drawn uniformly from `values` (int8; divide by the scale)."""
    shape = coupling_shape(topology, L)
    J = np.asarray(values, dtype=np.int8)[rng.integers(0, len(values), size=shape)]
    return (J * _mask(topology, L, shape)).astype(np.int8)


def geometric_temps(t_min, t_max, n):
    """T_k = t_min (t_max / t_min)^(k / (n-1)), k = 0 (coldest) .. n-1, float64."""
    if n == 1:
        return np.array([t_min], dtype=np.float64)
    k = np.arange(n, dtype=np.float64)
    return t_min * (t_max / t_min) ** (k / (n - 1))


def icm_cutoff(temps, t_cut=1.0):
    """Number of temperatures T_k <= t_cut (ICM only below the cutoff, T <~ J)."""
    return int(np.sum(np.asarray(temps) <= t_cut + 1e-12))


# Benchmark workloads: (name, topology, L, coupling kind, scale, K, T range, R, sweeps, instances)
WORKLOADS = {
    "2d_L8_pmJ_1inst": dict(config=0, topology=SQUARE2D, L=8, kind="pmJ", j_scale=1,
                            n_temps=16, t_min=0.2, t_max=1.6, n_replicas=2,
                            n_sweeps=4096, n_instances=1),
    "3d_L8_gauss_1024inst": dict(config=1, topology=CUBIC3D, L=8, kind="gauss", j_scale=1,
                                 n_temps=20, t_min=0.2, t_max=2.0, n_replicas=4,
                                 n_sweeps=1 << 14, n_instances=1024),
    "chimera_C12_int3_512inst": dict(config=2, topology=CHIMERA, L=12, kind="int3", j_scale=3,
                                     n_temps=30, t_min=0.2, t_max=3.0, n_replicas=2,
                                     n_sweeps=1 << 14, n_instances=512),
    # uneven batch: 256 instances of each side, in this order
    "3d_uneven_gauss_1536inst": dict(config=3, topology=CUBIC3D, L=None, sides=(4, 6, 8, 10, 12, 16),
                                     per_side=256, kind="gauss", j_scale=1,
                                     n_temps=24, t_min=0.2, t_max=2.0, n_replicas=4,
                                     n_sweeps=1 << 13, n_instances=1536),
    # the paper's simulation parameters (Table I): Gaussian disorder, two
    # replicas per temperature, ICM at the n_icm coldest temperatures; per_side
    # is the table's number of disorder instances per size, of which an
    # experiment takes the first few of every size
    "table1_2d_gauss": dict(config=5, topology=SQUARE2D, L=None, sides=(16, 24, 32), per_side=10000,
                            kind="gauss", j_scale=1, n_temps=30, t_min=0.2120, t_max=1.6325,
                            n_replicas=2, n_icm=30, n_sweeps=1 << 22, n_instances=30000),
    "table1_chimera_gauss": dict(config=6, topology=CHIMERA, L=None, sides=(4, 6, 8, 10, 12),
                                 per_side=10000, kind="gauss", j_scale=1, n_temps=30, t_min=0.2120,
                                 t_max=1.6325, n_replicas=2, n_icm=19, n_sweeps=1 << 22,
                                 n_instances=50000),
    "table1_3d_gauss": dict(config=7, topology=CUBIC3D, L=None, sides=(4, 6, 8, 10, 12), per_side=15000,
                            kind="gauss", j_scale=1, n_temps=26, t_min=0.42, t_max=1.8,
                            n_replicas=2, n_icm=13, n_sweeps=1 << 23, n_instances=75000),
}


def instance_side(spec, instance_index):
    """Side L (or chimera cells per side) of one instance of a workload."""
    if spec.get("sides"):
        return spec["sides"][instance_index // spec["per_side"]]
    return spec["L"]


def make_couplings(kind, topology, L, rng):
    if kind == "gauss":
        return gaussian_couplings(topology, L, rng)
    if kind == "pmJ":
        return pm_j_couplings(topology, L, rng)
    if kind == "int3":
        return int_couplings(topology, L, rng)
    raise ValueError(kind)


def workload_instance(name, instance_index, L=None):
    """(couplings, temps, icm_ntemps, spec) for one instance of a named workload."""
    spec = dict(WORKLOADS[name])
    spec["L"] = L if L is not None else instance_side(spec, instance_index)
    rng = make_rng(spec["config"], instance_index)
    J = make_couplings(spec["kind"], spec["topology"], spec["L"], rng)
    temps = geometric_temps(spec["t_min"], spec["t_max"], spec["n_temps"])
    kc = spec["n_icm"] if "n_icm" in spec else icm_cutoff(temps)
    return J, temps, kc, spec

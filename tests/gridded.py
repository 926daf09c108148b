"""Float couplings already on the library's coupling grid, for the GPU tests
that compare whole trajectories bit for bit with the oracle.

The library rounds float couplings to multiples of 2^-e (e = 20 whenever every
|J| < 8) before it simulates them; the oracle uses the float32 values exactly.
The two chains are the same chain only when nothing is rounded, so these tests
draw the workload's Gaussian couplings as usual and move each one to the
nearest multiple of 2^-20 here (Gaussian draws stay far below 8, so e = 20).
The seeded generators in paper_1501_05630_amd/inputs.py are left as they are:
the benchmark and the statistical test feed the raw float32 draws.
"""
import numpy as np

from paper_1501_05630_amd import inputs

GRID = 2.0 ** -20


def on_grid(J):
    J = np.asarray(J)
    if J.dtype.kind != "f":
        return J
    q = np.rint(J.astype(np.float64) / GRID) * GRID
    assert np.all(np.abs(q) < 8.0)
    return q.astype(np.float32)


def make_couplings(kind, topology, L, rng):
    return on_grid(inputs.make_couplings(kind, topology, L, rng))


def gaussian_couplings(topology, L, rng):
    return on_grid(inputs.gaussian_couplings(topology, L, rng))


def workload_instance(name, instance_index, L=None):
    J, temps, kc, spec = inputs.workload_instance(name, instance_index, L)
    return on_grid(J), temps, kc, spec

"""ctypes wrapper of the CPU oracle (oracle/oracle.cpp).

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this module.  It does not import the product
package, and the product package does not import it.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: another build of oracle.cpp (the pins' own mutation test runs
# them against copies with planted mistakes)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

SQUARE2D, CUBIC3D, CHIMERA, EXPLICIT = 0, 1, 2, 3
J_INT8, J_F32 = 0, 1
FLAG_2A, FLAG_PT, FLAG_SKIP_METRO, FLAG_MEASURE = 1, 2, 8, 16
OBS_BINS, OBS_FIELDS = 32, 4


class _Params(ctypes.Structure):
    _fields_ = [
        ("topology", ctypes.c_int32), ("L", ctypes.c_int32),
        ("n_sites", ctypes.c_int32), ("n_edges", ctypes.c_int32),
        ("edges", ctypes.c_void_p), ("colours", ctypes.c_void_p),
        ("jkind", ctypes.c_int32), ("j_scale", ctypes.c_int32),
        ("couplings", ctypes.c_void_p),
        ("n_temps", ctypes.c_int32), ("temps", ctypes.c_void_p),
        ("n_replicas", ctypes.c_int32), ("icm_ntemps", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("seed", ctypes.c_uint32),
        ("instance_key", ctypes.c_uint32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "metro_accepts", "icm_moves", "icm_nontrivial", "icm_cluster_sites",
        "icm_2a_flips", "pt_attempts", "pt_accepts")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: F401  (oracle/build.py)
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, U32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(P)]
    lib.orc_create.restype = ctypes.c_int
    lib.orc_destroy.argtypes = [P]
    for name in ("orc_n_sites", "orc_n_bonds"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = I32
    lib.orc_neighbours.argtypes = [P, I32, P, I32]
    lib.orc_neighbours.restype = I32
    lib.orc_colour.argtypes = [P, I32]
    lib.orc_colour.restype = I32
    lib.orc_init_hot.argtypes = [P]
    lib.orc_set_states.argtypes = [P, P, U32]
    lib.orc_run.argtypes = [P, U32]
    lib.orc_run_trace.argtypes = [P, U32, P]
    lib.orc_get_states.argtypes = [P, P]
    lib.orc_get_energies.argtypes = [P, P]
    lib.orc_get_walkers.argtypes = [P, P]
    lib.orc_get_sweep.argtypes = [P]
    lib.orc_get_sweep.restype = U32
    lib.orc_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.orc_get_labels.argtypes = [P, I32, I32, P, P, P]
    lib.orc_get_labels.restype = ctypes.c_int
    lib.orc_energy.argtypes = [P, P]
    lib.orc_energy.restype = I64
    lib.orc_bonds.argtypes = [P, P, P]
    lib.orc_get_observables.argtypes = [P, P, P]
    lib.orc_metro_accept_count.argtypes = [P, I32, I64]
    lib.orc_metro_accept_count.restype = ctypes.c_uint64
    lib.orc_percolation_smax.argtypes = [P, ctypes.c_double, U32, U32, P]
    lib.orc_percolation_smax.restype = None
    lib.orc_icm_step.argtypes = [P, I32, I32, U32]
    lib.orc_icm_step.restype = ctypes.c_int
    lib.orc_set_temperatures.argtypes = [P, P]
    lib.orc_set_temperatures.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: four uint32 words for counter ctr under key."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


class Sim:
    """One disorder instance with K temperatures x R replicas, run by the oracle."""

    def __init__(self, topology, L, couplings, temps, n_replicas, icm_ntemps,
                 flags=FLAG_2A | FLAG_PT, seed=0, instance_key=0, jkind=None,
                 j_scale=1, edges=None, colours=None, n_sites=0):
        lib = _load()
        couplings = np.asarray(couplings)
        if jkind is None:
            jkind = J_F32 if couplings.dtype.kind == "f" else J_INT8
        cj = np.ascontiguousarray(couplings, dtype=np.float32 if jkind == J_F32 else np.int8)
        temps = np.ascontiguousarray(temps, dtype=np.float64)
        p = _Params()
        p.topology, p.L = topology, L
        keep = [cj, temps]
        if topology == EXPLICIT:
            e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
            c = np.ascontiguousarray(colours, dtype=np.int32)
            keep += [e, c]
            p.n_sites, p.n_edges = int(n_sites or len(c)), e.shape[0]
            p.edges, p.colours = _ptr(e).value, _ptr(c).value
        p.jkind, p.j_scale = jkind, j_scale
        p.couplings = _ptr(cj).value
        p.n_temps, p.temps = len(temps), _ptr(temps).value
        p.n_replicas, p.icm_ntemps, p.flags = n_replicas, icm_ntemps, flags
        p.seed, p.instance_key = seed & 0xFFFFFFFF, instance_key & 0xFFFFFFFF
        h = ctypes.c_void_p()
        rc = lib.orc_create(ctypes.byref(p), ctypes.byref(h))
        if rc != 0:
            raise ValueError("oracle rejected the parameters")
        self._lib, self._h = lib, h
        self.K, self.R = len(temps), n_replicas
        self.N = lib.orc_n_sites(h)
        self.n_bonds = lib.orc_n_bonds(h)
        self.jkind, self.j_scale = jkind, j_scale
        self.temps = temps.copy()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_destroy(h)
            self._h = None

    def init_hot(self):
        self._lib.orc_init_hot(self._h)

    def set_states(self, spins, sweep0=0):
        s = np.ascontiguousarray(spins, dtype=np.int8).reshape(self.K, self.R, self.N)
        self._lib.orc_set_states(self._h, _ptr(s), sweep0)

    def run(self, n_sweeps):
        self._lib.orc_run(self._h, n_sweeps)

    def run_trace(self, n_sweeps):
        """Runs n steps; returns raw energies [n][K][R] after every step."""
        out = np.zeros((n_sweeps, self.K, self.R), dtype=np.int64)
        self._lib.orc_run_trace(self._h, n_sweeps, _ptr(out))
        return out

    def states(self):
        out = np.zeros((self.K, self.R, self.N), dtype=np.int8)
        self._lib.orc_get_states(self._h, _ptr(out))
        return out

    def energies_raw(self):
        out = np.zeros((self.K, self.R), dtype=np.int64)
        self._lib.orc_get_energies(self._h, _ptr(out))
        return out

    def energy_unit(self):
        return 1.0 / self.j_scale if self.jkind == J_INT8 else 2.0 ** -40

    def energies(self):
        return self.energies_raw().astype(np.float64) * self.energy_unit()

    def walkers(self):
        out = np.zeros((self.K, self.R), dtype=np.int32)
        self._lib.orc_get_walkers(self._h, _ptr(out))
        return out

    def sweep(self):
        return int(self._lib.orc_get_sweep(self._h))

    def stats(self):
        st = Stats()
        self._lib.orc_get_stats(self._h, ctypes.byref(st))
        return st.as_dict()

    def observables(self):
        """(sums [32][K][R/2][4], counts [32]): per logarithmic time bin and pair
        of chains, E_a + E_b (raw), N_b q_l, q^2 and the potential cluster sites
        min(n, N - n) summed over the steps in the bin."""
        sums = np.zeros((OBS_BINS, self.K, self.R // 2, OBS_FIELDS), dtype=np.int64)
        counts = np.zeros(OBS_BINS, dtype=np.int64)
        self._lib.orc_get_observables(self._h, _ptr(sums), _ptr(counts))
        return sums, counts

    def labels(self, k, p):
        lab = np.zeros(self.N, dtype=np.int32)
        seed, nm = ctypes.c_int32(), ctypes.c_int32()
        rc = self._lib.orc_get_labels(self._h, k, p, _ptr(lab), ctypes.byref(seed), ctypes.byref(nm))
        if rc != 0:
            raise ValueError("no ICM at this (k, pair)")
        return lab, int(seed.value), int(nm.value)

    def icm_step(self, k, p, u):
        """Steps 2a and 2b alone for pair p at temperature k with seed word u."""
        if self._lib.orc_icm_step(self._h, k, p, int(u) & 0xFFFFFFFF) != 0:
            raise ValueError("no ICM at this (k, pair)")

    def energy_raw(self, spins):
        s = np.ascontiguousarray(spins, dtype=np.int8)
        return int(self._lib.orc_energy(self._h, _ptr(s)))

    def bonds(self):
        ij = np.zeros((self.n_bonds, 2), dtype=np.int32)
        raw = np.zeros(self.n_bonds, dtype=np.int64)
        self._lib.orc_bonds(self._h, _ptr(ij), _ptr(raw))
        return ij, raw

    def neighbours(self, i):
        buf = np.zeros(64, dtype=np.int32)
        d = self._lib.orc_neighbours(self._h, i, _ptr(buf), 64)
        return buf[:d].copy()

    def colour(self, i):
        return int(self._lib.orc_colour(self._h, i))

    def metro_accept_count(self, k, dE_raw):
        return int(self._lib.orc_metro_accept_count(self._h, k, int(dE_raw)))

    def set_temperatures(self, temps):
        t = np.ascontiguousarray(temps, dtype=np.float64)
        assert t.shape == (self.K,)
        if self._lib.orc_set_temperatures(self._h, _ptr(t)) != 0:
            raise ValueError("invalid temperatures")

    def percolation_smax(self, p, n_samples, sample0=0):
        """Largest-cluster sizes [n_samples] of random site configurations on
        this simulation's graph (key = seed, instance_key)."""
        out = np.zeros(n_samples, dtype=np.int32)
        self._lib.orc_percolation_smax(self._h, float(p), sample0, n_samples, _ptr(out))
        return out

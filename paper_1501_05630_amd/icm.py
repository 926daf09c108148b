"""Thin ctypes binding of libicm (include/icm.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libicm.so.  PyTorch provides the device arena (a uint8 tensor) and
the HIP stream.  Importing this module never falls back to anything: if the
library is missing, loading it raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libicm.so")

ICM_OK, ICM_E_INVALID, ICM_E_NOMEM, ICM_E_DEVICE = 0, -1, -2, -3
ICM_E_NOTFOUND, ICM_E_BUSY, ICM_E_BUFSIZE = -4, -5, -6
TOPO_SQUARE2D, TOPO_CUBIC3D, TOPO_CHIMERA = 0, 1, 2
J_INT8, J_F32 = 0, 1
FLAG_2A, FLAG_PT, FLAG_RECORD_LABELS, FLAG_SKIP_METRO, FLAG_MEASURE = 1, 2, 4, 8, 16
OBS_BINS, OBS_FIELDS = 32, 4

_P = ctypes.c_void_p
_I32, _U32, _U64, _SZ = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t


class InstanceDesc(ctypes.Structure):
    _fields_ = [("topology", _I32), ("L", _I32), ("jkind", _I32), ("j_scale", _I32),
                ("couplings", _P), ("n_temps", _I32), ("temps", _P), ("n_replicas", _I32),
                ("icm_ntemps", _I32), ("flags", _U32), ("instance_key", _U32)]


class Stats(ctypes.Structure):
    _fields_ = [(n, _U64) for n in ("sweeps", "metro_accepts", "icm_moves", "icm_nontrivial",
                                    "icm_cluster_sites", "icm_2a_flips", "pt_attempts",
                                    "pt_accepts")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class RunConfig(ctypes.Structure):
    _fields_ = [("threads", _I32), ("sweeps_per_launch", _I32), ("use_graph", _I32),
                ("icm_slots", _I32), ("table_placement", _I32), ("class_threads", _I32 * 4)]


EXPORTS = {
    "icm_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, _P, _SZ, _U32]),
    "icm_destroy": (ctypes.c_int, [_P]),
    "icm_add_instance": (ctypes.c_int, [_P, ctypes.POINTER(InstanceDesc), ctypes.POINTER(_I32)]),
    "icm_remove_instance": (ctypes.c_int, [_P, _I32]),
    "icm_instance_bytes": (_SZ, [ctypes.POINTER(InstanceDesc)]),
    "icm_init_states": (ctypes.c_int, [_P, _I32]),
    "icm_set_states": (ctypes.c_int, [_P, _I32, _P, _U32]),
    "icm_run": (ctypes.c_int, [_P, _P, _I32, _U32]),
    "icm_run_per_instance": (ctypes.c_int, [_P, _P, _I32, _U32]),
    "icm_sync": (ctypes.c_int, [_P]),
    "icm_set_run_config": (ctypes.c_int, [_P, ctypes.POINTER(RunConfig)]),
    "icm_get_run_config": (ctypes.c_int, [_P, ctypes.POINTER(RunConfig)]),
    "icm_read_energies": (ctypes.c_int, [_P, _I32, _P, _P, _SZ]),
    "icm_read_states": (ctypes.c_int, [_P, _I32, _P, _SZ]),
    "icm_read_overlaps": (ctypes.c_int, [_P, _I32, _P, _P, _SZ]),
    "icm_read_labels": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _P, _P, _SZ]),
    "icm_read_stats": (ctypes.c_int, [_P, _I32, ctypes.POINTER(Stats)]),
    "icm_read_observables": (ctypes.c_int, [_P, _I32, _P, _P, _SZ]),
    "icm_read_walkers": (ctypes.c_int, [_P, _I32, _P, _SZ]),
    "icm_sweep_index": (_U32, [_P, _I32]),
    "icm_percolation_smax": (ctypes.c_int, [_P, _I32, _I32, ctypes.c_double, _U32, _U32, _U32, _P]),
    "icm_set_temperatures": (ctypes.c_int, [_P, _I32, _P]),
    "icm_serve_start": (ctypes.c_int, [_P, _I32]),
    "icm_serve_stop": (ctypes.c_int, [_P]),
    "icm_submit": (ctypes.c_int, [_P, ctypes.POINTER(InstanceDesc), _U32, ctypes.POINTER(_U64)]),
    "icm_poll": (ctypes.c_int, [_P, _U64, ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)]),
    "icm_take_result": (ctypes.c_int, [_P, _U64, _P, _P, _SZ, _SZ]),
    "icm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "icm_last_error": (ctypes.c_char_p, [_P]),
    "icm_arena_usage": (ctypes.c_int, [_P, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)]),
}

_lib = None


def load_library():
    """Loads libicm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libicm.so not found at {LIB_PATH}; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype, fn.argtypes = res, args
        _lib = lib
    return _lib


class IcmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def _check(ctx_handle, rc, what):
    if rc != ICM_OK:
        lib = load_library()
        # a busy context (the serving loop runs) does not set its last error
        detail = lib.icm_last_error(ctx_handle) if ctx_handle and rc != ICM_E_BUSY else lib.icm_strerror(rc)
        raise IcmError(rc, f"{what}: {detail.decode() if detail else ''}")


def coupling_kind(couplings):
    return J_F32 if np.asarray(couplings).dtype.kind == "f" else J_INT8


def size_class(n_sites):
    """Size class of a unit, as icm_run groups launches: sites <= 512, <= 1024,
    <= 2048, more."""
    return 0 if n_sites <= 512 else (1 if n_sites <= 1024 else (2 if n_sites <= 2048 else 3))


def launch_threads(n_sites, threads, class_threads=None):
    """Threads per workgroup that icm_run launches for units of n_sites sites
    (the rule the header states): the unit's size-class entry of class_threads
    if set (> 0), else `threads` if set, else for 0 / -1 the per-class default,
    256 up to 512 sites, 512 up to 1024, 1024 above."""
    if class_threads is not None and class_threads[size_class(n_sites)] > 0:
        return int(class_threads[size_class(n_sites)])
    if threads > 0:
        return int(threads)
    return 256 if n_sites <= 512 else (512 if n_sites <= 1024 else 1024)


def make_desc(topology, L, couplings, temps, n_replicas, icm_ntemps,
              flags=FLAG_2A | FLAG_PT, instance_key=0, j_scale=1, jkind=None):
    """InstanceDesc plus the numpy buffers it points into (keep both alive)."""
    if jkind is None:
        jkind = coupling_kind(couplings)
    cj = np.ascontiguousarray(couplings, dtype=np.float32 if jkind == J_F32 else np.int8)
    tp = np.ascontiguousarray(temps, dtype=np.float64)
    d = InstanceDesc(topology, L, jkind, j_scale, cj.ctypes.data, len(tp), tp.ctypes.data,
                     n_replicas, icm_ntemps, flags, instance_key & 0xFFFFFFFF)
    return d, (cj, tp)


def icm_instance_bytes(**kw):
    d, keep = make_desc(**kw)
    return int(load_library().icm_instance_bytes(ctypes.byref(d)))


class Context:
    """One icm_ctx on a torch device, with its arena and stream."""

    def __init__(self, arena_bytes=256 << 20, device=0, seed=150105630, stream=None):
        import torch
        lib = load_library()
        self.torch = torch
        self.device = device
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = _P()
        rc = lib.icm_create(ctypes.byref(h), device, _P(self.stream.cuda_stream),
                            _P(self.arena.data_ptr()), arena_bytes, seed & 0xFFFFFFFF)
        if rc != ICM_OK:
            raise IcmError(rc, "icm_create failed: " + lib.icm_strerror(rc).decode())
        self._lib, self.h = lib, h
        self.meta = {}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self._lib.icm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- instances -----------------------------------------------------------
    def icm_add_instance(self, topology, L, couplings, temps, n_replicas, icm_ntemps,
                         flags=FLAG_2A | FLAG_PT, instance_key=0, j_scale=1, jkind=None):
        d, keep = make_desc(topology, L, couplings, temps, n_replicas, icm_ntemps, flags,
                            instance_key, j_scale, jkind)
        out = _I32()
        _check(self.h, self._lib.icm_add_instance(self.h, ctypes.byref(d), ctypes.byref(out)),
               "icm_add_instance")
        n = {0: L * L, 1: L ** 3, 2: 8 * L * L}[topology]
        self.meta[out.value] = dict(K=len(keep[1]), R=n_replicas, N=n, Kc=icm_ntemps,
                                    jkind=d.jkind, j_scale=j_scale)
        return out.value

    def icm_remove_instance(self, h):
        _check(self.h, self._lib.icm_remove_instance(self.h, h), "icm_remove_instance")
        self.meta.pop(h, None)

    def icm_init_states(self, h):
        _check(self.h, self._lib.icm_init_states(self.h, h), "icm_init_states")

    def icm_set_states(self, h, spins, sweep0=0):
        m = self.meta[h]
        s = np.ascontiguousarray(spins, dtype=np.int8).reshape(m["K"], m["R"], m["N"])
        _check(self.h, self._lib.icm_set_states(self.h, h, _ptr(s), sweep0), "icm_set_states")

    # -- running ---------------------------------------------------------------
    def icm_run(self, handles, n_sweeps):
        hs = np.ascontiguousarray(np.atleast_1d(handles), dtype=np.int32)
        _check(self.h, self._lib.icm_run(self.h, _ptr(hs), len(hs), n_sweeps), "icm_run")

    def icm_run_per_instance(self, handles, n_sweeps):
        hs = np.ascontiguousarray(np.atleast_1d(handles), dtype=np.int32)
        _check(self.h, self._lib.icm_run_per_instance(self.h, _ptr(hs), len(hs), n_sweeps),
               "icm_run_per_instance")

    def icm_sync(self):
        _check(self.h, self._lib.icm_sync(self.h), "icm_sync")

    def icm_set_run_config(self, threads=0, sweeps_per_launch=0, use_graph=0, icm_slots=0,
                           table_placement=0, class_threads=(0, 0, 0, 0)):
        ct = (_I32 * 4)(*[int(x) for x in class_threads])
        cfg = RunConfig(threads, sweeps_per_launch, use_graph, icm_slots, table_placement, ct)
        _check(self.h, self._lib.icm_set_run_config(self.h, ctypes.byref(cfg)), "icm_set_run_config")

    def icm_get_run_config(self):
        cfg = RunConfig()
        _check(self.h, self._lib.icm_get_run_config(self.h, ctypes.byref(cfg)), "icm_get_run_config")
        return dict(threads=cfg.threads, sweeps_per_launch=cfg.sweeps_per_launch,
                    use_graph=cfg.use_graph, icm_slots=cfg.icm_slots,
                    table_placement=cfg.table_placement, class_threads=list(cfg.class_threads))

    # -- readout ---------------------------------------------------------------
    def icm_read_energies(self, h):
        m = self.meta[h]
        raw = np.zeros((m["K"], m["R"]), dtype=np.int64)
        real = np.zeros((m["K"], m["R"]), dtype=np.float64)
        _check(self.h, self._lib.icm_read_energies(self.h, h, _ptr(raw), _ptr(real), raw.size),
               "icm_read_energies")
        return raw, real

    def icm_read_states(self, h):
        m = self.meta[h]
        out = np.zeros((m["K"], m["R"], m["N"]), dtype=np.int8)
        _check(self.h, self._lib.icm_read_states(self.h, h, _ptr(out), out.size), "icm_read_states")
        return out

    def icm_read_walkers(self, h):
        m = self.meta[h]
        out = np.zeros((m["K"], m["R"]), dtype=np.int32)
        _check(self.h, self._lib.icm_read_walkers(self.h, h, _ptr(out), out.size), "icm_read_walkers")
        return out

    def icm_read_overlaps(self, h):
        m = self.meta[h]
        q = np.zeros((m["K"], m["R"] // 2), dtype=np.int32)
        ql = np.zeros_like(q)
        _check(self.h, self._lib.icm_read_overlaps(self.h, h, _ptr(q), _ptr(ql), q.size),
               "icm_read_overlaps")
        return q, ql

    def icm_read_labels(self, h, k, pair):
        m = self.meta[h]
        lab = np.zeros(m["N"], dtype=np.int32)
        seed, nm = _I32(), _I32()
        _check(self.h, self._lib.icm_read_labels(self.h, h, k, pair, _ptr(lab), ctypes.byref(seed),
                                                 ctypes.byref(nm), lab.size), "icm_read_labels")
        return lab, seed.value, nm.value

    def icm_read_stats(self, h):
        st = Stats()
        _check(self.h, self._lib.icm_read_stats(self.h, h, ctypes.byref(st)), "icm_read_stats")
        return st.as_dict()

    def icm_read_observables(self, h):
        """(sums [32][K][R/2][4] int64, counts [32] int64); see icm_read_observables."""
        m = self.meta[h]
        sums = np.zeros((OBS_BINS, m["K"], m["R"] // 2, OBS_FIELDS), dtype=np.int64)
        counts = np.zeros(OBS_BINS, dtype=np.int64)
        _check(self.h, self._lib.icm_read_observables(self.h, h, _ptr(sums), _ptr(counts), sums.size),
               "icm_read_observables")
        return sums, counts

    def icm_sweep_index(self, h):
        return int(self._lib.icm_sweep_index(self.h, h))

    def icm_set_temperatures(self, h, temps):
        t = np.ascontiguousarray(temps, dtype=np.float64)
        if t.shape != (self.meta[h]["K"],):
            raise ValueError("one temperature per temperature slot of the instance")
        _check(self.h, self._lib.icm_set_temperatures(self.h, h, _ptr(t)), "icm_set_temperatures")

    def icm_percolation_smax(self, topology, L, p, n_samples, sample0=0, key=0, out=None):
        """Largest-cluster sizes of n_samples random site configurations
        (icm_percolation_smax); returns a device int32 tensor [n_samples],
        written on the context stream."""
        t = self.torch
        if out is None:
            out = t.empty(n_samples, dtype=t.int32, device=self.arena.device)
        if out.dtype != t.int32 or not out.is_contiguous() or out.numel() < n_samples \
                or out.device != self.arena.device:
            raise ValueError("out must be a contiguous int32 tensor on the context's device")
        _check(self.h, self._lib.icm_percolation_smax(self.h, topology, L, float(p), sample0, n_samples, key,
                                                      ctypes.c_void_p(out.data_ptr())),
               "icm_percolation_smax")
        return out

    def icm_arena_usage(self):
        used, total = _SZ(), _SZ()
        _check(self.h, self._lib.icm_arena_usage(self.h, ctypes.byref(used), ctypes.byref(total)),
               "icm_arena_usage")
        return used.value, total.value

    # -- serving ---------------------------------------------------------------
    def icm_serve_start(self, sweeps_per_block=256):
        _check(self.h, self._lib.icm_serve_start(self.h, sweeps_per_block), "icm_serve_start")

    def icm_serve_stop(self):
        _check(self.h, self._lib.icm_serve_stop(self.h), "icm_serve_stop")

    def icm_submit(self, n_sweeps, **desc_kw):
        d, keep = make_desc(**desc_kw)
        t = _U64()
        _check(self.h, self._lib.icm_submit(self.h, ctypes.byref(d), n_sweeps, ctypes.byref(t)),
               "icm_submit")
        return t.value

    def icm_poll(self, ticket):
        done, lat = _I32(), ctypes.c_double()
        _check(self.h, self._lib.icm_poll(self.h, ticket, ctypes.byref(done), ctypes.byref(lat)),
               "icm_poll")
        return bool(done.value), lat.value

    def icm_take_result(self, ticket, K, R, N):
        e = np.zeros((K, R), dtype=np.int64)
        s = np.zeros((K, R, N), dtype=np.int8)
        _check(self.h, self._lib.icm_take_result(self.h, ticket, _ptr(e), _ptr(s), e.size, s.size),
               "icm_take_result")
        return e, s

"""Host-side checks of the C-ABI library (no GPU needed): every symbol that
include/icm.h declares is exported, and descriptor validation / sizing works."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1501_05630_amd import icm, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "icm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(icm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = icm.load_library()
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(icm.EXPORTS), set(names) ^ set(icm.EXPORTS)


def test_strerror_codes():
    lib = icm.load_library()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.icm_strerror(code)
    assert lib.icm_last_error(None) == b"null context"


def _bytes(**kw):
    base = dict(topology=inputs.CUBIC3D, L=8, couplings=np.zeros((512, 3), np.float32),
                temps=inputs.geometric_temps(0.2, 2.0, 20), n_replicas=4, icm_ntemps=14)
    base.update(kw)
    return icm.icm_instance_bytes(**base)


def test_instance_bytes_and_validation():
    n = _bytes()
    # spins 20 quads x 512 sites x 4 B dominate; couplings [N][6] float
    assert 40960 + 512 * 6 * 4 <= n < 80000
    assert _bytes(L=7) == 0                                    # odd L
    assert _bytes(n_replicas=3) == 0                           # odd R
    assert _bytes(icm_ntemps=21) == 0                          # K_c > K
    assert _bytes(temps=np.array([1.0, 0.5])) == 0             # not ascending
    assert _bytes(temps=np.array([0.0, 0.5])) == 0             # T = 0
    bad = np.zeros((512, 3), np.float32); bad[3, 1] = np.nan
    assert _bytes(couplings=bad) == 0                          # non-finite J
    bad[3, 1] = 100.0
    assert _bytes(couplings=bad) == 0                          # |J| > 64
    assert _bytes(L=18) == 0                                   # N > 4096 resident limit
    # chimera: slots that leave the grid must be zero
    Jc = inputs.int_couplings(inputs.CHIMERA, 3, inputs.make_rng(0, 0))
    ok = icm.icm_instance_bytes(topology=inputs.CHIMERA, L=3, couplings=Jc, temps=[0.5, 1.0],
                                n_replicas=2, icm_ntemps=2, j_scale=3)
    assert ok > 0
    Jc[8, 20] = 1
    assert icm.icm_instance_bytes(topology=inputs.CHIMERA, L=3, couplings=Jc, temps=[0.5, 1.0],
                                  n_replicas=2, icm_ntemps=2, j_scale=3) == 0


def test_integer_pt_table_too_long_is_rejected():
    # temperatures this close would need a PT threshold table longer than 2^16
    J = np.ones((16, 2), np.int8)
    assert icm.icm_instance_bytes(topology=inputs.SQUARE2D, L=4, couplings=J,
                                  temps=[1.0, 1.0 + 1e-6], n_replicas=2, icm_ntemps=0) == 0
    assert icm.icm_instance_bytes(topology=inputs.SQUARE2D, L=4, couplings=J,
                                  temps=[1.0, 1.0 + 1e-6], n_replicas=2, icm_ntemps=0,
                                  flags=icm.FLAG_2A) > 0


def test_create_without_device_fails_cleanly():
    lib = icm.load_library()
    h = ctypes.c_void_p()
    # null arena -> invalid, before any device call
    assert lib.icm_create(ctypes.byref(h), 0, None, None, 1 << 20, 1) == icm.ICM_E_INVALID


def test_binding_refuses_missing_library(monkeypatch, tmp_path):
    monkeypatch.setattr(icm, "_lib", None)
    monkeypatch.setattr(icm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        icm.load_library()

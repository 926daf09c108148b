"""Oracle pins for the counter-based generator (Philox4x32-10, Salmon et al. SC'11).

The oracle's Philox is checked against rocRAND's philox4x32_10 engine (an
independent third-party implementation, compiled here for the host) and
against basic statistical properties.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as orc

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rr")
    subprocess.check_call([hipcc, "-O1", "--offload-arch=gfx950",
                           os.path.join(HERE, "support", "rocrand_philox_ref.cpp"), "-o", exe],
                          cwd=d)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_matches_rocrand_engine(rocrand_ref):
    rng = np.random.default_rng(7)
    rows = rng.integers(0, 2 ** 32, size=(4000, 6), dtype=np.uint64)
    # The engine is positioned through a 64-bit word offset 4*(c0 + 2^32 c1),
    # so c1 stays below 2^30 here (c1 is the sweep index in the library).
    rows[:, 1] >>= 2
    rows[:8] = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0], [0, 0, 0, 1, 0, 0],
                [0xFFFFFFFF, 0x3FFFFFFF] + [0xFFFFFFFF] * 4, [5, 7, 9, 2, 150105630, 3], [0, 1, 2, 3, 4, 5],
                [7, 4095, 19, 0, 150105630, 1023], [1151, 16383, 14, 0, 150105630, 511]]
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    mine = np.array([orc.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint64)
    assert np.array_equal(mine, ref)


def _stream(n_blocks, key=(150105630, 1)):
    return np.concatenate([orc.philox4x32_10([i, 3, 5, 0], key) for i in range(n_blocks)])


def test_uniformity_and_bit_balance():
    w = _stream(1 << 15)  # 131072 words
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    exp = len(w) / 256
    chi2 = float(np.sum((counts - exp) ** 2 / exp))
    assert 150 < chi2 < 380  # 255 dof, ~5 sigma window
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(len(w)))


def test_avalanche_on_counter_and_key_bits():
    base_c, base_k = np.array([11, 22, 33, 44], np.uint32), np.array([55, 66], np.uint32)
    ref = orc.philox4x32_10(base_c, base_k)
    flips = []
    for word in range(4):
        for bit in range(32):
            c = base_c.copy(); c[word] ^= np.uint32(1 << bit)
            flips.append(sum(bin(int(a ^ b)).count("1") for a, b in zip(ref, orc.philox4x32_10(c, base_k))))
    for word in range(2):
        for bit in range(32):
            k = base_k.copy(); k[word] ^= np.uint32(1 << bit)
            flips.append(sum(bin(int(a ^ b)).count("1") for a, b in zip(ref, orc.philox4x32_10(base_c, k))))
    flips = np.array(flips)
    assert abs(flips.mean() - 64) < 2.5 and flips.min() > 35

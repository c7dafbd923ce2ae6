"""Oracle Philox4x32-10 pins.

The oracle's generator is checked against rocRAND's own Philox4x32-10 (an
independent implementation, compiled here from its public header and run on the
host), and by statistical properties every sound 128-bit block cipher output has.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

PROBE_SRC = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_probe.cpp")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("probe") / "probe")
    subprocess.run([hipcc, "-O1", "-o", exe, PROBE_SRC], check=True, capture_output=True)
    return exe


def _rocrand_blocks(exe, key, ctr, n):
    seed = (int(key[1]) << 32) | int(key[0])
    out = subprocess.run([exe, str(seed)] + [str(int(c)) for c in ctr] + [str(n)],
                         check=True, capture_output=True, text=True).stdout.split()
    return np.array([int(v) for v in out], dtype=np.uint64).astype(np.uint32).reshape(n, 4)


def test_philox_matches_rocrand(orc, probe):
    rng = np.random.default_rng(11)
    cases = [((0, 0), (0, 0, 0, 0)), ((1, 0), (0, 0, 0, 0)), ((0xFFFFFFFF, 0xFFFFFFFF), (0xFFFFFFF0, 7, 0, 0))]
    for _ in range(6):
        key = tuple(int(v) for v in rng.integers(0, 2**32, 2))
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        ctr[1] >>= 3  # rocRAND's 64-bit offset holds 4 * (c1:c0); keep it in range
        cases.append((key, tuple(ctr)))
    for key, ctr in cases:
        ref = _rocrand_blocks(probe, key, ctr, 4)
        for i in range(4):
            c = list(ctr)
            # consecutive blocks advance the 64-bit counter held in words (0, 1)
            lo = (c[0] + i) & 0xFFFFFFFF
            carry = (c[0] + i) >> 32
            c[0], c[1] = lo, (c[1] + carry) & 0xFFFFFFFF
            got = orc.philox(c, key)
            assert np.array_equal(got, ref[i]), (key, c, got, ref[i])


def _blocks(orc, n, key=(5, 9)):
    return np.array([orc.philox((i, 3, 1, 0), key) for i in range(n)], dtype=np.uint32)


def test_philox_bit_balance(orc):
    w = _blocks(orc, 4096).reshape(-1)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    sigma = 0.5 / np.sqrt(w.size)
    assert np.all(np.abs(frac - 0.5) < 5 * sigma), frac


def test_philox_avalanche(orc):
    rng = np.random.default_rng(3)
    flips = []
    for _ in range(64):
        key = [int(v) for v in rng.integers(0, 2**32, 2)]
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        base = orc.philox(ctr, key)
        word, bit = int(rng.integers(0, 6)), int(rng.integers(0, 32))
        c2, k2 = list(ctr), list(key)
        if word < 4:
            c2[word] ^= 1 << bit
        else:
            k2[word - 4] ^= 1 << bit
        out = orc.philox(c2, k2)
        flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, out)))
    assert 58 < np.mean(flips) < 70, np.mean(flips)


def test_philox_byte_uniformity(orc):
    from scipy.stats import chisquare

    w = _blocks(orc, 4096, key=(123, 456)).reshape(-1)
    by = np.frombuffer(w.tobytes(), dtype=np.uint8)
    counts = np.bincount(by, minlength=256)
    assert chisquare(counts).pvalue > 1e-4

"""Pins of the oracle's Philox generators (oracle/philox.py)."""
import os

import numpy as np
import pytest

from oracle.philox import philox4x32_10, philox4x64_10, philox4x32_10_vec

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox4x32_known_answers(ctr, key, out):
    assert philox4x32_10(ctr, key) == out


def test_philox4x32_vectorised_matches_scalar():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 2**32, size=(4, 50), dtype=np.uint64)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    v = philox4x32_10_vec(c[0], c[1], c[2], c[3], k0, k1)
    for i in range(50):
        ref = philox4x32_10([int(c[q, i]) for q in range(4)], [k0, k1])
        assert [int(v[q][i]) for q in range(4)] == ref
    # also the KAT through the vector path
    for ctr, key, out in _kat():
        v = philox4x32_10_vec(*[np.array([x], dtype=np.uint64) for x in ctr], *key)
        assert [int(x[0]) for x in v] == out


@pytest.mark.parametrize("key", [0, 1, 12345, 2**64 - 1, 0xDEADBEEFCAFEF00D1234])
def test_philox4x64_matches_numpy(key):
    # numpy's Philox bit generator is Philox4x64-10; it advances the 256-bit
    # counter by one before producing each block of four words.
    key &= (1 << 128) - 1
    k = [key & (2**64 - 1), key >> 64]
    for ctr0 in [0, 7, 2**64 - 2]:
        bg = np.random.Philox(key=key, counter=ctr0)
        raw = [int(x) for x in bg.random_raw(8)]
        c1 = ctr0 + 1
        c2 = ctr0 + 2
        ref = philox4x64_10([c1 & (2**64 - 1), c1 >> 64, 0, 0], k) + \
            philox4x64_10([c2 & (2**64 - 1), c2 >> 64, 0, 0], k)
        assert raw == ref

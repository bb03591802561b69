"""Oracle pins: the counter-based generator and the uniform/normal mappings.

Philox4x64-10 is checked bit for bit against numpy's independent
implementation (numpy increments its 256-bit counter before each block, so
block(c) is numpy's first output after setting counter c - 1).
"""
import numpy as np
import pytest

from oracle import oracle as O


def numpy_block(ctr, key):
    c = [int(x) for x in ctr]
    # 256-bit little-endian decrement
    val = sum(w << (64 * k) for k, w in enumerate(c))
    val = (val - 1) % (1 << 256)
    prev = [(val >> (64 * k)) & ((1 << 64) - 1) for k in range(4)]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(prev, dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_matches_numpy_random_counters():
    rng = np.random.default_rng(1234)
    for _ in range(2000):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] |= int(rng.integers(0, 2)) << 63
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert list(O.philox(ctr, key)) == list(numpy_block(ctr, key))


def test_philox_matches_numpy_method_counters():
    # the counter layout the method uses: (ion, step, purpose, sub), key (seed, system)
    for ion in (0, 1, 2, 1999, 1 << 20):
        for step in (0, 1, 199, 19999):
            for purpose in range(4):
                for sub in (0, 1, 7):
                    ctr = [ion, step, purpose, sub]
                    key = [1, 0]
                    assert list(O.philox(ctr, key)) == list(numpy_block(ctr, key))


def test_uniform_open_interval_and_exact():
    assert O.uniform(0) == 0.5 * 2.0**-52
    assert O.uniform(2**64 - 1) == 1.0 - 0.5 * 2.0**-52
    assert 0.0 < O.uniform(2**64 - 1) < 1.0
    # exactness: k + 1/2 is representable for every 52-bit k
    rng = np.random.default_rng(5)
    for w in rng.integers(0, 2**63, size=1000, dtype=np.int64):
        w = int(w) * 2 + 1
        k = w >> 12
        assert O.uniform(w) == (k + 0.5) / 2.0**52


def test_uniform_is_uniform():
    rng = np.random.default_rng(9)
    ws = rng.integers(0, 2**63, size=20000, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    us = np.array([O.uniform(int(w)) for w in ws])
    from scipy import stats
    assert stats.kstest(us, "uniform").pvalue > 1e-4

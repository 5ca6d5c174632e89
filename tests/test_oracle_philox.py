"""Pin: the oracle's Philox4x64-10 block function equals numpy.random.Philox
bit for bit (numpy implements the same published generator of Salmon et
al., SC'11).  numpy advances its 256-bit counter before producing a block, so
the block for counter c is the first block numpy returns when started at
c - 1."""
import numpy as np
import pytest

import oracle


def _numpy_block(counter, key):
    c = [int(x) for x in counter]
    v = sum(x << (64 * i) for i, x in enumerate(c))
    v = (v - 1) % (1 << 256)
    prev = np.array([(v >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev)
    return bg.random_raw(4)


def test_philox_matches_numpy_random_counters():
    rng = np.random.default_rng(1234)
    for _ in range(2000):
        ctr = rng.integers(0, 2**64, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**64, size=2, dtype=np.uint64)
        assert np.array_equal(oracle.philox4x64(ctr, key), _numpy_block(ctr, key))


@pytest.mark.parametrize("ctr", [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 7], [2**64 - 1, 0, 0, 0],
                                 [5, (3 << 32) | 17, 12, 6]])
def test_philox_matches_numpy_structured_counters(ctr):
    key = [987654321, 0]
    assert np.array_equal(oracle.philox4x64(ctr, key), _numpy_block(ctr, key))


def test_u01_is_53_bit():
    assert oracle.u01(0) == 0.0
    assert oracle.u01(2**64 - 1) == 1.0 - 2.0**-53
    assert oracle.u01(1 << 11) == 2.0**-53

"""Pins of the oracle's Philox4x64-10 against numpy's library implementation."""
import numpy as np
import pytest

from oracle import philox


def _numpy_block(counter, key):
    # numpy's Philox increments the counter before producing a block, so the
    # first four outputs for state counter c are the block of counter c + 1.
    c = [int(v) for v in counter]
    c0 = (c[0] - 1) % (1 << 64)
    borrow = c[0] == 0
    cc = [c0, c[1], c[2], c[3]]
    i = 1
    while borrow and i < 4:
        cc[i] = (cc[i] - 1) % (1 << 64)
        borrow = c[i] == 0
        i += 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(cc, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("seed", range(6))
def test_block_matches_numpy(seed):
    rng = np.random.Generator(np.random.PCG64(1234 + seed))
    for _ in range(20):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        assert list(philox.philox4x64_10(ctr, key)) == _numpy_block(ctr, key)


def test_zero_block_known_answer():
    # Published known-answer vector of Philox4x64-10 for zero counter and key.
    assert [hex(v) for v in philox.philox4x64_10((0, 0, 0, 0), (0, 0))] == [
        "0x16554d9eca36314c", "0xdb20fe9d672d0fdc", "0xd7e772cee186176b", "0x7e68b68aec7ba23b"]
    assert list(philox.philox4x64_10((0, 0, 0, 0), (0, 0))) == _numpy_block((0, 0, 0, 0), (0, 0))


def test_uniform_open_interval():
    assert philox.word_to_uniform(0) == 0.5 * 2.0 ** -53
    assert philox.word_to_uniform((1 << 64) - 1) == 1.0 - 0.5 * 2.0 ** -53
    us = [philox.uniform(3, 1, t, 2, 0, k) for t in range(10) for k in range(50)]
    assert all(0.0 < u < 1.0 for u in us)
    assert abs(np.mean(us) - 0.5) < 0.05

"""Pins of the oracle's Philox4x64-10 stream against NumPy's own Philox bit
generator, and of the uniform and normal transforms."""

import math

import numpy as np
import pytest

from oracle import philox as op


def _numpy_block(counter, key):
    """NumPy's Philox advances its 256-bit counter before producing a block,
    so the block for counter c comes from a generator started at c - 1."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(counter)) - 1
    c %= 1 << 256
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                         key=np.array([int(key[0]), int(key[1])], dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (14652, 3)),
    ((7, 1, 0, 0), (2**64 - 1, 2**63 + 5)),
    ((123456789, 0, 2**40, 0), (0xDEADBEEF, 17)),
    ((2**64 - 1, 2**64 - 1, 5, 9), (1, 2)),
])
def test_philox_matches_numpy(counter, key):
    ours = op.philox4x64(np.array([counter], dtype=np.uint64), key)[0]
    np.testing.assert_array_equal(ours, _numpy_block(counter, key))


def test_blocks_match_numpy_sequence():
    seed, chain, it = 2024, 5, 11
    ours = op.blocks(seed, chain, it, op.STREAM_MOMENTUM, 6)
    for b in range(6):
        np.testing.assert_array_equal(ours[b], _numpy_block((it, op.STREAM_MOMENTUM, b, 0), (seed, chain)))


def test_uniform_map_open_interval():
    w = np.array([0, 1 << 12, (1 << 64) - 1], dtype=np.uint64)
    u = op.to_uniform(w)
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.5 * 2.0 ** -52
    assert u[2] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_normals_are_standard_normal():
    from scipy import stats
    z = np.concatenate([op.normals(3, c, 0, 25001) for c in range(4)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_normals_box_muller_pairs():
    """Each pair shares a radius sqrt(-2 ln u) and its angle is 2 pi u'."""
    seed, chain, it = 1, 2, 3
    z = op.normals(seed, chain, it, 8).reshape(2, 4)
    u = op.to_uniform(_numpy_block((it, 0, 0, 0), (seed, chain)))
    for j in (0, 2):
        r = math.sqrt(-2 * math.log(u[j]))
        assert math.isclose(math.hypot(z[0, j], z[0, j + 1]), r, rel_tol=1e-14)
        ang = math.atan2(z[0, j + 1], z[0, j]) % (2 * math.pi)
        assert math.isclose(ang, 2 * math.pi * u[j + 1], rel_tol=1e-12)


def test_streams_and_chains_differ():
    a = op.normals(1, 0, 0, 16)
    assert not np.allclose(a, op.normals(1, 1, 0, 16))
    assert not np.allclose(a, op.normals(1, 0, 1, 16))
    assert not np.allclose(a, op.normals(2, 0, 0, 16))
    assert op.metropolis_uniform(1, 0, 0) != op.to_uniform(op.blocks(1, 0, 0, 0, 1))[0, 0]

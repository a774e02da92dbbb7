"""Pins of the oracle's two networks by brute force.

* Bitonic sorting network: the 0-1 principle (a comparator network sorts
  every input iff it sorts every 0/1 input), exhaustively for n <= 16, and
  random inputs against numpy's sort.
* Shift networks: compaction against a stable partition and expansion
  against a direct scatter, for every keep-mask of up to 12 positions."""
import itertools

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_bitonic_zero_one_principle(n):
    for bits in range(1 << n):
        a = np.array([(bits >> i) & 1 for i in range(n)], dtype=np.uint64)
        out = O.bitonic_sort(a)
        z = int(n - a.sum())
        assert (out[:z] == 0).all() and (out[z:] == 1).all(), bits


@pytest.mark.parametrize("n", [2, 32, 1024, 1 << 16])
def test_bitonic_random_against_sort(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, 2**64, size=n, dtype=np.uint64)
    assert (O.bitonic_sort(a) == np.sort(a)).all()
    small = rng.integers(0, 4, size=n, dtype=np.uint64)  # many ties
    assert (O.bitonic_sort(small) == np.sort(small)).all()


def test_bitonic_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        O.bitonic_sort(np.arange(6, dtype=np.uint64))


@pytest.mark.parametrize("m", range(1, 13))
def test_compaction_all_masks(m):
    payload = np.arange(100, 100 + m, dtype=np.uint32)
    for mask in range(1 << m):
        keep = np.array([(mask >> i) & 1 for i in range(m)], dtype=np.uint8)
        out, rc = O.compact(keep, payload)
        assert rc == 0
        kept = payload[keep == 1]
        assert (out[:kept.size] == kept).all()
        assert (out[kept.size:] == O.NONE32).all()


@pytest.mark.parametrize("m", range(2, 13))
def test_expansion_all_target_sets(m):
    for mask in range(1 << m):
        tgt = np.array([i for i in range(m) if (mask >> i) & 1], dtype=np.uint32)
        n = tgt.size
        payload = np.arange(7, 7 + n, dtype=np.uint32)
        out, rc = O.expand(tgt, payload, m)
        assert rc == 0
        want = np.full(m, O.NONE32, dtype=np.uint32)
        want[tgt] = payload  # direct scatter
        assert (out == want).all(), (m, mask)


def test_expansion_inverts_compaction_random():
    rng = np.random.default_rng(3)
    for m in (100, 4097, 1 << 15):
        keep = (rng.random(m) < 0.4).astype(np.uint8)
        payload = rng.integers(0, 2**31, m).astype(np.uint32)
        comp, rc = O.compact(keep, payload)
        assert rc == 0
        n = int(keep.sum())
        tgt = np.nonzero(keep)[0].astype(np.uint32)
        back, rc = O.expand(tgt, comp[:n], m)
        assert rc == 0
        want = np.where(keep == 1, payload, O.NONE32)
        assert (back == want).all()


def test_expansion_detects_invalid_targets():
    # targets not strictly increasing cannot be routed without a collision
    out, rc = O.expand(np.array([1, 1], np.uint32), np.array([5, 6], np.uint32), 4)
    assert rc != 0

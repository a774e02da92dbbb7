"""In-batch dedup under adversarial keys, against the oracle bit for bit.

The dedup kernel splits a batch into 64 partitions by the top bits of a
mix of the key, and folds each partition of up to 1024 commands through an
LDS hash table indexed by the low bits of the same mix (linear probing).
The mix is a bijection, so keys can be chosen by their mixed value: here
hundreds of distinct keys land in one partition and one hash slot (probe
chains as long as the table allows), and batches put more than 1024
commands into one partition (the sort path).
"""
import numpy as np
import pytest

from gpu_util import Twin

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1
MUL = 0xFF51AFD7ED558CCD
MUL_INV = pow(MUL, -1, 1 << 64)


def mix(k):
    x = k ^ (k >> 33)
    x = (x * MUL) & M64
    return x ^ (x >> 33)


def unmix(x):
    y = x ^ (x >> 33)
    y = (y * MUL_INV) & M64
    return y ^ (y >> 33)


def crafted_keys(n, part, slot, seed):
    """n distinct keys whose mix has top 6 bits `part` and low 11 bits `slot`."""
    rng = np.random.default_rng(seed)
    mids = np.unique(rng.integers(0, 1 << 40, 2 * n))[:n]
    assert mids.size == n
    out = []
    for m in mids.tolist():
        x = (part << 58) | (m << 11) | slot
        k = unmix(x)
        assert mix(k) == x
        out.append(k)
    return np.array(out, dtype=np.uint64)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


def _batch(rng, keys, q, vs, hot=None):
    pick = keys[rng.integers(0, keys.size, q)]
    if hot is not None:
        h = rng.random(q) < 0.4
        pick[h] = hot
    ops = rng.choice([0, 1, 2], size=q, p=[0.55, 0.3, 0.15]).astype(np.uint8)
    return ops, pick.astype(np.uint64), rng.integers(0, 256, (q, vs), dtype=np.uint8)


def _check(t, ops, keys, vals):
    (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
    assert rc_o == 0 and rc_g == 0 and st == 0, (rc_o, rc_g, st)
    assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o)


@pytest.mark.parametrize("observable", [0, 1])
def test_one_partition_one_hash_slot(observable):
    """Up to 1000 commands over 600 keys that share a partition and a hash
    slot (one probe chain through most of the table), with a hot key."""
    same = crafted_keys(600, 5, 123, 1)
    other = crafted_keys(200, 5, 2047, 2)  # the chain wraps past the table's end
    present = np.concatenate([same[:500], other[:150]])
    t = Twin(4096, 8, observable=observable)
    rng = np.random.default_rng(7)
    vals = rng.integers(0, 256, (present.size, 8), dtype=np.uint8)
    assert t.build(present, vals) == (0, 0, 0)
    pool = np.concatenate([same, other])  # absent keys too
    for b, q in enumerate([1000, 64, 1, 700, 1024, 333]):
        ops, keys, v = _batch(rng, pool, q, 8, hot=int(same[3]) if b % 2 == 0 else None)
        _check(t, ops, keys, v)
    t.assert_same_state()


def test_partition_over_1024_commands():
    """Batches that put 1025 .. 4096 commands into one partition (the
    partition is sorted instead of hashed), beside ordinary partitions."""
    same = crafted_keys(900, 9, 7, 3)
    t = Twin(8192, 16)
    rng = np.random.default_rng(11)
    vals = rng.integers(0, 256, (700, 16), dtype=np.uint8)
    assert t.build(same[:700], vals) == (0, 0, 0)
    for q in (1025, 2048, 4096):
        ops, keys, v = _batch(rng, same, q, 16, hot=int(same[0]))
        _check(t, ops, keys, v)
    # a batch mixing one huge partition with keys spread over all others
    spread = np.array([unmix((p << 58) | (int(r) << 11) | int(r & 2047)) for p, r in
                       zip(rng.integers(0, 64, 600).tolist(), rng.integers(0, 1 << 40, 600).tolist())],
                      dtype=np.uint64)
    ops, keys, v = _batch(rng, same, 3000, 16)
    ops2, keys2, v2 = _batch(rng, spread, 1000, 16)
    _check(t, np.concatenate([ops, ops2]), np.concatenate([keys, keys2]), np.concatenate([v, v2]))
    t.assert_same_state()

"""Seeded random mixes of batch sizes against the oracle, bit for bit.

Sizes are drawn from one command (the one-workgroup kernel), small batches
(pages written by their own rebuild), and large batches (pages rebuilt into
alternate halves of the outbox and sent during the next batch), in random
order with no flush between them, on both stores, plain and sealed, over a
key pool with hot keys, absent keys and inserts of new keys.  Every answer
is compared, and the whole state at the end (store, tags and write counts
of a sealed map, HBM bins, loads, stash, position map, trace).
"""
import numpy as np
import pytest

import synth
from gpu_util import Twin, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


def _size(rng):
    kind = rng.integers(0, 4)
    if kind == 0:
        return 1
    if kind == 1:
        return int(rng.integers(2, 256))
    if kind == 2:
        return int(rng.integers(256, 1200))
    return int(rng.integers(1200, 4097))


@pytest.mark.parametrize("observable,seal", [(0, False), (1, False), (0, True)])
def test_random_batch_sizes(observable, seal):
    t = Twin(6144, 16, observable=observable, seal=seal)
    k, v = workload(4500, 16, 7100 + observable + 2 * seal)
    assert t.build(k, v) == (0, 0, 0)
    fresh = synth.keys(1500, 7101, offset=10**9)
    hot = k[:24]
    rng = np.random.default_rng(7102 + observable + 2 * seal)
    for b in range(100):
        q = _size(rng)
        r = rng.random(q)
        keys = np.where(r < 0.3, hot[rng.integers(0, hot.size, q)],
                        np.where(r < 0.9, k[rng.integers(0, k.size, q)], fresh[rng.integers(0, fresh.size, q)]))
        # inserts of new keys only while the map has room (deletes free room again)
        ops = rng.choice([0, 1, 2], size=q, p=[0.6, 0.28, 0.12]).astype(np.uint8)
        if t.o.live > 5600:
            ops[(r >= 0.9) & (ops == 1)] = 0
        vals = rng.integers(0, 256, (q, 16), dtype=np.uint8)
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys.astype(np.uint64), vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, (b, q, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), (b, q)
    t.assert_same_state()

"""The write of a batch's rebuilt observable pages during the next batch.

Large batches on a pinned host store rebuild their pages in HBM, and the
next batch's fetch writes them to the store while it reads its own pages;
that fetch takes any page the previous batch rebuilt from HBM.  These tests
run batches back to back with no flush between them (large and small ones,
plain and sealed maps, one-map and many-map calls, explicit flushes), and
compare every answer and the final state (store, tags, write counts, HBM
bins, loads, stash, position map, trace) with the oracle, bit for bit.
"""
import numpy as np
import pytest

import synth
from gpu_util import Twin, dev_u64, dev_u8, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


def _batch(rng, keys, fresh, q, vs):
    r = rng.random(q)
    pick = np.where(r < 0.9, keys[rng.integers(0, keys.size, q)], fresh[rng.integers(0, fresh.size, q)])
    ops = rng.choice([0, 1, 2], size=q, p=[0.6, 0.3, 0.1]).astype(np.uint8)
    ops[(r >= 0.9) & (ops == 1)] = 0  # inserts only of present keys: the size stays as built
    return ops, pick.astype(np.uint64), rng.integers(0, 256, (q, vs), dtype=np.uint8)


def _launch(t, ops, keys, vals):
    """One batch on the GPU map without any flush or status call."""
    import torch

    q = len(ops)
    out = torch.zeros((q, t.vs), dtype=torch.uint8, device="cuda")
    st = torch.zeros(q, dtype=torch.uint8, device="cuda")
    rc = t.g.access(dev_u8(ops), dev_u64(keys), dev_u8(vals), out, st)
    return rc, out, st


@pytest.mark.parametrize("seal", [False, True])
def test_back_to_back_batches(seal):
    import torch

    t = Twin(8192, 16, seal=seal)
    k, v = workload(7000, 16, 4100 + seal)
    assert t.build(k, v) == (0, 0, 0)
    fresh = synth.keys(500, 4200, offset=10**9)
    rng = np.random.default_rng(17 + seal)
    sizes = [3000, 2000, 600, 40, 1, 2500, 256, 255, 4096, 3000, 700, 300]
    for b, q in enumerate(sizes):
        ops, keys, vals = _batch(rng, k, fresh, q, 16)
        rc_o, vo_o, st_o = t.o.access(ops, keys, vals)
        rc, out, st = _launch(t, ops, keys, vals)
        torch.cuda.synchronize()  # answers only: the pages may still wait to be written
        assert rc_o == 0 and rc == 0, (b, rc_o, rc)
        assert np.array_equal(st.cpu().numpy(), st_o) and np.array_equal(out.cpu().numpy(), vo_o), b
        if b == 5:
            assert t.g.flush() == 0
    t.assert_same_state()


def test_deferred_pages_then_many_map_calls():
    import torch
    import paper_2509_01742_amd as B

    twins, ks = [], []
    for j, seal in enumerate((False, True, False)):
        t = Twin(4096, 8, seal=seal, key=bytes((5 * j + i) & 255 for i in range(32)))
        k, v = workload(3500, 8, 4300 + j)
        assert t.build(k, v) == (0, 0, 0)
        twins.append(t)
        ks.append(k)
    fresh = synth.keys(300, 4400, offset=10**9)
    rng = np.random.default_rng(5)
    for rnd in range(3):
        # one large batch per map on its own (pages left for the next batch) ...
        for j, t in enumerate(twins):
            ops, keys, vals = _batch(rng, ks[j], fresh, 1500, 8)
            rc_o, vo_o, st_o = t.o.access(ops, keys, vals)
            rc, out, st = _launch(t, ops, keys, vals)
            torch.cuda.synchronize()
            assert rc_o == 0 and rc == 0
            assert np.array_equal(st.cpu().numpy(), st_o) and np.array_equal(out.cpu().numpy(), vo_o)
        # ... then one many-map call over all of them, which writes those pages first
        batches, host = [], []
        for j, t in enumerate(twins):
            q = int(rng.integers(200, 1200))
            ops, keys, vals = _batch(rng, ks[j], fresh, q, 8)
            batches.append((dev_u8(ops), dev_u64(keys), dev_u8(vals),
                            torch.zeros((q, 8), dtype=torch.uint8, device="cuda"),
                            torch.zeros(q, dtype=torch.uint8, device="cuda")))
            host.append((ops, keys, vals))
        assert B.access_many([t.g for t in twins], batches) == 0
        torch.cuda.synchronize()
        for j, t in enumerate(twins):
            rc_o, vo_o, st_o = t.o.access(*host[j])
            assert rc_o == 0
            assert np.array_equal(batches[j][3].cpu().numpy(), vo_o)
            assert np.array_equal(batches[j][4].cpu().numpy(), st_o)
    for t in twins:
        assert t.g.status() == 0
        t.assert_same_state()


def test_alternating_halves_with_hot_keys():
    """Batches that rebuild into alternate halves of the outbox (and small
    ones that write the store themselves) over a few hot keys, so that
    consecutive batches rebuild the same pages while the previous batch's
    are still being sent; no flush until the end."""
    import torch

    t = Twin(8192, 16)
    k, v = workload(7500, 16, 4500)
    assert t.build(k, v) == (0, 0, 0)
    hot = k[:40]
    rng = np.random.default_rng(4501)
    sizes = [4096, 4096, 300, 255, 4096, 1, 2048, 256, 4096, 4096, 100, 4096]
    for b, q in enumerate(sizes):
        pick = np.where(rng.random(q) < 0.5, hot[rng.integers(0, hot.size, q)], k[rng.integers(0, k.size, q)])
        ops = rng.choice([0, 1, 2], size=q, p=[0.5, 0.4, 0.1]).astype(np.uint8)
        vals = rng.integers(0, 256, (q, 16), dtype=np.uint8)
        rc_o, vo_o, st_o = t.o.access(ops, pick.astype(np.uint64), vals)
        rc, out, st = _launch(t, ops, pick.astype(np.uint64), vals)
        torch.cuda.synchronize()
        assert rc_o == 0 and rc == 0, (b, rc_o, rc)
        assert np.array_equal(st.cpu().numpy(), st_o) and np.array_equal(out.cpu().numpy(), vo_o), b
    t.assert_same_state()

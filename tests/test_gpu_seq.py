"""Batch sequences (bolt_access_seq): one call with several batches of a map
gives exactly what the batches give one call at a time, while each batch's
dedup and key hashes run beside the batch before it.

* Against the oracle run batch by batch: answers, statuses, observable
  pages, HBM bins, loads, stash, position map and the whole trace, bit for
  bit.  One-round and several-round batches, one-command batches, both
  stores, sealed pages, the decomposed store.
* A rejected batch (a bad op code) inside a sequence: its successor's tape
  positions were taken on the guess that it is accepted and must be
  re-derived on the device; the oracle decides the right ones.
* Against a twin map given the same batches by separate calls.
* Argument errors."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import Twin, dev_u64, dev_u8, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


def _batches(rng, present, fresh, sizes, vs, cap, bad_at=()):
    out = []
    live = set(present)
    for b, q in enumerate(sizes):
        pool = np.array(sorted(live), dtype=np.uint64) if live else fresh[:10]
        r = rng.random(q)
        keys = np.where(r < 0.3, pool[rng.integers(0, min(5, pool.size), q)],
                        np.where(r < 0.85, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
        ops = rng.choice([0, 1, 2], size=q, p=[0.5, 0.35, 0.15]).astype(np.uint8)
        if len(live) + q > cap:
            ops[ops == 1] = 2
        if b in bad_at:
            ops[rng.integers(0, q)] = 7
        else:
            for op, key in zip(ops.tolist(), keys.tolist()):
                if op == 1:
                    live.add(int(key))
                elif op == 2:
                    live.discard(int(key))
        out.append((ops, keys.astype(np.uint64), rng.integers(0, 256, (q, vs), dtype=np.uint8)))
    return out


def _seq_on_gpu(m, batches, vs):
    import torch

    qs = [len(b[0]) for b in batches]
    ops = np.concatenate([b[0] for b in batches])
    keys = np.concatenate([b[1] for b in batches])
    vals = np.concatenate([b[2] for b in batches])
    vo = torch.zeros((ops.size, vs), dtype=torch.uint8, device="cuda")
    st = torch.zeros(ops.size, dtype=torch.uint8, device="cuda")
    rc = m.access_seq(dev_u8(ops), dev_u64(keys), dev_u8(vals), vo, st, qs)
    torch.cuda.synchronize()
    return rc, vo.cpu().numpy(), st.cpu().numpy()


def _check_against_oracle(t, batches, vs, bad_at=()):
    rc, vo, st = _seq_on_gpu(t.g, batches, vs)
    assert rc == 0 and t.g.status() == 0, (rc, t.g.status())
    at = 0
    for b, (ops, keys, vals) in enumerate(batches):
        rc_o, vo_o, st_o = t.o.access(ops, keys, vals)
        q = len(ops)
        if b in bad_at:
            assert rc_o == O.EINVAL
            assert (st[at:at + q] == 0xFF).all() and (vo[at:at + q] == 0).all(), b
        else:
            assert rc_o == 0, (b, rc_o)
            assert np.array_equal(st[at:at + q], st_o), b
            assert np.array_equal(vo[at:at + q], vo_o), b
        at += q
    t.assert_same_state()


@pytest.mark.parametrize("cap,n,vs,observable,kw,sizes", [
    (2048, 1500, 16, 0, {}, [1, 200, 37, 1, 150, 9, 64, 1, 300, 5, 2, 3]),  # several-round and one-command batches
    (4096, 3000, 64, 1, dict(alpha_permille=600), [500, 1, 1, 333, 80, 600, 2, 1, 450, 12]),
    (1 << 15, 30000, 8, 0, {}, [4096, 1, 2000, 8192, 1, 700, 3000]),
    (1 << 20, (1 << 20) - 100, 16, 0, {}, [4096, 3000, 4096, 1, 4096, 4096, 256, 255]),  # one-round batches
    (1 << 20, 1 << 19, 64, 1, {}, [4096] * 6),
])
def test_sequence_matches_the_oracle(cap, n, vs, observable, kw, sizes):
    t = Twin(cap, vs, observable=observable, **kw)
    k, v = workload(n, vs, 50 + n)
    assert t.build(k, v) == (0, 0, 0)
    rng = np.random.default_rng(n + vs)
    fresh = synth.keys(40000, n + 3, offset=10**8)
    for rnd in range(2):  # two calls in a row: the second starts from the first's state
        bs = _batches(rng, set(int(x) for x in t.o.logical_contents()), fresh, sizes, vs, cap)
        _check_against_oracle(t, bs, vs)


@pytest.mark.parametrize("bad_at,sizes", [
    ((1,), [300, 200, 400, 100]),
    ((0, 2), [4096, 4096, 4096, 4096, 17]),
    ((3,), [1, 1, 1, 1, 1, 1]),
    ((4,), [2000, 50, 4096, 9, 700]),  # the last batch rejected: nothing follows it
])
def test_rejected_batch_inside_a_sequence(bad_at, sizes):
    t = Twin(1 << 16, 16)
    k, v = workload(50000, 16, 77)
    assert t.build(k, v) == (0, 0, 0)
    rng = np.random.default_rng(len(sizes))
    fresh = synth.keys(20000, 78, offset=10**8)
    bs = _batches(rng, set(int(x) for x in k), fresh, sizes, 16, 1 << 16, bad_at=bad_at)
    _check_against_oracle(t, bs, 16, bad_at=bad_at)


def test_sequence_sealed_and_decomposed_stores():
    for kw in (dict(seal=True), dict(decomposed=True), dict(seal=True, decomposed=True, observable=1)):
        t = Twin(4096, 16, alpha_permille=300, **kw)
        k, v = workload(3500, 16, 41)
        assert t.build(k, v) == (0, 0, 0)
        rng = np.random.default_rng(42)
        bs = _batches(rng, set(int(x) for x in k), synth.keys(5000, 43, offset=10**8), [1, 300, 1, 1000, 64, 2, 900],
                      16, 4096)
        _check_against_oracle(t, bs, 16)


def test_sequence_equals_separate_calls():
    """Two GPU maps with one key: one gets a sequence, the other the same
    batches one call at a time (pinned store, config-2 layout at 2^20)."""
    import torch
    import paper_2509_01742_amd as B

    cap, vs = (1 << 20) + (1 << 12), 64
    key = bytes(range(90, 122))
    maps = []
    for _ in range(2):
        p = B.params(cap, vs, key=key)
        p.flags |= B.BOLT_F_TRACE
        maps.append(B.Map(p))
    k, v = workload(1 << 20, vs, 5)
    for m in maps:
        assert m.build(dev_u64(k), dev_u8(v)) == 0
    rng = np.random.default_rng(6)
    bs = _batches(rng, set(int(x) for x in k[:5000]), synth.keys(9000, 7, offset=10**8), [4096] * 8 + [1, 100], vs,
                  cap)
    rc, vo, st = _seq_on_gpu(maps[0], bs, vs)
    assert rc == 0
    outs = []
    for ops, keys, vals in bs:
        o = torch.zeros((len(ops), vs), dtype=torch.uint8, device="cuda")
        s = torch.zeros(len(ops), dtype=torch.uint8, device="cuda")
        assert maps[1].access(dev_u8(ops), dev_u64(keys), dev_u8(vals), o, s) == 0
        outs.append((o, s))
    torch.cuda.synchronize()
    assert np.array_equal(vo, np.concatenate([o.cpu().numpy() for o, _ in outs]))
    assert np.array_equal(st, np.concatenate([s.cpu().numpy() for _, s in outs]))
    a, b = maps
    assert a.status() == 0 and b.status() == 0
    assert np.array_equal(a.observable(), b.observable())
    assert np.array_equal(a.hbm_bins(), b.hbm_bins())
    assert np.array_equal(a.loads(), b.loads())
    assert np.array_equal(a.trace(), b.trace())
    assert a.stats()["steps"] == b.stats()["steps"]
    for m in maps:
        m.close()


def test_sequence_argument_errors():
    import torch
    import paper_2509_01742_amd as B

    t = Twin(1024, 8)
    k, v = workload(500, 8, 9)
    assert t.build(k, v) == (0, 0, 0)
    z8 = torch.zeros(16, dtype=torch.uint8, device="cuda")
    zk = dev_u64(k[:16])
    zv = torch.zeros((16, 8), dtype=torch.uint8, device="cuda")
    zo = torch.zeros((16, 8), dtype=torch.uint8, device="cuda")
    for qs in ([], [0], [3, 0, 2], [B.BOLT_MAX_BATCH + 1]):
        assert t.g.access_seq(z8, zk, zv, zo, z8, qs) == B.BOLT_EINVAL, qs
    torch.cuda.synchronize()
    assert t.g.status() == 0 and t.g.stats()["steps"] == 0

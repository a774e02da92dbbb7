"""Sealed observable store (BOLT_F_SEAL, ChaCha20-Poly1305 per page) on the
GPU against the sealed oracle, bit for bit: cipher text, tags, write counts,
answers and trace; and refusal of changed and replayed pages."""
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


def _mixed(rng, present, fresh, q, vs):
    pool = np.array(sorted(present), dtype=np.uint64) if present else fresh[:10]
    r = rng.random(q)
    keys = np.where(r < 0.3, pool[rng.integers(0, min(5, pool.size), q)],
                    np.where(r < 0.85, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
    ops = rng.choice([0, 1, 2], size=q, p=[0.5, 0.35, 0.15]).astype(np.uint8)
    return ops, keys.astype(np.uint64), rng.integers(0, 256, (q, vs), dtype=np.uint8)


def _run(t, k, cap, vs, nb, qmax, seed):
    rng = np.random.default_rng(seed)
    fresh = synth.keys(30000, seed + 7, offset=10**8)
    present = set(int(x) for x in k)
    for b in range(nb):
        q = int(rng.integers(1, qmax + 1))
        ops, keys, vals = _mixed(rng, present, fresh, q, vs)
        if len(present) > cap - q:
            ops[ops == 1] = 2
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, (b, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), b
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == 1:
                present.add(int(key))
            elif op == 2:
                present.discard(int(key))


@pytest.mark.parametrize("cap,n,vs,observable,qmax", [
    (2048, 1500, 16, 0, 300), (4096, 3000, 64, 1, 600), (1 << 15, 30000, 8, 0, 4096),
    (1 << 18, 1 << 17, 8, 1, 2000),  # one-round batches
    (1000, 900, 256, 0, 200),        # 4 KiB pages
])
def test_sealed_parity(cap, n, vs, observable, qmax):
    t = Twin(cap, vs, seal=True, observable=observable)
    k, v = workload(n, vs, 600 + n)
    assert t.build(k, v) == (0, 0, 0)
    t.assert_same_state()
    _run(t, k, cap, vs, 12, qmax, n)
    t.assert_same_state()


def _read_many(t, k, q=2000):
    import torch

    q = min(q, k.size)
    ops = np.zeros(q, np.uint8)
    vals = np.zeros((q, t.vs), np.uint8)
    rc_o, _, _ = t.o.access(ops, k[:q], vals)
    d_out = torch.zeros((q, t.vs), dtype=torch.uint8, device="cuda")
    d_st = torch.zeros(q, dtype=torch.uint8, device="cuda")
    rc_g = t.g.access(dev_u8(ops), dev_u64(k[:q]), dev_u8(vals), d_out, d_st)
    torch.cuda.synchronize()
    return rc_o, rc_g, t.g.status()


@pytest.mark.parametrize("where,observable", [("page", 0), ("tag", 0), ("page", 1)])
def test_sealed_refuses_a_changed_page(where, observable):
    import paper_2509_01742_amd as B

    t = Twin(3000, 16, seal=True, trace=False, observable=observable)
    k, v = workload(2500, 16, 17)
    assert t.build(k, v) == (0, 0, 0)
    pb = t.g.sizes["page_bytes"]
    for m in (t.g, t.o):  # the same change in both stores
        raw = bytearray(m.raw_page(3))
        raw[40 if where == "page" else pb + 7] ^= 0x10
        m.put_raw_page(3, bytes(raw))
    for _ in range(30):
        rc_o, rc_g, st = _read_many(t, k)
        if rc_o != 0 or st != 0:
            break
    assert rc_o == O.ETAMPER and st == B.BOLT_ETAMPER


def test_sealed_refuses_a_replayed_page():
    import paper_2509_01742_amd as B

    t = Twin(3000, 16, seal=True, trace=False)
    k, v = workload(2500, 16, 18)
    assert t.build(k, v) == (0, 0, 0)
    M = t.g.sizes["M"]
    old = [t.g.raw_page(p) for p in range(M)]
    v0 = t.g.versions()
    rc_o, rc_g, st = _read_many(t, k)
    assert rc_o == 0 and st == 0
    v1 = t.g.versions()
    assert np.array_equal(v1, t.o.versions())
    p = int(np.nonzero(v1 != v0)[0][0])
    for m in (t.g, t.o):
        m.put_raw_page(p, old[p])  # a valid seal, one write old
    for _ in range(30):
        rc_o, rc_g, st = _read_many(t, k)
        if rc_o != 0 or st != 0:
            break
    assert rc_o == O.ETAMPER and st == B.BOLT_ETAMPER


def test_sealed_and_plain_maps_together():
    """Many-map build and access over sealed and unsealed maps at once, and a
    sealed map replaying captured graphs."""
    import torch
    import paper_2509_01742_amd as B

    specs = [(2048, 1500, 16, True), (2048, 1500, 16, False), (8192, 7000, 64, True), (1 << 14, 9000, 8, False)]
    twins, inputs, ks = [], [], []
    for j, (cap, n, vs, seal) in enumerate(specs):
        t = Twin(cap, vs, seal=seal, key=bytes((9 * j + i) & 255 for i in range(32)))
        k, v = workload(n, vs, 700 + j)
        assert t.o.build(k, v) == 0
        twins.append(t)
        inputs.append((dev_u64(k), dev_u8(v)))
        ks.append(k)
    assert B.build_many([t.g for t in twins], inputs) == 0
    torch.cuda.synchronize()
    for t in twins:
        assert t.g.status() == 0
        t.assert_same_state()
    rng = np.random.default_rng(3)
    for rnd in range(4):
        batches, host = [], []
        for j, (cap, n, vs, seal) in enumerate(specs):
            q = int(rng.integers(1, 1500))
            ops, keys, vals = _mixed(rng, set(int(x) for x in ks[j][:200]), synth.keys(100, j + 50, offset=10**8),
                                     q, vs)
            ops[ops == 1] = 0  # no inserts: the key sets stay as built
            batches.append((dev_u8(ops), dev_u64(keys), dev_u8(vals),
                            torch.zeros((q, vs), dtype=torch.uint8, device="cuda"),
                            torch.zeros(q, dtype=torch.uint8, device="cuda")))
            host.append((ops, keys, vals))
        assert B.access_many([t.g for t in twins], batches) == 0
        torch.cuda.synchronize()
        for j, t in enumerate(twins):
            rc_o, vo_o, st_o = t.o.access(*host[j])
            assert rc_o == 0 and t.g.status() == 0
            assert np.array_equal(batches[j][3].cpu().numpy(), vo_o) and np.array_equal(batches[j][4].cpu().numpy(),
                                                                                         st_o)
    for t in twins:
        t.assert_same_state()
    g = Twin(4096, 16, seal=True, flags=B.BOLT_F_GRAPHS)
    k, v = workload(3500, 16, 777)
    assert g.build(k, v) == (0, 0, 0)
    _run(g, k, 4096, 16, 8, 1000, 31)
    g.assert_same_state()

"""Parity of the HIP path with the oracle, bit for bit, through the C ABI.

Every case feeds the library and the oracle the same seeded inputs and the
same PRF key, then compares answers, status bytes, the observable pages, the
HBM bins, the bin loads, the stash and the position map (as sets), and the
trace of observable accesses."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import Twin, dev_u64, dev_u8, host_u64, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


# ------------------------------------------------------------------ primitives

def test_prf_matches_oracle():
    import torch
    import paper_2509_01742_amd as B

    key = bytes(range(50, 82))
    x = np.concatenate([np.array([0, 1, 2**64 - 1, 2**63], np.uint64), synth.keys(997, 3)])
    for domain in (1, 2, 3, 0xAB):
        out = torch.zeros(4 * x.size, dtype=torch.int64, device="cuda")
        assert B.prf(key, domain, dev_u64(x), out) == 0
        got = host_u64(out).reshape(-1, 4)
        for i in range(x.size):
            assert tuple(int(v) for v in got[i]) == O.prf(key, domain, int(x[i])), (domain, i)


@pytest.mark.parametrize("n", [1, 2, 4, 64, 1024, 8192, 16384, 1 << 17, 1 << 20])
def test_sort_matches_numpy(n):
    import torch
    import paper_2509_01742_amd as B

    rng = np.random.default_rng(n)
    for a in (rng.integers(0, 2**64, n, dtype=np.uint64), rng.integers(0, 3, n, dtype=np.uint64),
              np.arange(n, dtype=np.uint64)[::-1].copy()):
        d = dev_u64(a)
        assert B.sort_u64(d) == 0
        torch.cuda.synchronize()
        assert np.array_equal(host_u64(d), np.sort(a))


def test_sort_zero_one_principle():
    import torch
    import paper_2509_01742_amd as B

    n = 8
    for bits in range(1 << n):
        a = np.array([(bits >> i) & 1 for i in range(n)], dtype=np.uint64)
        d = dev_u64(a)
        assert B.sort_u64(d) == 0
        torch.cuda.synchronize()
        assert np.array_equal(host_u64(d), np.sort(a)), bits


@pytest.mark.parametrize("m,frac", [(2, 0.5), (100, 0.3), (4097, 0.6), ((1 << 16) + 3, 0.5), (1 << 20, 0.9)])
def test_expand_matches_oracle(m, frac):
    import torch
    import paper_2509_01742_amd as B

    rng = np.random.default_rng(m)
    keep = rng.random(m) < frac
    tgt = np.nonzero(keep)[0].astype(np.uint32)
    n = tgt.size
    pay = rng.integers(0, 2**31, n).astype(np.uint32)
    want, rc = O.expand(tgt, pay, m)
    assert rc == 0
    el = np.full(m, 2**64 - 1, dtype=np.uint64)
    el[:n] = (tgt.astype(np.uint64) << np.uint64(32)) | pay.astype(np.uint64)
    d = dev_u64(el)
    tmp = torch.zeros(m, dtype=torch.int64, device="cuda")
    assert B.expand_u64(d, tmp) == 0
    torch.cuda.synchronize()
    got = host_u64(d)
    empty = got == np.uint64(2**64 - 1)
    assert np.array_equal(empty, want == O.NONE32)
    assert np.array_equal((got[~empty] & np.uint64(0xFFFFFFFF)).astype(np.uint32), want[~empty])
    assert np.array_equal((got[~empty] >> np.uint64(32)).astype(np.int64), np.nonzero(~empty)[0])


# ------------------------------------------------------------------ build

@pytest.mark.parametrize("cap,n,vs,kw", [
    (64, 0, 8, {}), (64, 1, 8, {}), (64, 64, 8, {}), (1000, 777, 16, dict(alpha_permille=0)),
    (1000, 999, 8, dict(alpha_permille=500)), (4096, 3000, 64, {}), (1 << 14, (1 << 14) - 5, 8, dict(alpha_permille=10)),
    (5000, 4321, 24, dict(alpha_permille=999)), (1 << 16, 1 << 16, 8, {}), (100000, 99999, 64, dict(c=4)),
    (1 << 17, 100000, 8, dict(pm_choices=2, pm_keys_per_row=8))])
def test_build_parity(cap, n, vs, kw):
    t = Twin(cap, vs, **kw)
    k, v = workload(n, vs, 1000 + n)
    rc_o, rc_g, st = t.build(k, v)
    assert rc_o == 0 and rc_g == 0 and st == 0
    t.assert_same_state()


def test_build_parity_device_observable():
    t = Twin(3000, 16, observable=1)
    k, v = workload(2900, 16, 5)
    assert t.build(k, v) == (0, 0, 0)
    t.assert_same_state()


def test_build_trace_identical_across_datasets():
    traces = []
    for seed in (1, 2, 3):
        t = Twin(5000, 8, key=bytes([seed]) * 32)
        k, v = workload(4500, 8, 77 * seed)
        assert t.build(k, v) == (0, 0, 0)
        traces.append(t.g.trace())
    M = traces[0].size
    assert M == Twin(5000, 8).o.s["M"]
    for tr in traces:
        assert np.array_equal(tr, traces[0])
        assert (tr["kind"] == 1).all() and np.array_equal(tr["page"], np.arange(M))


def test_build_errors():
    import paper_2509_01742_amd as B

    k, v = workload(300, 8, 9)
    kd = k.copy()
    kd[10] = kd[200]
    t = Twin(512, 8)
    rc_o, rc_g, st = t.build(kd, v)
    assert rc_o == O.EDUPKEY and rc_g == 0 and st == B.BOLT_EDUPKEY
    assert t.g.build(dev_u64(k), dev_u8(v)) == B.BOLT_ESTATE
    t = Twin(512, 8, bin_slots=1)
    rc_o, rc_g, st = t.build(k, v)
    assert rc_o == O.EOVERFLOW and st == B.BOLT_EOVERFLOW
    t = Twin(512, 8, pm_row_slots=1)
    rc_o, rc_g, st = t.build(k, v)
    assert rc_o == O.EOVERFLOW and st == B.BOLT_EOVERFLOW
    t = Twin(256, 8)
    assert t.g.build(dev_u64(k), dev_u8(v)) == B.BOLT_EINVAL  # more keys than capacity
    assert t.g.build(dev_u64(k[:200]), dev_u8(v[:200])) == 0
    assert t.g.build(dev_u64(k[:200]), dev_u8(v[:200])) == B.BOLT_EINVAL  # once per map


# ------------------------------------------------------------------ access

def _mixed_batch(rng, present, fresh, q, vs, hot=5, p=(0.5, 0.35, 0.15)):
    pool = np.array(sorted(present), dtype=np.uint64) if present else fresh[:10]
    r = rng.random(q)
    keys = np.where(r < 0.3, pool[rng.integers(0, min(hot, pool.size), q)],
                    np.where(r < 0.85, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
    ops = rng.choice([0, 1, 2], size=q, p=list(p)).astype(np.uint8)
    vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
    return ops, keys.astype(np.uint64), vals


@pytest.mark.parametrize("cap,n,vs,kw,qmax,nb", [
    (2048, 1500, 16, {}, 200, 40),
    (2048, 1500, 8, dict(alpha_permille=0), 300, 30),
    (4096, 3000, 64, dict(alpha_permille=600), 500, 30),
    (1 << 15, 30000, 8, {}, 4096, 12),
    (1 << 12, 4000, 8, dict(alpha_permille=500), 8192, 4),
    (512, 0, 8, {}, 64, 30),
    # one-round batches (q <= ceil(B/16) and q <= ceil(R/16)): the thread-per-command remap
    (1 << 20, (1 << 20) - 100, 16, {}, 4096, 8),
    (1 << 20, 1 << 19, 8, dict(alpha_permille=0), 3000, 6),
])
def test_access_parity(cap, n, vs, kw, qmax, nb):
    t = Twin(cap, vs, **kw)
    k, v = workload(n, vs, 31 + n)
    assert t.build(k, v) == (0, 0, 0)
    rng = np.random.default_rng(n + qmax)
    fresh = synth.keys(50000, 4242, offset=10**8)
    present = set(int(x) for x in k)
    for b in range(nb):
        q = int(rng.integers(1, qmax + 1))
        ops, keys, vals = _mixed_batch(rng, present, fresh, q, vs)
        if len(present) > cap - q:
            ops[ops == 1] = 2
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, (b, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o), b
        assert np.array_equal(vo_g, vo_o), b
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == 1:
                present.add(int(key))
            elif op == 2:
                present.discard(int(key))
        if b % 5 == 4 or b == nb - 1:
            t.assert_same_state()


def test_access_edge_keys_and_single_ops():
    t = Twin(256, 8)
    k = np.array([0, 2**64 - 1, 1, 2**63], dtype=np.uint64)
    v = np.arange(32, dtype=np.uint8).reshape(4, 8)
    assert t.build(k, v) == (0, 0, 0)
    seq = [(0, 0), (0, 2**64 - 1), (2, 0), (0, 0), (1, 0), (0, 0), (0, 12345), (2, 12345), (1, 2**64 - 2)]
    for op, key in seq:
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(np.array([op], np.uint8), np.array([key], np.uint64),
                                                               np.full((1, 8), 7, np.uint8))
        assert rc_o == rc_g == st == 0
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o)
    t.assert_same_state()


def test_get_put_wrappers():
    import torch

    t = Twin(4096, 16)
    k, v = workload(3000, 16, 8)
    assert t.build(k, v) == (0, 0, 0)
    P = O.PlainMap(16)
    P.build(k, v)
    rng = np.random.default_rng(2)
    keys = np.concatenate([k[rng.integers(0, 3000, 500)], synth.keys(100, 99, offset=10**9)])
    vo = torch.zeros((keys.size, 16), dtype=torch.uint8, device="cuda")
    found = torch.zeros(keys.size, dtype=torch.uint8, device="cuda")
    assert t.g.get(dev_u64(keys), vo, found) == 0
    wo, wst = P.access(np.zeros(keys.size, np.uint8), keys, np.zeros((keys.size, 16), np.uint8))
    assert t.g.status() == 0
    assert np.array_equal(found.cpu().numpy(), wst) and np.array_equal(vo.cpu().numpy(), wo)
    pk = np.concatenate([k[:50], synth.keys(30, 98, offset=10**9)])
    pv = rng.integers(0, 256, (pk.size, 16), dtype=np.uint8)
    st = torch.zeros(pk.size, dtype=torch.uint8, device="cuda")
    assert t.g.put(dev_u64(pk), dev_u8(pv), st) == 0
    _, wst = P.access(np.ones(pk.size, np.uint8), pk, pv)
    assert t.g.status() == 0
    assert np.array_equal(st.cpu().numpy(), wst)


def test_access_rejects_bad_op_without_change():
    t = Twin(1024, 8)
    k, v = workload(900, 8, 4)
    assert t.build(k, v) == (0, 0, 0)
    obs0 = t.g.observable()
    (rc_o, _, _), (rc_g, st, vo_g, st_g) = t.access(np.array([0, 7], np.uint8), k[:2], np.zeros((2, 8), np.uint8))
    assert rc_o == O.EINVAL and rc_g == 0 and st == 0
    assert (st_g == 0xFF).all() and (vo_g == 0).all()
    assert np.array_equal(t.g.observable(), obs0)
    assert t.g.stats()["steps"] == 0


def test_access_capacity_errors():
    import paper_2509_01742_amd as B

    t = Twin(64, 8)
    k, v = workload(60, 8, 1)
    assert t.build(k, v) == (0, 0, 0)
    new = synth.keys(10, 999, offset=10**9)
    (rc_o, _, _), (rc_g, st, _, _) = t.access(np.ones(10, np.uint8), new, np.zeros((10, 8), np.uint8))
    assert rc_o == O.EFULL and st == B.BOLT_EFULL
    import torch

    z = torch.zeros(1, dtype=torch.uint8, device="cuda")
    assert t.g.access(z, dev_u64(k[:1]), dev_u8(np.zeros((1, 8))), torch.zeros((1, 8), dtype=torch.uint8,
                                                                                device="cuda"), z) == B.BOLT_ESTATE
    t = Twin(256, 8, pm_row_slots=1, pm_keys_per_row=64)
    assert t.build(np.zeros(0, np.uint64), np.zeros((0, 8), np.uint8)) == (0, 0, 0)
    (rc_o, _, _), (rc_g, st, _, _) = t.access(np.ones(8, np.uint8), synth.keys(8, 4), np.zeros((8, 8), np.uint8))
    assert rc_o == O.EOVERFLOW and st == B.BOLT_EOVERFLOW


@pytest.mark.parametrize("observable", [0, 1])
def test_access_parity_through_captured_graphs(observable):
    """BOLT_F_GRAPHS: every batch replays the graph of its size class.  Sizes
    cross the one-round / several-round threshold and revisit classes, and an
    eager map's batches run between the replays; every replay is checked, and
    at the end the state and the whole trace of the replayed map (grids sized
    for the class, each kernel stopping at the plan's q)."""
    import paper_2509_01742_amd as B

    t = Twin(1 << 15, 16, observable=observable, flags=B.BOLT_F_GRAPHS)
    e = Twin(1 << 12, 8, trace=False)  # eager work between the replays
    k, v = workload(30000, 16, 77)
    ke, ve = workload(3000, 8, 78)
    assert t.build(k, v) == (0, 0, 0) and e.build(ke, ve) == (0, 0, 0)
    rng = np.random.default_rng(99)
    fresh = synth.keys(40000, 4243, offset=10**8)
    present = set(int(x) for x in k)
    pe = set(int(x) for x in ke)
    sizes = [1, 1, 2, 3, 64, 65, 128, 129, 5, 4096, 8192, 100, 1, 2000, 4095, 7, 8192, 3]
    for b, q in enumerate(sizes):
        ops, keys, vals = _mixed_batch(rng, present, fresh, q, 16)
        if len(present) > (1 << 15) - q:
            ops[ops == 1] = 2
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, (b, q, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), (b, q)
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == 1:
                present.add(int(key))
            elif op == 2:
                present.discard(int(key))
        opse, kse, vse = _mixed_batch(rng, pe, fresh, 50, 8)
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = e.access(opse, kse, vse)
        assert rc_o == 0 and rc_g == 0 and np.array_equal(vo_g, vo_o)
        for op, key in zip(opse.tolist(), kse.tolist()):
            if op == 1:
                pe.add(int(key))
            elif op == 2:
                pe.discard(int(key))
    t.assert_same_state()  # the replays' trace too
    e.assert_same_state(trace=False)


def _oracle_marks(o, K, marks):
    """The bound marks after a batch, from the oracle's state: the largest
    bin load, the items of the K HBM bins, their high-water marks, and the
    stash high-water mark."""
    ld = o.loads().astype(np.int64)
    hbm = int(ld[:K].sum())
    marks["load_hw"] = max(marks.get("load_hw", 0), int(ld.max()))
    marks["hbm_hw"] = max(marks.get("hbm_hw", 0), hbm)
    return int(ld.max()), hbm


def test_watch_marks_follow_every_batch():
    """BOLT_F_WATCH: after each batch the map reports the largest bin load
    and the items of its HBM bins, with high-water marks.  Every mark is
    compared after every batch with the same quantities computed from the
    oracle's loads, and the stash high-water mark with the oracle's."""
    import paper_2509_01742_amd as B

    t = Twin(1 << 14, 8, trace=False, flags=B.BOLT_F_WATCH, alpha_permille=300)
    k, v = workload(15000, 8, 91)
    assert t.build(k, v) == (0, 0, 0)
    K = t.g.sizes["K"]
    rng = np.random.default_rng(5)
    fresh = synth.keys(20000, 4244, offset=10**8)
    present = set(int(x) for x in k)
    marks = {}
    for b in range(12):
        q = int(rng.integers(1, 3000))
        ops, keys, vals = _mixed_batch(rng, present, fresh, q, 8)
        if len(present) > (1 << 14) - q:
            ops[ops == 1] = 2
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0 and np.array_equal(vo_g, vo_o)
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == 1:
                present.add(int(key))
            elif op == 2:
                present.discard(int(key))
        mx, hbm = _oracle_marks(t.o, K, marks)
        s = t.g.stats()
        assert s["hbm_load"] == hbm and s["hbm_load_highwater"] == marks["hbm_hw"], b
        assert s["load_highwater"] == marks["load_hw"] and s["max_load"] == mx, b
        assert s["stash_highwater"] == t.o.stash_highwater, b
    t.assert_same_state(trace=False)


@pytest.mark.parametrize("c,alpha", [(8, 200), (16, 500), (16, 10)])
def test_dynamics_marks_match_the_oracle(c, alpha):
    """The bound validation's setting (Sec. 4.3, dimensions in practice) at a
    size the oracle runs in seconds: N = 2^16 keys, a long stream of uniform
    GETs in batches of 4096 on the device store; after every batch the
    GPU's marks (largest bin load, HBM-bin items, their high-water marks,
    the stash high-water mark) equal those of the oracle's state, and at the
    end the whole state does."""
    import paper_2509_01742_amd as B

    n = 1 << 16
    t = Twin(n, 8, trace=False, observable=B.BOLT_OBS_DEVICE, flags=B.BOLT_F_WATCH, c=c, alpha_permille=alpha)
    k, v = workload(n, 8, 300 + c + alpha)
    assert t.build(k, v) == (0, 0, 0)
    K = t.g.sizes["K"]
    rng = np.random.default_rng(c * 1000 + alpha)
    marks = {}  # high-water marks over batch ends (the build's loads are not among them)
    ops = np.zeros(4096, np.uint8)
    vals = np.zeros((4096, 8), np.uint8)
    for b in range(48):
        keys = k[rng.integers(0, n, 4096)]
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0 and np.array_equal(vo_g, vo_o) and (st_g == 1).all()
        mx, hbm = _oracle_marks(t.o, K, marks)
        s = t.g.stats()
        assert (s["max_load"], s["load_highwater"], s["hbm_load"], s["hbm_load_highwater"]) == (
            mx, marks["load_hw"], hbm, marks["hbm_hw"]), b
        assert s["stash_highwater"] == t.o.stash_highwater and s["stash_live"] == t.o.stash_live, b
        assert mx <= t.g.sizes["Z"] and t.o.stash_highwater <= t.g.sizes["stash_bound"]
    t.assert_same_state(trace=False)
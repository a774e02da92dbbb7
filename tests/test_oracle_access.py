"""Pins of the oracle's batched access (Alg. 1, module order of Sec. 5.1).

* Answers: exhaustive small key sets against the plain dictionary (O1), for
  every op sequence up to length 3 and both batch splits, plus long random
  mixed streams.
* State: after every batch, the stored items decode to exactly the
  dictionary, each mapped key sits in one of its two mapped bins, and the
  load of every bin equals its items plus its stash items.
* Trace (Claim 4.1 and its simulator): each op reveals two distinct bins;
  with alpha = 0 the schedule of reads and writes is the same for every
  dataset and query stream; the revealed pairs follow the pair law even for
  adversarial streams.
* Dynamics: bin loads stay within l_max (Claim 4.2) and the stash settles
  near the drift equilibrium (Claim 4.4) and under its bound."""
import itertools

import numpy as np
import pytest

import oracle as O
import synth

KEY = bytes(range(7, 39))


def _mk(cap, vs, n, seed, alpha=200, trace=False, **kw):
    m = O.OracleMap(cap, vs, alpha_pm=alpha, key=KEY, trace=trace, **kw)
    k, v = synth.keys(n, seed), synth.values(n, vs, seed + 1)
    assert m.build(k, v) == O.OK
    p = O.PlainMap(vs)
    p.build(k, v)
    return m, p, k


def _check_state(m, p):
    s = m.s
    Z, vs, K, B = s["Z"], s["vs"], s["K"], s["B"]
    assert m.logical_contents() == p.d
    assert m.live == len(p.d)
    bins = np.concatenate([m.hbm_bins(), m.observable()])
    where = {}
    count = np.zeros(B, dtype=np.int64)
    for b, page in enumerate(bins):
        items = O.decode_page(page, Z, vs)
        keys = [x[0] for x in items]
        assert keys == sorted(keys)
        count[b] += len(items)
        for key in keys:
            where[key] = b
    for key, dest, _ in m.stash():
        assert dest >= K  # only host bins have stash items
        count[dest] += 1
        where[key] = dest
    assert (count == m.loads()).all()
    assert m.loads().max() <= Z
    pm = m.pmap()
    assert sorted(e[1] for e in pm) == sorted(p.d)
    for _, key, p1, p2 in pm:
        assert p1 != p2 and where[key] in (p1, p2)


# ---------------------------------------------------------------- answers

def _exhaustive_cases():
    ka, kb, kc = 0x1111, 0x2222, 0xFFFFFFFFFFFFFFFF
    universe = [ka, kb, kc]
    vals = {1: bytes([1] * 8), 2: bytes([2] * 8)}
    kinds = [(op, v) for op, v in ((O.GET, 0), (O.PUT, 1), (O.PUT, 2), (O.DEL, 0))]
    steps = [(op, v, k) for (op, v) in kinds for k in universe]
    seqs = []
    for L in (1, 2, 3):
        seqs.extend(itertools.product(steps, repeat=L))
    return universe, vals, seqs


def test_exhaustive_small_key_sets():
    universe, vals, seqs = _exhaustive_cases()
    zero = bytes(8)
    n_cases = 0
    for init_mask in range(8):
        init = [k for i, k in enumerate(universe) if (init_mask >> i) & 1]
        for seq in seqs:
            for split in (1, len(seq)):
                m = O.OracleMap(16, 8, alpha_pm=500, key=KEY)  # B = 2: one HBM bin, one page
                ik = np.array(init, dtype=np.uint64)
                iv = np.array([[0x30 + j] * 8 for j in range(len(init))], dtype=np.uint8).reshape(-1, 8)
                assert m.build(ik, iv) == O.OK
                p = O.PlainMap(8)
                p.build(ik, iv)
                ops = np.array([s[0] for s in seq], np.uint8)
                keys = np.array([s[2] for s in seq], np.uint64)
                vin = np.array([list(vals.get(s[1], zero)) for s in seq], np.uint8)
                for a in range(0, len(seq), split):
                    rc, vo, st = m.access(ops[a:a + split], keys[a:a + split], vin[a:a + split])
                    assert rc == O.OK
                    wo, wst = p.access(ops[a:a + split], keys[a:a + split], vin[a:a + split])
                    assert (st == wst).all() and (vo == wo).all(), (init, seq, split)
                assert m.logical_contents() == p.d
                n_cases += 1
    assert n_cases == 8 * 1884 * 2


@pytest.mark.parametrize("alpha", [0, 200, 600])
def test_random_mixed_stream(alpha):
    vs = 16
    n, cap = 1500, 2048
    m, p, k = _mk(cap, vs, n, 321 + alpha, alpha=alpha)
    rng = np.random.default_rng(alpha)
    fresh = synth.keys(30000, 777, offset=10**6)
    fi = 0
    for b in range(120):
        q = int(rng.integers(1, 200))
        pool = np.array(sorted(p.d), dtype=np.uint64) if p.d else k
        hot = pool[rng.integers(0, min(5, pool.size), q)]  # repeated keys in a batch
        cold = pool[rng.integers(0, pool.size, q)]
        new = fresh[fi:fi + q]
        fi += q
        r = rng.random(q)
        keys = np.where(r < 0.3, hot, np.where(r < 0.85, cold, new)).astype(np.uint64)
        ops = rng.choice([O.GET, O.PUT, O.DEL], size=q, p=[0.5, 0.35, 0.15]).astype(np.uint8)
        if len(p.d) > cap - 250:
            ops[ops == O.PUT] = O.DEL
        vin = rng.integers(0, 256, (q, vs), dtype=np.uint8)
        rc, vo, st = m.access(ops, keys, vin)
        assert rc == O.OK
        wo, wst = p.access(ops, keys, vin)
        assert (st == wst).all() and (vo == wo).all()
        if b % 10 == 0:
            _check_state(m, p)
    _check_state(m, p)


# ---------------------------------------------------------------- trace

def _batches(kind, keys, rng, nb, q):
    out = []
    for b in range(nb):
        if kind == "same":
            ks = np.full(q, keys[0], np.uint64)
        elif kind == "absent":
            ks = synth.keys(q, 55, offset=10**7 + b * q)
        elif kind == "sequential":
            ks = keys[(b * q + np.arange(q)) % keys.size]
        else:
            ks = keys[rng.integers(0, keys.size, q)]
        ops = np.zeros(q, np.uint8)
        out.append((ops, ks, np.zeros((q, 8), np.uint8)))
    return out


def test_alpha0_schedule_identical_across_data_and_streams():
    """With alpha = 0 every op reads exactly two pages, so the schedule
    (count, order, read/write kinds) is the same whatever the data."""
    shapes = []
    for seed, kind in ((1, "uniform"), (2, "same"), (3, "absent"), (4, "sequential")):
        m, p, k = _mk(1024, 8, 1000, 10 * seed, alpha=0, trace=True)
        m.trace_clear()
        rng = np.random.default_rng(seed)
        for b, (ops, ks, vi) in enumerate(_batches(kind, k, rng, 20, 32)):
            rc, _, _ = m.access(ops, ks, vi)
            assert rc == O.OK
        t = m.trace()
        per_batch = []
        for b in range(1, 21):
            tb = t[t["batch"] == b]
            reads = tb[tb["kind"] == 0]["page"]
            writes = tb[tb["kind"] == 1]["page"]
            assert (tb["kind"][:reads.size] == 0).all()  # reads first, then writes
            assert reads.size == 64
            assert (reads[0::2] != reads[1::2]).all()  # two distinct bins per op
            assert list(writes) == sorted(set(reads.tolist()))  # each page read, written once, ascending
            per_batch.append((reads.size, writes.size))
        shapes.append([r for r, _ in per_batch])
    assert all(s == shapes[0] for s in shapes)


@pytest.mark.parametrize("kind", ["same", "absent", "sequential"])
def test_revealed_pairs_uniform_for_adversarial_streams(kind):
    """Claim 4.1: each access reveals a uniform pair of distinct bins, even
    when the same key is asked again and again."""
    m, p, k = _mk(128, 8, 100, 5, alpha=0, trace=True)  # B = M = 16
    M = m.s["M"]
    m.trace_clear()
    rng = np.random.default_rng(9)
    for ops, ks, vi in _batches(kind, k, rng, 240, 25):
        assert m.access(ops, ks, vi)[0] == O.OK
    t = m.trace()
    reads = t[t["kind"] == 0]["page"].reshape(-1, 2)
    counts = np.zeros((M, M))
    for a, b in reads:
        counts[a, b] += 1
    assert np.trace(counts) == 0
    obs = counts[~np.eye(M, dtype=bool)]
    exp = reads.shape[0] / (M * (M - 1))
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert chi2 < 340, chi2  # 239 dof: the 0.9999 quantile is about 335


def test_alpha_positive_reads_are_host_bins_only():
    m, p, k = _mk(2048, 8, 2000, 8, alpha=500, trace=True)
    m.trace_clear()
    rng = np.random.default_rng(1)
    n_reads = 0
    for ops, ks, vi in _batches("uniform", k, rng, 50, 40):
        assert m.access(ops, ks, vi)[0] == O.OK
    t = m.trace()
    reads = t[t["kind"] == 0]
    frac = reads.size / (2 * 50 * 40)
    assert 0.4 < frac < 0.6  # about 1 - alpha of the 2q bins are pages
    assert (t["page"] < m.s["M"]).all()


# ---------------------------------------------------------------- dynamics

@pytest.mark.parametrize("alpha", [10, 200, 500])
def test_stash_dynamics_and_max_load(alpha):
    n = cap = 1 << 12
    m, p, k = _mk(cap, 8, n, 42, alpha=alpha)
    s = m.s
    M = s["M"]
    rng = np.random.default_rng(alpha)
    occ = []
    for b in range(2500):
        ks = k[rng.integers(0, n, 32)]
        assert m.access(np.zeros(32, np.uint8), ks, np.zeros((32, 8), np.uint8))[0] == O.OK
        if b >= 500:
            occ.append(m.stash_live)
        assert m.loads().max() <= s["Z"]
    mean = float(np.mean(occ))
    lo = 0.6 * M / 2
    hi = 1.2 * (1 + alpha / 1000) * M / 2
    assert lo < mean < hi, (mean, lo, hi)
    assert m.stash_highwater <= s["stash_bound"]


# ---------------------------------------------------------------- errors

def test_access_errors():
    m, p, k = _mk(64, 8, 60, 1)
    bad = np.array([0, 3], np.uint8)
    rc, _, _ = m.access(bad, k[:2], np.zeros((2, 8), np.uint8))
    assert rc == O.EINVAL
    assert m.access(np.zeros(2, np.uint8), k[:2], np.zeros((2, 8), np.uint8))[0] == O.OK  # not poisoned
    new = synth.keys(10, 999, offset=10**9)
    rc, _, st = m.access(np.ones(10, np.uint8), new, np.zeros((10, 8), np.uint8))
    assert rc == O.EFULL  # 70 live keys > capacity 64
    assert m.access(np.zeros(1, np.uint8), k[:1], np.zeros((1, 8), np.uint8))[0] == O.ESTATE
    m2 = O.OracleMap(64, 8, key=KEY)
    assert m2.access(np.zeros(1, np.uint8), k[:1], np.zeros((1, 8), np.uint8))[0] == O.EINVAL  # not built


def test_rejected_batch_keeps_its_number_and_records_nothing():
    m, p, k = _mk(64, 8, 60, 1, trace=True)
    n0 = m.trace().size
    assert m.access(np.array([0, 5], np.uint8), k[:2], np.zeros((2, 8), np.uint8))[0] == O.EINVAL
    assert m.trace().size == n0 and m.ctr == 0
    assert m.access(np.zeros(1, np.uint8), k[:1], np.zeros((1, 8), np.uint8))[0] == O.OK
    t = m.trace()[n0:]
    assert t.size > 0 and (t["batch"] == 2).all()


def test_row_overflow_on_insert():
    m = O.OracleMap(256, 8, W=1, kpr=64, key=KEY)  # 4 rows of one slot
    assert m.build(np.zeros(0, np.uint64), np.zeros((0, 8), np.uint8)) == O.OK
    new = synth.keys(8, 4)
    rc, _, _ = m.access(np.ones(8, np.uint8), new, np.zeros((8, 8), np.uint8))
    assert rc == O.EOVERFLOW


def test_empty_batch_and_empty_map():
    m = O.OracleMap(64, 8, key=KEY, trace=True)
    assert m.build(np.zeros(0, np.uint64), np.zeros((0, 8), np.uint8)) == O.OK
    rc, vo, st = m.access(np.zeros(0, np.uint8), np.zeros(0, np.uint64), np.zeros((0, 8), np.uint8))
    assert rc == O.OK and vo.shape == (0, 8)
    assert m.ctr == 0
    p = O.PlainMap(8)
    k = synth.keys(5, 2)
    ops = np.array([0, 1, 0, 2, 0], np.uint8)
    vin = np.arange(40, dtype=np.uint8).reshape(5, 8)
    rc, vo, st = m.access(ops, k[[0, 0, 0, 0, 0]], vin)
    wo, wst = p.access(ops, k[[0, 0, 0, 0, 0]], vin)
    assert rc == O.OK and (st == wst).all() and (vo == wo).all()
    assert list(st) == [0, 2, 1, 3, 0]

"""Pins of the oracle's build (the oblivious form of the 'fast data
initialization' of Sec. 5.2).

The network procedure (PRF, P2C rounds, bitonic sort, rank, expansion,
write-out) must end in exactly the state of the plain definition (bucket
each key into its P2C bin, write canonical pages), and that state must
satisfy what the paper fixes: every item sits in one of its two random bins
(Sec. 4.1), the less loaded one at the time it was placed (P2C), bins stay
within l_max (Claim 4.2), and the only observable accesses are the writes
of pages 0..M-1 in order, whatever the data (Sec. 5.3, obliviousness
analysis)."""
import numpy as np
import pytest

import oracle as O
import synth

KEY = bytes(range(100, 132))


def _data(n, vs, seed):
    return synth.keys(n, seed), synth.values(n, vs, seed + 1)


def _prf_pairs(keys, B):
    return [O.pair(*O.prf(KEY, 1, int(k))[:2], B) for k in keys]


def _pm_rows(key, R):
    w = O.prf(KEY, 2, int(key))
    return [(w[j] * R) >> 64 for j in range(4)]


def _check_pages(arr, Z, vs, page_bytes):
    for page in arr:
        mask = int(page[:8].view("<u8")[0])
        n = bin(mask).count("1")
        assert mask == (1 << n) - 1  # real slots first
        keys = page[8:8 + 8 * Z].view("<u8")
        assert list(keys[:n]) == sorted(keys[:n])
        assert (keys[n:] == 0).all()
        vals = page[8 + 8 * Z:8 + 8 * Z + vs * Z]
        assert (vals[n * vs:] == 0).all()
        assert (page[8 + 8 * Z + vs * Z:] == 0).all()


@pytest.mark.parametrize("cap,n,vs,alpha", [
    (64, 0, 8, 200), (64, 1, 8, 200), (64, 64, 8, 200), (1000, 777, 16, 0), (1000, 999, 8, 500),
    (4096, 3000, 64, 200), (1 << 14, (1 << 14) - 5, 8, 10), (5000, 4321, 24, 999)])
def test_network_build_equals_plain_definition(cap, n, vs, alpha):
    k, v = _data(n, vs, 11 + n)
    a = O.OracleMap(cap, vs, alpha_pm=alpha, key=KEY, trace=True)
    b = O.OracleMap(cap, vs, alpha_pm=alpha, key=KEY, trace=True)
    assert a.build(k, v, mode=0) == O.OK
    assert b.build(k, v, mode=1) == O.OK
    assert (a.observable() == b.observable()).all()
    assert (a.hbm_bins() == b.hbm_bins()).all()
    assert (a.loads() == b.loads()).all()
    assert a.pmap() == b.pmap()


@pytest.mark.parametrize("cap,n,alpha", [(2000, 2000, 200), (3001, 2500, 0), (8192, 8000, 500)])
def test_build_state_invariants(cap, n, alpha):
    vs = 8
    k, v = _data(n, vs, 99)
    m = O.OracleMap(cap, vs, alpha_pm=alpha, key=KEY)
    assert m.build(k, v) == O.OK
    s = m.s
    B, K, Z = s["B"], s["K"], s["Z"]
    # contents are exactly the input
    assert m.logical_contents() == {int(a): bytes(b) for a, b in zip(k, v)}
    _check_pages(m.observable(), Z, vs, s["page_bytes"])
    _check_pages(m.hbm_bins(), Z, vs, s["page_bytes"])
    # where each key landed
    where = {}
    for b, page in enumerate(np.concatenate([m.hbm_bins(), m.observable()])):
        for key, _ in O.decode_page(page, Z, vs):
            where[key] = b
    loads = m.loads()
    assert (np.bincount(list(where.values()), minlength=B) == loads).all()
    assert loads.max() <= Z
    pairs = _prf_pairs(k, B)
    # P2C in rounds of ceil(B/16): the second bin only when strictly less
    # loaded at the start of the key's round
    rs = (B + 15) // 16
    start = np.zeros(B, dtype=np.int64)
    for r0 in range(0, n, rs):
        for i in range(r0, min(n, r0 + rs)):
            p1, p2 = pairs[i]
            dest = where[int(k[i])]
            assert dest in (p1, p2)
            assert dest == (p2 if start[p2] < start[p1] else p1)
        for i in range(r0, min(n, r0 + rs)):
            start[where[int(k[i])]] += 1
    # position map: each key once, with its pair, in its least-loaded row
    pm = m.pmap()
    assert sorted(e[1] for e in pm) == sorted(int(x) for x in k)
    row_of = {e[1]: e[0] for e in pm}
    for (row, key, p1, p2) in pm:
        i = int(np.nonzero(k == np.uint64(key))[0][0])
        assert (p1, p2) == pairs[i]
    R = s["R_pm"]
    rs = (R + 15) // 16
    cnt = np.zeros(R, dtype=np.int64)
    for r0 in range(0, n, rs):
        for i in range(r0, min(n, r0 + rs)):
            rows = _pm_rows(k[i], R)
            best = rows[0]
            for r in rows[1:]:
                if cnt[r] < cnt[best]:
                    best = r
            assert row_of[int(k[i])] == best
        for i in range(r0, min(n, r0 + rs)):
            cnt[row_of[int(k[i])]] += 1
    assert m.pm_max_row() <= s["W"]


def test_build_trace_is_data_independent():
    cap, n, vs = 3000, 2500, 16
    traces = []
    for seed in (1, 2, 3):
        k, v = _data(n, vs, 1000 * seed)
        m = O.OracleMap(cap, vs, key=bytes([seed]) * 32, trace=True)
        assert m.build(k, v) == O.OK
        traces.append(m.trace())
    M = O.sizing(cap, vs)["M"]
    want = np.zeros(M, dtype=O.TRACE_DTYPE)
    want["kind"] = 1
    want["page"] = np.arange(M)
    for t in traces:
        assert (t == want).all()


def test_max_load_at_2_20_within_lmax():
    """Claim 4.2 with constant 1 at N = 2^20, c = 8: max load <= 14 (the
    paper's simulation shows 12, two below the bound)."""
    n = 1 << 20
    m = O.OracleMap(n, 8, key=KEY)
    k, v = _data(n, 8, 5)
    assert m.build(k, v, mode=1) == O.OK
    mx = int(m.loads().max())
    assert mx <= m.s["lmax"] == 14
    assert mx >= 10  # P2C, not a perfect spread


def test_build_errors():
    vs = 8
    k, v = _data(100, vs, 3)
    m = O.OracleMap(64, vs, key=KEY)
    assert m.build(k, v) == O.EINVAL  # more keys than capacity
    m = O.OracleMap(128, vs, key=KEY)
    kd = k.copy()
    kd[7] = kd[50]
    assert m.build(kd, v) == O.EDUPKEY
    assert m.build(k, v) == O.ESTATE  # poisoned after an error
    m = O.OracleMap(128, vs, bin_slots=1, key=KEY)
    assert m.build(k, v) == O.EOVERFLOW
    m = O.OracleMap(128, vs, W=1, key=KEY)
    assert m.build(k, v) == O.EOVERFLOW
    m = O.OracleMap(128, vs, key=KEY)
    assert m.build(k, v) == O.OK
    assert m.build(k, v) == O.EINVAL  # one build per map

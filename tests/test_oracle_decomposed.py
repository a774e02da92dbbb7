"""The decomposed HBM store (Sec. 5.2, "Decomposed HBM storage" and "Dynamic
HBM management") in the oracle, pinned against the page layout it replaces.

The decomposed store changes only where the items of the K HBM bins are
kept (value-pool entries listed under their bin, instead of dummy-padded
pages); which bin holds which key, every load, every host page, the
position map, the answers and the trace are those of the page layout.  So a
map with the decomposed store and one without, fed the same inputs, must
agree on all of those, and the decomposed map's pool must hold exactly the
page layout's HBM-bin items plus its stash."""
import numpy as np
import pytest

import oracle as O
import synth

KEY = bytes(range(160, 192))


def _items(m):
    """(key, bin, value) of every stored item outside the host pages."""
    s = m.s
    out = set(m.stash())
    for b, page in enumerate(m.hbm_bins()):
        for k, v in O.decode_page(page, s["Z"], s["vs"]):
            out.add((k, b, v))
    return out


def _agree(a, d):
    assert np.array_equal(a.observable(), d.observable())
    assert np.array_equal(a.loads(), d.loads())
    assert a.pmap() == d.pmap()
    assert np.array_equal(a.trace(), d.trace())
    assert not d.hbm_bins().any()  # no HBM pages in the decomposed store
    assert _items(a) == _items(d)
    assert a.stash_live == d.stash_live and a.live == d.live and a.ctr == d.ctr
    K = a.s["K"]
    assert d.hbm_live == int(d.loads()[:K].sum()) <= d.s["hbm_bound"]
    assert a.logical_contents() == d.logical_contents()


@pytest.mark.parametrize("cap,n,vs,alpha,c", [(2048, 1500, 16, 200, 8), (4096, 4000, 8, 600, 8), (1000, 900, 24, 0, 8),
                                              (8192, 7000, 8, 500, 4), (1 << 14, 12000, 64, 999, 8)])
def test_decomposed_store_agrees_with_the_page_layout(cap, n, vs, alpha, c):
    a = O.OracleMap(cap, vs, alpha_pm=alpha, c=c, key=KEY, trace=True)
    d = O.OracleMap(cap, vs, alpha_pm=alpha, c=c, key=KEY, trace=True, decomposed=True)
    k, v = synth.keys(n, 80 + vs), synth.values(n, vs, 81)
    assert a.build(k, v) == d.build(k, v) == O.OK
    _agree(a, d)
    rng = np.random.default_rng(alpha + vs)
    fresh = synth.keys(40000, 82, offset=10**8)
    present = set(int(x) for x in k)
    for step in range(40):
        q = int(rng.integers(1, 600))
        pool = np.array(sorted(present), dtype=np.uint64)
        r = rng.random(q)
        keys = np.where(r < 0.3, pool[rng.integers(0, 5, q)],
                        np.where(r < 0.85, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
        ops = rng.choice([O.GET, O.PUT, O.DEL], size=q, p=[0.5, 0.3, 0.2]).astype(np.uint8)
        if len(present) + q > cap:
            ops[ops == O.PUT] = O.DEL
        vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
        ra, voa, sta = a.access(ops, keys, vals)
        rd, vod, std = d.access(ops, keys, vals)
        assert ra == rd == O.OK and np.array_equal(voa, vod) and np.array_equal(sta, std)
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == O.PUT:
                present.add(int(key))
            elif op == O.DEL:
                present.discard(int(key))
        if step % 10 == 9:
            _agree(a, d)
    _agree(a, d)


def test_hbm_bound_is_claim43_rounded_up():
    for cap, c, alpha in ((1 << 16, 8, 200), ((1 << 24) + (1 << 16), 8, 200), (1 << 20, 16, 500), (1000, 8, 0)):
        s = O.sizing(cap, 8, c=c, alpha_pm=alpha)
        exact = O.claim43_bound(s["K"], c, s["lmax"], cap)
        assert s["hbm_bound"] == int(np.ceil(exact))
        assert s["hbm_bound"] >= s["K"] * c  # at least the mean load of the HBM bins

"""The decomposed HBM store on the GPU (BOLT_F_DECOMPOSED; Sec. 5.2,
"Decomposed HBM storage" and "Dynamic HBM management"): the HBM bins' items
are value-pool entries listed under their bin, taken from and returned to a
free-address ring.

* Against the oracle's decomposed store, bit for bit: observable pages,
  loads, position map, trace, answers; the pool (every entry in use, HBM-bin
  items and stash alike) as a set of (key, bin, value), read through the
  ring (an entry in the ring's free range twice, or one out of range, fails
  the read).  Builds of every shape, one-round, several-round and
  one-command batches, both stores, sealed pages, many-map calls mixing
  both layouts.
* At config-2 size (N = 2^24, 64-byte values), a decomposed map and a page
  map fed the same inputs end with the same answers, pages, loads,
  position map and trace; the decomposed map needs less HBM."""
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


def _stream(t, k, cap, vs, sizes, seed, check_every=5):
    rng = np.random.default_rng(seed)
    fresh = synth.keys(40000, seed + 7, offset=10**8)
    present = set(int(x) for x in k)
    for b, q in enumerate(sizes):
        ops, keys, vals = _mixed(rng, present, fresh, q, vs)
        if len(present) > cap - q:
            ops[ops == 1] = 2
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, (b, q, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), (b, q)
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == 1:
                present.add(int(key))
            elif op == 2:
                present.discard(int(key))
        if b % check_every == check_every - 1:
            t.assert_same_state()
    t.assert_same_state()


@pytest.mark.parametrize("cap,n,vs,kw", [
    (64, 0, 8, {}), (64, 1, 8, {}), (64, 64, 8, {}), (1000, 999, 8, dict(alpha_permille=500)),
    (4096, 3000, 64, {}), (5000, 4321, 24, dict(alpha_permille=999)), (100000, 99999, 64, dict(c=4)),
    (1 << 17, 100000, 8, dict(pm_choices=2, pm_keys_per_row=8))])
def test_decomposed_build_matches_the_oracle(cap, n, vs, kw):
    t = Twin(cap, vs, decomposed=True, **kw)
    k, v = workload(n, vs, 900 + n)
    assert t.build(k, v) == (0, 0, 0)
    t.assert_same_state()
    assert not t.g.hbm_bins().any()
    K = t.g.sizes["K"]
    assert len(t.g.stash()) == int(t.g.loads()[:K].sum())  # after the build the pool holds the HBM bins' items


@pytest.mark.parametrize("cap,n,vs,observable,kw,sizes", [
    (2048, 1500, 16, 0, {}, [1, 200, 37, 1, 150, 9, 64, 1, 300, 5] * 3),
    (4096, 3000, 64, 1, dict(alpha_permille=600), [500, 1, 1, 333, 80, 600, 2, 1, 450, 12] * 2),
    (1 << 15, 30000, 8, 0, {}, [4096, 1, 2000, 8192, 1, 700, 3000]),
    (1 << 20, (1 << 20) - 100, 16, 0, {}, [4096, 3000, 4096, 1, 4096]),  # one-round batches
    (1 << 18, 1 << 17, 8, 1, dict(alpha_permille=999), [2000, 1, 2000, 777]),
])
def test_decomposed_access_matches_the_oracle(cap, n, vs, observable, kw, sizes):
    t = Twin(cap, vs, observable=observable, decomposed=True, **kw)
    k, v = workload(n, vs, 300 + n)
    assert t.build(k, v) == (0, 0, 0)
    _stream(t, k, cap, vs, sizes, n + vs)


def test_decomposed_sealed_store_matches_the_oracle():
    t = Twin(4096, 16, seal=True, decomposed=True, alpha_permille=300)
    k, v = workload(3500, 16, 41)
    assert t.build(k, v) == (0, 0, 0)
    _stream(t, k, 4096, 16, [1, 300, 1, 1000, 64, 2, 900], 42)


def test_many_map_calls_mix_both_layouts():
    import torch
    import paper_2509_01742_amd as B

    specs = [(2048, 1500, 16, True), (2048, 1500, 16, False), (1 << 14, 12000, 8, True), (5000, 400, 64, True)]
    twins, inputs, ks = [], [], []
    for j, (cap, n, vs, dec) in enumerate(specs):
        t = Twin(cap, vs, decomposed=dec, key=bytes((11 * j + i) & 255 for i in range(32)))
        k, v = workload(n, vs, 1700 + j)
        assert t.o.build(k, v) == 0
        twins.append(t)
        inputs.append((dev_u64(k), dev_u8(v)))
        ks.append(k)
    assert B.build_many([t.g for t in twins], inputs) == 0
    torch.cuda.synchronize()
    for t in twins:
        assert t.g.status() == 0
        t.assert_same_state()
    rng = np.random.default_rng(8)
    for rnd in range(4):
        batches, host = [], []
        for j, (cap, n, vs, dec) in enumerate(specs):
            q = int(rng.integers(1, 1500))
            ops, keys, vals = _mixed(rng, set(int(x) for x in ks[j][:300]), synth.keys(100, j + 70, offset=10**8),
                                     q, vs)
            ops[ops == 1] = 0
            batches.append((dev_u8(ops), dev_u64(keys), dev_u8(vals),
                            torch.zeros((q, vs), dtype=torch.uint8, device="cuda"),
                            torch.zeros(q, dtype=torch.uint8, device="cuda")))
            host.append((ops, keys, vals))
        assert B.access_many([t.g for t in twins], batches) == 0
        torch.cuda.synchronize()
        for j, t in enumerate(twins):
            rc_o, vo_o, st_o = t.o.access(*host[j])
            assert rc_o == 0 and t.g.status() == 0
            assert np.array_equal(batches[j][3].cpu().numpy(), vo_o)
            assert np.array_equal(batches[j][4].cpu().numpy(), st_o)
    for t in twins:
        t.assert_same_state()


@pytest.mark.timeout(600)
def test_config2_decomposed_equals_page_layout():
    import torch
    import paper_2509_01742_amd as B

    wl = synth.config2(n_batches=16)
    key = bytes(range(50, 82))
    maps = []
    for dec in (False, True):
        p = B.params(wl.cap, wl.vs, key=key)
        p.flags |= B.BOLT_F_TRACE | (B.BOLT_F_DECOMPOSED if dec else 0)
        maps.append(B.Map(p))
    for m in maps:
        assert m.build(dev_u64(wl.build_keys), dev_u8(wl.build_vals)) == 0
    outs = [[], []]
    for ops, keys, vals in wl.batches:
        d = (dev_u8(ops), dev_u64(keys), dev_u8(vals))
        for j, m in enumerate(maps):
            vo = torch.zeros((ops.size, wl.vs), dtype=torch.uint8, device="cuda")
            st = torch.zeros(ops.size, dtype=torch.uint8, device="cuda")
            assert m.access(*d, vo, st) == 0
            outs[j].append((vo, st))
    torch.cuda.synchronize()
    page, dec = maps
    assert page.status() == 0 and dec.status() == 0
    for (a, sa), (b, sb) in zip(*outs):
        assert torch.equal(a, b) and torch.equal(sa, sb)
    assert np.array_equal(page.observable(), dec.observable())
    assert np.array_equal(page.loads(), dec.loads())
    assert np.array_equal(page.trace(), dec.trace())
    pa, da = page.pmap_arrays(), dec.pmap_arrays()
    o1, o2 = np.argsort(pa[1]), np.argsort(da[1])
    for x, y in zip(pa, da):
        assert np.array_equal(x[o1], y[o2])
    # the decomposed pool = the page map's HBM-bin items plus its stash
    K, Z, vs = page.sizes["K"], page.sizes["Z"], wl.vs
    hb = page.hbm_bins()
    cnt = page.loads()[:K].astype(np.int64)  # a page bin's items are its first cnt slots
    real = np.arange(Z)[None, :] < cnt[:, None]
    assert np.array_equal(hb[:, :8].copy().view("<u8")[:, 0], (np.uint64(1) << cnt.astype(np.uint64)) - np.uint64(1))
    hk = np.ascontiguousarray(hb[:, 8:8 + 8 * Z]).view("<u8").reshape(K, Z)[real]
    hbin = np.repeat(np.arange(K, dtype=np.uint32), cnt)
    hv = np.ascontiguousarray(hb[:, 8 + 8 * Z:8 + 8 * Z + vs * Z]).reshape(K, Z, vs)[real]
    sk, sb, sv = page.stash_arrays()
    want_k, want_b, want_v = np.concatenate([hk, sk]), np.concatenate([hbin, sb]), np.concatenate([hv, sv])
    dk, db, dv = dec.stash_arrays()
    ow, od = np.argsort(want_k), np.argsort(dk)
    assert np.array_equal(want_k[ow], dk[od]) and np.array_equal(want_b[ow], db[od])
    assert np.array_equal(want_v[ow], dv[od])
    sp, sd = page.stats(), dec.stats()
    assert sp["stash_live"] == sd["stash_live"] and sp["live"] == sd["live"]
    assert B.footprint(dec.p)[0] < B.footprint(page.p)[0]
    for m in maps:
        m.close()

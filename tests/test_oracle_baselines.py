"""The CPU baselines the benchmark times beside the GPU.

* O1 in C (a hash table with linear probing and backward-shift deletion)
  gives exactly the answers of the dictionary definition, over streams that
  delete and re-insert often inside small, crowded tables.
* The oracle built with OpenMP (the parallel baseline of the same
  procedure) ends every build and every batch in exactly the state of the
  single-thread oracle: pages, HBM bins, loads, stash, position map,
  answers and, where a trace is kept, the trace."""
import numpy as np
import pytest

import oracle as O
import synth

KEY = bytes(range(90, 122))


@pytest.mark.parametrize("cap,universe,seed", [(8, 12, 1), (64, 100, 2), (1000, 3000, 3), (5, 5, 4)])
def test_plain_c_matches_the_dictionary(cap, universe, seed):
    rng = np.random.default_rng(seed)
    vs = 8
    keys_u = synth.keys(universe, 600 + seed)
    p, c = O.PlainMap(vs), O.PlainMapC(cap, vs)
    n0 = min(cap // 2, universe)
    k0, v0 = keys_u[:n0], synth.values(n0, vs, seed)
    p.build(k0, v0)
    assert c.build(k0, v0) == O.OK
    for b in range(300):
        q = int(rng.integers(1, 40))
        keys = keys_u[rng.integers(0, universe, q)]
        ops = rng.choice([O.GET, O.PUT, O.DEL], size=q, p=[0.4, 0.3, 0.3]).astype(np.uint8)
        # keep the live set within the capacity
        live = set(p.d)
        for i in range(q):
            if ops[i] == O.PUT and int(keys[i]) not in live:
                if len(live) >= cap:
                    ops[i] = O.DEL
                else:
                    live.add(int(keys[i]))
            elif ops[i] == O.DEL:
                live.discard(int(keys[i]))
        vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
        wvo, wst = p.access(ops, keys, vals)
        rc, vo, st = c.access(ops, keys, vals)
        assert rc == O.OK and np.array_equal(st, wst) and np.array_equal(vo, wvo), b
        assert len(c) == len(p.d)
    # every key of the universe still answers as the dictionary says
    ops = np.zeros(universe, np.uint8)
    wvo, wst = p.access(ops, keys_u, np.zeros((universe, vs), np.uint8))
    rc, vo, st = c.access(ops, keys_u, np.zeros((universe, vs), np.uint8))
    assert rc == O.OK and np.array_equal(st, wst) and np.array_equal(vo, wvo)
    assert c.access(np.array([3], np.uint8), keys_u[:1], np.zeros((1, vs), np.uint8))[0] == O.EINVAL


def _same(a, b, trace):
    assert np.array_equal(a.observable(), b.observable())
    assert np.array_equal(a.hbm_bins(), b.hbm_bins())
    assert np.array_equal(a.loads(), b.loads())
    assert a.stash() == b.stash()
    assert a.pmap() == b.pmap()
    assert (a.ctr, a.live, a.stash_live) == (b.ctr, b.live, b.stash_live)
    if trace:
        assert np.array_equal(a.trace(), b.trace())


@pytest.mark.parametrize("cap,n,vs,alpha,trace", [(1 << 15, 30000, 16, 200, False), (1 << 14, 16000, 8, 0, True),
                                                  (5000, 4000, 64, 600, False)])
def test_openmp_oracle_equals_the_single_thread_oracle(cap, n, vs, alpha, trace):
    omp = O.load_openmp()
    a = O.OracleMap(cap, vs, alpha_pm=alpha, key=KEY, trace=trace)
    b = O.OracleMap(cap, vs, alpha_pm=alpha, key=KEY, trace=trace, lib=omp)
    k, v = synth.keys(n, 70 + vs), synth.values(n, vs, 71)
    assert a.build(k, v) == O.OK and b.build(k, v) == O.OK
    _same(a, b, trace)
    rng = np.random.default_rng(vs)
    fresh = synth.keys(20000, 72, offset=10**8)
    for step in range(6):
        q = int(rng.integers(1, 4000))
        keys = np.where(rng.random(q) < 0.85, k[rng.integers(0, n, q)], fresh[rng.integers(0, fresh.size, q)])
        ops = rng.choice([O.GET, O.PUT, O.DEL], size=q, p=[0.6, 0.2, 0.2]).astype(np.uint8)
        if n + q > cap:
            ops[ops == O.PUT] = O.GET
        vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
        ra, voa, sta = a.access(ops, keys, vals)
        rb, vob, stb = b.access(ops, keys, vals)
        assert ra == rb == O.OK and np.array_equal(voa, vob) and np.array_equal(sta, stb)
    _same(a, b, trace)
    dk = np.concatenate([k[:100], k[:1]])  # a duplicate key: both refuse the build
    a2 = O.OracleMap(cap, vs, key=KEY)
    b2 = O.OracleMap(cap, vs, key=KEY, lib=omp)
    assert a2.build(dk, synth.values(101, vs, 1)) == b2.build(dk, synth.values(101, vs, 1)) == O.EDUPKEY

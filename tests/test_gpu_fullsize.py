"""The measured workloads at their full sizes, in the launch configuration
the benchmark times.

* Config 1 (N = 2^16, 2^14 single GETs then 2^12 single PUTs, one command
  per call): every answer, the final state and the whole trace against the
  oracle, bit for bit.
* Config 2 (N = 2^24 with 2^16 insert headroom, 64-byte values, 1 KiB
  pages, 24 Zipf batches of 4096 commands on the pinned host store, the
  rebuilt pages of each batch sent during the next one, no flush until the
  end): every answer against the oracle and the plain definition, then the
  whole state (observable pages, HBM bins, loads, stash, position map) and
  the whole trace against the oracle, bit for bit.  The oracle runs on a
  thread of its own beside the GPU (about a minute at this size).  A second
  map built from another dataset of the same size writes the same build
  trace.
* Config 3 (N = 2^26, 8-byte values, then 2^16 uniform GETs): every answer
  against the build arrays, and the same invariants.
"""
import numpy as np
import pytest

import synth
from gpu_util import Twin, dev_u64, dev_u8

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


def test_config1_single_commands_against_the_oracle():
    wl = synth.config1()
    t = Twin(wl.cap, wl.vs)
    assert t.build(wl.build_keys, wl.build_vals) == (0, 0, 0)
    for b, (ops, keys, vals) in enumerate(wl.batches):
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, b
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), b
    t.assert_same_state()


def _plain_answers(build_keys, build_vals, batches):
    """Expected (values, status) of each batch by the plain definition: the
    commands one by one in order; a dictionary holds the keys they changed."""
    order = np.argsort(build_keys)
    sk, sv = build_keys[order], build_vals[order]
    changed = {}
    vs = build_vals.shape[1]
    zero = np.zeros(vs, np.uint8)
    out = []
    for ops, keys, vals in batches:
        vo = np.zeros((ops.size, vs), np.uint8)
        st = np.zeros(ops.size, np.uint8)
        pos = np.searchsorted(sk, keys)
        for i in range(ops.size):
            k = int(keys[i])
            if k in changed:
                cur = changed[k]
            else:
                j = int(pos[i])
                cur = sv[j] if j < sk.size and int(sk[j]) == k else None
            op = int(ops[i])
            if op == 0:
                st[i] = cur is not None
                vo[i] = cur if cur is not None else zero
            elif op == 1:
                st[i] = 1 if cur is not None else 2
                changed[k] = vals[i].copy()
            else:
                st[i] = 3 if cur is not None else 0
                changed[k] = None
        out.append((vo, st))
    ck = np.array(list(changed), dtype=np.uint64)
    j = np.searchsorted(sk, ck)
    in_build = (j < sk.size) & (sk[np.minimum(j, sk.size - 1)] == ck)
    alive = np.array([changed[int(k)] is not None for k in ck], dtype=bool)
    live = build_keys.size + int((~in_build & alive).sum()) - int((in_build & ~alive).sum())
    return out, live


def _invariants(m, live, steps):
    s = m.sizes
    loads = m.loads()
    assert int(loads.max()) <= s["Z"]
    assert int(loads.sum(dtype=np.uint64)) == live
    st = m.stats()
    assert st["live"] == live and st["steps"] == steps
    assert st["stash_live"] <= s["stash_bound"] and st["stash_highwater"] <= s["stash_bound"]


def _run_batches(m, batches, vs):
    import torch

    got = []
    for ops, keys, vals in batches:
        q = ops.size
        out = torch.zeros((q, vs), dtype=torch.uint8, device="cuda")
        st = torch.zeros(q, dtype=torch.uint8, device="cuda")
        assert m.access(dev_u8(ops), dev_u64(keys), dev_u8(vals), out, st) == 0
        got.append((out, st))
    torch.cuda.synchronize()
    assert m.status() == 0
    return [(o.cpu().numpy(), s.cpu().numpy()) for o, s in got]


def _sorted_rows(arrs, by):
    order = np.argsort(arrs[by], kind="stable")
    return [a[order] for a in arrs]


@pytest.mark.timeout(900)
def test_config2_full_size_state_and_trace_match_the_oracle():
    import threading

    import torch

    import oracle as O
    import paper_2509_01742_amd as B

    wl = synth.config2(n_batches=24)
    key = bytes(range(100, 132))
    print("config 2 at full size: oracle on a thread, GPU beside it", flush=True)
    o = O.OracleMap(wl.cap, wl.vs, key=key, trace=True)
    o_out = {}

    def run_oracle():
        o_out["build"] = o.build(wl.build_keys, wl.build_vals)
        o_out["batches"] = [o.access(ops, keys, vals) for ops, keys, vals in wl.batches]

    th = threading.Thread(target=run_oracle)
    th.start()
    try:
        p = B.params(wl.cap, wl.vs, key=key)
        p.flags |= B.BOLT_F_TRACE
        g = B.Map(p)
        assert g.build(dev_u64(wl.build_keys), dev_u8(wl.build_vals)) == 0
        torch.cuda.synchronize()
        assert g.status() == 0
        build_trace = g.trace()
        # another dataset of the same size writes the same build trace
        p2 = B.params(wl.cap, wl.vs, key=bytes(range(7, 39)))
        p2.flags |= B.BOLT_F_TRACE
        g2 = B.Map(p2)
        k2, v2 = synth.keys(wl.n, 0xB0170F00), synth.values(wl.n, wl.vs, 0xB0170F01)
        assert g2.build(dev_u64(k2), dev_u8(v2)) == 0
        torch.cuda.synchronize()
        assert g2.status() == 0
        assert np.array_equal(g2.trace(), build_trace), "build traces differ across datasets"
        g2.close()
        del k2, v2
        got = _run_batches(g, wl.batches, wl.vs)  # no flush between batches
    finally:
        th.join()
    assert o_out["build"] == 0
    want, live = _plain_answers(wl.build_keys, wl.build_vals, wl.batches)
    for b, ((vo, st), (rc_o, vo_o, st_o), (wvo, wst)) in enumerate(zip(got, o_out["batches"], want)):
        assert rc_o == 0, b
        assert np.array_equal(st_o, wst) and np.array_equal(vo_o, wvo), b
        assert np.array_equal(st, st_o), b
        assert np.array_equal(vo, vo_o), b
    print("answers match; comparing state", flush=True)
    M = o.s["M"]
    assert build_trace.size == M
    assert np.array_equal(g.observable(), o.observable()), "observable pages differ"
    assert np.array_equal(g.hbm_bins(), o.hbm_bins()), "HBM bins differ"
    assert np.array_equal(g.loads(), o.loads()), "bin loads differ"
    gs, os_ = _sorted_rows(g.stash_arrays(), 0), _sorted_rows(o.stash_arrays(), 0)
    assert gs[0].size == os_[0].size and gs[0].size > 0
    for a, b_ in zip(gs, os_):
        assert np.array_equal(a, b_), "stash differs"
    gp, op = _sorted_rows(g.pmap_arrays(), 1), _sorted_rows(o.pmap_arrays(), 1)
    assert gp[1].size == op[1].size == live
    for a, b_ in zip(gp, op):
        assert np.array_equal(a, b_), "position map differs"
    st = g.stats()
    assert st["live"] == o.live == live and st["steps"] == o.ctr == 24 * 4096
    assert st["stash_live"] == o.stash_live
    tg, to = g.trace(), o.trace()
    assert tg.size == to.size, (tg.size, to.size)
    assert np.array_equal(tg[:M], to[:M]) and np.array_equal(tg, to), "trace differs"
    _invariants(g, live, 24 * 4096)
    g.close()
    o.close()


def test_config3_full_size_build_and_gets():
    import torch
    import paper_2509_01742_amd as B

    wl = synth.config3()
    m = B.Map(B.params(wl.cap, wl.vs))
    assert m.build(dev_u64(wl.build_keys), dev_u8(wl.build_vals)) == 0
    torch.cuda.synchronize()
    assert m.status() == 0
    _invariants(m, wl.n, 0)
    got = _run_batches(m, wl.batches, wl.vs)
    order = np.argsort(wl.build_keys)
    sk, sv = wl.build_keys[order], wl.build_vals[order]
    for (ops, keys, _), (vo, st) in zip(wl.batches, got):
        j = np.searchsorted(sk, keys)
        assert (st == 1).all()
        assert np.array_equal(vo, sv[j])
    _invariants(m, wl.n, sum(b[0].size for b in wl.batches))
    m.close()

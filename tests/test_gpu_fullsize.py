"""The measured workloads at their full sizes, in the launch configuration
the benchmark times.

* Config 1 (N = 2^16, 2^14 single GETs then 2^12 single PUTs, one command
  per call): every answer, the final state and the whole trace against the
  oracle, bit for bit.
* Config 2 (N = 2^24, 64-byte values, Zipf batches of 4096 commands on the
  pinned host store): the oracle would take minutes at this size, so every
  answer is checked against the plain definition (a dictionary of the keys
  the stream changed, over the build arrays), and the state against the
  invariants that hold at any size (bin loads at most Z and summing to the
  live keys, the stash within its bound, one tape step per command).
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


def test_config2_full_size_batches():
    import torch
    import paper_2509_01742_amd as B

    wl = synth.config2(n_batches=24)
    m = B.Map(B.params(wl.cap, wl.vs))
    assert m.build(dev_u64(wl.build_keys), dev_u8(wl.build_vals)) == 0
    torch.cuda.synchronize()
    assert m.status() == 0
    got = _run_batches(m, wl.batches, wl.vs)
    want, live = _plain_answers(wl.build_keys, wl.build_vals, wl.batches)
    for b, ((vo, st), (wvo, wst)) in enumerate(zip(got, want)):
        assert np.array_equal(st, wst), b
        assert np.array_equal(vo, wvo), b
    _invariants(m, live, sum(b[0].size for b in wl.batches))
    m.close()


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

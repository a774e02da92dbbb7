"""Sealed commands and responses on the GPU (BOLT_F_SEAL_CMDS; Sec. 3, the
host relays only encrypted instructions and results; Sec. 5.1, the decode
and response modules).  The client side is the oracle's: its records are
pinned against OpenSSL, and nothing of the library seals the commands
here.

* One map, a stream of sealed requests of mixed sizes and ops: every
  response record equals, byte for byte, the oracle's seal of the oracle
  map's answers; the state and trace end as the oracle's.
* A changed, truncated or replayed request changes nothing and poisons the
  map with BOLT_ETAMPER.
* Serving: sealed maps beside plain ones on one server; every opened
  response equals the plain dictionary's answer, alone and in the mix."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import Twin, dev_u8, workload

pytestmark = pytest.mark.gpu

SKEY = bytes((7 * i + 3) & 255 for i in range(32))


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


def _mixed(rng, present, fresh, q, vs, bad_op=False):
    pool = np.array(sorted(present), dtype=np.uint64)
    r = rng.random(q)
    keys = np.where(r < 0.3, pool[rng.integers(0, 5, q)],
                    np.where(r < 0.85, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
    ops = rng.choice([0, 1, 2], size=q, p=[0.5, 0.35, 0.15]).astype(np.uint8)
    if bad_op:
        ops[q // 2] = 9
    return ops, keys.astype(np.uint64), rng.integers(0, 256, (q, vs), dtype=np.uint8)


def _gpu_sealed(t, req, q, vs):
    import torch

    d_resp = torch.zeros((q, 24 + vs), dtype=torch.uint8, device="cuda")
    rc = t.g.access_sealed(dev_u8(req), d_resp)
    torch.cuda.synchronize()
    return rc, t.g.status(), d_resp.cpu().numpy()


def _oracle_sealed(t, seq, req, vs):
    """The oracle's side: open, run, seal (a rejected batch answers 0xFF and zeros)."""
    bad, ops, keys, vals = O.cmd_open(SKEY, seq, req, vs)
    assert bad == 0
    rc, vo, st = t.o.access(ops, keys, vals)
    if rc == O.EINVAL:
        st = np.full(ops.size, 0xFF, np.uint8)
        vo = np.zeros_like(vo)
    return rc, O.resp_seal(SKEY, seq, st, vo, vs), (ops, keys, vals)


@pytest.mark.parametrize("observable,vs", [(0, 16), (1, 64)])
def test_sealed_requests_match_the_oracle(observable, vs):
    t = Twin(1 << 14, vs, observable=observable, session_key=SKEY)
    k, v = workload(12000, vs, 501 + vs)
    assert t.build(k, v) == (0, 0, 0)
    p = O.PlainMap(vs)
    p.build(k, v)
    rng = np.random.default_rng(vs)
    fresh = synth.keys(20000, 4411, offset=10**8)
    present = set(int(x) for x in k)
    for seq, q in enumerate([1, 7, 300, 1, 4096, 2, 1000, 1, 8192, 55], start=1):
        ops, keys, vals = _mixed(rng, present, fresh, q, vs, bad_op=(seq == 6))
        if len(present) > (1 << 14) - q:
            ops[ops == 1] = 2
        req = O.cmd_seal(SKEY, seq, ops, keys, vals, vs)  # the client's records
        rc_o, want, _ = _oracle_sealed(t, seq, req, vs)
        rc_g, st, got = _gpu_sealed(t, req, q, vs)
        assert rc_g == 0 and st == 0, (seq, rc_g, st)
        assert np.array_equal(got, want), seq  # every response record, byte for byte
        bad, st_r, vo_r = O.resp_open(SKEY, seq, got, vs)
        assert bad == 0
        if seq == 6:
            assert rc_o == O.EINVAL and (st_r == 0xFF).all()
            continue
        assert rc_o == 0
        wvo, wst = p.access(ops, keys, vals)
        assert np.array_equal(st_r, wst) and np.array_equal(vo_r, wvo), seq
        for op, key in zip(ops.tolist(), keys.tolist()):
            if op == 1:
                present.add(int(key))
            elif op == 2:
                present.discard(int(key))
    t.assert_same_state()


@pytest.mark.parametrize("how", ["changed", "truncated", "replayed", "other_session"])
def test_tampered_sealed_request_changes_nothing_and_poisons(how):
    import paper_2509_01742_amd as B

    vs = 16
    t = Twin(4096, vs, session_key=SKEY)
    k, v = workload(3000, vs, 77)
    assert t.build(k, v) == (0, 0, 0)
    rng = np.random.default_rng(5)
    present = set(int(x) for x in k)
    fresh = synth.keys(100, 991, offset=10**8)
    ops, keys, vals = _mixed(rng, present, fresh, 200, vs)
    req1 = O.cmd_seal(SKEY, 1, ops, keys, vals, vs)
    rc_o, want, _ = _oracle_sealed(t, 1, req1, vs)
    rc_g, st, got = _gpu_sealed(t, req1, 200, vs)
    assert rc_o == 0 and rc_g == 0 and st == 0 and np.array_equal(got, want)
    ops2, keys2, vals2 = _mixed(rng, present, fresh, 50, vs)
    if how == "changed":
        req = O.cmd_seal(SKEY, 2, ops2, keys2, vals2, vs)
        req[17, 9] ^= 0x10
    elif how == "truncated":
        req = O.cmd_seal(SKEY, 2, ops2, keys2, vals2, vs)[:49]
    elif how == "replayed":
        req = req1
    else:
        req = O.cmd_seal(bytes(32), 2, ops2, keys2, vals2, vs)
    rc_g, st, got = _gpu_sealed(t, req, req.shape[0], vs)
    assert st == B.BOLT_ETAMPER
    # the rejected request changed nothing: the state is the oracle's after request 1
    t.assert_same_state()


def test_sealed_serving_alone_equals_mix_equals_reference():
    import paper_2509_01742_amd as B

    specs = [(1 << 12, 3000, 16, True), (1 << 14, 12000, 64, False), (1 << 15, 30000, 64, True)]
    maps = [(cap, synth.keys(n, 7300 + j), synth.values(n, vs, 7400 + j), vs, sealed)
            for j, (cap, n, vs, sealed) in enumerate(specs)]
    rng = np.random.default_rng(21)
    reqs = []
    for r in range(150):
        j = int(rng.integers(0, len(maps)))
        cap, k, v, vs, sealed = maps[j]
        q = int(min(600, max(1, int(2 ** (np.log2(600) * rng.random())))))
        keys = k[synth.zipf_ranks(k.size, q, 0.99, rng)].astype(np.uint64)
        ops = rng.choice([0, 1, 2], size=q, p=[0.8, 0.15, 0.05]).astype(np.uint8)
        reqs.append((j, ops, keys, rng.integers(0, 256, (q, vs), dtype=np.uint8)))
    pm = [O.PlainMap(vs) for _, _, _, vs, _ in maps]
    for (cap, k, v, vs, _), p in zip(maps, pm):
        p.build(k, v)
    ref = [pm[j].access(ops, keys, vals) for j, ops, keys, vals in reqs]

    def run(server_maps, order):
        srv = B.Server(streams=4)
        ids = {j: srv.open_map(B.params(maps[j][0], maps[j][3], **({"session_key": SKEY} if maps[j][4] else {})),
                               maps[j][1], maps[j][2]) for j in server_maps}
        seq = {j: 0 for j in server_maps}
        out = {}
        pending = []
        for i in order:
            j, ops, keys, vals = reqs[i]
            vs = maps[j][3]
            if maps[j][4]:
                seq[j] += 1
                tk, resp = srv.submit_sealed(ids[j], O.cmd_seal(SKEY, seq[j], ops, keys, vals, vs), vs)
                assert resp is not None, tk
                pending.append((i, tk, ("sealed", seq[j], resp)))
            else:
                tk, vo, st = srv.submit(ids[j], ops, keys, vals)
                assert vo is not None, tk
                pending.append((i, tk, ("plain", vo, st)))
        assert srv.drain(120000) == 0
        for i, tk, res in pending:
            assert srv.poll(tk) == 0
            if res[0] == "sealed":
                bad, st, vo = O.resp_open(SKEY, res[1], res[2], maps[reqs[i][0]][3])
                assert bad == 0
                out[i] = (vo, st)
            else:
                out[i] = (res[1].copy(), res[2].copy())
        s = srv.stats()
        srv.close()
        return out, s

    mix, s = run(range(len(maps)), range(len(reqs)))
    assert s["failed"] == 0 and s["launches"] < len(reqs)
    for j in range(len(maps)):
        alone, _ = run([j], [i for i in range(len(reqs)) if reqs[i][0] == j])
        for i, res in alone.items():
            assert np.array_equal(res[0], mix[i][0]) and np.array_equal(res[1], mix[i][1]), i
    for i in range(len(reqs)):
        assert np.array_equal(mix[i][1], ref[i][1]) and np.array_equal(mix[i][0], ref[i][0]), i


def test_plain_and_sealed_submissions_are_kept_apart():
    import paper_2509_01742_amd as B

    srv = B.Server(streams=1)
    k, v = workload(100, 8, 3)
    sid = srv.open_map(B.params(256, 8, session_key=SKEY), k, v)
    pid = srv.open_map(B.params(256, 8), k, v)
    ops, keys, vals = np.zeros(2, np.uint8), k[:2], np.zeros((2, 8), np.uint8)
    assert srv.submit(sid, ops, keys, vals)[0] == B.BOLT_EINVAL  # a sealed map takes no plain commands
    assert srv.submit_sealed(pid, O.cmd_seal(SKEY, 1, ops, keys, vals, 8), 8)[0] == B.BOLT_EINVAL
    srv.close()

"""The serving loop through the C ABI: continuous batching over several
resident maps, admission by HBM footprint, and results that are the same
for a request alone and in the mix (tolerance 0: integers only)."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


MAPS = [(1 << 12, 3000, 16), (1 << 14, 12000, 64), (5000, 4000, 8), (1 << 15, 30000, 64)]


def _maps():
    out = []
    for j, (cap, n, vs) in enumerate(MAPS):
        out.append((cap, synth.keys(n, 7100 + j), synth.values(n, vs, 7200 + j), vs))
    return out


def _requests(maps, n_req, seed, qmax=600):
    """(map, ops, keys, vals) in arrival order: Zipf keys over each map's
    present keys plus absent ones, GET / PUT / DEL, sizes log-uniform."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        j = int(rng.integers(0, len(maps)))
        cap, k, v, vs = maps[j]
        q = int(min(qmax, max(1, int(2 ** (np.log2(qmax) * rng.random())))))
        ranks = synth.zipf_ranks(k.size, q, 0.99, rng)
        keys = k[ranks].copy()
        absent = rng.random(q) < 0.05
        keys[absent] = synth.keys(int(absent.sum()), 9000 + r, offset=10**9)
        ops = rng.choice([0, 1, 2], size=q, p=[0.8, 0.15, 0.05]).astype(np.uint8)
        ops[absent & (ops == 1)] = 0  # no inserts: capacity is never approached
        vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
        reqs.append((j, ops, keys.astype(np.uint64), vals))
    return reqs


def _plain(maps, reqs):
    """Answers of the non-oblivious reference map, request by request."""
    pm = [O.PlainMap(vs) for _, _, _, vs in maps]
    for (cap, k, v, vs), p in zip(maps, pm):
        p.build(k, v)
    out = []
    for j, ops, keys, vals in reqs:
        vo, st = pm[j].access(ops, keys, vals)
        out.append((vo, st))
    return out


def test_serving_alone_equals_mix_equals_reference():
    import paper_2509_01742_amd as B

    maps = _maps()
    reqs = _requests(maps, 300, 11)
    ref = _plain(maps, reqs)
    # the mix: every map on one server, all requests queued at once so the
    # loop coalesces them and overlaps maps
    srv = B.Server(streams=4)
    ids = [srv.open_map(B.params(cap, vs), k, v) for cap, k, v, vs in maps]
    got = []
    for j, ops, keys, vals in reqs:
        t, vo, st = srv.submit(ids[j], ops, keys, vals)
        assert vo is not None, t
        got.append((t, vo, st))
    assert srv.drain(120000) == 0
    for t, _, _ in got:
        assert srv.poll(t) == 0
    s = srv.stats()
    assert s["completed"] == len(reqs) and s["failed"] == 0
    assert s["launches"] < len(reqs)  # requests were batched together
    mix = [(vo.copy(), st.copy()) for _, vo, st in got]
    srv.close()
    # alone: one map per server, one request at a time
    alone = [None] * len(reqs)
    for j, (cap, k, v, vs) in enumerate(maps):
        srv = B.Server(streams=1)
        mid = srv.open_map(B.params(cap, vs), k, v)
        for i, (jj, ops, keys, vals) in enumerate(reqs):
            if jj != j:
                continue
            t, vo, st = srv.submit(mid, ops, keys, vals)
            assert srv.wait(t, 60000) == 0
            alone[i] = (vo.copy(), st.copy())
        srv.close()
    for i in range(len(reqs)):
        assert np.array_equal(mix[i][1], alone[i][1]) and np.array_equal(mix[i][0], alone[i][0]), i
        assert np.array_equal(mix[i][1], ref[i][1]) and np.array_equal(mix[i][0], ref[i][0]), i


def test_serving_admission_by_budget():
    import paper_2509_01742_amd as B

    maps = _maps()[:3]
    fps = []
    for cap, k, v, vs in maps:
        hbm, _ = B.footprint(B.params(cap, vs))
        fps.append(hbm)
    # room for the first two maps plus their command staging (about 1.5 MiB
    # together), not for the third as well
    budget = int(fps[0] + fps[1] + 3 * (1 << 20))
    assert fps[2] > 3 * (1 << 20) and fps[0] > fps[2]
    srv = B.Server(hbm_budget=budget, streams=2)
    ids = [srv.open_map(B.params(cap, vs), k, v) for cap, k, v, vs in maps]
    reqs = _requests(maps, 60, 12)
    ref = _plain(maps, reqs)
    got = [srv.submit(ids[j], ops, keys, vals) for j, ops, keys, vals in reqs]
    first = [g for g, r in zip(got, reqs) if r[0] != 2]
    for t, _, _ in first:
        assert srv.wait(t, 60000) == 0
    assert srv.map_state(ids[2])[0] == B.BOLT_SRV_WAITING
    third = [g for g, r in zip(got, reqs) if r[0] == 2]
    assert third and all(srv.poll(t) == 1 for t, _, _ in third)  # waiting for admission
    s = srv.stats()
    assert s["maps_waiting"] == 1 and s["hbm_used"] <= budget
    assert srv.close_map(ids[0]) == 0  # frees room: the third map is admitted
    assert srv.drain(120000) == 0
    assert srv.map_state(ids[0])[0] == B.BOLT_SRV_CLOSED and srv.map_state(ids[2])[0] == B.BOLT_SRV_RESIDENT
    for (t, vo, st), r, (rvo, rst) in zip(got, reqs, ref):
        assert np.array_equal(st, rst) and np.array_equal(vo, rvo)
    s = srv.stats()
    assert s["hbm_peak"] <= budget and s["maps_admitted"] == 3
    srv.close()


def test_serving_refusals_and_failed_maps():
    import paper_2509_01742_amd as B

    cap, k, v, vs = _maps()[2]
    srv = B.Server(max_batch=256)
    mid = srv.open_map(B.params(cap, vs), k, v)
    ops = np.zeros(4, np.uint8)
    vals = np.zeros((4, vs), np.uint8)
    assert srv.submit(mid, np.array([0, 9, 0, 0], np.uint8), k[:4], vals)[0] == B.BOLT_EINVAL  # bad op code
    assert srv.submit(mid, np.zeros(300, np.uint8), k[:300], np.zeros((300, vs), np.uint8))[0] == B.BOLT_EINVAL
    assert srv.submit(99, ops, k[:4], vals)[0] == B.BOLT_EINVAL
    t, vo, st = srv.submit(mid, ops, k[:4], vals)
    assert srv.wait(t) == 0 and (st == 1).all() and np.array_equal(vo, v[:4])
    # a map whose build input repeats a key fails, and so do its requests
    kd = k.copy()
    kd[10] = kd[20]
    bad = srv.open_map(B.params(cap, vs), kd, v)
    t2, _, _ = srv.submit(bad, ops, k[:4], vals)
    assert srv.wait(t2) == B.BOLT_EDUPKEY
    assert srv.map_state(bad) == (B.BOLT_SRV_FAILED, B.BOLT_EDUPKEY)
    assert srv.submit(bad, ops, k[:4], vals)[0] == B.BOLT_ESTATE
    # a map that could never fit the budget is refused at once
    small = B.Server(hbm_budget=1 << 20)
    with pytest.raises(B.BoltError):
        small.open_map(B.params(cap, vs), k, v)
    small.close()
    assert srv.close_map(mid) == 0 and srv.close_map(mid) == B.BOLT_EINVAL
    assert srv.submit(mid, ops, k[:4], vals)[0] == B.BOLT_EINVAL
    assert srv.drain(10000) == 0
    srv.close()

"""Multi-map batching through the C ABI (bolt_access_many): one call runs a
batch on each of several maps, and every map must end exactly where the
one-map call (bolt_access_batch) and the oracle take it: answers, status
bytes, pages, bins, stash, position map and trace, bit for bit."""
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


def _mixed_batch(rng, present, fresh, q, vs):
    pool = np.array(sorted(present), dtype=np.uint64) if present else fresh[:10]
    r = rng.random(q)
    keys = np.where(r < 0.3, pool[rng.integers(0, min(5, pool.size), q)],
                    np.where(r < 0.85, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
    ops = rng.choice([0, 1, 2], size=q, p=[0.5, 0.35, 0.15]).astype(np.uint8)
    vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
    return ops, keys.astype(np.uint64), vals


def _apply(present, ops, keys):
    for op, key in zip(ops.tolist(), keys.tolist()):
        if op == 1:
            present.add(int(key))
        elif op == 2:
            present.discard(int(key))


# (capacity, build keys, value bytes, params, largest batch)
MIX = [
    (2048, 1500, 16, {}, 200),
    (1 << 15, 30000, 8, {}, 4096),
    (4096, 3000, 64, dict(alpha_permille=600), 500),
    (1 << 18, 1 << 17, 8, {}, 1000),        # one-round batches (q <= B/16)
    (512, 0, 8, {}, 64),                    # empty build
    (1 << 12, 4000, 8, dict(alpha_permille=500), 8192),
]


def test_access_many_matches_oracle():
    import torch
    import paper_2509_01742_amd as B

    twins, present, fresh = [], [], []
    for j, (cap, n, vs, kw, _) in enumerate(MIX):
        t = Twin(cap, vs, key=bytes((j * 7 + i) & 255 for i in range(32)), **kw)
        k, v = workload(n, vs, 500 + j)
        assert t.build(k, v) == (0, 0, 0), j
        twins.append(t)
        present.append(set(int(x) for x in k))
        fresh.append(synth.keys(20000, 777 + j, offset=10**8))
    rng = np.random.default_rng(2025)
    for rnd in range(10):
        batches, host = [], []
        for j, (cap, n, vs, kw, qmax) in enumerate(MIX):
            q = 0 if (rnd + j) % 7 == 6 else int(rng.integers(1, qmax + 1))
            ops, keys, vals = _mixed_batch(rng, present[j], fresh[j], q, vs)
            if len(present[j]) > cap - q:
                ops[ops == 1] = 2
            vout = torch.zeros((q, vs), dtype=torch.uint8, device="cuda")
            st = torch.zeros(q, dtype=torch.uint8, device="cuda")
            batches.append((dev_u8(ops), dev_u64(keys), dev_u8(vals), vout, st))
            host.append((ops, keys, vals))
        # A rotating order: the plan table must not assume sorted sizes.
        order = [(rnd + j) % len(MIX) for j in range(len(MIX))]
        rc = B.access_many([twins[j].g for j in order], [batches[j] for j in order])
        torch.cuda.synchronize()
        assert rc == 0, (rnd, rc)
        for j, t in enumerate(twins):
            ops, keys, vals = host[j]
            if ops.size == 0:
                continue
            rc_o, vo_o, st_o = t.o.access(ops, keys, vals)
            assert rc_o == 0 and t.g.status() == 0, (rnd, j)
            assert np.array_equal(batches[j][4].cpu().numpy(), st_o), (rnd, j)
            assert np.array_equal(batches[j][3].cpu().numpy(), vo_o), (rnd, j)
            _apply(present[j], ops, keys)
        if rnd % 3 == 2 or rnd == 9:
            for t in twins:
                t.assert_same_state()


def test_access_many_rejects_one_map_only():
    import torch
    import paper_2509_01742_amd as B

    a, b = Twin(1024, 8), Twin(1024, 8, key=bytes(range(1, 33)))
    ka, va = workload(900, 8, 4)
    kb, vb = workload(700, 8, 5)
    assert a.build(ka, va) == (0, 0, 0) and b.build(kb, vb) == (0, 0, 0)
    obs0 = a.g.observable()
    bad = (dev_u8(np.array([0, 7], np.uint8)), dev_u64(ka[:2]), dev_u8(np.zeros((2, 8))),
           torch.zeros((2, 8), dtype=torch.uint8, device="cuda"), torch.zeros(2, dtype=torch.uint8, device="cuda"))
    ops = np.zeros(64, np.uint8)
    good = (dev_u8(ops), dev_u64(kb[:64]), dev_u8(np.zeros((64, 8))),
            torch.zeros((64, 8), dtype=torch.uint8, device="cuda"), torch.zeros(64, dtype=torch.uint8, device="cuda"))
    assert B.access_many([a.g, b.g], [bad, good]) == 0
    torch.cuda.synchronize()
    assert (bad[4].cpu().numpy() == 0xFF).all() and (bad[3].cpu().numpy() == 0).all()
    assert np.array_equal(a.g.observable(), obs0) and a.g.stats()["steps"] == 0
    rc_o, vo_o, st_o = b.o.access(ops, kb[:64], np.zeros((64, 8), np.uint8))
    assert rc_o == 0 and np.array_equal(good[3].cpu().numpy(), vo_o) and (good[4].cpu().numpy() == 1).all()
    b.assert_same_state()


def test_access_many_argument_errors():
    import torch
    import paper_2509_01742_amd as B

    a = Twin(1024, 8)
    k, v = workload(500, 8, 6)
    assert a.build(k, v) == (0, 0, 0)
    one = (dev_u8(np.zeros(4, np.uint8)), dev_u64(k[:4]), dev_u8(np.zeros((4, 8))),
           torch.zeros((4, 8), dtype=torch.uint8, device="cuda"), torch.zeros(4, dtype=torch.uint8, device="cuda"))
    assert B.access_many([a.g, a.g], [one, one]) == B.BOLT_EINVAL  # one batch per map and call
    unbuilt = B.Map(B.params(1024, 8))
    assert B.access_many([a.g, unbuilt], [one, one]) == B.BOLT_EINVAL
    assert B.access_many([], []) == 0
    torch.cuda.synchronize()
    assert a.g.stats()["steps"] == 0  # nothing ran


# (capacity, keys, value bytes, params): tiny, empty, one-key, odd sizes,
# a device-observable map, and maps past one sort tile and one expansion tile.
BUILD_MIX = [
    (64, 0, 8, {}), (64, 1, 8, {}), (64, 64, 8, {}), (1000, 777, 16, dict(alpha_permille=0)),
    (4096, 3000, 64, {}), (1 << 14, (1 << 14) - 5, 8, dict(alpha_permille=10)),
    (5000, 4321, 24, dict(alpha_permille=999)), (1 << 16, 1 << 16, 8, {}), (100000, 99999, 64, dict(c=4)),
    (3000, 2900, 16, dict(observable=1)), (1 << 17, 100000, 8, dict(pm_choices=2, pm_keys_per_row=8)),
]


def test_build_many_matches_oracle_then_access_many():
    import torch
    import paper_2509_01742_amd as B

    twins, inputs, keys = [], [], []
    for j, (cap, n, vs, kw) in enumerate(BUILD_MIX):
        t = Twin(cap, vs, key=bytes((5 * j + i) & 255 for i in range(32)), **kw)
        k, v = workload(n, vs, 900 + j)
        assert t.o.build(k, v) == 0
        twins.append(t)
        inputs.append((dev_u64(k) if n else None, dev_u8(v) if n else None))
        keys.append(k)
    order = list(range(len(BUILD_MIX)))[::-1]  # the largest map first
    assert B.build_many([twins[j].g for j in order], [inputs[j] for j in order]) == 0
    torch.cuda.synchronize()
    for j, t in enumerate(twins):
        assert t.g.status() == 0, j
        t.assert_same_state()
    # then one access round on all of them, checked against the oracle
    rng = np.random.default_rng(7)
    batches, host = [], []
    for j, (cap, n, vs, kw) in enumerate(BUILD_MIX):
        present = set(int(x) for x in keys[j])
        q = int(rng.integers(1, min(cap, 2000) + 1))
        ops, ks, vals = _mixed_batch(rng, present, synth.keys(5000, 31 + j, offset=10**8), q, vs)
        if len(present) > cap - q:
            ops[ops == 1] = 2
        batches.append((dev_u8(ops), dev_u64(ks), dev_u8(vals), torch.zeros((q, vs), dtype=torch.uint8, device="cuda"),
                        torch.zeros(q, dtype=torch.uint8, device="cuda")))
        host.append((ops, ks, vals))
    assert B.access_many([t.g for t in twins], batches) == 0
    torch.cuda.synchronize()
    for j, t in enumerate(twins):
        rc_o, vo_o, st_o = t.o.access(*host[j])
        assert rc_o == 0 and t.g.status() == 0, j
        assert np.array_equal(batches[j][4].cpu().numpy(), st_o), j
        assert np.array_equal(batches[j][3].cpu().numpy(), vo_o), j
        t.assert_same_state()


def test_build_many_errors_stay_per_map():
    import torch
    import paper_2509_01742_amd as B

    good, dup, full = Twin(2000, 8), Twin(2000, 8), Twin(256, 8, pm_row_slots=1, pm_keys_per_row=64)
    kg, vg = workload(1500, 8, 11)
    kd, vd = workload(1500, 8, 12)
    kd[700] = kd[3]  # a repeated key
    kf, vf = workload(200, 8, 13)
    assert good.o.build(kg, vg) == 0 and dup.o.build(kd, vd) == O.EDUPKEY and full.o.build(kf, vf) == O.EOVERFLOW
    maps = [good.g, dup.g, full.g]
    assert B.build_many(maps, [(dev_u64(kg), dev_u8(vg)), (dev_u64(kd), dev_u8(vd)), (dev_u64(kf), dev_u8(vf))]) == 0
    torch.cuda.synchronize()
    assert good.g.status() == 0 and dup.g.status() == B.BOLT_EDUPKEY and full.g.status() == B.BOLT_EOVERFLOW
    good.assert_same_state()
    # argument errors: nothing runs
    fresh = [Twin(500, 8), Twin(500, 8)]
    k, v = workload(400, 8, 14)
    one = (dev_u64(k), dev_u8(v))
    assert B.build_many([fresh[0].g, fresh[0].g], [one, one]) == B.BOLT_EINVAL
    assert B.build_many([fresh[0].g, good.g], [one, one]) == B.BOLT_EINVAL  # already built
    big = workload(600, 8, 15)
    assert B.build_many([fresh[0].g, fresh[1].g], [one, (dev_u64(big[0]), dev_u8(big[1]))]) == B.BOLT_EINVAL
    assert B.build_many([fresh[0].g, fresh[1].g], [one, one]) == 0
    torch.cuda.synchronize()
    assert fresh[0].o.build(k, v) == 0
    fresh[0].assert_same_state()


def _gpu_map(cap, vs, key):
    import paper_2509_01742_amd as B

    return B.Map(B.params(cap, vs, key=key))


def test_many_equals_per_call_at_full_size():
    """Sixty-four maps of 2^10..2^22 keys, each built and then given one GET
    batch of up to 8192 commands: the batched build and access and sixty-four
    one-map calls on twin maps leave identical pages and answers, and every
    answer is the value the key was built with (absent keys answer not-found
    with a zero value)."""
    import torch
    import paper_2509_01742_amd as B

    work = synth.config4()
    many, single, batches, expect, inputs = [], [], [], [], []
    for j, w in enumerate(work):
        key = bytes((j + i * 3) & 255 for i in range(32))
        g1, g2 = _gpu_map(w.cap, w.vs, key), _gpu_map(w.cap, w.vs, key)
        dk, dv = dev_u64(w.build_keys), dev_u8(w.build_vals)
        inputs.append((dk, dv))
        assert g2.build(dk, dv) == 0
        ops, keys, _ = w.batches[0]
        q = ops.size
        batches.append((dev_u8(ops), dev_u64(keys), dev_u8(np.zeros((q, w.vs))),
                        torch.zeros((q, w.vs), dtype=torch.uint8, device="cuda"),
                        torch.zeros(q, dtype=torch.uint8, device="cuda")))
        order = np.argsort(w.build_keys, kind="stable")
        sk = w.build_keys[order]
        at = np.minimum(np.searchsorted(sk, keys), sk.size - 1)
        hit = sk[at] == keys
        vals = np.where(hit[:, None], w.build_vals[order[at]], 0).astype(np.uint8)
        expect.append((hit.astype(np.uint8), vals))
        many.append(g1)
        single.append(g2)
    assert B.build_many(many, inputs) == 0  # the batched build, against 64 one-map builds
    torch.cuda.synchronize()
    for j in range(len(work)):
        assert many[j].status() == 0
        assert np.array_equal(many[j].observable(), single[j].observable()), j
        assert np.array_equal(many[j].hbm_bins(), single[j].hbm_bins()), j
    assert B.access_many(many, batches) == 0
    torch.cuda.synchronize()
    got = [(b[3].cpu().numpy().copy(), b[4].cpu().numpy().copy()) for b in batches]
    for j, g in enumerate(single):
        b = batches[j]
        b[3].zero_()
        b[4].zero_()
        assert g.access(b[0], b[1], b[2], b[3], b[4]) == 0
        torch.cuda.synchronize()
        assert np.array_equal(b[3].cpu().numpy(), got[j][0]), j
        assert np.array_equal(b[4].cpu().numpy(), got[j][1]), j
        assert np.array_equal(got[j][1], expect[j][0]), j
        assert np.array_equal(got[j][0], expect[j][1]), j
        assert many[j].status() == 0 and g.status() == 0
        assert np.array_equal(many[j].observable(), g.observable()), j
        assert np.array_equal(many[j].hbm_bins(), g.hbm_bins()), j
        assert many[j].stats() == g.stats(), j
    for g in many + single:
        g.close()

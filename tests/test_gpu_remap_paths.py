"""The several-round remap (a batch with more keys to place than one P2C
round of ceil(B/16) holds; Alg. 1's P2C_load_balance per key, in rounds in
command order) runs two ways on the GPU, chosen by the map's bin count: one
wave with the loads in LDS, one to kWaveKeys keys per lane and round
(B <= 24576), or the workgroup on the loads in HBM.  Each side of the
boundaries (one key per lane or two; the largest map kept in LDS and the
next), alone and in one many-map call, against the oracle bit for bit
(answers, pages, HBM bins, loads, stash, position map, trace)."""
import numpy as np
import pytest

import synth
from gpu_util import Twin, dev_u64, dev_u8, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


# capacities whose bin count (c = 8) sits on each side of the boundaries
CAPS = [(8 * 1024, "one key a lane, LDS loads"), (8 * 1040, "two keys a lane, LDS loads"),
        (8 * 7952, "eight keys a lane, LDS loads"), (8 * 24576, "24 keys a lane, LDS loads"),
        (8 * 24592, "workgroup, HBM loads")]


def _batch(rng, present, fresh, q, vs, cap):
    pool = np.array(sorted(present), dtype=np.uint64) if present else fresh[:10]
    r = rng.random(q)
    keys = np.where(r < 0.15, pool[rng.integers(0, min(5, pool.size), q)],
                    np.where(r < 0.8, pool[rng.integers(0, pool.size, q)], fresh[rng.integers(0, fresh.size, q)]))
    ops = rng.choice([0, 1, 2], size=q, p=[0.6, 0.3, 0.1]).astype(np.uint8)
    if len(present) + q > cap:  # no room for every PUT to insert: those become GETs
        ops[ops == 1] = 0
    return ops, keys.astype(np.uint64), rng.integers(0, 256, (q, vs), dtype=np.uint8)


def _apply(present, ops, keys):
    for op, key in zip(ops.tolist(), keys.tolist()):
        if op == 1:
            present.add(int(key))
        elif op == 2:
            present.discard(int(key))


@pytest.mark.parametrize("cap,what", CAPS)
@pytest.mark.parametrize("alpha", [0, 300])
def test_several_round_remap_each_side_of_the_boundaries(cap, what, alpha):
    vs = 16
    t = Twin(cap, vs, alpha_permille=alpha)
    k, v = workload(cap * 3 // 4, vs, cap + alpha)
    assert t.build(k, v) == (0, 0, 0)
    B = t.g.sizes["B"]
    rng = np.random.default_rng(cap + alpha)
    fresh = synth.keys(20000, cap, offset=10**8)
    present = set(int(x) for x in k)
    for q in (8192, 3 * ((B + 15) // 16) + 5, 8192):
        ops, keys, vals = _batch(rng, present, fresh, q, vs, cap)
        (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, vals)
        assert rc_o == 0 and rc_g == 0 and st == 0, (what, q, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), (what, q)
        _apply(present, ops, keys)
    t.assert_same_state()


def test_several_round_remaps_in_one_many_map_call():
    import torch
    import paper_2509_01742_amd as B

    vs = 8
    specs = [(128 * 8, 0), (1024 * 8, 200), (1040 * 8, 0), (7952 * 8, 500), (24576 * 8, 200), (24592 * 8, 0)]
    twins, present = [], []
    for j, (cap, alpha) in enumerate(specs):
        t = Twin(cap, vs, alpha_permille=alpha, key=bytes((9 * j + i) & 255 for i in range(32)))
        k, v = workload(cap // 2, vs, 4000 + j)
        assert t.build(k, v) == (0, 0, 0)
        twins.append(t)
        present.append(set(int(x) for x in k))
    rng = np.random.default_rng(99)
    for rnd in range(3):
        batches, host = [], []
        for j, (cap, _) in enumerate(specs):
            q = int(rng.integers(2000, 8193))
            ops, keys, vals = _batch(rng, present[j], synth.keys(20000, 70 + j, offset=10**8), q, vs, cap)
            batches.append((dev_u8(ops), dev_u64(keys), dev_u8(vals),
                            torch.zeros((q, vs), dtype=torch.uint8, device="cuda"),
                            torch.zeros(q, dtype=torch.uint8, device="cuda")))
            host.append((ops, keys, vals))
        assert B.access_many([t.g for t in twins], batches) == 0
        torch.cuda.synchronize()
        for j, t in enumerate(twins):
            rc_o, vo_o, st_o = t.o.access(*host[j])
            assert rc_o == 0 and t.g.status() == 0, (rnd, j)
            assert np.array_equal(batches[j][4].cpu().numpy(), st_o), (rnd, j)
            assert np.array_equal(batches[j][3].cpu().numpy(), vo_o), (rnd, j)
            _apply(present[j], host[j][0], host[j][1])
    for t in twins:
        t.assert_same_state()

"""Batches of one command, which a plain map runs as one workgroup (every
step of the batch in one launch), against the oracle bit for bit.

Covered: every op on present and absent keys, on both stores and with HBM
bins at several ratios; a rejected op code; a full map and a full
position-map row; single commands between large batches (whose pages are
still waiting to be written); a page too large for the one-workgroup form
(the batched kernels run instead); and a map without a trace.
"""
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


def _one(t, op, key, val):
    (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(np.array([op], np.uint8), np.array([key], np.uint64),
                                                           val.reshape(1, -1))
    return rc_o, vo_o, st_o, rc_g, st, vo_g, st_g


def _stream(t, k, fresh, n, seed):
    rng = np.random.default_rng(seed)
    for c in range(n):
        key = int(k[rng.integers(0, k.size)]) if rng.random() < 0.8 else int(fresh[rng.integers(0, fresh.size)])
        op = int(rng.choice([0, 1, 2], p=[0.5, 0.3, 0.2]))
        val = rng.integers(0, 256, t.vs, dtype=np.uint8)
        rc_o, vo_o, st_o, rc_g, st, vo_g, st_g = _one(t, op, key, val)
        assert rc_o == 0 and rc_g == 0 and st == 0, (c, rc_o, rc_g, st)
        assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o), c


@pytest.mark.parametrize("observable,alpha", [(0, 200), (1, 200), (1, 600), (0, 0)])
def test_single_command_stream(observable, alpha):
    t = Twin(2048, 16, observable=observable, alpha_permille=alpha)
    k, v = workload(1500, 16, 700 + alpha + observable)
    assert t.build(k, v) == (0, 0, 0)
    _stream(t, k, synth.keys(200, 701, offset=10**9), 400, 3 + observable)
    t.assert_same_state()


def test_single_command_rejected_op():
    t = Twin(1024, 8)
    k, v = workload(900, 8, 4)
    assert t.build(k, v) == (0, 0, 0)
    obs0 = t.g.observable()
    rc_o, _, _, rc_g, st, vo_g, st_g = _one(t, 7, int(k[0]), np.zeros(8, np.uint8))
    assert rc_o == O.EINVAL and rc_g == 0 and st == 0
    assert (st_g == 0xFF).all() and (vo_g == 0).all()
    assert np.array_equal(t.g.observable(), obs0)
    assert t.g.stats()["steps"] == 0
    # the map goes on as before
    _stream(t, k, synth.keys(50, 5, offset=10**9), 40, 6)
    t.assert_same_state()


def test_single_command_full_map():
    t = Twin(64, 8)
    k, v = workload(63, 8, 1)
    assert t.build(k, v) == (0, 0, 0)
    new = synth.keys(4, 999, offset=10**9)
    codes = []
    for key in new.tolist():
        rc_o, _, _, rc_g, st, _, _ = _one(t, 1, key, np.full(8, 3, np.uint8))
        codes.append((rc_o, st))
        if rc_o != 0:
            break
    assert codes[0] == (0, 0)
    assert codes[-1][0] == O.EFULL and codes[-1][1] == t.B.BOLT_EFULL, codes


def test_single_command_full_position_map_row():
    t = Twin(256, 8, pm_row_slots=1, pm_keys_per_row=64)
    assert t.build(np.zeros(0, np.uint64), np.zeros((0, 8), np.uint8)) == (0, 0, 0)
    for c, key in enumerate(synth.keys(64, 4).tolist()):
        rc_o, _, st_o, rc_g, st, _, st_g = _one(t, 1, key, np.full(8, c & 255, np.uint8))
        if rc_o != 0:
            assert rc_o == O.EOVERFLOW and st == t.B.BOLT_EOVERFLOW, (c, rc_o, st)
            return
        assert rc_g == 0 and st == 0 and np.array_equal(st_g, st_o), c
    pytest.fail("no row filled up")


def test_single_commands_between_large_batches():
    import torch

    t = Twin(8192, 16, observable=0)  # pinned store: large batches leave their pages to the next call
    k, v = workload(7000, 16, 91)
    assert t.build(k, v) == (0, 0, 0)
    fresh = synth.keys(300, 92, offset=10**9)
    rng = np.random.default_rng(93)
    for rnd in range(4):
        q = 3000
        ops = rng.choice([0, 1, 2], size=q, p=[0.6, 0.3, 0.1]).astype(np.uint8)
        keys = k[rng.integers(0, k.size, q)]
        vals = rng.integers(0, 256, (q, 16), dtype=np.uint8)
        rc_o, vo_o, st_o = t.o.access(ops, keys, vals)
        out = torch.zeros((q, 16), dtype=torch.uint8, device="cuda")
        st = torch.zeros(q, dtype=torch.uint8, device="cuda")
        assert t.g.access(dev_u8(ops), dev_u64(keys), dev_u8(vals), out, st) == 0 and rc_o == 0
        torch.cuda.synchronize()
        assert np.array_equal(st.cpu().numpy(), st_o) and np.array_equal(out.cpu().numpy(), vo_o)
        _stream(t, k, fresh, 25, 100 + rnd)
    t.assert_same_state()


@pytest.mark.parametrize("vs", [1024, 2048])
def test_single_commands_large_pages(vs):
    """1 KiB values (13 KiB pages) fit three rebuild waves in one workgroup's
    64 KiB of LDS; 2 KiB values do not, and run through the batched kernels."""
    t = Twin(512, vs)
    k, v = workload(400, vs, 40 + vs)
    assert t.build(k, v) == (0, 0, 0)
    _stream(t, k, synth.keys(50, 41, offset=10**9), 60, 42)
    t.assert_same_state()


def test_single_commands_without_trace():
    t = Twin(2048, 32, trace=False)
    k, v = workload(1800, 32, 51)
    assert t.build(k, v) == (0, 0, 0)
    _stream(t, k, synth.keys(100, 52, offset=10**9), 200, 53)
    t.assert_same_state(trace=False)


def test_timed_map_counts_the_one_command_kernel():
    """BOLT_F_TIMING: a one-command batch is one launch of its own kernel
    class, a larger batch one launch of each batched kernel; answers and
    state as without timing."""
    import paper_2509_01742_amd as B

    t = Twin(2048, 16, flags=B.BOLT_F_TIMING)
    k, v = workload(1500, 16, 61)
    assert t.build(k, v) == (0, 0, 0)
    t.g.kernel_times_reset()
    _stream(t, k, synth.keys(50, 62, offset=10**9), 3, 63)
    rng = np.random.default_rng(64)
    ops = rng.choice([0, 1], size=300, p=[0.8, 0.2]).astype(np.uint8)
    keys = k[rng.integers(0, k.size, 300)]
    (rc_o, vo_o, st_o), (rc_g, st, vo_g, st_g) = t.access(ops, keys, rng.integers(0, 256, (300, 16), dtype=np.uint8))
    assert rc_o == 0 and rc_g == 0 and st == 0
    assert np.array_equal(st_g, st_o) and np.array_equal(vo_g, vo_o)
    times = t.g.kernel_times()
    assert times["acc_solo"][0] == 3
    assert times["acc_fetch"][0] == 1 and times["acc_dedup"][0] == 1 and times["acc_compose"][0] == 1
    t.assert_same_state()

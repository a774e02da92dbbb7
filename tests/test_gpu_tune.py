"""The autotuner of the network schedules: every schedule it may choose sorts
and expands exactly as the oracle does, its results survive a cache file,
and a build under a tuned table still matches the oracle bit for bit."""
import os

import numpy as np
import pytest

import oracle as O
from gpu_util import Twin, dev_u64, host_u64, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd as B

    yield
    B.bolt_tune_reset()


def _check_sort(B, n, seed):
    import torch

    rng = np.random.default_rng(seed)
    for a in (rng.integers(0, 2**64, n, dtype=np.uint64), rng.integers(0, 3, n, dtype=np.uint64)):
        d = dev_u64(a)
        assert B.sort_u64(d) == 0
        torch.cuda.synchronize()
        assert np.array_equal(host_u64(d), np.sort(a))


def _check_expand(B, m, seed):
    import torch

    rng = np.random.default_rng(seed)
    keep = rng.random(m) < 0.6
    tgt = np.nonzero(keep)[0].astype(np.uint32)
    n = tgt.size
    pay = rng.integers(0, 2**31, n).astype(np.uint32)
    want, rc = O.expand(tgt, pay, m)
    assert rc == 0
    el = np.full(m, 2**64 - 1, dtype=np.uint64)
    el[:n] = (tgt.astype(np.uint64) << np.uint64(32)) | pay.astype(np.uint64)
    d = dev_u64(el)
    tmp = torch.zeros(m, dtype=torch.int64, device="cuda")
    assert B.expand_u64(d, tmp) == 0
    torch.cuda.synchronize()
    got = host_u64(d)
    empty = got == np.uint64(2**64 - 1)
    assert np.array_equal(empty, want == O.NONE32)
    assert np.array_equal((got[~empty] & np.uint64(0xFFFFFFFF)).astype(np.uint32), want[~empty])


@pytest.mark.parametrize("L", [14, 16])
def test_every_schedule_is_the_same_network(L):
    import paper_2509_01742_amd as B

    n = 1 << L
    for tile in (11, 12, 13):
        for f in (1, 2, 3, 4, 5, 6):
            assert B.tune_set([dict(log2_n=L, sort_tile_log=tile, sort_pass_strides=f,
                                    expand_pass_stages=min(f, 4))]) == 0
            _check_sort(B, n, 100 * tile + f)
            _check_expand(B, n - 5, 10 * f + L)  # class 2^L, ragged length
    assert B.bolt_tune_reset() == 0
    bad = dict(log2_n=L, sort_tile_log=10, sort_pass_strides=1, expand_pass_stages=1)
    assert B.tune_set([bad]) == B.BOLT_EINVAL


def test_autotune_cache_and_tuned_build(tmp_path):
    import torch
    import paper_2509_01742_amd as B

    path = str(tmp_path / "bolt.tune")
    assert B.bolt_tune_reset() == 0
    assert B.autotune(1 << 17, path) == 0
    t1 = B.tune_table()
    assert [e["log2_n"] for e in t1] == [14, 15, 16, 17]
    for e in t1:
        assert 11 <= e["sort_tile_log"] <= 13 and 1 <= e["sort_pass_strides"] <= 6
        assert 1 <= e["expand_pass_stages"] <= 4 and e["sort_ms"] > 0 and e["expand_ms"] > 0
    assert os.path.getsize(path) > 0
    assert B.bolt_tune_reset() == 0 and B.tune_table() == []
    assert B.autotune(1 << 17, path) == 0  # loaded from the cache, not measured again
    t2 = B.tune_table()
    assert [(e["log2_n"], e["sort_tile_log"], e["sort_pass_strides"], e["expand_pass_stages"]) for e in t2] == \
        [(e["log2_n"], e["sort_tile_log"], e["sort_pass_strides"], e["expand_pass_stages"]) for e in t1]
    # a build whose sort (npad 2^17) and expansion run the tuned schedules
    t = Twin(100000, 8)
    k, v = workload(99000, 8, 4242)
    assert t.build(k, v) == (0, 0, 0)
    t.assert_same_state()
    _check_sort(B, 1 << 17, 5)
    torch.cuda.synchronize()

"""Duplicate build keys end the build in BOLT_EDUPKEY (the build keys,
sorted by the same network as the tags, are distinct iff no two neighbours
are equal).  The oracle finds them in the position map's rows (Sec. 5.2:
each key in the least loaded of its d rows, in rounds of ceil(R/16) keys),
so copies placed in one round, copies rounds apart, three copies, the
largest and the smallest key value, with several row shapes, one map at a
time and in one many-map build: each status against the oracle's, and a
clean build of the same keys against its state."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import Twin, dev_u64, dev_u8

pytestmark = pytest.mark.gpu

TOP = np.uint64(2**64 - 1)


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2509_01742_amd  # noqa: F401  (fails loudly when the library is missing)


# (capacity, row parameters): default rows (d = 4, 32 slots, 16 keys a row),
# two choices with short rows, one choice (every copy in one row)
SHAPES = [(4096, {}), (4096, dict(pm_choices=2, pm_row_slots=8, pm_keys_per_row=4)),
          (1 << 16, dict(pm_choices=1)), (1 << 16, {})]


def _round_len(cap, kw):
    kpr = kw.get("pm_keys_per_row", 16)
    R = (cap + kpr - 1) // kpr
    return (R + 15) // 16


def _cases(n, rs):
    """(name, list of (copy index, source index)) with every copy index
    distinct from its source."""
    return [
        ("same round", [(5, 4)]),
        ("rounds apart", [(5 * rs + 3, 1)]),
        ("first and last", [(n - 1, 0)]),
        ("three copies", [(rs + 2, 2), (n - 2, 2)]),
        ("largest key twice", [(7, 6), (3 * rs, 6)]),
        ("smallest key twice", [(9 * rs + 1, 8)]),
    ]


@pytest.mark.parametrize("cap,kw", SHAPES)
def test_duplicates_found_like_the_oracle(cap, kw):
    vs = 8
    n = cap * 3 // 4
    rs = _round_len(cap, kw)
    assert 10 * rs < n
    base = synth.keys(n, cap + 17)
    base[6], base[8] = TOP, 0  # the extreme key values, each present once
    vals = synth.values(n, vs, 3)
    t = Twin(cap, vs, trace=False, **kw)
    assert t.build(base, vals) == (0, 0, 0)  # every key distinct, the extremes included
    t.assert_same_state(trace=False)
    for name, copies in _cases(n, rs):
        k = base.copy()
        for at, src in copies:
            k[at] = k[src]
        assert np.unique(k).size < n, name
        t = Twin(cap, vs, trace=False, **kw)
        rc_o, rc_g, st = t.build(k, vals)
        assert rc_o == O.EDUPKEY and rc_g == 0 and st == t.B.BOLT_EDUPKEY, (name, rc_o, rc_g, st)


def test_duplicates_in_one_many_map_build():
    import torch
    import paper_2509_01742_amd as B

    vs = 8
    twins, inputs, want = [], [], []
    for j, (cap, kw) in enumerate(SHAPES):
        n = cap * 3 // 4
        rs = _round_len(cap, kw)
        k = synth.keys(n, 900 + j)
        if j % 2 == 0:  # a copy in the same round on even maps, rounds apart on odd ones
            k[11] = k[10]
        else:
            k[7 * rs] = k[3]
        twins.append(Twin(cap, vs, trace=False, **kw))
        inputs.append((k, synth.values(n, vs, 40 + j)))
        want.append(O.EDUPKEY)
    clean = synth.keys(3000, 77)
    twins.append(Twin(4096, vs, trace=False))
    inputs.append((clean, synth.values(3000, vs, 78)))
    want.append(0)
    for t, (k, v), w in zip(twins, inputs, want):
        assert t.o.build(k, v) == w
    assert B.build_many([t.g for t in twins], [(dev_u64(k), dev_u8(v)) for k, v in inputs]) == 0
    torch.cuda.synchronize()
    for j, t in enumerate(twins):
        assert t.g.status() == (B.BOLT_EDUPKEY if want[j] else 0), j
    twins[-1].assert_same_state(trace=False)

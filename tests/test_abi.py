"""The C-ABI library loads, exports every entry point include/bolt.h declares,
and its host-side sizing agrees with the oracle's (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bolt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bolt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2509_01742_amd as B

    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(B.lib, name), name
    assert sorted(B.EXPORTED) == declared


@pytest.mark.parametrize("cap,vs,kw", [
    (1 << 16, 8, {}), ((1 << 24) + (1 << 16), 64, {}), (1 << 26, 8, {}), (1000, 16, dict(alpha_permille=0)),
    (12345, 24, dict(alpha_permille=999, c=4)), (1 << 20, 8, dict(c=16)), (4096, 8, dict(bin_slots=20)),
    (1 << 22, 64, {}), ((1 << 22) + 8, 64, {}), (1 << 23, 8, dict(c=16)),
    (777, 8, dict(pm_keys_per_row=4, pm_row_slots=8, pm_choices=2))])
def test_sizes_agree_with_oracle(cap, vs, kw):
    import paper_2509_01742_amd as B

    p = B.params(cap, vs, **kw)
    s = B.sizes_of(p)
    o = O.sizing(cap, vs, c=p.c, alpha_pm=p.alpha_permille, bin_slots=p.bin_slots, d=p.pm_choices,
                 kpr=p.pm_keys_per_row, W=p.pm_row_slots)
    assert (s["B"], s["K"], s["M"], s["Z"], s["page_bytes"], s["pm_rows"], s["stash_bound"], s["lmax"],
            s["hbm_bound"]) == (o["B"], o["K"], o["M"], o["Z"], o["page_bytes"], o["R_pm"], o["stash_bound"],
                                o["lmax"], o["hbm_bound"])
    assert s["stash_pool"] == s["stash_bound"] + B.BOLT_MAX_BATCH
    pd = B.params(cap, vs, **kw)
    pd.flags |= B.BOLT_F_DECOMPOSED  # the pool also holds the HBM bins' items; no HBM pages
    sd = B.sizes_of(pd)
    assert sd["stash_pool"] == s["stash_bound"] + B.BOLT_MAX_BATCH + s["hbm_bound"]
    if s["K"] and vs >= 32:  # a pool entry costs key + value + 12 bytes, a page slot key + value
        assert B.footprint(pd)[0] < B.footprint(p)[0]


@pytest.mark.parametrize("kw", [dict(capacity=1), dict(value_bytes=12), dict(value_bytes=0),
                                dict(alpha_permille=1000), dict(pm_choices=5), dict(pm_row_slots=33),
                                dict(c=0), dict(bin_slots=63), dict(observable=2)])
def test_sizes_reject(kw):
    import paper_2509_01742_amd as B

    p = B.params(1024, 8)
    for k, v in kw.items():
        setattr(p, k, v)
    assert B.bolt_sizes_of(C.byref(p), None) == B.BOLT_EINVAL
    h = C.c_void_p()
    assert B.bolt_create(C.byref(p), None, C.byref(h)) == B.BOLT_EINVAL


def test_footprint_grows_with_capacity_and_mode():
    import paper_2509_01742_amd as B

    small = B.footprint(B.params(1 << 16, 64))
    big = B.footprint(B.params(1 << 24, 64))
    dev = B.footprint(B.params(1 << 24, 64, observable=B.BOLT_OBS_DEVICE))
    assert big[0] > small[0] and big[1] > small[1]
    assert dev[0] == big[0] + big[1]  # device-observable mode keeps the pages in HBM too
    s = B.sizes_of(B.params(1 << 24, 64))
    assert big[1] == s["M"] * s["page_bytes"]


def test_null_map_calls_are_rejected():
    import paper_2509_01742_amd as B

    assert B.bolt_destroy(None) == B.BOLT_OK
    assert B.bolt_status(None) == B.BOLT_EINVAL
    assert B.bolt_build(None, None, None, 0, None) == B.BOLT_EINVAL
    assert B.bolt_access_batch(None, None, None, None, None, None, 1, None) == B.BOLT_EINVAL
    assert B.bolt_sort_u64(None, 4, None) == B.BOLT_EINVAL


def test_sealing_under_a_fixed_key_needs_the_reuse_flag():
    """A fixed PRF key fixes the page key, so sealed maps sharing it would
    repeat key streams: bolt_create refuses that unless the caller says the
    reuse is meant (tests only).  The check comes before any device call."""
    import paper_2509_01742_amd as B

    p = B.params(1024, 8, key=bytes(32))
    p.flags |= B.BOLT_F_SEAL
    h = C.c_void_p()
    assert B.bolt_create(C.byref(p), None, C.byref(h)) == B.BOLT_EINVAL and not h.value

"""Pins of the oracle's sizing against the numbers the paper prints.

* The validation slack table (Sec. 4.3, "Dimensions in practice") fixes the
  bin capacity l_max at N = 2^20 (14 for c = 8, 22 for c = 16) and, through
  the printed relative slacks, the shapes of the bounds of Claims 4.3 and 4.4.
* The HBM-usage example after Claim 5.2 (Sec. 5.3) fixes the Claim 5.2
  formula to within the paper's rounding.
"""
import json
import math
import os

import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table():
    return json.load(open(os.path.join(GOLDEN, "slack_table.json")))


@pytest.mark.parametrize("c,lmax", [(8, 14), (16, 22)])
def test_bin_capacity_matches_slack_table(c, lmax):
    t = _table()
    s = O.sizing(t["N"], 8, c=c, alpha_pm=200)
    assert s["lmax"] == lmax
    for abs_slack, rel in t["c"][str(c)]["bin_load"]:
        assert abs(abs_slack / s["lmax"] - rel) < 0.0015
    # at N = 2^20 a batch fills a sizeable part of a placement round
    # (B <= 2^19): the default capacity keeps one slot above l_max
    assert s["B"] <= 1 << 19 and s["Z"] == lmax + 1


def test_default_capacity_margin_follows_the_round_fill():
    """One slot above l_max exactly when B <= 64 * 8192 (the largest batch
    then fills at least 1/64 of the bins in one placement round)."""
    for cap, c in ((1 << 16, 8), (1 << 20, 16), (1 << 22, 8), ((1 << 22) + 8, 8), (1 << 23, 16), (1 << 24, 8),
                   ((1 << 24) + (1 << 16), 8), (1 << 26, 8)):
        s = O.sizing(cap, 8, c=c)
        assert s["Z"] == s["lmax"] + (1 if s["B"] <= 64 * 8192 else 0), (cap, c)
        assert O.sizing(cap, 8, c=c, bin_slots=s["lmax"])["Z"] == s["lmax"]  # an explicit capacity is kept


@pytest.mark.parametrize("c", [8, 16])
def test_hbm_load_bound_matches_slack_table(c):
    """Claim 4.3 bound with K = alpha B real-valued reproduces the printed
    relative slack of the 'HBM Ld' row to its printed digits."""
    t = _table()
    N = t["N"]
    B = N / c
    lmax = O.sizing(N, 8, c=c)["lmax"]
    for alpha, (abs_slack, rel) in zip(t["alphas"], t["c"][str(c)]["hbm_load"]):
        bound = O.claim43_bound(alpha * B, c, lmax, N)
        emp = bound - abs_slack
        assert emp > alpha * B * c * 0.95  # the simulated sum is near its mean K c
        assert abs(abs_slack / bound - rel) < 0.0015, (alpha, bound, abs_slack / bound, rel)


@pytest.mark.parametrize("c", [8, 16])
def test_stash_bound_matches_slack_table(c):
    """Claim 4.4 bound reproduces the printed relative slack of the 'Stash'
    row to about one point (the paper's own rounding of its inputs is not
    stated); the implied simulated maxima stay under the 6.5 % / 3.3 % of N
    stated in the same section."""
    t = _table()
    N = t["N"]
    B = N / c
    lmax = O.sizing(N, 8, c=c)["lmax"]
    for alpha, (abs_slack, rel) in zip(t["alphas"], t["c"][str(c)]["stash"]):
        M = (1 - alpha) * B
        bound = O.claim44_bound(M, alpha, lmax, N)
        assert abs(abs_slack / bound - rel) < 0.0075, (alpha, bound, abs_slack / bound, rel)
        assert (bound - abs_slack) / N <= t["text_stash_max_fraction_of_N"][str(c)] + 1e-9


def test_integer_stash_bound_is_claim44_rounded_up():
    for cap, vs, alpha in ((1 << 16, 8, 200), ((1 << 24) + (1 << 16), 64, 200), (1 << 26, 8, 200),
                           (1 << 20, 8, 10), (1 << 20, 8, 500), (1000, 8, 0)):
        s = O.sizing(cap, vs, alpha_pm=alpha)
        exact = O.claim44_bound(s["M"], alpha / 1000, s["lmax"], cap)
        assert s["stash_bound"] == math.ceil(exact)


def test_claim52_example():
    """Sec. 5.3: with the HBM store off, HBM needs 26 % / 12 % / 7 % of the raw
    data for 64 B / 256 B / 1 KiB values at 10^9 items.  The formula gives
    25.4 / 11.3 / 7.6 %, inside one point of each printed value."""
    g = json.load(open(os.path.join(GOLDEN, "claim52_example.json")))
    N, ks, c = g["N"], g["key_bits"], g["c"]
    M = N / c  # alpha = 0: every bin is a host page
    lmax = c + math.ceil(math.log2(math.ceil(math.log2(N)))) + 1
    beta2 = O.claim44_bound(M, 0.0, lmax, N)
    R = N / g["keys_per_row"]
    for vs_bytes, printed in g["printed_percent"].items():
        vs_bits = 8 * int(vs_bytes)
        bits = O.claim52_bits(N, ks, vs_bits, 0.0, beta2, R, g["d"])
        pct = 100 * bits / (N * (ks + vs_bits))
        assert abs(pct - printed) <= 1.0, (vs_bytes, pct, printed)


def test_sizing_formulas_on_configs():
    s = O.sizing(1 << 16, 8)
    assert (s["B"], s["K"], s["M"], s["lmax"], s["Z"], s["page_bytes"], s["R_pm"]) == (
        8192, 1638, 6554, 13, 14, 256, 4096)
    s = O.sizing((1 << 24) + (1 << 16), 64)
    assert (s["B"], s["K"], s["M"], s["Z"], s["page_bytes"]) == (2105344, 421068, 1684276, 14, 1024)
    s = O.sizing(1 << 26, 8)
    assert (s["B"], s["K"], s["M"], s["Z"], s["page_bytes"]) == (8388608, 1677721, 6710887, 14, 256)
    # alpha = K / (K + M) (Claim 4.4), not K / (K + N)
    assert s["K"] == (200 * s["B"]) // 1000 and s["K"] + s["M"] == s["B"]


@pytest.mark.parametrize("bad", [dict(cap=1), dict(vs=12), dict(vs=0), dict(alpha_pm=1000), dict(d=5), dict(W=33),
                                 dict(c=0), dict(bin_slots=65)])
def test_sizing_rejects(bad):
    args = dict(cap=1024, vs=8)
    args.update(bad)
    with pytest.raises(ValueError):
        O.sizing(**args)

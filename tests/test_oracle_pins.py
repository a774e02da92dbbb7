"""Independent pins of the oracle's batched access, written from the paper's
rules without the oracle's code:

* the remap (Alg. 1, random_remap then P2C_load_balance; Sec. 5.1 step 5):
  every key present at the end of a batch moves to the less loaded bin of
  its fresh pair R(s), loads counted after every removal of the batch, the
  second bin only when strictly less loaded, in rounds of ceil(B/16) keys in
  command order that see the loads at their round's start;
* the pairs each command reveals (Claim 4.1 and its simulator): a leader
  whose key is mapped reads the pair its key got at its last placement; any
  other command reads the fresh pair F(s) of its own step.  Every revealed
  pair is therefore a PRF or tape value never revealed before, and revealed
  exactly once (the injectivity the simulator rests on);
* batch numbers: a call with at least one command on a built map takes the
  next number whether it runs or is rejected for its op codes, so the labels
  of the trace depend on the sequence of calls alone.

The model here uses hashlib for the PRF and plain Python for the rules; it
reads the oracle's state only through its snapshots.  A last group of tests
compiles copies of the oracle with a plausible mistake planted in them and
checks that these pins catch each one."""
import hashlib
import os
import subprocess

import numpy as np
import pytest

import oracle as O
import synth

KEY = bytes(range(40, 72))
ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "bolt_oracle.c")


# ------------------------------------------------------------ the model

def prf_words(key: bytes, domain: int, x: int):
    """The keyed PRF: BLAKE2s-256 of domain || LE64(x), as four LE64 words."""
    d = hashlib.blake2s(bytes([domain]) + int(x).to_bytes(8, "little"), key=key, digest_size=32).digest()
    return [int.from_bytes(d[8 * j:8 * j + 8], "little") for j in range(4)]


def distinct_pair(w0: int, w1: int, B: int):
    """Two distinct bins from two words by multiply-high range reduction."""
    p1 = (w0 * B) >> 64
    return p1, (p1 + 1 + ((w1 * (B - 1)) >> 64)) % B


def pair_of(source, key: bytes, B: int):
    """The pair behind a revealed source: a key's build pair (domain 1),
    the remap pair R(s) (domain 3, words 2 and 3) or the fetch pair F(s)
    (domain 3, words 0 and 1)."""
    kind, x = source
    if kind == "build":
        w = prf_words(key, 1, x)
        return distinct_pair(w[0], w[1], B)
    w = prf_words(key, 3, x)
    return distinct_pair(w[2], w[3], B) if kind == "R" else distinct_pair(w[0], w[1], B)


def where_items(m):
    """key -> bin of every stored item (page, HBM bin or stash entry)."""
    s = m.s
    Z, vs, K = s["Z"], s["vs"], s["K"]
    out = {}
    for b, page in enumerate(m.hbm_bins()):
        for k, _ in O.decode_page(page, Z, vs):
            out[k] = b
    for p, page in enumerate(m.observable()):
        for k, _ in O.decode_page(page, Z, vs):
            out[k] = K + p
    for k, dest, _ in m.stash():
        out[k] = dest
    return out


def leaders_of(keys):
    first = {}
    for i, k in enumerate(keys.tolist()):
        first.setdefault(int(k), i)
    return first


def predicted_placement(key, B, ctr, loads_before, where_before, keys, present_after):
    """Bins and loads after one batch, by the remap rule alone."""
    L = loads_before.astype(np.int64).copy()
    first = leaders_of(keys)
    for k in first:
        if k in where_before:  # a present key leaves its bin
            L[where_before[k]] -= 1
    movers = sorted((i, k) for k, i in first.items() if k in present_after)
    where = {k: b for k, b in where_before.items() if k in present_after}
    rs = (B + 15) // 16
    for r0 in range(0, len(movers), rs):
        chunk = movers[r0:r0 + rs]
        chosen = []
        for i, k in chunk:
            r1, r2 = pair_of(("R", ctr + i), key, B)
            chosen.append(r2 if L[r2] < L[r1] else r1)
        for (i, k), b in zip(chunk, chosen):
            L[b] += 1
            where[k] = b
    return where, L


def random_batches(rng, pool_keys, fresh, nb, qmax, hot=6):
    fi = 0
    for _ in range(nb):
        q = int(rng.integers(1, qmax + 1))
        hotk = pool_keys[rng.integers(0, hot, q)]
        cold = pool_keys[rng.integers(0, pool_keys.size, q)]
        new = fresh[fi:fi + q]
        fi += q
        r = rng.random(q)
        keys = np.where(r < 0.3, hotk, np.where(r < 0.8, cold, new)).astype(np.uint64)
        ops = rng.choice([O.GET, O.PUT, O.DEL], size=q, p=[0.55, 0.3, 0.15]).astype(np.uint8)
        vals = rng.integers(0, 256, (q, 8), dtype=np.uint8)
        yield ops, keys, vals


def _fresh_map(cap, n, alpha, seed, lib=None, trace=False):
    m = O.OracleMap(cap, 8, alpha_pm=alpha, key=KEY, trace=trace, lib=lib)
    k, v = synth.keys(n, seed), synth.values(n, 8, seed + 1)
    assert m.build(k, v) == O.OK
    p = O.PlainMap(8)
    p.build(k, v)
    return m, p, k


def check_remap_rule(lib=None, alpha=200, cap=2048, n=1500, nb=40, qmax=120, seed=5):
    """Runs a random stream and compares every batch's bins and loads with
    the model; returns the first mismatch as a string, or None."""
    m, p, k = _fresh_map(cap, n, alpha, seed, lib=lib)
    B = m.s["B"]
    rng = np.random.default_rng(seed)
    fresh = synth.keys(nb * qmax, seed + 7, offset=10**8)
    for b, (ops, keys, vals) in enumerate(random_batches(rng, k, fresh, nb, qmax)):
        where0, loads0, ctr = where_items(m), m.loads(), m.ctr
        rc, _, _ = m.access(ops, keys, vals)
        if rc != O.OK:
            return "batch %d: rc %d" % (b, rc)
        p.access(ops, keys, vals)
        want_where, want_loads = predicted_placement(KEY, B, ctr, loads0, where0, keys, p.d)
        got_where = where_items(m)
        if got_where != want_where:
            bad = [x for x in want_where if got_where.get(x) != want_where[x]][:3]
            return "batch %d: bins of %d keys differ, e.g. %s" % (b, len(bad), bad)
        if not np.array_equal(m.loads().astype(np.int64), want_loads):
            return "batch %d: loads differ" % b
    return None


def check_revealed_pairs(lib=None, alpha=0, cap=1024, n=800, nb=60, qmax=64, seed=9):
    """Replays the fetch rule: the observable reads of each batch must be
    the pages of the pairs the model says each command reveals, in command
    and role order; no source may be revealed twice.  Returns the first
    mismatch as a string, or None."""
    m, p, k = _fresh_map(cap, n, alpha, seed, lib=lib, trace=True)
    B, K = m.s["B"], m.s["K"]
    m.trace_clear()
    source = {int(x): ("build", int(x)) for x in k.tolist()}
    seen = set()
    rng = np.random.default_rng(seed)
    fresh = synth.keys(nb * qmax, seed + 3, offset=10**8)
    for b, (ops, keys, vals) in enumerate(random_batches(rng, k, fresh, nb, qmax)):
        ctr = m.ctr
        n_before = m.trace().size
        rc, _, _ = m.access(ops, keys, vals)
        if rc != O.OK:
            return "batch %d: rc %d" % (b, rc)
        p.access(ops, keys, vals)
        first = leaders_of(keys)
        want = []
        for i, x in enumerate(keys.tolist()):
            x = int(x)
            src = source[x] if (first[x] == i and x in source) else ("F", ctr + i)
            if src in seen:
                return "batch %d: source %s revealed twice" % (b, src)
            seen.add(src)
            for bin_ in pair_of(src, KEY, B):
                if bin_ >= K:
                    want.append(bin_ - K)
        t = m.trace()[n_before:]
        reads = t[t["kind"] == 0]["page"].tolist()
        if reads != want:
            return "batch %d: revealed pages differ from the model" % b
        for x, i in first.items():
            if x in p.d:
                source[x] = ("R", ctr + i)
            else:
                source.pop(x, None)
    return None


# ------------------------------------------------------------ the pins

@pytest.mark.parametrize("alpha,cap,qmax", [(200, 2048, 120), (0, 2048, 120), (500, 1024, 90), (200, 256, 40)])
def test_remap_rule_matches_an_independent_model(alpha, cap, qmax):
    """B = cap/8 bins, so ceil(B/16) = 16 keys (or 2 at cap 256) per round:
    most batches take several rounds."""
    assert check_remap_rule(alpha=alpha, cap=cap, n=cap * 3 // 4, qmax=qmax) is None


@pytest.mark.parametrize("alpha", [0, 200, 700])
def test_revealed_pairs_are_fresh_and_revealed_once(alpha):
    assert check_revealed_pairs(alpha=alpha) is None


def test_batch_numbers_count_calls_with_commands():
    """Rule of the boundary: each call with q >= 1 on a built map takes the
    next batch number, also when its op codes reject it (it then records no
    access); a call with q = 0 takes none.  Labels follow the calls alone."""
    m, p, k = _fresh_map(256, 200, 200, 3, trace=True)
    n0 = m.trace().size
    z = np.zeros((4, 8), np.uint8)
    good = np.zeros(4, np.uint8)
    bad = np.array([0, 1, 7, 0], np.uint8)
    calls = [good, bad, None, good, bad, bad, good]
    expect = []
    label = 0
    for c in calls:
        if c is None:
            assert m.access(np.zeros(0, np.uint8), k[:0], np.zeros((0, 8), np.uint8))[0] == O.OK
            continue
        label += 1
        rc = m.access(c, k[:4], z)[0]
        assert rc == (O.OK if c is good else O.EINVAL)
        if c is good:
            expect.append(label)
    t = m.trace()[n0:]
    assert sorted(set(t["batch"].tolist())) == expect == [1, 3, 6]
    assert m.ctr == 12  # rejected calls use no tape step


# ------------------------------------------------------------ planted mistakes

MUTANTS = {
    # the second bin also on a tie
    "ties_to_second": [("chosen[o] = m->load[r2[i]] < m->load[r1[i]] ? r2[i] : r1[i];",
                        "chosen[o] = m->load[r2[i]] <= m->load[r1[i]] ? r2[i] : r1[i];")],
    # the more loaded bin
    "picks_reversed": [("chosen[o] = m->load[r2[i]] < m->load[r1[i]] ? r2[i] : r1[i];",
                        "chosen[o] = m->load[r2[i]] < m->load[r1[i]] ? r1[i] : r2[i];")],
    # every key of the batch in one round
    "one_round": [("  uint64_t rs = (s->B + 15) / 16;\n  uint32_t* ord",
                   "  uint64_t rs = q;\n  uint32_t* ord")],
    # one key at a time
    "sequential": [("  uint64_t rs = (s->B + 15) / 16;\n  uint32_t* ord",
                    "  uint64_t rs = 1;\n  uint32_t* ord")],
    # P2C on the loads before the batch's removals (removals applied after)
    "pre_removal_loads": [
        ("  int broken = 0;\n", "  int broken = 0;\n  uint32_t* pre_rm = malloc(2ull * q * sizeof(uint32_t));\n"
                                "  uint32_t npre = 0;\n"),
        ("        m->load[b]--;\n", "        pre_rm[npre++] = (uint32_t)b;\n"),
        ("  for (uint32_t o = 0; o < nplace; ++o)\n    if (m->load[chosen[o]] > s->Z) over = 1;",
         "  for (uint32_t x = 0; x < npre; ++x) m->load[pre_rm[x]]--;\n"
         "  for (uint32_t o = 0; o < nplace; ++o)\n    if (m->load[chosen[o]] > s->Z) over = 1;"),
    ],
    # the remap takes the fetch words of the tape
    "remap_from_fetch_words": [("or_pair(w[2], w[3], s->B, &r1[i], &r2[i]);",
                                "or_pair(w[0], w[1], s->B, &r1[i], &r2[i]);")],
    # repeated keys read the mapped pair again instead of a fresh one
    "repeats_read_mapped_pair": [
        ("    if (hit[i]) {\n      pr[0] = m->rows[hrow[i] * s->W + hidx[i]].p1;\n"
         "      pr[1] = m->rows[hrow[i] * s->W + hidx[i]].p2;\n    }",
         "    if (hit[leader[i]]) {\n      pr[0] = m->rows[hrow[leader[i]] * s->W + hidx[leader[i]]].p1;\n"
         "      pr[1] = m->rows[hrow[leader[i]] * s->W + hidx[leader[i]]].p2;\n    }")],
}


def _build_mutant(tmp_path, name):
    src = open(ORACLE_SRC).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    c = tmp_path / ("or_%s.c" % name)
    c.write_text(src)
    so = tmp_path / ("or_%s.so" % name)
    subprocess.run(["gcc", "-O2", "-std=c11", "-w", "-shared", "-fPIC", "-o", str(so), str(c), "-lm"], check=True)
    return O.load_variant(str(so))


@pytest.mark.parametrize("name", ["ties_to_second", "picks_reversed", "one_round", "sequential",
                                  "pre_removal_loads", "remap_from_fetch_words"])
def test_remap_pin_catches_planted_mistake(tmp_path, name):
    lib = _build_mutant(tmp_path, name)
    assert check_remap_rule(lib=lib) is not None


@pytest.mark.parametrize("name", ["repeats_read_mapped_pair", "remap_from_fetch_words"])
def test_reveal_pin_catches_planted_mistake(tmp_path, name):
    lib = _build_mutant(tmp_path, name)
    assert check_revealed_pairs(lib=lib) is not None

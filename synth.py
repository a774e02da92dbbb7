"""Seeded synthetic inputs for the oblivious-map workloads.

This module holds no arithmetic of the map itself; it only draws keys,
values and query streams, and both the HIP path's tests and the oracle are
fed from it.  The inputs stand in for the paper's YCSB-like workload
(Sec. 6.2), which is not available here:

* keys: key_i = mix64(seed + i), with mix64 the SplitMix64 finalizer (a
  bijection on 64-bit words), so keys are distinct;
* absent keys: mix64(seed + N + j), disjoint from the present keys;
* values: bytes from numpy's PCG64 generator;
* Zipf(s) ranks by inverse CDF over a float64 table (numpy's own ``zipf``
  needs s > 1); ranks map to keys through a seeded permutation so the hot
  keys are spread out.

Seeds are 0xB0170000 + config number, with fixed sub-seeds per stream.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 0xB0170000
GET, PUT, DEL = 0, 1, 2
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finalizer, elementwise on uint64."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def keys(n: int, seed: int, offset: int = 0) -> np.ndarray:
    """n distinct keys mix64(seed + offset + i)."""
    with np.errstate(over="ignore"):
        ctr = np.uint64(seed) + np.uint64(offset) + np.arange(n, dtype=np.uint64)
    return mix64(ctr)


def values(n: int, vs: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 256, size=(n, vs), dtype=np.uint8)


def zipf_ranks(n_items: int, count: int, s: float, rng: np.random.Generator) -> np.ndarray:
    """count ranks in [0, n_items) with P(r) proportional to (r + 1)^-s."""
    w = np.arange(1, n_items + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(count)
    return np.minimum(np.searchsorted(cdf, u, side="right"), n_items - 1)


class Workload:
    """A built map's inputs plus a stream of (ops, keys, vals) batches."""

    def __init__(self, name, cap, vs, build_keys, build_vals, batches):
        self.name = name
        self.cap = cap
        self.vs = vs
        self.build_keys = build_keys
        self.build_vals = build_vals
        self.batches = batches  # list of (ops u8[q], keys u64[q], vals u8[q, vs])

    @property
    def n(self):
        return int(self.build_keys.size)

    @property
    def n_ops(self):
        return int(sum(b[0].size for b in self.batches))


def config1(n: int = 1 << 16, n_get: int = 1 << 14, n_put: int = 1 << 12) -> Workload:
    """N=2^16, u64 keys/values; 2^14 single GETs (90 % present, 10 % absent)
    and 2^12 single PUTs that overwrite present keys."""
    seed = SEED_BASE + 1
    vs = 8
    k = keys(n, seed)
    v = values(n, vs, seed + 1)
    rng = np.random.Generator(np.random.PCG64(seed + 2))
    absent = keys(n_get, seed, offset=n)
    present = rng.random(n_get) < 0.9
    gk = np.where(present, k[rng.integers(0, n, n_get)], absent)
    pk = k[rng.integers(0, n, n_put)]
    pv = values(n_put, vs, seed + 3)
    batches = []
    for i in range(n_get):
        batches.append((np.array([GET], np.uint8), gk[i:i + 1].copy(), np.zeros((1, vs), np.uint8)))
    for i in range(n_put):
        batches.append((np.array([PUT], np.uint8), pk[i:i + 1].copy(), pv[i:i + 1].copy()))
    return Workload("plain-omap-n16", n, vs, k, v, batches)


def config2(n: int = 1 << 24, n_ops: int = 1 << 20, batch: int = 4096, vs: int = 64,
            zipf_s: float = 0.99, absent_frac: float = 0.05, put_frac: float = 0.10,
            headroom: int = 1 << 16, n_batches: int | None = None) -> Workload:
    """N=2^24, 64-byte values; n_ops ops in batches of 4096, Zipf(0.99) over
    present keys with 5 % absent keys, 90 % GET / 10 % PUT.  Absent PUTs insert,
    so the capacity is N + 2^16."""
    seed = SEED_BASE + 2
    k = keys(n, seed)
    v = values(n, vs, seed + 1)
    rng = np.random.Generator(np.random.PCG64(seed + 2))
    perm = rng.permutation(n)
    total = n_ops if n_batches is None else n_batches * batch
    ranks = zipf_ranks(n, total, zipf_s, rng)
    qk = k[perm[ranks]]
    is_absent = rng.random(total) < absent_frac
    qk = np.where(is_absent, keys(total, seed, offset=n + rng.integers(0, 1 << 30)), qk)
    ops = np.where(rng.random(total) < put_frac, PUT, GET).astype(np.uint8)
    qv = values(total, vs, seed + 3)
    batches = [(ops[i:i + batch], qk[i:i + batch], qv[i:i + batch]) for i in range(0, total, batch)]
    return Workload("plain-omap-n24-v64-zipf", n + headroom, vs, k, v, batches)


def config3(n: int = 1 << 26, n_get: int = 1 << 16, batch: int = 4096) -> Workload:
    """Build-heavy: N=2^26, 8-byte values, then 2^16 uniform GETs."""
    seed = SEED_BASE + 3
    vs = 8
    k = keys(n, seed)
    v = values(n, vs, seed + 1)
    rng = np.random.Generator(np.random.PCG64(seed + 2))
    gk = k[rng.integers(0, n, n_get)]
    batches = [(np.zeros(min(batch, n_get - i), np.uint8), gk[i:i + batch], np.zeros((min(batch, n_get - i), vs), np.uint8))
               for i in range(0, n_get, batch)]
    return Workload("build-heavy-n26-v8", n, vs, k, v, batches)


def config4(n_maps: int = 64, lo: int = 10, hi: int = 22, qmax: int = 8192, vs: int = 8,
            absent_frac: float = 0.10) -> list:
    """64 maps with N log-uniform in [2^lo, 2^hi], each with one GET batch of
    size uniform in [1, qmax] (uniform present keys, 10 % absent)."""
    seed = SEED_BASE + 4
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for m in range(n_maps):
        n = int(2 ** (lo + (hi - lo) * rng.random()))
        q = int(rng.integers(1, qmax + 1))
        ms = seed + 1000 * (m + 1)
        k = keys(n, ms)
        v = values(n, vs, ms + 1)
        r2 = np.random.Generator(np.random.PCG64(ms + 2))
        qk = np.where(r2.random(q) < absent_frac, keys(q, ms, offset=n), k[r2.integers(0, n, q)])
        out.append(Workload("multi-map-%d" % m, n, vs, k, v,
                            [(np.zeros(q, np.uint8), qk.astype(np.uint64), np.zeros((q, vs), np.uint8))]))
    return out


def config5_maps(n_maps: int = 16, lo: int = 16, hi: int = 24, vs: int = 64) -> list:
    """16 resident maps with N log-uniform in [2^lo, 2^hi], 64-byte values."""
    seed = SEED_BASE + 5
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for m in range(n_maps):
        n = int(2 ** (lo + (hi - lo) * rng.random()))
        ms = seed + 1000 * (m + 1)
        out.append((n, keys(n, ms), values(n, vs, ms + 1), ms))
    return out


def request_stream(n_keys_map: dict, key_arrays: dict, vs: int, rate_hz: float, duration_s: float,
                   qmax: int = 4096, zipf_s: float = 0.99, put_frac: float = 0.10, seed: int = SEED_BASE + 50):
    """Poisson arrivals of request batches over several maps: size
    floor(2^(12u)) clipped to [1, qmax], 90 % GET / 10 % PUT, Zipf keys.
    Yields (t_arrival, map_id, ops, keys, vals) in arrival order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ids = sorted(n_keys_map)
    t = 0.0
    zcache: dict = {}
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s:
            return
        mid = ids[int(rng.integers(0, len(ids)))]
        q = int(min(qmax, max(1, int(2 ** (12 * rng.random())))))
        n = n_keys_map[mid]
        if mid not in zcache:
            w = np.arange(1, n + 1, dtype=np.float64) ** (-zipf_s)
            c = np.cumsum(w)
            zcache[mid] = (c / c[-1], rng.permutation(n))
        cdf, perm = zcache[mid]
        ranks = np.minimum(np.searchsorted(cdf, rng.random(q), side="right"), n - 1)
        ks = key_arrays[mid][perm[ranks]]
        ops = np.where(rng.random(q) < put_frac, PUT, GET).astype(np.uint8)
        vals = rng.integers(0, 256, size=(q, vs), dtype=np.uint8)
        yield t, mid, ops, ks, vals

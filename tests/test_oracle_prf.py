"""Pins of the oracle's PRF (keyed BLAKE2s) and of its pair reduction.

The PRF is checked against Python's hashlib (a separate BLAKE2s
implementation) and against the RFC 7693 test vector; the pair reduction
against the pair law in the proof of Claim 4.1 (every ordered pair of
distinct bins equally likely)."""
import hashlib
import json
import os
import struct

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_rfc7693_vector():
    g = json.load(open(os.path.join(GOLDEN, "rfc7693_blake2s_abc.json")))
    out = O.blake2s(bytes.fromhex(g["key_hex"]), bytes.fromhex(g["msg_hex"]))
    assert out.hex() == g["digest_hex"]


@pytest.mark.parametrize("klen", [0, 1, 16, 31, 32])
@pytest.mark.parametrize("mlen", [0, 1, 9, 55, 63, 64, 65, 128, 200])
def test_blake2s_matches_hashlib(klen, mlen):
    rng = np.random.default_rng(klen * 1000 + mlen)
    key = bytes(rng.integers(0, 256, klen, dtype=np.uint8))
    msg = bytes(rng.integers(0, 256, mlen, dtype=np.uint8))
    assert O.blake2s(key, msg) == hashlib.blake2s(msg, key=key, digest_size=32).digest()
    assert O.blake2s(key, msg, 16) == hashlib.blake2s(msg, key=key, digest_size=16).digest()


def test_prf_is_blake2s_of_domain_and_le64():
    key = bytes(range(32))
    for domain in (1, 2, 3):
        for x in (0, 1, 0xFFFFFFFFFFFFFFFF, 0x0123456789ABCDEF):
            d = hashlib.blake2s(bytes([domain]) + struct.pack("<Q", x), key=key, digest_size=32).digest()
            assert O.prf(key, domain, x) == struct.unpack("<4Q", d)


def test_pair_distinct_and_in_range():
    rng = np.random.default_rng(7)
    for B in (2, 3, 7, 1000, 2105344, 8388608):
        for _ in range(200):
            w0, w1 = (int(v) for v in rng.integers(0, 2**63, 2, dtype=np.uint64) * 2 + rng.integers(0, 2, 2))
            a, b = O.pair(w0, w1, B)
            assert 0 <= a < B and 0 <= b < B and a != b


def test_pair_extremes():
    # w = 0 gives the lowest bin; w = 2^64 - 1 the highest offsets.
    assert O.pair(0, 0, 10) == (0, 1)
    top = 2**64 - 1
    assert O.pair(top, 0, 10) == (9, 0)
    assert O.pair(0, top, 10) == (0, 9)
    assert O.pair(top, top, 10) == (9, 8)


def test_pair_law_chi_square():
    """Claim 4.1: Pr[(b1, b2)] = 1 / (B (B - 1)) for every ordered distinct pair."""
    B = 12
    n = 132 * 150
    key = bytes(32)
    counts = np.zeros((B, B))
    for s in range(n):
        w = O.prf(key, 3, s)
        a, b = O.pair(w[0], w[1], B)
        counts[a, b] += 1
    assert np.trace(counts) == 0
    obs = counts[~np.eye(B, dtype=bool)]
    exp = n / (B * (B - 1))
    chi2 = ((obs - exp) ** 2 / exp).sum()
    # 131 degrees of freedom: the 0.999 quantile is about 190.
    assert chi2 < 190, chi2

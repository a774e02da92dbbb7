"""Sealed command and response records (Sec. 3: the host relays only
encrypted instructions and results; Sec. 5.1: the decode module opens them,
the response module seals results).

* The oracle's records against OpenSSL's ChaCha20-Poly1305 (libcrypto through
  ctypes), which shares nothing with it: every record is the RFC 8439 AEAD
  of its plain fields under the stated nonce and associated data.
* Changed records, changed counts (a truncated request), other request
  numbers (a replay) and swapped records fail their tags.
* The library's client helpers (host code, no GPU) seal and open exactly
  the oracle's records, byte for byte."""
import ctypes.util

import numpy as np
import pytest

import oracle as O

_crypto = ctypes.util.find_library("crypto")
KEY = bytes((3 * i + 1) & 255 for i in range(32))


def _cmds(q, vs, seed):
    rng = np.random.default_rng(seed)
    ops = rng.integers(0, 3, q).astype(np.uint8)
    keys = rng.integers(0, 2**63, q, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    vals = rng.integers(0, 256, (q, vs), dtype=np.uint8)
    return ops, keys, vals


def _nonce(direction, i, seq):
    return ((direction << 31) | i).to_bytes(4, "little") + seq.to_bytes(8, "little")


@pytest.mark.skipif(_crypto is None, reason="no libcrypto to pin against")
@pytest.mark.parametrize("q,vs,seq", [(1, 8, 1), (5, 64, 7), (3, 24, 2**40 + 3), (2, 256, 99)])
def test_records_are_rfc8439_aead_of_their_fields(q, vs, seq):
    from test_oracle_seal import _ssl_aead

    ops, keys, vals = _cmds(q, vs, q + vs)
    recs = O.cmd_seal(KEY, seq, ops, keys, vals, vs)
    aad = q.to_bytes(8, "little")
    for i in range(q):
        plain = int(ops[i]).to_bytes(8, "little") + int(keys[i]).to_bytes(8, "little") + bytes(vals[i])
        ct, tag = _ssl_aead(KEY, _nonce(0, i, seq), aad, plain)
        assert bytes(recs[i]) == ct + tag
    st = np.array([1, 2, 0, 3, 0xFF][:q] * (q // 5 + 1), np.uint8)[:q]
    rv = O.resp_seal(KEY, seq, st, vals, vs)
    for i in range(q):
        plain = int(st[i]).to_bytes(8, "little") + bytes(vals[i])
        ct, tag = _ssl_aead(KEY, _nonce(1, i, seq), aad, plain)
        assert bytes(rv[i]) == ct + tag


def test_records_open_only_as_sealed():
    q, vs, seq = 6, 16, 5
    ops, keys, vals = _cmds(q, vs, 1)
    recs = O.cmd_seal(KEY, seq, ops, keys, vals, vs)
    bad, o, k, v = O.cmd_open(KEY, seq, recs, vs)
    assert bad == 0 and np.array_equal(o, ops) and np.array_equal(k, keys) and np.array_equal(v, vals)
    assert O.cmd_open(KEY, seq + 1, recs, vs)[0] == q          # another request number: a replay
    assert O.cmd_open(KEY, seq, recs[:q - 1], vs)[0] == q - 1  # truncated: the count is bound in
    assert O.cmd_open(bytes(32), seq, recs, vs)[0] == q        # another session
    sw = recs[[1, 0, 2, 3, 4, 5]]
    assert O.cmd_open(KEY, seq, sw, vs)[0] == 2                 # swapped records
    for at in (0, 17, 16 + vs + 3):                              # cipher text or tag changed
        x = recs.copy()
        x[2, at] ^= 0x40
        bad, o, k, v = O.cmd_open(KEY, seq, x, vs)
        assert bad == 1 and o[2] == 0xFF and k[2] == 0 and not v[2].any()
    rv = O.resp_seal(KEY, seq, np.arange(q, dtype=np.uint8), vals, vs)
    assert O.resp_open(KEY, seq, rv, vs)[0] == 0
    assert O.resp_open(KEY, seq + 1, rv, vs)[0] == q


@pytest.mark.parametrize("q,vs,seq", [(1, 8, 1), (64, 64, 3), (7, 4096, 2**33 + 1), (300, 16, 12)])
def test_library_client_helpers_match_the_oracle(q, vs, seq):
    import paper_2509_01742_amd as B

    ops, keys, vals = _cmds(q, vs, 11 * q + vs)
    got = B.seal_requests(KEY, seq, ops, keys, vals, vs)
    assert np.array_equal(got, O.cmd_seal(KEY, seq, ops, keys, vals, vs))
    st = np.random.default_rng(q).integers(0, 4, q).astype(np.uint8)
    rv = O.resp_seal(KEY, seq, st, vals, vs)
    rc, st2, v2 = B.open_responses(KEY, seq, rv, vs)
    assert rc == B.BOLT_OK and np.array_equal(st2, st) and np.array_equal(v2, vals)
    rv[q // 2, 5] ^= 1
    rc, st3, v3 = B.open_responses(KEY, seq, rv, vs)
    assert rc == B.BOLT_ETAMPER and st3[q // 2] == 0 and not v3[q // 2].any()
    assert B.open_responses(KEY, seq + 1, O.resp_seal(KEY, seq, st, vals, vs), vs)[0] == B.BOLT_ETAMPER

"""The oracle's ChaCha20-Poly1305 (RFC 8439), which seals observable pages,
pinned against an implementation it shares nothing with: the system's
OpenSSL libcrypto, called through ctypes (EVP_chacha20 for the raw key
stream, EVP_chacha20_poly1305 for the AEAD)."""
import ctypes as C
import ctypes.util

import numpy as np
import pytest

import oracle as O
from oracle import OK

_name = ctypes.util.find_library("crypto")
pytestmark = pytest.mark.skipif(_name is None, reason="no libcrypto to pin against")

EVP_CTRL_AEAD_SET_IVLEN = 0x9  # openssl/evp.h
EVP_CTRL_AEAD_GET_TAG = 0x10


def _ssl():
    lib = C.CDLL(_name)
    P = C.c_void_p
    lib.EVP_CIPHER_CTX_new.restype = P
    lib.EVP_chacha20_poly1305.restype = P
    lib.EVP_chacha20.restype = P
    lib.EVP_EncryptInit_ex.argtypes = [P, P, P, P, P]
    lib.EVP_EncryptUpdate.argtypes = [P, P, C.POINTER(C.c_int), P, C.c_int]
    lib.EVP_EncryptFinal_ex.argtypes = [P, P, C.POINTER(C.c_int)]
    lib.EVP_CIPHER_CTX_ctrl.argtypes = [P, C.c_int, C.c_int, P]
    lib.EVP_CIPHER_CTX_free.argtypes = [P]
    return lib


def _ssl_aead(key, nonce, aad, pt):
    lib = _ssl()
    ctx = lib.EVP_CIPHER_CTX_new()
    assert lib.EVP_EncryptInit_ex(ctx, lib.EVP_chacha20_poly1305(), None, None, None) == 1
    assert lib.EVP_CIPHER_CTX_ctrl(ctx, EVP_CTRL_AEAD_SET_IVLEN, 12, None) == 1
    assert lib.EVP_EncryptInit_ex(ctx, None, None, O._buf(key), O._buf(nonce)) == 1
    n = C.c_int()
    if aad:
        assert lib.EVP_EncryptUpdate(ctx, None, C.byref(n), O._buf(aad), len(aad)) == 1
    out = (C.c_uint8 * (len(pt) + 16))()
    total = 0
    if pt:
        assert lib.EVP_EncryptUpdate(ctx, out, C.byref(n), O._buf(pt), len(pt)) == 1
        total = n.value
    assert lib.EVP_EncryptFinal_ex(ctx, C.byref(out, total), C.byref(n)) == 1
    tag = (C.c_uint8 * 16)()
    assert lib.EVP_CIPHER_CTX_ctrl(ctx, EVP_CTRL_AEAD_GET_TAG, 16, tag) == 1
    lib.EVP_CIPHER_CTX_free(ctx)
    return bytes(out)[:len(pt)], bytes(tag)


def _ssl_stream(key, counter, nonce, n):
    """n bytes of ChaCha20 key stream from block `counter` (IV = LE32(counter) || nonce)."""
    lib = _ssl()
    ctx = lib.EVP_CIPHER_CTX_new()
    iv = counter.to_bytes(4, "little") + nonce
    assert lib.EVP_EncryptInit_ex(ctx, lib.EVP_chacha20(), None, O._buf(key), O._buf(iv)) == 1
    out = (C.c_uint8 * n)()
    m = C.c_int()
    assert lib.EVP_EncryptUpdate(ctx, out, C.byref(m), O._buf(bytes(n)), n) == 1
    lib.EVP_CIPHER_CTX_free(ctx)
    return bytes(out)


def test_chacha20_block_matches_libcrypto():
    rng = np.random.default_rng(1)
    for counter in (0, 1, 7, 2**32 - 1):
        key = rng.bytes(32)
        nonce = rng.bytes(12)
        assert O.chacha20_block(key, counter, nonce) == _ssl_stream(key, counter, nonce, 64)


@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 63, 64, 65, 127, 128, 1000, 1024, 4096, 4099])
def test_aead_matches_libcrypto(n):
    rng = np.random.default_rng(n + 3)
    for aad_len in (0, 12, 33):
        key, nonce, aad, pt = rng.bytes(32), rng.bytes(12), rng.bytes(aad_len), rng.bytes(n)
        ct, tag = O.aead_seal(key, nonce, aad, pt)
        assert (ct, tag) == _ssl_aead(key, nonce, aad, pt), (n, aad_len)
        assert O.aead_open(key, nonce, aad, ct, tag) == pt


def test_poly1305_limits():
    """Blocks whose sums reach and pass p = 2^130 - 5, with the key's r clamped
    to its largest value: Poly1305 against the AEAD's own definition via
    libcrypto on all-0xFF texts (the carry and final reduction paths)."""
    key = bytes([0xFF] * 32)
    for n in (16, 32, 48, 4096):
        pt = bytes([0xFF] * n)
        nonce = bytes(12)
        assert O.aead_seal(key, nonce, b"", pt) == _ssl_aead(key, nonce, b"", pt)


def test_open_rejects_any_change():
    rng = np.random.default_rng(9)
    key, nonce, pt = rng.bytes(32), rng.bytes(12), rng.bytes(1024)
    ct, tag = O.aead_seal(key, nonce, b"", pt)
    for pos in (0, 511, 1023):
        bad = bytearray(ct)
        bad[pos] ^= 1
        assert O.aead_open(key, nonce, b"", bytes(bad), tag) is None
    bt = bytearray(tag)
    bt[15] ^= 0x80
    assert O.aead_open(key, nonce, b"", ct, bytes(bt)) is None
    other = bytearray(nonce)
    other[4] ^= 1  # another version of the same page
    assert O.aead_open(key, bytes(other), b"", ct, tag) is None


# ------------------------------------------------------------------ sealed map

def _maps(cap=3000, n=2500, vs=16, seed=3):
    import synth

    k, v = synth.keys(n, seed), synth.values(n, vs, seed + 1)
    plain = O.OracleMap(cap, vs, key=bytes(range(32)), trace=True)
    sealed = O.OracleMap(cap, vs, key=bytes(range(32)), trace=True, seal=True)
    assert plain.build(k, v) == 0 and sealed.build(k, v) == 0
    return plain, sealed, k


def _open_all(m):
    """Every observable page of a sealed oracle map, opened with its key."""
    key = b"".join(int(w).to_bytes(8, "little") for w in O.prf(bytes(range(32)), 4, 0))
    obs, tags, ver = m.observable(), m.tags(), m.versions()
    out = []
    for p in range(obs.shape[0]):
        nonce = int(p).to_bytes(4, "little") + int(ver[p]).to_bytes(8, "little")
        pt = O.aead_open(key, nonce, b"", obs[p].tobytes(), tags[p].tobytes())
        assert pt is not None, p
        out.append(np.frombuffer(pt, dtype=np.uint8))
    return np.stack(out)


def test_sealed_map_is_the_plain_map_under_the_seal():
    """Sealing changes the bytes in the store, not the procedure: the same
    answers, the same trace, and every page opens to the unsealed map's page
    with the version that counts its writes."""
    plain, sealed, k = _maps()
    rng = np.random.default_rng(4)
    for b in range(12):
        q = int(rng.integers(1, 400))
        ops = rng.choice([0, 1, 2], size=q, p=[0.6, 0.3, 0.1]).astype(np.uint8)
        keys = k[rng.integers(0, k.size, q)]
        vals = rng.integers(0, 256, (q, 16), dtype=np.uint8)
        ra, va, sa = plain.access(ops, keys, vals)
        rb, vb, sb = sealed.access(ops, keys, vals)
        assert ra == rb == 0 and np.array_equal(va, vb) and np.array_equal(sa, sb)
    assert np.array_equal(plain.trace(), sealed.trace())
    assert np.array_equal(_open_all(sealed), plain.observable())
    assert not np.array_equal(sealed.observable(), plain.observable())
    tr = sealed.trace()
    writes = np.bincount(tr["page"][tr["kind"] == 1].astype(np.int64), minlength=sealed.s["M"])
    assert np.array_equal(sealed.versions(), writes)  # one more per write, from the build's 1


def _read_all(m, k):
    """A batch that reads the pages of many keys."""
    q = min(2000, k.size)
    return m.access(np.zeros(q, np.uint8), k[:q], np.zeros((q, m.s["vs"]), np.uint8))[0]


@pytest.mark.parametrize("where", ["page", "tag"])
def test_sealed_map_refuses_a_changed_page(where):
    _, sealed, k = _maps()
    pb = sealed.s["page_bytes"]
    raw = bytearray(sealed.raw_page(5))
    raw[17 if where == "page" else pb + 3] ^= 0x40
    sealed.put_raw_page(5, bytes(raw))
    rc = OK
    for _ in range(50):  # until some batch reads page 5
        rc = _read_all(sealed, k)
        if rc != OK:
            break
    assert rc == O.ETAMPER
    assert _read_all(sealed, k) == O.ESTATE  # poisoned


def test_sealed_map_refuses_a_replayed_page():
    _, sealed, k = _maps()
    old = [sealed.raw_page(p) for p in range(sealed.s["M"])]
    v0 = sealed.versions()
    rc = _read_all(sealed, k)  # rewrites every page it read
    assert rc == OK
    moved = np.nonzero(sealed.versions() != v0)[0]
    assert moved.size > 0
    p = int(moved[0])
    sealed.put_raw_page(p, old[p])  # the page as it was one write ago: a valid old seal
    rc = OK
    for _ in range(50):
        rc = _read_all(sealed, k)
        if rc != OK:
            break
    assert rc == O.ETAMPER

"""The oracle's ChaCha20-Poly1305 (RFC 8439), which seals observable pages,
pinned against an implementation it shares nothing with: the system's
OpenSSL libcrypto, called through ctypes (EVP_chacha20 for the raw key
stream, EVP_chacha20_poly1305 for the AEAD)."""
import ctypes as C
import ctypes.util

import numpy as np
import pytest

import oracle as O

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

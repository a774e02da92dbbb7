"""Reference oracle for the BOLT oblivious map (arxiv 2509.01742).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this package.  The product path
(the HIP library and its binding) never imports it.  It shares no code with
that path.

Two oracles live here:

* ``PlainMap`` (O1) is the plain definition of the answers: a dictionary
  with the Get/Put/Delete semantics of Sec. 2.1 (delete = a tombstone put).
* ``OracleMap`` (O2) is a scalar, single-threaded C implementation of the
  same oblivious procedure the GPU runs (``bolt_oracle.c``).  It covers the
  build (PRF, P2C rounds, bitonic network, expansion network, page
  write-out, position map) and batched access (Alg. 1 in the module order
  of Sec. 5.1), and it records every access to the observable store.

The C file is compiled by ``oracle/build.py`` into ``oracle/liboracle.so``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, EDUPKEY, EOVERFLOW, EFULL, ESTATE, EBROKEN = 0, -1, -2, -3, -4, -5, -7, -99
ETAMPER = -9
GET, PUT, DEL = 0, 1, 2
ST_ABSENT, ST_FOUND, ST_UPDATED, ST_INSERTED, ST_DELETED = 0, 1, 1, 2, 3
NONE32 = 0xFFFFFFFF


class _Sizes(C.Structure):
    _fields_ = [
        ("cap", C.c_uint64), ("vs", C.c_uint32), ("c", C.c_uint32), ("alpha_pm", C.c_uint32),
        ("Z", C.c_uint32), ("d", C.c_uint32), ("kpr", C.c_uint32), ("W", C.c_uint32),
        ("B", C.c_uint64), ("K", C.c_uint64), ("M", C.c_uint64), ("R_pm", C.c_uint64),
        ("page_bytes", C.c_uint64), ("stash_bound", C.c_uint64), ("lmax", C.c_uint32),
        ("hbm_bound", C.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


TRACE_DTYPE = np.dtype([("batch", "<u4"), ("kind", "<u4"), ("page", "<u8")])

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    _lib = _configure(C.CDLL(_LIB_PATH))
    return _lib


def load_openmp():
    """The same oracle built with OpenMP (the parallel CPU baseline); its
    thread count follows OMP_NUM_THREADS."""
    path = os.path.join(_HERE, "liboracle_omp.so")
    if not os.path.exists(path):
        from . import build as _build

        _build.build()
    return _configure(C.CDLL(path))


def load_variant(path: str):
    """Loads another build of the oracle's C source (the tests compile
    copies with a planted mistake, to show that the pins catch it)."""
    return _configure(C.CDLL(path))


def _configure(lib):
    P, U8P, U32P, U64P = C.c_void_p, C.POINTER(C.c_uint8), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
    lib.or_blake2s.argtypes = [P, C.c_uint32, P, C.c_uint32, P, C.c_uint64]
    lib.or_prf.argtypes = [P, C.c_uint8, C.c_uint64, P]
    lib.or_pair.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, P, P]
    lib.or_sizing.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                              C.c_uint32, C.c_uint32, C.POINTER(_Sizes)]
    lib.or_stash_bound.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64]
    lib.or_stash_bound.restype = C.c_uint64
    for name, n in (("or_claim43_bound", 4), ("or_claim44_bound", 4), ("or_claim52_bits", 7)):
        getattr(lib, name).argtypes = [C.c_double] * n
        getattr(lib, name).restype = C.c_double
    lib.or_bitonic_sort_u64.argtypes = [P, C.c_uint64]
    lib.or_expand.argtypes = [P, P, C.c_uint64, C.c_uint64, P]
    lib.or_compact.argtypes = [P, P, C.c_uint64, P]
    lib.or_create.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                              C.c_uint32, C.c_uint32, P, C.c_int]
    lib.or_create.restype = C.c_void_p
    lib.or_destroy.argtypes = [P]
    lib.or_build.argtypes = [P, P, P, C.c_uint64, C.c_int]
    lib.or_access.argtypes = [P, P, P, P, P, P, C.c_uint32]
    lib.or_get_sizes.argtypes = [P]
    lib.or_get_sizes.restype = C.POINTER(_Sizes)
    for name in ("or_obs_ptr", "or_hbm_ptr"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = C.c_void_p
    lib.or_load_ptr.argtypes = [P]
    lib.or_load_ptr.restype = C.c_void_p
    for name in ("or_ctr", "or_live", "or_stash_live", "or_stash_highwater", "or_trace_len"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = C.c_uint64
    lib.or_trace_copy.argtypes = [P, P, C.c_uint64]
    lib.or_trace_copy.restype = C.c_uint64
    lib.or_trace_clear.argtypes = [P]
    lib.or_stash_copy.argtypes = [P, P, P, P, C.c_uint64]
    lib.or_stash_copy.restype = C.c_uint64
    lib.or_pm_copy.argtypes = [P, P, P, P, P, C.c_uint64]
    lib.or_pm_copy.restype = C.c_uint64
    lib.or_pm_max_row.argtypes = [P]
    lib.or_pm_max_row.restype = C.c_uint32
    lib.or_chacha20_block.argtypes = [P, C.c_uint32, P, P]
    lib.or_set_seal.argtypes = [P]
    lib.or_set_decomposed.argtypes = [P]
    lib.or_hbm_live.argtypes = [P]
    lib.or_hbm_live.restype = C.c_uint64
    for name in ("or_tags_ptr", "or_ver_ptr"):
        getattr(lib, name).argtypes = [P]
        getattr(lib, name).restype = C.c_void_p
    lib.or_obs_raw.argtypes = [P, C.c_uint64, P, C.c_int]
    lib.or_poly1305.argtypes = [P, P, C.c_uint64, P]
    lib.or_aead_seal.argtypes = [P, P, P, C.c_uint64, P, C.c_uint64, P, P]
    lib.or_aead_open.argtypes = [P, P, P, C.c_uint64, P, C.c_uint64, P, P]
    lib.or_plain_create.argtypes = [C.c_uint64, C.c_uint32]
    lib.or_plain_create.restype = C.c_void_p
    lib.or_plain_destroy.argtypes = [P]
    lib.or_plain_build.argtypes = [P, P, P, C.c_uint64]
    lib.or_plain_access.argtypes = [P, P, P, P, P, P, C.c_uint32]
    lib.or_plain_size.argtypes = [P]
    lib.or_plain_size.restype = C.c_uint64
    lib.or_cmd_seal.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P, P, P, P]
    lib.or_cmd_open.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P, P, P, P]
    lib.or_cmd_open.restype = C.c_uint32
    lib.or_resp_seal.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P, P, P]
    lib.or_resp_open.argtypes = [P, C.c_uint64, C.c_uint32, C.c_uint32, P, P, P]
    lib.or_resp_open.restype = C.c_uint32
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------

def blake2s(key: bytes, msg: bytes, nn: int = 32) -> bytes:
    """Keyed BLAKE2s (RFC 7693)."""
    lib = _load()
    out = (C.c_uint8 * 32)()
    kb = (C.c_uint8 * max(1, len(key))).from_buffer_copy(key or b"\0")
    mb = (C.c_uint8 * max(1, len(msg))).from_buffer_copy(msg or b"\0")
    rc = lib.or_blake2s(out, nn, kb, len(key), mb, len(msg))
    if rc:
        raise ValueError("bad BLAKE2s lengths")
    return bytes(out)[:nn]


def prf(key: bytes, domain: int, x: int) -> tuple:
    """PRF_K(domain, x) = BLAKE2s_K(domain || LE64(x)) as four LE64 words."""
    lib = _load()
    w = (C.c_uint64 * 4)()
    kb = (C.c_uint8 * 32).from_buffer_copy(key)
    lib.or_prf(kb, domain, x, w)
    return tuple(int(v) for v in w)


def _buf(b: bytes):
    return (C.c_uint8 * max(1, len(b))).from_buffer_copy(b or b"\0")


def chacha20_block(key: bytes, counter: int, nonce: bytes) -> bytes:
    """One ChaCha20 block (RFC 8439, Sec. 2.3)."""
    out = (C.c_uint8 * 64)()
    _load().or_chacha20_block(_buf(key), counter, _buf(nonce), out)
    return bytes(out)


def poly1305(key: bytes, msg: bytes) -> bytes:
    """Poly1305 tag of msg under a 32-byte one-time key (RFC 8439, Sec. 2.5)."""
    tag = (C.c_uint8 * 16)()
    _load().or_poly1305(_buf(key), _buf(msg), len(msg), tag)
    return bytes(tag)


def aead_seal(key: bytes, nonce: bytes, aad: bytes, pt: bytes) -> tuple:
    """AEAD_CHACHA20_POLY1305 (RFC 8439, Sec. 2.8): (ciphertext, tag)."""
    ct = (C.c_uint8 * max(1, len(pt)))()
    tag = (C.c_uint8 * 16)()
    _load().or_aead_seal(_buf(key), _buf(nonce), _buf(aad), len(aad), _buf(pt), len(pt), ct, tag)
    return bytes(ct)[:len(pt)], bytes(tag)


def aead_open(key: bytes, nonce: bytes, aad: bytes, ct: bytes, tag: bytes):
    """The plain text, or None when the tag does not check."""
    pt = (C.c_uint8 * max(1, len(ct)))()
    rc = _load().or_aead_open(_buf(key), _buf(nonce), _buf(aad), len(aad), _buf(ct), len(ct), _buf(tag), pt)
    return None if rc else bytes(pt)[:len(ct)]


def cmd_seal(key: bytes, seq: int, ops, keys, vals, vs: int) -> np.ndarray:
    """q command records (q x (32 + vs) bytes) of request seq."""
    o = np.ascontiguousarray(ops, dtype=np.uint8)
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    v = np.ascontiguousarray(vals, dtype=np.uint8).reshape(-1)
    q = o.size
    out = np.zeros((max(1, q), 32 + vs), dtype=np.uint8)
    _load().or_cmd_seal(_buf(key), seq, q, vs, _ptr(o), _ptr(k), _ptr(v) if v.size else None, _ptr(out))
    return out[:q]


def cmd_open(key: bytes, seq: int, records, vs: int):
    """(failures, ops, keys, vals) of q command records."""
    r = np.ascontiguousarray(records, dtype=np.uint8).reshape(-1, 32 + vs)
    q = r.shape[0]
    o, k = np.zeros(max(1, q), np.uint8), np.zeros(max(1, q), np.uint64)
    v = np.zeros((max(1, q), vs), np.uint8)
    bad = _load().or_cmd_open(_buf(key), seq, q, vs, _ptr(r), _ptr(o), _ptr(k), _ptr(v))
    return int(bad), o[:q], k[:q], v[:q]


def resp_seal(key: bytes, seq: int, status, vals, vs: int) -> np.ndarray:
    """q response records (q x (24 + vs) bytes) of request seq."""
    st = np.ascontiguousarray(status, dtype=np.uint8)
    v = np.ascontiguousarray(vals, dtype=np.uint8).reshape(-1)
    q = st.size
    out = np.zeros((max(1, q), 24 + vs), dtype=np.uint8)
    _load().or_resp_seal(_buf(key), seq, q, vs, _ptr(st), _ptr(v) if v.size else None, _ptr(out))
    return out[:q]


def resp_open(key: bytes, seq: int, records, vs: int):
    """(failures, status, vals) of q response records."""
    r = np.ascontiguousarray(records, dtype=np.uint8).reshape(-1, 24 + vs)
    q = r.shape[0]
    st = np.zeros(max(1, q), np.uint8)
    v = np.zeros((max(1, q), vs), np.uint8)
    bad = _load().or_resp_open(_buf(key), seq, q, vs, _ptr(r), _ptr(st), _ptr(v))
    return int(bad), st[:q], v[:q]


def pair(w0: int, w1: int, B: int) -> tuple:
    lib = _load()
    a, b = C.c_uint32(), C.c_uint32()
    lib.or_pair(w0, w1, B, C.byref(a), C.byref(b))
    return a.value, b.value


def sizing(cap, vs, c=8, alpha_pm=200, bin_slots=0, d=4, kpr=16, W=32) -> dict:
    lib = _load()
    s = _Sizes()
    if lib.or_sizing(cap, vs, c, alpha_pm, bin_slots, d, kpr, W, C.byref(s)):
        raise ValueError("invalid parameters")
    return s.as_dict()


def stash_bound(M, alpha_pm, Z, cap) -> int:
    return int(_load().or_stash_bound(M, alpha_pm, Z, cap))


def claim43_bound(K, c, lmax, N) -> float:
    """Claim 4.3 bound on the summed HBM bin loads (O() constant 1)."""
    return float(_load().or_claim43_bound(K, c, lmax, N))


def claim44_bound(M, alpha, lmax, N) -> float:
    """Claim 4.4 bound on the stash size (O() constant 1)."""
    return float(_load().or_claim44_bound(M, alpha, lmax, N))


def claim52_bits(N, ks_bits, vs_bits, beta1, beta2, R, d) -> float:
    """Claim 5.2 bound on HBM usage, in bits."""
    return float(_load().or_claim52_bits(N, ks_bits, vs_bits, beta1, beta2, R, d))


def bitonic_sort(a) -> np.ndarray:
    """Scalar bitonic sorting network (ascending); len(a) a power of two."""
    x = np.ascontiguousarray(a, dtype=np.uint64).copy()
    if _load().or_bitonic_sort_u64(_ptr(x), x.size):
        raise ValueError("length must be a power of two")
    return x


def expand(target, payload, m: int):
    """Expansion (shift) network; returns (payload per position, collision flag)."""
    t = np.ascontiguousarray(target, dtype=np.uint32)
    p = np.ascontiguousarray(payload, dtype=np.uint32)
    out = np.empty(m, dtype=np.uint32)
    rc = _load().or_expand(_ptr(t), _ptr(p), t.size, m, _ptr(out))
    return out, rc


def compact(keep, payload):
    """Order-preserving compaction (shift) network; returns (out, collision flag)."""
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    p = np.ascontiguousarray(payload, dtype=np.uint32)
    out = np.empty(k.size, dtype=np.uint32)
    rc = _load().or_compact(_ptr(k), _ptr(p), k.size, _ptr(out))
    return out, rc


# --------------------------------------------------------------------------
# page format (shared reading of the paper's "flag bit, key, value" tuples)
# --------------------------------------------------------------------------

def decode_page(page: np.ndarray, Z: int, vs: int) -> list:
    """[(key, value bytes)] of the real slots of one page, in slot order."""
    page = np.asarray(page, dtype=np.uint8)
    mask = int(page[:8].view("<u8")[0])
    keys = page[8:8 + 8 * Z].view("<u8")
    out = []
    for j in range(Z):
        if (mask >> j) & 1:
            off = 8 + 8 * Z + j * vs
            out.append((int(keys[j]), bytes(page[off:off + vs])))
    return out


# --------------------------------------------------------------------------
# O1: the plain definition of the answers
# --------------------------------------------------------------------------

class PlainMap:
    """Dictionary semantics of Get / Put / Delete (Sec. 2.1)."""

    def __init__(self, vs: int):
        self.vs = vs
        self.d: dict = {}

    def build(self, keys, vals) -> None:
        vals = np.asarray(vals, dtype=np.uint8).reshape(len(keys), self.vs)
        for k, v in zip(np.asarray(keys, dtype=np.uint64).tolist(), vals):
            self.d[int(k)] = bytes(v)

    def access(self, ops, keys, vals_in):
        q = len(ops)
        vals_in = np.asarray(vals_in, dtype=np.uint8).reshape(q, self.vs)
        out = np.zeros((q, self.vs), dtype=np.uint8)
        st = np.zeros(q, dtype=np.uint8)
        zero = bytes(self.vs)
        for i, (op, k) in enumerate(zip(np.asarray(ops).tolist(), np.asarray(keys, dtype=np.uint64).tolist())):
            k = int(k)
            had = k in self.d
            if op == GET:
                st[i] = ST_FOUND if had else ST_ABSENT
                out[i] = np.frombuffer(self.d.get(k, zero), dtype=np.uint8)
            elif op == PUT:
                st[i] = ST_UPDATED if had else ST_INSERTED
                self.d[k] = bytes(vals_in[i])
            elif op == DEL:
                st[i] = ST_DELETED if had else ST_ABSENT
                self.d.pop(k, None)
            else:
                raise ValueError("bad op")
        return out, st


class PlainMapC:
    """The same definition as PlainMap, as a C hash table (the timed plain
    baseline)."""

    def __init__(self, cap: int, vs: int):
        self._lib = _load()
        self.vs = vs
        self._h = self._lib.or_plain_create(cap, vs)
        if not self._h:
            raise MemoryError("plain map")

    def close(self):
        if self._h:
            self._lib.or_plain_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, keys, vals) -> int:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        v = np.ascontiguousarray(vals, dtype=np.uint8).reshape(-1)
        return int(self._lib.or_plain_build(self._h, _ptr(k), _ptr(v), k.size))

    def access(self, ops, keys, vals_in):
        o = np.ascontiguousarray(ops, dtype=np.uint8)
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        q = o.size
        vi = np.ascontiguousarray(vals_in, dtype=np.uint8).reshape(-1)
        vo = np.zeros(max(1, q * self.vs), np.uint8)
        st = np.zeros(max(1, q), np.uint8)
        rc = int(self._lib.or_plain_access(self._h, _ptr(o), _ptr(k), _ptr(vi), _ptr(vo), _ptr(st), q))
        return rc, vo[:q * self.vs].reshape(q, self.vs), st[:q]

    def __len__(self):
        return int(self._lib.or_plain_size(self._h))


# --------------------------------------------------------------------------
# O2: the scalar procedure
# --------------------------------------------------------------------------

class OracleMap:
    def __init__(self, cap, vs, c=8, alpha_pm=200, bin_slots=0, d=4, kpr=16, W=32, key=bytes(32),
                 trace=False, seal=False, lib=None, decomposed=False):
        lib = lib if lib is not None else _load()
        kb = (C.c_uint8 * 32).from_buffer_copy(bytes(key))
        self._h = lib.or_create(cap, vs, c, alpha_pm, bin_slots, d, kpr, W, kb, 1 if trace else 0)
        if not self._h:
            raise ValueError("invalid parameters")
        self._lib = lib
        self.s = lib.or_get_sizes(self._h).contents.as_dict()
        self.sealed = bool(seal)
        if seal and lib.or_set_seal(self._h):
            raise ValueError("sealing")
        self.decomposed = bool(decomposed)
        if decomposed and lib.or_set_decomposed(self._h):
            raise ValueError("decomposed")

    def tags(self) -> np.ndarray:
        """(M, 16) Poly1305 tags of the sealed pages."""
        M = self.s["M"]
        p = self._lib.or_tags_ptr(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint8)), shape=(M * 16,)).reshape(M, 16).copy()

    def versions(self) -> np.ndarray:
        M = self.s["M"]
        p = self._lib.or_ver_ptr(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint64)), shape=(M,)).copy()

    def raw_page(self, page: int) -> bytes:
        """An adversary's read of a sealed page and its tag."""
        buf = (C.c_uint8 * (self.s["page_bytes"] + 16))()
        if self._lib.or_obs_raw(self._h, page, buf, 0):
            raise ValueError("raw page")
        return bytes(buf)

    def put_raw_page(self, page: int, data: bytes):
        """An adversary's write of a page and tag (for example an old copy)."""
        buf = (C.c_uint8 * len(data)).from_buffer_copy(data)
        if self._lib.or_obs_raw(self._h, page, buf, 1):
            raise ValueError("raw page")

    def close(self):
        if self._h:
            self._lib.or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, keys, vals, mode: int = 0) -> int:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        v = np.ascontiguousarray(vals, dtype=np.uint8).reshape(-1)
        assert v.size == k.size * self.s["vs"]
        return int(self._lib.or_build(self._h, _ptr(k), _ptr(v), k.size, mode))

    def access(self, ops, keys, vals_in):
        o = np.ascontiguousarray(ops, dtype=np.uint8)
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        q = o.size
        vs = self.s["vs"]
        vi = np.ascontiguousarray(vals_in, dtype=np.uint8).reshape(q * vs) if q else np.zeros(1, np.uint8)
        vo = np.zeros(max(1, q * vs), dtype=np.uint8)
        st = np.zeros(max(1, q), dtype=np.uint8)
        rc = int(self._lib.or_access(self._h, _ptr(o), _ptr(k), _ptr(vi), _ptr(vo), _ptr(st), q))
        return rc, vo[:q * vs].reshape(q, vs), st[:q]

    # --- state ----------------------------------------------------------
    def observable(self) -> np.ndarray:
        M, pb = self.s["M"], self.s["page_bytes"]
        p = self._lib.or_obs_ptr(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint8)), shape=(M * pb,)).reshape(M, pb).copy()

    def hbm_bins(self) -> np.ndarray:
        K, pb = self.s["K"], self.s["page_bytes"]
        if K == 0:
            return np.zeros((0, pb), dtype=np.uint8)
        p = self._lib.or_hbm_ptr(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint8)), shape=(K * pb,)).reshape(K, pb).copy()

    def loads(self) -> np.ndarray:
        p = self._lib.or_load_ptr(self._h)
        return np.ctypeslib.as_array(C.cast(p, C.POINTER(C.c_uint32)), shape=(self.s["B"],)).copy()

    def stash(self) -> list:
        """[(key, dest bin, value bytes)] sorted."""
        n = int(self._lib.or_stash_copy(self._h, None, None, None, 0))
        k = np.zeros(max(1, n), np.uint64)
        d = np.zeros(max(1, n), np.uint32)
        v = np.zeros(max(1, n) * self.s["vs"], np.uint8)
        self._lib.or_stash_copy(self._h, _ptr(k), _ptr(d), _ptr(v), n)
        vs = self.s["vs"]
        return sorted((int(k[i]), int(d[i]), bytes(v[i * vs:(i + 1) * vs])) for i in range(n))

    def pmap(self) -> list:
        """[(row, key, p1, p2)] sorted."""
        n = int(self._lib.or_pm_copy(self._h, None, None, None, None, 0))
        r = np.zeros(max(1, n), np.uint64)
        k = np.zeros(max(1, n), np.uint64)
        a = np.zeros(max(1, n), np.uint32)
        b = np.zeros(max(1, n), np.uint32)
        self._lib.or_pm_copy(self._h, _ptr(r), _ptr(k), _ptr(a), _ptr(b), n)
        return sorted((int(r[i]), int(k[i]), int(a[i]), int(b[i])) for i in range(n))

    def stash_arrays(self):
        """The stash as arrays (key u64[n], dest bin u32[n], values u8[n, vs]),
        unsorted: for comparisons at sizes where a list of tuples is slow."""
        n = int(self._lib.or_stash_copy(self._h, None, None, None, 0))
        vs = self.s["vs"]
        k, d = np.zeros(max(1, n), np.uint64), np.zeros(max(1, n), np.uint32)
        v = np.zeros(max(1, n) * vs, np.uint8)
        self._lib.or_stash_copy(self._h, _ptr(k), _ptr(d), _ptr(v), n)
        return k[:n], d[:n], v[:n * vs].reshape(n, vs)

    def pmap_arrays(self):
        """The position map as arrays (row u64[n], key u64[n], p1 u32[n],
        p2 u32[n]), unsorted."""
        n = int(self._lib.or_pm_copy(self._h, None, None, None, None, 0))
        m = max(1, n)
        r, k = np.zeros(m, np.uint64), np.zeros(m, np.uint64)
        a, b = np.zeros(m, np.uint32), np.zeros(m, np.uint32)
        self._lib.or_pm_copy(self._h, _ptr(r), _ptr(k), _ptr(a), _ptr(b), n)
        return r[:n], k[:n], a[:n], b[:n]

    def pm_max_row(self) -> int:
        return int(self._lib.or_pm_max_row(self._h))

    def trace(self) -> np.ndarray:
        n = int(self._lib.or_trace_len(self._h))
        out = np.zeros(n, dtype=TRACE_DTYPE)
        if n:
            self._lib.or_trace_copy(self._h, _ptr(out), n)
        return out

    def trace_clear(self):
        self._lib.or_trace_clear(self._h)

    @property
    def ctr(self):
        return int(self._lib.or_ctr(self._h))

    @property
    def live(self):
        return int(self._lib.or_live(self._h))

    @property
    def stash_live(self):
        return int(self._lib.or_stash_live(self._h))

    @property
    def hbm_live(self):
        """Items of the HBM bins held in the value pool (decomposed store)."""
        return int(self._lib.or_hbm_live(self._h))

    @property
    def stash_highwater(self):
        return int(self._lib.or_stash_highwater(self._h))

    def logical_contents(self) -> dict:
        """key -> value over HBM bins, observable pages and the stash."""
        Z, vs = self.s["Z"], self.s["vs"]
        out = {}
        for arr in (self.hbm_bins(), self.observable()):
            for page in arr:
                for k, v in decode_page(page, Z, vs):
                    assert k not in out, "key stored twice"
                    out[k] = v
        for k, _, v in self.stash():
            assert k not in out, "key stored twice"
            out[k] = v
        return out

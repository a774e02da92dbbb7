"""Python binding of the oblivious-map library ``libbolt.so`` (include/bolt.h).

The binding only marshals arguments: every step of the build and of the
batched get/put runs in the library's HIP kernels.  PyTorch supplies device
memory and streams.  If the library is not built this module raises at
import: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbolt.so")

BOLT_OK, BOLT_EINVAL, BOLT_ENOMEM, BOLT_EDUPKEY, BOLT_EOVERFLOW, BOLT_EFULL, BOLT_EHIP, BOLT_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
BOLT_OP_GET, BOLT_OP_PUT, BOLT_OP_DEL = 0, 1, 2
BOLT_ST_ABSENT, BOLT_ST_FOUND, BOLT_ST_UPDATED, BOLT_ST_INSERTED, BOLT_ST_DELETED = 0, 1, 1, 2, 3
BOLT_OBS_HOST_PINNED, BOLT_OBS_DEVICE = 0, 1
BOLT_F_TRACE, BOLT_F_FIXED_KEY, BOLT_F_TIMING, BOLT_F_GRAPHS, BOLT_F_WATCH, BOLT_F_SEAL = 1, 2, 4, 8, 16, 32
BOLT_F_SEAL_KEY_REUSE = 64
BOLT_F_SEAL_CMDS = 128
BOLT_F_DECOMPOSED = 256
BOLT_MAX_BATCH = 8192
BOLT_NOALLOC_EXPAND_MAX = 1 << 21
BOLT_ETIMEOUT = -8
BOLT_ETAMPER = -9
BOLT_SRV_WAITING, BOLT_SRV_BUILDING, BOLT_SRV_RESIDENT, BOLT_SRV_CLOSED, BOLT_SRV_FAILED = 0, 1, 2, 3, 4

_NAMES = {0: "BOLT_OK", -1: "BOLT_EINVAL", -2: "BOLT_ENOMEM", -3: "BOLT_EDUPKEY", -4: "BOLT_EOVERFLOW",
          -5: "BOLT_EFULL", -6: "BOLT_EHIP", -7: "BOLT_ESTATE", -8: "BOLT_ETIMEOUT",
          -9: "BOLT_ETAMPER"}


class BoltError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, _NAMES.get(rc, "?"), rc))
        self.rc = rc


class bolt_params(C.Structure):
    _fields_ = [
        ("capacity", C.c_uint64), ("value_bytes", C.c_uint32), ("c", C.c_uint32),
        ("alpha_permille", C.c_uint32), ("bin_slots", C.c_uint32), ("pm_choices", C.c_uint32),
        ("pm_keys_per_row", C.c_uint32), ("pm_row_slots", C.c_uint32), ("observable", C.c_uint32),
        ("flags", C.c_uint32), ("trace_words", C.c_uint64), ("key", C.c_uint8 * 32),
        ("session_key", C.c_uint8 * 32),
    ]


class bolt_sizes(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("B", "K", "M", "Z", "page_bytes", "pm_rows", "stash_bound", "stash_pool",
                                          "lmax", "hbm_bound")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class bolt_stats(C.Structure):
    _fields_ = [("live", C.c_uint64), ("steps", C.c_uint64), ("batches", C.c_uint64), ("stash_live", C.c_uint64),
                ("stash_highwater", C.c_uint64), ("max_load", C.c_uint32), ("max_row", C.c_uint32),
                ("load_highwater", C.c_uint32), ("hbm_load", C.c_uint64), ("hbm_load_highwater", C.c_uint64)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class bolt_trace_rec(C.Structure):
    _fields_ = [("batch", C.c_uint32), ("kind", C.c_uint32), ("page", C.c_uint64)]


class bolt_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint64), ("total_ms", C.c_double)]


class bolt_batch(C.Structure):
    _fields_ = [("d_ops", C.c_void_p), ("d_keys", C.c_void_p), ("d_vals_in", C.c_void_p),
                ("d_vals_out", C.c_void_p), ("d_status", C.c_void_p), ("q", C.c_uint32)]


class bolt_server_params(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("streams", C.c_uint32), ("max_batch", C.c_uint32),
                ("flags", C.c_uint32)]


class bolt_server_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "failed", "commands", "launches", "queued",
                                           "queue_peak", "maps_admitted", "maps_resident", "maps_waiting",
                                           "hbm_used", "hbm_peak")] + \
               [(n, C.c_double) for n in ("lat_p50_ms", "lat_p99_ms", "lat_max_ms", "lat_mean_ms", "span_s",
                                          "mean_group_maps", "mean_group_commands")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class bolt_tune_entry(C.Structure):
    _fields_ = [("log2_n", C.c_uint32), ("sort_tile_log", C.c_uint32), ("sort_pass_strides", C.c_uint32),
                ("expand_pass_stages", C.c_uint32), ("sort_ms", C.c_float), ("expand_ms", C.c_float)]


TRACE_DTYPE = np.dtype([("batch", "<u4"), ("kind", "<u4"), ("page", "<u8")])

# (name, restype, argtypes) of every entry point in include/bolt.h
_P, _U8, _U32, _U64, _I = C.c_void_p, C.c_uint8, C.c_uint32, C.c_uint64, C.c_int
_SIGS = [
    ("bolt_params_default", None, [C.POINTER(bolt_params), _U64, _U32]),
    ("bolt_sizes_of", _I, [C.POINTER(bolt_params), C.POINTER(bolt_sizes)]),
    ("bolt_footprint", _I, [C.POINTER(bolt_params), C.POINTER(_U64), C.POINTER(_U64)]),
    ("bolt_create", _I, [C.POINTER(bolt_params), _P, C.POINTER(_P)]),
    ("bolt_build", _I, [_P, _P, _P, _U64, _P]),
    ("bolt_access_batch", _I, [_P, _P, _P, _P, _P, _P, _U32, _P]),
    ("bolt_access_many", _I, [_P, _P, _U32, _P]),
    ("bolt_build_many", _I, [_P, _P, _P, _P, _U32, _P]),
    ("bolt_get_batch", _I, [_P, _P, _U32, _P, _P, _P]),
    ("bolt_access_sealed", _I, [_P, _P, _U32, _P, _P]),
    ("bolt_seal_requests", _I, [_P, _U64, _U32, _U32, _P, _P, _P, _P]),
    ("bolt_open_responses", _I, [_P, _U64, _U32, _U32, _P, _P, _P]),
    ("bolt_put_batch", _I, [_P, _P, _P, _U32, _P, _P]),
    ("bolt_destroy", _I, [_P]),
    ("bolt_status", _I, [_P]),
    ("bolt_flush", _I, [_P, _P]),
    ("bolt_map_sizes", _I, [_P, C.POINTER(bolt_sizes)]),
    ("bolt_get_stats", _I, [_P, C.POINTER(bolt_stats)]),
    ("bolt_trace_read", _I, [_P, _P, _U64, C.POINTER(_U64)]),
    ("bolt_trace_clear", _I, [_P]),
    ("bolt_observable_snapshot", _I, [_P, _P, _U64]),
    ("bolt_hbm_snapshot", _I, [_P, _P, _U64]),
    ("bolt_tags_snapshot", _I, [_P, _P, _U64]),
    ("bolt_versions_snapshot", _I, [_P, _P, _U64]),
    ("bolt_observable_raw", _I, [_P, _U64, _P, _I]),
    ("bolt_loads_snapshot", _I, [_P, _P, _U64]),
    ("bolt_stash_snapshot", _I, [_P, _P, _P, _P, _U64, C.POINTER(_U64)]),
    ("bolt_pm_snapshot", _I, [_P, _P, _P, _P, _P, _U64, C.POINTER(_U64)]),
    ("bolt_kernel_times", _I, [_P, _P, _U32, C.POINTER(_U32)]),
    ("bolt_kernel_times_reset", _I, [_P]),
    ("bolt_now_ns", _U64, []),
    ("bolt_server_footprint", _I, [C.POINTER(bolt_params), _U32, C.POINTER(_U64)]),
    ("bolt_server_create", _I, [C.POINTER(bolt_server_params), C.POINTER(_P)]),
    ("bolt_server_open_map", _I, [_P, C.POINTER(bolt_params), _P, _P, _U64, C.POINTER(_U32)]),
    ("bolt_server_close_map", _I, [_P, _U32]),
    ("bolt_server_map_state", _I, [_P, _U32, C.POINTER(_I), C.POINTER(_I)]),
    ("bolt_server_map", _P, [_P, _U32]),
    ("bolt_server_submit", _I, [_P, _U32, _P, _P, _P, _P, _P, _U32, _U64, C.POINTER(_U64)]),
    ("bolt_server_submit_sealed", _I, [_P, _U32, _P, _U32, _P, _U64, C.POINTER(_U64)]),
    ("bolt_server_poll", _I, [_P, _U64, C.POINTER(_I)]),
    ("bolt_server_wait", _I, [_P, _U64, _U32]),
    ("bolt_server_drain", _I, [_P, _U32]),
    ("bolt_server_get_stats", _I, [_P, C.POINTER(bolt_server_stats)]),
    ("bolt_server_reset_stats", _I, [_P]),
    ("bolt_server_destroy", _I, [_P]),
    ("bolt_autotune", _I, [_U64, C.c_char_p, _P]),
    ("bolt_tune_get", _I, [C.POINTER(bolt_tune_entry), _U32, C.POINTER(_U32)]),
    ("bolt_tune_set", _I, [C.POINTER(bolt_tune_entry), _U32]),
    ("bolt_tune_reset", _I, []),
    ("bolt_prf", _I, [_P, _U8, _P, _U64, _P, _P]),
    ("bolt_sort_u64", _I, [_P, _U64, _P]),
    ("bolt_expand_u64", _I, [_P, _P, _U64, _P]),
    ("bolt_expand_u64_noalloc", _I, [_P, _U64, _P]),
]
EXPORTED = [s[0] for s in _SIGS]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbolt.so is not built (run __graft_entry__.build() or paper_2509_01742_amd/build.py); "
                          "there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in _SIGS:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()

# Module-level names identical to the C ABI.
for _name, _, _ in _SIGS:
    globals()[_name] = getattr(lib, _name)


# --------------------------------------------------------------------------
# marshalling helpers (torch only for device memory and streams)
# --------------------------------------------------------------------------

_raw_stream = None


def _stream(stream=None):
    """The HIP stream handle of `stream`, else of torch's current stream on
    the current device (read without building a Stream object)."""
    global _raw_stream
    if stream is not None:
        return stream.cuda_stream
    if _raw_stream is None:
        import torch

        get, dev = torch._C._cuda_getCurrentRawStream, torch._C._cuda_getDevice
        _raw_stream = lambda: get(dev())  # noqa: E731
    return _raw_stream()


def _dptr(t):
    return None if t is None else t.data_ptr()


def check(rc: int, what: str) -> int:
    if rc != BOLT_OK:
        raise BoltError(rc, what)
    return rc


def params(capacity: int, value_bytes: int, **kw) -> bolt_params:
    p = bolt_params()
    bolt_params_default(C.byref(p), capacity, value_bytes)
    key = kw.pop("key", None)
    if key is not None:
        key = bytes(key)
        assert len(key) == 32
        C.memmove(p.key, key, 32)
        p.flags |= BOLT_F_FIXED_KEY
    skey = kw.pop("session_key", None)
    if skey is not None:
        skey = bytes(skey)
        assert len(skey) == 32
        C.memmove(p.session_key, skey, 32)
        p.flags |= BOLT_F_SEAL_CMDS
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown parameter %s" % k)
        setattr(p, k, v)
    return p


def seal_requests(session_key: bytes, seq: int, ops, keys, vals, vs: int) -> np.ndarray:
    """Client side: q command records (q x (32 + vs) bytes) of request seq."""
    o = np.ascontiguousarray(ops, dtype=np.uint8)
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    v = np.ascontiguousarray(vals, dtype=np.uint8)
    q = o.size
    out = np.zeros((q, 32 + vs), dtype=np.uint8)
    kb = (C.c_uint8 * 32).from_buffer_copy(bytes(session_key))
    check(bolt_seal_requests(kb, seq, q, vs, o.ctypes.data_as(C.c_void_p), k.ctypes.data_as(C.c_void_p),
                             v.ctypes.data_as(C.c_void_p), out.ctypes.data_as(C.c_void_p)), "bolt_seal_requests")
    return out


def open_responses(session_key: bytes, seq: int, records, vs: int):
    """Client side: (rc, status u8[q], values u8[q, vs]) of q response records."""
    r = np.ascontiguousarray(records, dtype=np.uint8).reshape(-1, 24 + vs)
    q = r.shape[0]
    st = np.zeros(max(1, q), dtype=np.uint8)
    vo = np.zeros((max(1, q), vs), dtype=np.uint8)
    kb = (C.c_uint8 * 32).from_buffer_copy(bytes(session_key))
    rc = bolt_open_responses(kb, seq, q, vs, r.ctypes.data_as(C.c_void_p), st.ctypes.data_as(C.c_void_p),
                             vo.ctypes.data_as(C.c_void_p))
    return rc, st[:q], vo[:q]


def sizes_of(p: bolt_params) -> dict:
    s = bolt_sizes()
    check(bolt_sizes_of(C.byref(p), C.byref(s)), "bolt_sizes_of")
    return s.as_dict()


def footprint(p: bolt_params) -> tuple:
    h, o = C.c_uint64(), C.c_uint64()
    check(bolt_footprint(C.byref(p), C.byref(h), C.byref(o)), "bolt_footprint")
    return int(h.value), int(o.value)


class Map:
    """One oblivious map on the current device (owns a bolt_map*)."""

    def __init__(self, p: bolt_params, stream=None):
        h = C.c_void_p()
        check(bolt_create(C.byref(p), _stream(stream), C.byref(h)), "bolt_create")
        self.h = h
        self.p = p
        self.sizes = sizes_of(p)
        self.vs = int(p.value_bytes)

    def close(self):
        if self.h is not None and self.h.value:
            bolt_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- the path -------------------------------------------------------
    def build(self, keys, vals, stream=None) -> int:
        """keys: int64/uint64 cuda tensor [n]; vals: uint8 cuda tensor [n, vs]."""
        n = 0 if keys is None else keys.numel()
        return bolt_build(self.h, _dptr(keys), _dptr(vals), n, _stream(stream))

    def access(self, ops, keys, vals_in, vals_out, status, stream=None) -> int:
        q = ops.numel()
        return bolt_access_batch(self.h, _dptr(ops), _dptr(keys), _dptr(vals_in), _dptr(vals_out), _dptr(status),
                                 q, _stream(stream))

    def access_sealed(self, req, resp, stream=None) -> int:
        """One sealed request: req / resp device tensors of q command and q
        response records."""
        q = req.numel() // (32 + self.vs)
        return bolt_access_sealed(self.h, _dptr(req), q, _dptr(resp), _stream(stream))

    def get(self, keys, vals_out, found, stream=None) -> int:
        return bolt_get_batch(self.h, _dptr(keys), keys.numel(), _dptr(vals_out), _dptr(found), _stream(stream))

    def put(self, keys, vals, status, stream=None) -> int:
        return bolt_put_batch(self.h, _dptr(keys), _dptr(vals), keys.numel(), _dptr(status), _stream(stream))

    def flush(self, stream=None) -> int:
        return bolt_flush(self.h, _stream(stream))

    # --- state ----------------------------------------------------------
    def status(self) -> int:
        return bolt_status(self.h)

    def stats(self) -> dict:
        s = bolt_stats()
        check(bolt_get_stats(self.h, C.byref(s)), "bolt_get_stats")
        return s.as_dict()

    def trace(self) -> np.ndarray:
        n = C.c_uint64()
        rc = bolt_trace_read(self.h, None, 0, C.byref(n))
        if rc not in (BOLT_OK,):
            raise BoltError(rc, "bolt_trace_read")
        out = np.zeros(int(n.value), dtype=TRACE_DTYPE)
        if n.value:
            check(bolt_trace_read(self.h, out.ctypes.data_as(C.c_void_p), n.value, C.byref(n)), "bolt_trace_read")
        return out

    def kernel_times(self) -> dict:
        """{class: (launches, total_ms)} since create or the last reset (BOLT_F_TIMING)."""
        arr = (bolt_kernel_time * 32)()
        n = C.c_uint32()
        check(bolt_kernel_times(self.h, arr, 32, C.byref(n)), "bolt_kernel_times")
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}

    def kernel_times_reset(self):
        check(bolt_kernel_times_reset(self.h), "bolt_kernel_times_reset")

    def trace_clear(self):
        check(bolt_trace_clear(self.h), "bolt_trace_clear")

    def observable(self) -> np.ndarray:
        M, pb = self.sizes["M"], self.sizes["page_bytes"]
        out = np.zeros((M, pb), dtype=np.uint8)
        check(bolt_observable_snapshot(self.h, out.ctypes.data_as(C.c_void_p), out.nbytes), "observable_snapshot")
        return out

    def tags(self) -> np.ndarray:
        """BOLT_F_SEAL: (M, 16) tags of the sealed observable pages."""
        M = self.sizes["M"]
        out = np.zeros((M, 16), dtype=np.uint8)
        check(bolt_tags_snapshot(self.h, out.ctypes.data_as(C.c_void_p), out.size), "tags_snapshot")
        return out

    def versions(self) -> np.ndarray:
        """BOLT_F_SEAL: each observable page's write count."""
        M = self.sizes["M"]
        out = np.zeros(M, dtype=np.uint64)
        check(bolt_versions_snapshot(self.h, out.ctypes.data_as(C.c_void_p), M), "versions_snapshot")
        return out

    def raw_page(self, page: int) -> bytes:
        """BOLT_F_SEAL: an adversary's read of a sealed page and its tag."""
        buf = (C.c_uint8 * (self.sizes["page_bytes"] + 16))()
        check(bolt_observable_raw(self.h, page, buf, 0), "observable_raw")
        return bytes(buf)

    def put_raw_page(self, page: int, data: bytes):
        """BOLT_F_SEAL: an adversary's write of a page and its tag."""
        buf = (C.c_uint8 * len(data)).from_buffer_copy(data)
        check(bolt_observable_raw(self.h, page, buf, 1), "observable_raw")

    def hbm_bins(self) -> np.ndarray:
        K, pb = self.sizes["K"], self.sizes["page_bytes"]
        out = np.zeros((K, pb), dtype=np.uint8)
        check(bolt_hbm_snapshot(self.h, out.ctypes.data_as(C.c_void_p), out.nbytes), "hbm_snapshot")
        return out

    def loads(self) -> np.ndarray:
        out = np.zeros(self.sizes["B"], dtype=np.uint32)
        check(bolt_loads_snapshot(self.h, out.ctypes.data_as(C.c_void_p), out.nbytes), "loads_snapshot")
        return out

    def stash(self) -> list:
        n = C.c_uint64()
        check(bolt_stash_snapshot(self.h, None, None, None, 0, C.byref(n)), "stash_snapshot")
        k = np.zeros(max(1, n.value), np.uint64)
        b = np.zeros(max(1, n.value), np.uint32)
        v = np.zeros(max(1, n.value) * self.vs, np.uint8)
        check(bolt_stash_snapshot(self.h, k.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                                  v.ctypes.data_as(C.c_void_p), n.value, C.byref(n)), "stash_snapshot")
        vs = self.vs
        return sorted((int(k[i]), int(b[i]), bytes(v[i * vs:(i + 1) * vs])) for i in range(int(n.value)))

    def pmap(self) -> list:
        n = C.c_uint64()
        check(bolt_pm_snapshot(self.h, None, None, None, None, 0, C.byref(n)), "pm_snapshot")
        m = max(1, n.value)
        r, k = np.zeros(m, np.uint64), np.zeros(m, np.uint64)
        a, b = np.zeros(m, np.uint32), np.zeros(m, np.uint32)
        check(bolt_pm_snapshot(self.h, r.ctypes.data_as(C.c_void_p), k.ctypes.data_as(C.c_void_p),
                               a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), n.value, C.byref(n)),
              "pm_snapshot")
        return sorted((int(r[i]), int(k[i]), int(a[i]), int(b[i])) for i in range(int(n.value)))

    def stash_arrays(self):
        """The stash as arrays (key u64[n], dest bin u32[n], values u8[n, vs]),
        in the library's pool order."""
        n = C.c_uint64()
        check(bolt_stash_snapshot(self.h, None, None, None, 0, C.byref(n)), "stash_snapshot")
        k = np.zeros(max(1, n.value), np.uint64)
        b = np.zeros(max(1, n.value), np.uint32)
        v = np.zeros(max(1, n.value) * self.vs, np.uint8)
        check(bolt_stash_snapshot(self.h, k.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                                  v.ctypes.data_as(C.c_void_p), n.value, C.byref(n)), "stash_snapshot")
        c = int(n.value)
        return k[:c], b[:c], v[:c * self.vs].reshape(c, self.vs)

    def pmap_arrays(self):
        """The position map as arrays (row u64[n], key u64[n], p1 u32[n],
        p2 u32[n]), in the library's slot order."""
        n = C.c_uint64()
        check(bolt_pm_snapshot(self.h, None, None, None, None, 0, C.byref(n)), "pm_snapshot")
        m = max(1, n.value)
        r, k = np.zeros(m, np.uint64), np.zeros(m, np.uint64)
        a, b = np.zeros(m, np.uint32), np.zeros(m, np.uint32)
        check(bolt_pm_snapshot(self.h, r.ctypes.data_as(C.c_void_p), k.ctypes.data_as(C.c_void_p),
                               a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), n.value, C.byref(n)),
              "pm_snapshot")
        c = int(n.value)
        return r[:c], k[:c], a[:c], b[:c]


def build_many(maps, inputs, stream=None) -> int:
    """Builds every map of `maps` from its (keys, vals) device tensors, one launch per phase for all."""
    n = len(maps)
    if n != len(inputs):
        raise ValueError("one input per map")
    k = max(n, 1)
    hs = (C.c_void_p * k)(*[m.h for m in maps])
    ks = (C.c_void_p * k)(*[_dptr(a) for a, _ in inputs])
    vs = (C.c_void_p * k)(*[_dptr(b) for _, b in inputs])
    ns = (C.c_uint64 * k)(*[0 if a is None else a.numel() for a, _ in inputs])
    return bolt_build_many(hs, ks, vs, ns, n, _stream(stream))


def access_many(maps, batches, stream=None) -> int:
    """One batch per map, every phase launched once for all maps.

    maps: sequence of Map; batches: sequence of (ops, keys, vals_in, vals_out, status) device tensors."""
    n = len(maps)
    if n != len(batches):
        raise ValueError("one batch per map")
    hs = (C.c_void_p * max(n, 1))(*[m.h for m in maps])
    bs = (bolt_batch * max(n, 1))()
    for i, (ops, keys, vin, vout, status) in enumerate(batches):
        bs[i] = bolt_batch(_dptr(ops), _dptr(keys), _dptr(vin), _dptr(vout),
                           _dptr(status), 0 if ops is None else ops.numel())
    return bolt_access_many(hs, bs, n, _stream(stream))


def server_footprint(p: bolt_params, max_batch: int = 0) -> int:
    b = C.c_uint64()
    check(bolt_server_footprint(C.byref(p), max_batch, C.byref(b)), "bolt_server_footprint")
    return int(b.value)


class Server:
    """A serving loop over many resident maps (requests are host numpy arrays)."""

    def __init__(self, hbm_budget: int = 0, streams: int = 0, max_batch: int = 0):
        sp = bolt_server_params(hbm_budget, streams, max_batch, 0)
        h = C.c_void_p()
        check(bolt_server_create(C.byref(sp), C.byref(h)), "bolt_server_create")
        self.h = h
        self._live = {}  # ticket -> the request's buffers (kept alive until done)

    def close(self):
        if self.h is not None and self.h.value:
            bolt_server_destroy(self.h)
        self.h = None
        self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open_map(self, p: bolt_params, keys, vals) -> int:
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        v = np.ascontiguousarray(vals, dtype=np.uint8)
        mid = C.c_uint32()
        check(bolt_server_open_map(self.h, C.byref(p), k.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                   k.size, C.byref(mid)), "bolt_server_open_map")
        return mid.value

    def close_map(self, mid: int) -> int:
        return bolt_server_close_map(self.h, mid)

    def map_state(self, mid: int):
        st, err = C.c_int(), C.c_int()
        check(bolt_server_map_state(self.h, mid, C.byref(st), C.byref(err)), "bolt_server_map_state")
        return st.value, err.value

    def submit(self, mid: int, ops, keys, vals_in, arrival_ns: int = 0):
        """Queues one request; returns (ticket, vals_out, status), the last two
        filled when the request completes."""
        ops = np.ascontiguousarray(ops, dtype=np.uint8)
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        vals_in = np.ascontiguousarray(vals_in, dtype=np.uint8)
        q = ops.size
        vs = vals_in.size // max(q, 1)
        vout = np.zeros((q, vs), np.uint8)
        st = np.zeros(q, np.uint8)
        t = C.c_uint64()
        rc = bolt_server_submit(self.h, mid, ops.ctypes.data_as(C.c_void_p), keys.ctypes.data_as(C.c_void_p),
                                vals_in.ctypes.data_as(C.c_void_p), vout.ctypes.data_as(C.c_void_p),
                                st.ctypes.data_as(C.c_void_p), q, arrival_ns, C.byref(t))
        if rc != BOLT_OK:
            return rc, None, None
        self._live[t.value] = (ops, keys, vals_in, vout, st)
        return t.value, vout, st

    def submit_sealed(self, mid: int, records, vs: int, arrival_ns: int = 0):
        """Queues one sealed request (q command records); returns (ticket,
        response records), the latter filled when the request completes."""
        rec = np.ascontiguousarray(records, dtype=np.uint8).reshape(-1, 32 + vs)
        q = rec.shape[0]
        resp = np.zeros((q, 24 + vs), np.uint8)
        t = C.c_uint64()
        rc = bolt_server_submit_sealed(self.h, mid, rec.ctypes.data_as(C.c_void_p), q,
                                       resp.ctypes.data_as(C.c_void_p), arrival_ns, C.byref(t))
        if rc != BOLT_OK:
            return rc, None
        self._live[t.value] = (rec, resp)
        return t.value, resp

    def poll(self, ticket: int) -> int:
        r = C.c_int()
        check(bolt_server_poll(self.h, ticket, C.byref(r)), "bolt_server_poll")
        if r.value != 1:
            self._live.pop(ticket, None)
        return r.value

    def wait(self, ticket: int, timeout_ms: int = 60000) -> int:
        rc = bolt_server_wait(self.h, ticket, timeout_ms)
        if rc != BOLT_ETIMEOUT:
            self._live.pop(ticket, None)
        return rc

    def drain(self, timeout_ms: int = 120000) -> int:
        rc = bolt_server_drain(self.h, timeout_ms)
        if rc == BOLT_OK:
            self._live.clear()
        return rc

    def stats(self) -> dict:
        s = bolt_server_stats()
        check(bolt_server_get_stats(self.h, C.byref(s)), "bolt_server_get_stats")
        return s.as_dict()

    def reset_stats(self):
        check(bolt_server_reset_stats(self.h), "bolt_server_reset_stats")


def autotune(n_max: int, cache_path=None, stream=None) -> int:
    """Tunes (or loads from cache_path) the network schedules up to arrays of n_max."""
    path = None if cache_path is None else os.fsencode(cache_path)
    return bolt_autotune(n_max, path, _stream(stream))


def tune_table() -> list:
    arr = (bolt_tune_entry * 64)()
    n = C.c_uint32()
    check(bolt_tune_get(arr, 64, C.byref(n)), "bolt_tune_get")
    return [{f: getattr(arr[i], f) for f, _ in bolt_tune_entry._fields_} for i in range(min(n.value, 64))]


def tune_set(entries) -> int:
    arr = (bolt_tune_entry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = bolt_tune_entry(e["log2_n"], e["sort_tile_log"], e["sort_pass_strides"], e["expand_pass_stages"],
                                 e.get("sort_ms", 0.0), e.get("expand_ms", 0.0))
    return bolt_tune_set(arr, len(entries))


def prf(key: bytes, domain: int, x, out, stream=None) -> int:
    """out[4 * i:4 * i + 4] = PRF_key(domain, x[i]) (device tensors)."""
    kb = (C.c_uint8 * 32).from_buffer_copy(bytes(key))
    return bolt_prf(kb, domain, _dptr(x), x.numel(), _dptr(out), _stream(stream))


def sort_u64(data, stream=None) -> int:
    return bolt_sort_u64(_dptr(data), data.numel(), _stream(stream))


def expand_u64(elems, tmp, stream=None) -> int:
    return bolt_expand_u64(_dptr(elems), _dptr(tmp), elems.numel(), _stream(stream))


def expand_u64_noalloc(elems, stream=None) -> int:
    return bolt_expand_u64_noalloc(_dptr(elems), elems.numel(), _stream(stream))

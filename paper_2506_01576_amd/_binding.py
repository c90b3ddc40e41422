"""ctypes binding of libidx.so -- argument marshalling only.

Tensors are device buffers; their ``data_ptr()`` values and the current HIP
stream handle are passed straight through the C ABI of ``include/idx.h``.
Every computation happens inside the library's HIP kernels.  If the library
has not been built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libidx.so")

IDX_BS, IDX_EBS, IDX_EKS = 0, 1, 2
IDX_KEY_U32, IDX_KEY_U64, IDX_SOA, IDX_AOS, IDX_AOS_PADDED = 0, 1, 0, 2, 4
IDX_MISS = 0xFFFFFFFF
IDX_OK = 0
IDX_ERR_ARG = -1
IDX_ERR_RESERVED_ROWID = -2
IDX_ERR_NOMEM = -3
IDX_ERR_HIP = -4
IDX_ERR_CAPACITY = -5
IDX_ERR_SCRATCH = -6
IDX_NOALLOC_MAX_RANGES = 1 << 23

LAYOUTS = {"bs": IDX_BS, "ebs": IDX_EBS, "eks": IDX_EKS}


class IdxError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = lib().idx_strerror(status).decode()
        if status == IDX_ERR_HIP:
            msg += f" (hip error {lib().idx_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{status}]")


class idx_allocator(ctypes.Structure):
    _fields_ = [
        ("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
        ("release", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)),
        ("ctx", ctypes.c_void_p),
    ]


class idx_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("slots", ctypes.c_uint64),
        ("footprint_bytes", ctypes.c_uint64),
        ("layout", ctypes.c_int32),
        ("k", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("unique", ctypes.c_uint32),
        ("levels", ctypes.c_uint32),
        ("full_levels", ctypes.c_uint32),
        ("bottom_keys", ctypes.c_uint64),
        ("build_ms_sort", ctypes.c_float),
        ("build_ms_permute", ctypes.c_float),
    ]


class idx_lookup_params(ctypes.Structure):
    _fields_ = [
        ("group", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("per_lane", ctypes.c_uint32),
        ("lds_levels", ctypes.c_uint32),
        ("persistent", ctypes.c_uint32),
        ("reorder", ctypes.c_uint32),
        ("early_exit", ctypes.c_uint32),
        ("model", ctypes.c_uint32),
        ("window_rounds", ctypes.c_uint32),
        ("range_scan", ctypes.c_uint32),
        ("leaf_lines", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


IDX_FEATURE_AUTO, IDX_FEATURE_LINEAR, IDX_FEATURE_LOG, IDX_FEATURE_SPLINE = 0, 1, 2, 3


class idx_learn_stats(ctypes.Structure):
    _fields_ = [
        ("leaves", ctypes.c_uint32),
        ("epochs", ctypes.c_uint32),
        ("feature", ctypes.c_uint32),
        ("root_a0", ctypes.c_float),
        ("root_a1", ctypes.c_float),
        ("root_loss", ctypes.c_double),
        ("leaf_loss", ctypes.c_double),
        ("mean_window", ctypes.c_double),
        ("max_window", ctypes.c_double),
        ("segments", ctypes.c_uint32),
        ("bin_feature", ctypes.c_uint32),
    ]


_lib = None

# Every symbol include/idx.h declares, with its ctypes signature.
_P = ctypes.c_void_p
_U64 = ctypes.c_uint64
_U32 = ctypes.c_uint32
_I = ctypes.c_int
SIGNATURES = {
    "idx_build": (_I, [_P, _P, _U64, _I, _U32, _U32, ctypes.POINTER(idx_allocator), _P, ctypes.POINTER(_P)]),
    "idx_relayout": (_I, [_P, _I, _U32, _U32, ctypes.POINTER(idx_allocator), _P, ctypes.POINTER(_P)]),
    "idx_point": (_I, [_P, _P, _U64, _P, _P]),
    "idx_range": (_I, [_P, _P, _P, _U64, _P, _P, _U64, ctypes.POINTER(_U64), _P]),
    "idx_range_noalloc": (_I, [_P, _P, _P, _U64, _P, _P, _U64, ctypes.POINTER(_U64), _P]),
    "idx_destroy": (_I, [_P]),
    "idx_strerror": (ctypes.c_char_p, [_I]),
    "idx_last_hip_error": (_I, []),
    "idx_get_info": (_I, [_P, ctypes.POINTER(idx_info)]),
    "idx_export": (_I, [_P, _P, _P, _P]),
    "idx_slot_rank": (_U64, [_U64, _U32, _U64]),
    "idx_rank_slot": (_U64, [_U64, _U32, _U64]),
    "idx_set_params": (_I, [_P, ctypes.POINTER(idx_lookup_params)]),
    "idx_get_params": (_I, [_P, ctypes.POINTER(idx_lookup_params)]),
    "idx_probe_random": (_I, [_P, _U64, _U32, _U64, _U32, _U64, _P, _P]),
    "idx_batch_create": (_I, [ctypes.POINTER(_P), _U32, _P, ctypes.POINTER(_P)]),
    "idx_batch_point": (_I, [_P, _P, _P, _P, _U32, _P]),
    "idx_batch_destroy": (_I, [_P]),
    "idx_merge": (_I, [_P, _P, _P, _U64, _I, _U32, _U32, ctypes.POINTER(idx_allocator), _P, ctypes.POINTER(_P)]),
    "idx_save": (_I, [_P, _P, _U64, ctypes.POINTER(_U64), _P]),
    "idx_load": (_I, [_P, _U64, ctypes.POINTER(idx_allocator), _P, ctypes.POINTER(_P)]),
    "idx_batch_mixed": (_I, [_P, _U64, _P, _P, _P, _P, _P, _P, _P, _U64, ctypes.POINTER(_U64), _P]),
    "idx_learn_batch": (_I, [ctypes.POINTER(_P), _U32, ctypes.POINTER(_U32), _U32, _U32, _P]),
    "idx_learn": (_I, [_P, _U32, _U32, _U32, _P]),
    "idx_learn_stats_get": (_I, [_P, ctypes.POINTER(idx_learn_stats)]),
    "idx_learn_export": (_I, [_P, _P, _P]),
    "idx_unlearn": (_I, [_P]),
    "idx_learn_eval": (_I, [_P, _U32, ctypes.POINTER(ctypes.c_float), _U32, _P, ctypes.POINTER(ctypes.c_double), _P,
                            _P]),
}


def probe_random(buf: torch.Tensor, group: int, lanes: int, steps: int, seed: int = 1, stream=None):
    """Launch the random-access probe over `buf` (a device tensor of 8-byte
    words); returns the number of word loads it issues."""
    _dev(buf, "buf")
    sink = torch.zeros(1, dtype=torch.int64, device=buf.device)
    words = buf.numel() * buf.element_size() // 8
    _check(lib().idx_probe_random(buf.data_ptr(), words, group, lanes, steps, seed, sink.data_ptr(),
                                  _stream(stream)), "idx_probe_random")
    return lanes * steps * 8


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check(status: int, what: str):
    if status != IDX_OK:
        raise IdxError(status, what)


def _key_flag(t: torch.Tensor) -> int:
    if t.element_size() == 8:
        return IDX_KEY_U64
    if t.element_size() == 4:
        return IDX_KEY_U32
    raise TypeError("keys must be 32- or 64-bit integers (their bits are read as unsigned)")


def _aos_flags(aos) -> int:
    if aos == "padded":
        return IDX_AOS | IDX_AOS_PADDED
    return IDX_AOS if aos else IDX_SOA


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")


def _keys_of(t: torch.Tensor, name: str, key_bits: int):
    """A device tensor of keys of the index's width (bit patterns are read as
    unsigned, so signed and unsigned integer dtypes of that width both work)."""
    _dev(t, name)
    if t.dtype.is_floating_point or t.dtype.is_complex or t.element_size() * 8 != key_bits:
        raise ValueError(f"{name}: {key_bits}-bit integer keys expected, got {t.dtype}")
    if t.dim() != 1:
        raise ValueError(f"{name} must be one-dimensional")


def _out_u32(t: torch.Tensor, name: str, length: int):
    _dev(t, name)
    if t.dtype not in (torch.int32, torch.uint32) or t.dim() != 1 or len(t) < length:
        raise ValueError(f"{name} must be a 32-bit integer device tensor of at least {length} entries")


def _offsets_of(t: torch.Tensor, name: str, count: int):
    """Per-index query offsets: int64 (or uint64), count + 1 entries."""
    _dev(t, name)
    if t.dtype not in (torch.int64, torch.uint64) or t.dim() != 1 or len(t) != count + 1:
        raise ValueError(f"{name} must be a 64-bit integer device tensor of {count + 1} entries")


class Index:
    """A static index over (keys, rowids) device tensors.

    keys: 32- or 64-bit integer tensor (bit pattern read as unsigned);
    rowids: int32/uint32 tensor of row IDs (0xFFFFFFFF is reserved).
    layout: "bs", "ebs" or "eks"; k: fan-out for "eks"; aos: interleave rowids.
    """

    def __init__(self, keys: torch.Tensor, rowids: torch.Tensor, layout: str = "eks", k: int = 9,
                 aos: bool = False, stream=None):
        _dev(keys, "keys")
        _dev(rowids, "rowids")
        if rowids.element_size() != 4 or len(rowids) != len(keys):
            raise ValueError("rowids must be 32-bit and as long as keys")
        self.layout = layout
        self.key_bits = keys.element_size() * 8
        self.key_dtype = keys.dtype
        lay = LAYOUTS[layout]
        kk = {IDX_BS: 1, IDX_EBS: 2, IDX_EKS: k}[lay]
        flags = _key_flag(keys) | _aos_flags(aos)
        h = ctypes.c_void_p()
        st = lib().idx_build(keys.data_ptr(), rowids.data_ptr(), len(keys), lay, kk, flags, None, _stream(stream),
                             ctypes.byref(h))
        _check(st, "idx_build")
        self._h = h
        self.n = len(keys)
        self.k = kk

    @classmethod
    def _wrap(cls, h, n, k, layout, key_bits, key_dtype):
        self = cls.__new__(cls)
        self._h = h
        self.n, self.k, self.layout = n, k, layout
        self.key_bits, self.key_dtype = key_bits, key_dtype
        return self

    def relayout(self, layout: str, k: int = 9, aos: bool | str = False, stream=None) -> "Index":
        """Another layout of this (BS, SoA) index's key set, built by the
        permutation alone (no second sort).  aos: False, True or "padded"."""
        lay = LAYOUTS[layout]
        kk = {IDX_BS: 1, IDX_EBS: 2, IDX_EKS: k}[lay]
        flags = (IDX_KEY_U64 if self.key_bits == 64 else IDX_KEY_U32) | _aos_flags(aos)
        h = ctypes.c_void_p()
        _check(lib().idx_relayout(self._h, lay, kk, flags, None, _stream(stream), ctypes.byref(h)), "idx_relayout")
        return Index._wrap(h, self.n, kk, layout, self.key_bits, self.key_dtype)

    def merge(self, keys: torch.Tensor, rowids: torch.Tensor, layout: str = "bs", k: int = 9,
              aos: bool | str = False, stream=None) -> "Index":
        """A new index over this (BS, SoA) index's pairs plus (keys, rowids),
        laid out as asked (idx_merge); this index is unchanged."""
        _dev(keys, "keys")
        _dev(rowids, "rowids")
        if len(keys) != len(rowids):
            raise ValueError("keys and rowids differ in length")
        lay = LAYOUTS[layout]
        kk = {IDX_BS: 1, IDX_EBS: 2, IDX_EKS: k}[lay]
        flags = (IDX_KEY_U64 if self.key_bits == 64 else IDX_KEY_U32) | _aos_flags(aos)
        h = ctypes.c_void_p()
        _check(lib().idx_merge(self._h, keys.data_ptr() if len(keys) else None,
                               rowids.data_ptr() if len(keys) else None, len(keys), lay, kk, flags, None,
                               _stream(stream), ctypes.byref(h)), "idx_merge")
        return Index._wrap(h, self.n + len(keys), kk, layout, self.key_bits, self.key_dtype)

    def save(self, stream=None) -> bytes:
        """The handle as a host byte blob (idx_save)."""
        size = ctypes.c_uint64(0)
        _check(lib().idx_save(self._h, None, 0, ctypes.byref(size), _stream(stream)), "idx_save(size)")
        buf = ctypes.create_string_buffer(size.value)
        _check(lib().idx_save(self._h, buf, size.value, ctypes.byref(size), _stream(stream)), "idx_save")
        return buf.raw

    @classmethod
    def load(cls, blob: bytes, stream=None) -> "Index":
        """A handle from a blob written by save() (idx_load)."""
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().idx_load(buf, len(blob), None, _stream(stream), ctypes.byref(h)), "idx_load")
        ix = cls._wrap(h, 0, 1, "bs", 32, torch.int32)
        info = ix.info()
        ix.n, ix.k = info["n"], info["k"]
        ix.layout = {v: name for name, v in LAYOUTS.items()}[info["layout"]]
        ix.key_bits = 64 if info["flags"] & IDX_KEY_U64 else 32
        ix.key_dtype = torch.int64 if ix.key_bits == 64 else torch.int32
        return ix

    # -- lifecycle
    def close(self):
        """Free the index.  Raises IdxError (and keeps the index) while a
        Batch holds it: close the batch first."""
        if getattr(self, "_h", None):
            _check(lib().idx_destroy(self._h), "idx_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- lookups
    def point(self, queries: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _keys_of(queries, "queries", self.key_bits)
        if out is None:
            out = torch.empty(len(queries), dtype=torch.int32, device=queries.device)
        _out_u32(out, "out", len(queries))
        _check(lib().idx_point(self._h, queries.data_ptr(), len(queries), out.data_ptr(), _stream(stream)),
               "idx_point")
        return out

    def range(self, lo: torch.Tensor, hi: torch.Tensor, capacity: int | None = None, count_only: bool = False,
              stream=None):
        """Returns (offsets[m+1] int64, rowids[total] int32)."""
        _keys_of(lo, "lo", self.key_bits)
        _keys_of(hi, "hi", self.key_bits)
        m = len(lo)
        if len(hi) != m:
            raise ValueError("lo and hi differ in length")
        offsets = torch.empty(m + 1, dtype=torch.int64, device=lo.device)
        total = ctypes.c_uint64(0)
        s = _stream(stream)
        if count_only or capacity is None:
            _check(lib().idx_range(self._h, lo.data_ptr(), hi.data_ptr(), m, offsets.data_ptr(), None, 0,
                                   ctypes.byref(total), s), "idx_range(count)")
            if count_only:
                return offsets, None
            capacity = total.value
        out = torch.empty(max(1, capacity), dtype=torch.int32, device=lo.device)
        _check(lib().idx_range(self._h, lo.data_ptr(), hi.data_ptr(), m, offsets.data_ptr(), out.data_ptr(),
                               capacity, ctypes.byref(total), s), "idx_range")
        return offsets, out[: total.value]

    def range_noalloc(self, lo: torch.Tensor, hi: torch.Tensor, offsets: torch.Tensor,
                      rowids: torch.Tensor | None = None, stream=None) -> int:
        """Range lookups into caller-given outputs with no device allocation
        (idx_range_noalloc): offsets int64[m + 1]; rowids a 32-bit tensor
        whose length is the capacity, or None to count only.  At most
        IDX_NOALLOC_MAX_RANGES ranges.  Returns the total number of matches."""
        _keys_of(lo, "lo", self.key_bits)
        _keys_of(hi, "hi", self.key_bits)
        m = len(lo)
        if len(hi) != m:
            raise ValueError("lo and hi differ in length")
        _offsets_of(offsets, "offsets", m)
        cap = 0
        if rowids is not None:
            _out_u32(rowids, "rowids", 0)
            cap = len(rowids)
        total = ctypes.c_uint64(0)
        _check(lib().idx_range_noalloc(self._h, lo.data_ptr(), hi.data_ptr(), m, offsets.data_ptr(),
                                       rowids.data_ptr() if rowids is not None and cap else None, cap,
                                       ctypes.byref(total), _stream(stream)), "idx_range_noalloc")
        return total.value

    # -- introspection and tuning
    def info(self) -> dict:
        i = idx_info()
        _check(lib().idx_get_info(self._h, ctypes.byref(i)), "idx_get_info")
        return {f: getattr(i, f) for f, _ in i._fields_}

    def export(self, stream=None):
        info = self.info()
        keys = torch.empty(info["slots"], dtype=self.key_dtype, device="cuda")
        rows = torch.empty(info["slots"], dtype=torch.int32, device="cuda")
        _check(lib().idx_export(self._h, keys.data_ptr(), rows.data_ptr(), _stream(stream)), "idx_export")
        return keys, rows

    # -- learned rank model (sorted-array indexes)
    def learn(self, leaves: int = 4096, epochs: int = 2, feature: int = IDX_FEATURE_AUTO, stream=None) -> dict:
        _check(lib().idx_learn(self._h, leaves, epochs, feature, _stream(stream)), "idx_learn")
        return self.learn_stats()

    def learn_stats(self) -> dict:
        st = idx_learn_stats()
        _check(lib().idx_learn_stats_get(self._h, ctypes.byref(st)), "idx_learn_stats_get")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def learn_export(self, stream=None) -> torch.Tensor:
        """The leaf table as a (leaves, 8) int32 tensor of raw 32-byte records."""
        L = self.learn_stats()["leaves"]
        t = torch.empty((L, 8), dtype=torch.int32, device="cuda")
        _check(lib().idx_learn_export(self._h, t.data_ptr(), _stream(stream)), "idx_learn_export")
        return t

    def unlearn(self):
        _check(lib().idx_unlearn(self._h), "idx_unlearn")

    def learn_eval(self, feature: int, root_ab, leaves: int, leaf_ab: torch.Tensor | None = None, stream=None):
        """(root sums[6], leaf sums (leaves, 6) or None) of the training
        kernels at the given parameters; see idx_learn_eval."""
        ra = (ctypes.c_float * 2)(*[float(v) for v in root_ab])
        racc = (ctypes.c_double * 6)()
        lacc = None
        lp = None
        if leaf_ab is not None:
            _dev(leaf_ab, "leaf_ab")
            lacc = torch.zeros((leaves, 6), dtype=torch.float64, device=leaf_ab.device)
            lp = leaf_ab.data_ptr()
        _check(lib().idx_learn_eval(self._h, feature, ra, leaves, lp, racc, None if lacc is None else lacc.data_ptr(),
                                    _stream(stream)), "idx_learn_eval")
        return list(racc), lacc

    def set_params(self, **kw):
        p = idx_lookup_params(**kw)
        _check(lib().idx_set_params(self._h, ctypes.byref(p)), "idx_set_params")
        return self.params()

    def reset_params(self):
        _check(lib().idx_set_params(self._h, None), "idx_set_params")

    def params(self) -> dict:
        p = idx_lookup_params()
        _check(lib().idx_get_params(self._h, ctypes.byref(p)), "idx_get_params")
        return p.as_dict()


IDX_BATCH_GRAPH = 1


def learn_batch(indexes, leaves, epochs: int = 2, feature: int = IDX_FEATURE_AUTO, stream=None):
    """Train the models of many sorted-array indexes with one launch sequence
    (idx_learn_batch); `leaves` is one count per index.  Returns each
    index's model statistics."""
    indexes = list(indexes)
    leaves = list(leaves)
    if len(leaves) != len(indexes):
        raise ValueError("one leaf count per index")
    arr = (ctypes.c_void_p * len(indexes))(*[ix._h.value for ix in indexes])
    lv = (ctypes.c_uint32 * len(leaves))(*leaves)
    _check(lib().idx_learn_batch(arr, len(indexes), lv, epochs, feature, _stream(stream)), "idx_learn_batch")
    return [ix.learn_stats() for ix in indexes]


class Batch:
    """Many indexes served by one persistent launch (idx_batch_*).  The
    indexes must stay open while the batch is used."""

    def __init__(self, indexes, stream=None):
        self._indexes = list(indexes)
        if not self._indexes:
            raise ValueError("a batch needs at least one index")
        self.key_bits = self._indexes[0].key_bits
        self.count = len(self._indexes)
        self._total_seen = {}
        arr = (ctypes.c_void_p * len(self._indexes))(*[ix._h.value for ix in self._indexes])
        h = ctypes.c_void_p()
        _check(lib().idx_batch_create(arr, len(self._indexes), _stream(stream), ctypes.byref(h)), "idx_batch_create")
        self._h = h

    def _check_total(self, offsets: torch.Tensor, m: int, exact: bool):
        """The kernels read offsets[count] entries of the query arrays: it may
        not exceed their length (exact: must equal it).  Read once per offsets
        tensor and version."""
        key = (offsets.data_ptr(), offsets._version, len(offsets))
        total = self._total_seen.get(key)
        if total is None:
            total = int(offsets[-1].item())
            self._total_seen = {key: total}
        if total > m or (exact and total != m):
            raise ValueError(f"offsets[-1] = {total} does not fit the {m} queries given")

    def point(self, queries: torch.Tensor, offsets: torch.Tensor, out: torch.Tensor | None = None,
              graph: bool = False, stream=None) -> torch.Tensor:
        _keys_of(queries, "queries", self.key_bits)
        _offsets_of(offsets, "offsets", self.count)
        self._check_total(offsets, len(queries), exact=False)
        if out is None:
            out = torch.empty(len(queries), dtype=torch.int32, device=queries.device)
        _out_u32(out, "out", len(queries))
        _check(lib().idx_batch_point(self._h, queries.data_ptr(), offsets.data_ptr(), out.data_ptr(),
                                     IDX_BATCH_GRAPH if graph else 0, _stream(stream)), "idx_batch_point")
        return out

    def mixed(self, lo: torch.Tensor, hi: torch.Tensor, kind: torch.Tensor, offsets: torch.Tensor,
              capacity: int | None = None, stream=None):
        """Mixed point/range stream (idx_batch_mixed).  Returns (rowid[m]
        int32, range_offsets[m+1] int64, range_rowids[total] int32)."""
        _keys_of(lo, "lo", self.key_bits)
        _keys_of(hi, "hi", self.key_bits)
        _dev(kind, "kind")
        if kind.dtype != torch.uint8:
            raise TypeError("kind must be uint8")
        m = len(lo)
        if len(hi) != m or len(kind) != m:
            raise ValueError("lo, hi and kind differ in length")
        _offsets_of(offsets, "offsets", self.count)
        self._check_total(offsets, m, exact=True)
        out = torch.empty(m, dtype=torch.int32, device=lo.device)
        offs = torch.empty(m + 1, dtype=torch.int64, device=lo.device)
        total = ctypes.c_uint64(0)
        s = _stream(stream)
        if capacity is None:
            _check(lib().idx_batch_mixed(self._h, m, lo.data_ptr(), hi.data_ptr(), kind.data_ptr(), offsets.data_ptr(),
                                         out.data_ptr(), offs.data_ptr(), None, 0, ctypes.byref(total), s),
                   "idx_batch_mixed(count)")
            capacity = total.value
        rows = torch.empty(max(1, capacity), dtype=torch.int32, device=lo.device)
        _check(lib().idx_batch_mixed(self._h, m, lo.data_ptr(), hi.data_ptr(), kind.data_ptr(), offsets.data_ptr(),
                                     out.data_ptr(), offs.data_ptr(), rows.data_ptr(), capacity, ctypes.byref(total),
                                     s), "idx_batch_mixed")
        return out, offs, rows[: total.value]

    def close(self):
        if getattr(self, "_h", None):
            lib().idx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

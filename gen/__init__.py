"""Seeded synthetic inputs (numpy arrays) for the static index.

Thin ctypes wrapper over ``gen/libgen.so``.  This module is shared input
plumbing for the CPU oracle side and the GPU side; it holds no indexing
arithmetic.  Every function is a pure function of its seed.

Workload recipes follow the paper's synthetic setups (Section 8.1: unique
uniform build keys, uniform lookups drawn from the build set; Section 8.9:
Zipf-skewed lookups) and the configurations the benchmark names.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgen.so")
MISS = 0xFFFFFFFF
BASE_SEED = 0x250601576

_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def build_lib(force: bool = True) -> str:
    """Compile libgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
             os.path.join(_HERE, "gen.c"), "-o", _SO + ".tmp", "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_lib()
        L = ctypes.CDLL(_SO)
        L.gen_draw.restype = _u64
        L.gen_draw.argtypes = [_u64, _u64, _u64]
        L.gen_bij.restype = _u64
        L.gen_bij.argtypes = [_u64, ctypes.c_int, _u64]
        L.gen_perm.restype = _u64
        L.gen_perm.argtypes = [_u64, _u64, _u64]
        L.gen_unique_keys.argtypes = [_u64, ctypes.c_int, _u64, _p, ctypes.c_int, _p]
        L.gen_point_queries.argtypes = [_u64, ctypes.c_int, _u64, _u64, _u64, _p, ctypes.c_int, _p]
        L.gen_zipf_ranks.argtypes = [_u64, ctypes.c_double, _u64, _u64, _p]
        L.gen_zipf_queries.argtypes = [_u64, ctypes.c_int, ctypes.c_double, _p, _u64, _u64, _u64, _p,
                                       ctypes.c_int, _p]
        L.gen_lognormal_params.argtypes = [_u64, _p, _p]
        L.gen_lognormal_keys.restype = ctypes.c_int
        L.gen_lognormal_keys.argtypes = [_u64, _u64, _p, _p]
        L.gen_log_uniform.argtypes = [_u64, _u64, _u64, _u64, _u64, _p]
        L.gen_ranges.argtypes = [_u64, _p, ctypes.c_int, _u64, _u64, _u64, _u64, _p, _p, _p, _p]
        L.gen_uniform_values.argtypes = [_u64, _u64, ctypes.c_int, _u64, _p, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _kdt(key_bits: int):
    if key_bits not in (32, 64):
        raise ValueError("key_bits must be 32 or 64")
    return np.uint32 if key_bits == 32 else np.uint64


def bij(seed: int, w: int, x: int) -> int:
    """The keyed bijection f on [0, 2^w) behind unique_keys(seed, w, ...)."""
    return lib().gen_bij(lib().gen_draw(seed, 1, 0), w, x)


def unique_keys(seed: int, n: int, key_bits: int = 32, w: int | None = None):
    """n distinct keys f(0..n-1) in [0, 2^w) and rowids 0..n-1 (insertion order)."""
    w = key_bits if w is None else w
    keys = np.empty(n, dtype=_kdt(key_bits))
    rowids = np.empty(n, dtype=np.uint32)
    lib().gen_unique_keys(seed, w, n, _ptr(keys), key_bits // 8, _ptr(rowids))
    return keys, rowids


def point_queries(seed: int, n: int, m: int, hit_fraction: float, key_bits: int = 32, w: int | None = None):
    """m queries against unique_keys(seed, n): round(m*hit_fraction) hits at
    seeded positions, misses uniform over the complement of the set.
    Returns (queries, expected rowid or MISS)."""
    w = key_bits if w is None else w
    q = np.empty(m, dtype=_kdt(key_bits))
    e = np.empty(m, dtype=np.uint32)
    n_hits = int(round(m * hit_fraction)) if n > 0 else 0
    lib().gen_point_queries(seed, w, n, m, n_hits, _ptr(q), key_bits // 8, _ptr(e))
    return q, e


def zipf_ranks(seed: int, s: float, N: int, m: int) -> np.ndarray:
    out = np.empty(m, dtype=np.uint64)
    lib().gen_zipf_ranks(seed, s, N, m, _ptr(out))
    return out


def zipf_queries(seed: int, s: float, n: int, m: int, miss_fraction: float, key_bits: int = 64,
                 w: int | None = None, keys: np.ndarray | None = None):
    """Zipf(s)-popular hits plus round(m*miss_fraction) misses.  keys=None means
    the set is unique_keys(seed, n, key_bits, w)."""
    w = key_bits if w is None else w
    q = np.empty(m, dtype=_kdt(key_bits))
    e = np.empty(m, dtype=np.uint32)
    if keys is not None:
        keys = np.ascontiguousarray(keys, dtype=_kdt(key_bits))
    lib().gen_zipf_queries(seed, w, s, _ptr(keys), n, m, int(round(m * miss_fraction)), _ptr(q), key_bits // 8,
                           _ptr(e))
    return q, e


def lognormal_params(seed: int):
    mu = np.empty(64, dtype=np.float64)
    sg = np.empty(64, dtype=np.float64)
    lib().gen_lognormal_params(seed, _ptr(mu), _ptr(sg))
    return mu, sg


def lognormal_keys(seed: int, n: int):
    """n distinct uint64 keys from the 64-component lognormal mixture, in
    seeded random order; rowids 0..n-1."""
    keys = np.empty(n, dtype=np.uint64)
    rowids = np.empty(n, dtype=np.uint32)
    if lib().gen_lognormal_keys(seed, n, _ptr(keys), _ptr(rowids)) != 0:
        raise MemoryError("lognormal key generation failed")
    return keys, rowids


def log_uniform(seed: int, stream: int, lo: int, hi: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().gen_log_uniform(seed, stream, lo, hi, count, _ptr(out))
    return out


def ranges(seed: int, keys: np.ndarray, m: int, cmin: int, cmax: int, with_ranks: bool = False):
    """m range queries [lo, hi] over the build set `keys` covering c ~ U{cmin..cmax}
    consecutive build keys each.  The set is put in ascending order with
    numpy's sort (input preparation only).  Returns (lo, hi, c), and with
    with_ranks also r, the ascending-order rank of each range's first key
    (the range covers ranks r .. r + c - 1 of a set of distinct keys)."""
    kb = keys.dtype.itemsize * 8
    ordered = np.sort(keys, kind="stable")
    lo = np.empty(m, dtype=keys.dtype)
    hi = np.empty(m, dtype=keys.dtype)
    c = np.empty(m, dtype=np.uint32)
    r = np.empty(m, dtype=np.uint64) if with_ranks else None
    lib().gen_ranges(seed, _ptr(ordered), kb // 8, len(keys), m, cmin, cmax, _ptr(lo), _ptr(hi), _ptr(c), _ptr(r))
    return (lo, hi, c, r) if with_ranks else (lo, hi, c)


def uniform_values(seed: int, stream: int, m: int, key_bits: int = 32, w: int | None = None) -> np.ndarray:
    w = key_bits if w is None else w
    out = np.empty(m, dtype=_kdt(key_bits))
    lib().gen_uniform_values(seed, stream, w, m, _ptr(out), key_bits // 8)
    return out


def mixed_queries_device(seed: int, keys, m: int, range_fraction: float = 0.3, miss_fraction: float = 0.1,
                         cmin: int = 1, cmax: int = 256, rows=None):
    """A seeded mixed lookup stream over one build set, made on the device
    with torch's own sort and random generator (input preparation only; no
    index code is involved).  `keys` is a device tensor of int64 key bit
    patterns below 2^63 (so signed order is key order).  Each of the m
    queries is a range with probability range_fraction -- c ~ U{cmin..cmax}
    consecutive build keys, L = the key of a uniform rank r, U = the key of
    rank r + c - 1 (clamped to the largest) -- else a point lookup of a
    uniform build key, replaced with probability miss_fraction by an odd
    value uniform in [0, 2^63) (absent unless it happens to be a key).
    Returns device tensors (lo, hi, kind) with kind 1 for ranges; hi = lo
    for points.  With the keys' row IDs `rows` (device int32) and distinct
    keys, also the answers known by construction: (lo, hi, kind, expect,
    count) with expect the row ID of every hit point lookup (-1 for the
    misses and the ranges) and count the number of keys each range covers
    (0 for points)."""
    import torch

    dev = keys.device
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed) & ((1 << 63) - 1))
    n = len(keys)
    ordered, perm = torch.sort(keys, stable=True)
    kind = (torch.rand(m, generator=g, device=dev) < range_fraction).to(torch.uint8)
    pick = torch.randint(0, n, (m,), generator=g, device=dev)
    hit = ordered[pick]
    miss = torch.randint(0, 1 << 62, (m,), generator=g, device=dev) * 2 + 1
    is_hit = torch.rand(m, generator=g, device=dev) < 1.0 - miss_fraction
    lo = torch.where(is_hit, hit, miss)
    c = torch.randint(cmin, cmax + 1, (m,), generator=g, device=dev)
    r = torch.randint(0, n, (m,), generator=g, device=dev)
    e = torch.clamp(r + c - 1, max=n - 1)
    rk = kind.bool()
    hi = torch.where(rk, ordered[e], lo)
    lo = torch.where(rk, ordered[r], lo)
    if rows is None:
        return lo, hi, kind
    expect = torch.where(is_hit & ~rk, rows[perm[pick]], torch.full_like(rows[:1], -1).expand(m))
    count = torch.where(rk, e - r + 1, torch.zeros_like(e))
    return lo, hi, kind, expect, count

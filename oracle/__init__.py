"""CPU oracle for the static index -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline leg may import this package.  It shares no code with the GPU library
(``paper_2506_01576_amd``) and never imports it.  It is the plain definition
of what the index computes:

* ``stable_sort``  -- stable sort of (key, rowid) pairs by key (Section 1
  problem statement; Section 3: the BS index is a key-value sort).
* ``point``        -- lower bound + equality test, miss sentinel 0xFFFFFFFF
  (Section 1 point lookup).
* ``range_lookup`` -- every rowid with L <= key <= U, ascending key order
  (Section 1 range lookup).
* ``eytzinger_ranks`` / ``eytzinger_layout`` -- level-order linearisation of
  the complete search tree by an in-order walk (Section 3, Figures 4-5;
  k-ary: Section 6, Figure 10).  Deliberately not the closed-form
  permutation of Sections 4 and 6.1, which is what the GPU build evaluates.

Keys are unsigned 32- or 64-bit integers; 32-bit keys are widened to 64 bits
before the C code sees them (widening preserves order).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
MISS = 0xFFFFFFFF

_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def build_lib(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, IEEE float, no contraction)."""
    if force or not os.path.exists(_SO):
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-pthread",
             os.path.join(_HERE, "oracle.c"), "-o", _SO + ".tmp", "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build_lib()
        L = ctypes.CDLL(_SO)
        L.orc_stable_sort.restype = ctypes.c_int
        L.orc_stable_sort.argtypes = [_p, _p, _u64, _p, _p]
        L.orc_point.argtypes = [_p, _p, _u64, _p, _u64, _p, ctypes.c_int]
        L.orc_range_count.argtypes = [_p, _u64, _p, _p, _u64, _p, _p, ctypes.c_int]
        L.orc_range_fill.argtypes = [_p, _p, _p, _u64, _p, _p]
        L.orc_eytzinger_ranks.restype = ctypes.c_int
        L.orc_eytzinger_ranks.argtypes = [_u64, _u64, _p]
        L.orc_leaf_grad.argtypes = [_p, _p, _p, _u64, _p, ctypes.c_uint32, _p, _p, _p]
        L.orc_root_grad.argtypes = [_p, _p, _u64, _p, _p, _p, _p]
        L.orc_key_feature.restype = ctypes.c_float
        L.orc_key_feature.argtypes = [_u64, ctypes.c_uint32]
        L.orc_spline_build.argtypes = [_p, _u64, ctypes.c_uint32, ctypes.c_uint32, _p, _p, _p, _p, _p]
        L.orc_spline_build.restype = None
        L.orc_spline_assign.argtypes = [_p, ctypes.c_uint32, ctypes.c_uint32, _p, _p, _p, _p, _p, _u64, _p]
        L.orc_spline_assign.restype = None
        L.orc_assign_leaves.argtypes = [_p, _u64, ctypes.c_uint32, ctypes.c_float, ctypes.c_float, ctypes.c_uint32,
                                        _p, _p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _u64arr(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype not in (np.uint32, np.uint64):
        raise TypeError("keys must be uint32 or uint64")
    return np.ascontiguousarray(a, dtype=np.uint64)


def stable_sort(keys, rowids):
    """(sorted keys as the input dtype, rowids) -- ties keep input order."""
    keys = np.asarray(keys)
    k64 = _u64arr(keys)
    r = np.ascontiguousarray(rowids, dtype=np.uint32)
    n = len(k64)
    ok = np.empty(n, dtype=np.uint64)
    orr = np.empty(n, dtype=np.uint32)
    if lib().orc_stable_sort(_ptr(k64), _ptr(r), n, _ptr(ok), _ptr(orr)) != 0:
        raise MemoryError("oracle sort scratch allocation failed")
    return ok.astype(keys.dtype, copy=False), orr


def point(sorted_keys, sorted_rowids, queries, nthreads: int = 1) -> np.ndarray:
    """Rowid of the first match of each query in the sorted build set, or MISS."""
    K = _u64arr(sorted_keys)
    R = np.ascontiguousarray(sorted_rowids, dtype=np.uint32)
    q = _u64arr(queries)
    out = np.empty(len(q), dtype=np.uint32)
    lib().orc_point(_ptr(K), _ptr(R), len(K), _ptr(q), len(q), _ptr(out), nthreads)
    return out


def range_count(sorted_keys, lo, hi, nthreads: int = 1):
    """(rank of first match, match count) per query [lo, hi]."""
    K = _u64arr(sorted_keys)
    L = _u64arr(lo)
    U = _u64arr(hi)
    m = len(L)
    lr = np.empty(m, dtype=np.uint64)
    c = np.empty(m, dtype=np.uint64)
    lib().orc_range_count(_ptr(K), len(K), _ptr(L), _ptr(U), m, _ptr(lr), _ptr(c), nthreads)
    return lr, c


def range_lookup(sorted_keys, sorted_rowids, lo, hi, nthreads: int = 1, count_only: bool = False):
    """(offsets[m+1] uint64, rowids in key order per query)."""
    lr, c = range_count(sorted_keys, lo, hi, nthreads)
    m = len(lr)
    R = np.ascontiguousarray(sorted_rowids, dtype=np.uint32)
    off = np.empty(m + 1, dtype=np.uint64)
    total = int(c.sum())
    out = None if count_only else np.empty(total, dtype=np.uint32)
    lib().orc_range_fill(_ptr(R), _ptr(lr), _ptr(c), m, _ptr(off), _ptr(out))
    return off, out


def eytzinger_ranks(n: int, k: int) -> np.ndarray:
    """slot -> sorted rank for the level-order k-ary Eytzinger tree (0-based slots)."""
    out = np.empty(n, dtype=np.uint64)
    if lib().orc_eytzinger_ranks(n, k, _ptr(out)) != 0:
        raise ValueError("k must be >= 2")
    return out


def eytzinger_layout(sorted_keys, sorted_rowids, k: int, one_based: bool):
    """Keys and rowids in Eytzinger order.  one_based=True is the binary
    layout with its empty slot 0 (returned as key 0, rowid MISS)."""
    sk = np.asarray(sorted_keys)
    sr = np.asarray(sorted_rowids, dtype=np.uint32)
    ranks = eytzinger_ranks(len(sk), k)
    keys = sk[ranks] if len(sk) else sk.copy()
    rows = sr[ranks] if len(sr) else sr.copy()
    if one_based:
        keys = np.concatenate([np.zeros(1, dtype=sk.dtype), keys])
        rows = np.concatenate([np.array([MISS], dtype=np.uint32), rows])
    return keys, rows


def leaf_grad(d, y, leaf, params, L: int):
    """Per-leaf (loss, grad[L,2], hess[L,3]) of sum (a*d + b - y)^2 in float64."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    leaf = np.ascontiguousarray(leaf, dtype=np.uint32)
    params = np.ascontiguousarray(params, dtype=np.float64)
    loss = np.empty(L)
    grad = np.empty(2 * L)
    hess = np.empty(3 * L)
    lib().orc_leaf_grad(_ptr(d), _ptr(y), _ptr(leaf), len(d), _ptr(params), L, _ptr(loss), _ptr(grad), _ptr(hess))
    return loss, grad.reshape(L, 2), hess.reshape(L, 3)


def key_feature(key: int, mode: int) -> float:
    return lib().orc_key_feature(key, mode)


def assign_leaves(sorted_keys, mode: int, a0: float, a1: float, L: int):
    """(leaf per key, root feature per key as float32) under the root model."""
    K = _u64arr(sorted_keys)
    leaf = np.empty(len(K), dtype=np.uint32)
    x = np.empty(len(K), dtype=np.float32)
    lib().orc_assign_leaves(_ptr(K), len(K), mode, a0, a1, L, _ptr(leaf), _ptr(x))
    return leaf, x


def spline_bins(n: int) -> int:
    """Bins available to the spline root for n keys: the largest power of two
    <= 65536 with at least 64 keys per bin (1 for tiny sets)."""
    B = 1
    while B < 65536 and B * 2 * 64 <= n:
        B *= 2
    return B


def spline_root(sorted_keys, L: int, bfeat: int) -> dict:
    """The spline root over the sorted build keys with L leaves and bin feature
    bfeat (1 = the key, 2 = the log-like code): geometry and bin records."""
    S = _u64arr(sorted_keys)
    B = spline_bins(len(S))
    geo = np.zeros(3, dtype=np.uint64)
    anchor = np.zeros(B, dtype=np.uint64)
    mul, first, sh = (np.zeros(B, dtype=np.uint32) for _ in range(3))
    lib().orc_spline_build(_ptr(S), len(S), L, bfeat, _ptr(geo), _ptr(anchor), _ptr(mul), _ptr(first), _ptr(sh))
    nb = int(geo[2])
    return {"L": L, "bfeat": bfeat, "f_lo": int(geo[0]), "shift": int(geo[1]), "nb": nb, "geo": geo,
            "anchor": anchor[:nb].copy(), "mul": mul[:nb].copy(), "first": first[:nb].copy(), "sh": sh[:nb].copy()}


def spline_leaves(root: dict, keys):
    """Leaf of each key under a spline root from spline_root."""
    K = _u64arr(keys)
    leaf = np.zeros(len(K), dtype=np.uint32)
    lib().orc_spline_assign(_ptr(root["geo"]), root["bfeat"], root["L"], _ptr(root["anchor"]), _ptr(root["mul"]),
                            _ptr(root["first"]), _ptr(root["sh"]), _ptr(K), len(K), _ptr(leaf))
    return leaf


def leaf_frame(sorted_keys, leaf, L: int):
    """Per key: leaf-local feature d = f32(key - first key of its leaf) and
    target y = rank - rank of that first key; per leaf: base rank and size.
    Keys are sorted and leaves non-decreasing, so each leaf is one run."""
    K = _u64arr(sorted_keys)
    n = len(K)
    size = np.bincount(leaf, minlength=L).astype(np.uint64)
    base = np.zeros(L, dtype=np.uint64)
    base[1:] = np.cumsum(size)[:-1]
    kmin = np.where(size > 0, K[np.minimum(base, max(n - 1, 0))], 0).astype(np.uint64)
    rank = np.arange(n, dtype=np.uint64)
    d = (K - kmin[leaf]).astype(np.float32).astype(np.float64)
    y = (rank - base[leaf]).astype(np.float64)
    return d, y, base, size


def root_grad(x, t, params):
    x = np.ascontiguousarray(x, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64)
    params = np.ascontiguousarray(params, dtype=np.float64)
    loss = np.empty(1)
    grad = np.empty(2)
    hess = np.empty(3)
    lib().orc_root_grad(_ptr(x), _ptr(t), len(x), _ptr(params), _ptr(loss), _ptr(grad), _ptr(hess))
    return float(loss[0]), grad, hess

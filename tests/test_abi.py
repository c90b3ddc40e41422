"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/idx.h declares, rejects bad arguments before touching
the device, and its host evaluation of the build permutation agrees with the
oracle's in-order-walk layout."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "idx.h")

idx = pytest.importorskip("paper_2506_01576_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(idx_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = idx.lib()
    names = declared_functions()
    assert "idx_build" in names and "idx_point" in names and "idx_range" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(idx.SIGNATURES), "binding signatures out of step with the header"


def test_strerror():
    L = idx.lib()
    for st in (0, -1, -2, -3, -4, -5, 99):
        assert isinstance(L.idx_strerror(st), bytes)
    assert L.idx_strerror(idx.IDX_ERR_CAPACITY) != L.idx_strerror(idx.IDX_ERR_ARG)


def _build(keys=1, rows=1, n=10, layout=0, k=2, flags=0, alloc=None, out=True):
    h = ctypes.c_void_p()
    return idx.lib().idx_build(keys, rows, n, layout, k, flags, alloc, None, ctypes.byref(h) if out else None), h


def test_build_argument_errors():
    E = idx.IDX_ERR_ARG
    assert _build(out=False)[0] == E
    assert _build(layout=3)[0] == E
    assert _build(layout=-1)[0] == E
    assert _build(layout=idx.IDX_EBS, k=3)[0] == E
    assert _build(layout=idx.IDX_EKS, k=1)[0] == E
    assert _build(layout=idx.IDX_EKS, k=66)[0] == E
    assert _build(n=0xFFFFFFFF)[0] == E
    assert _build(keys=None)[0] == E
    assert _build(rows=None)[0] == E
    assert _build(flags=8)[0] == E
    assert _build(flags=idx.IDX_AOS_PADDED)[0] == E  # padding only applies to AoS
    st, h = _build()
    assert h.value is None


def test_allocator_failure_is_reported_before_device_use():
    calls = []

    def alloc(ctx, nbytes, stream):
        calls.append(nbytes)
        return None

    def release(ctx, p, stream):
        raise AssertionError("nothing was allocated")

    A = idx.idx_allocator(idx.idx_allocator._fields_[0][1](alloc), idx.idx_allocator._fields_[1][1](release), None)
    for layout, k, flags in ((0, 1, 0), (1, 2, 1), (2, 9, 3)):
        st, h = _build(layout=layout, k=k, flags=flags, alloc=ctypes.byref(A))
        assert st == idx.IDX_ERR_NOMEM and h.value is None
    assert len(calls) == 3 and all(c > 0 for c in calls)
    # an allocator missing a callback is an argument error
    B = idx.idx_allocator(idx.idx_allocator._fields_[0][1](alloc), idx.idx_allocator._fields_[1][1](), None)
    assert _build(alloc=ctypes.byref(B))[0] == idx.IDX_ERR_ARG


def test_null_handle_errors():
    L = idx.lib()
    E = idx.IDX_ERR_ARG
    assert L.idx_point(None, 1, 1, 1, None) == E
    assert L.idx_range(None, 1, 1, 1, 1, None, 0, None, None) == E
    assert L.idx_destroy(None) == idx.IDX_OK
    assert L.idx_get_info(None, None) == E
    assert L.idx_export(None, None, None, None) == E
    assert L.idx_set_params(None, None) == E
    assert L.idx_get_params(None, None) == E


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 65])
def test_build_permutation_matches_oracle(k):
    """The closed-form inverse permutation the build kernel evaluates (host
    copy of the same function) equals the oracle's in-order-walk layout."""
    L = idx.lib()
    ns = list(range(0, 300)) + [k ** 3 - 1, k ** 3, k ** 3 + 1, 4097, 65535, 65536]
    for n in ns:
        if n > 70000:
            continue
        want = oracle.eytzinger_ranks(n, k)
        got = np.fromiter((L.idx_slot_rank(n, k, t) for t in range(n)), dtype=np.uint64, count=n)
        assert np.array_equal(got, want), (k, n)
    assert L.idx_slot_rank(5, 1, 0) == 2**64 - 1
    assert L.idx_slot_rank(5, 2, 5) == 2**64 - 1


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 64, 65])
def test_build_rank_slot_matches_oracle(k):
    """The rank-to-slot map the layout build kernels evaluate (host copy of
    the same function) places every sorted rank where the oracle's
    in-order-walk layout holds it."""
    L = idx.lib()
    ns = list(range(0, 300)) + [k ** 2 - 1, k ** 2, k ** 3 - 1, k ** 3 + 1, 4097, 65535, 65536]
    for n in ns:
        if n > 70000:
            continue
        ranks = oracle.eytzinger_ranks(n, k)  # rank held by each slot
        want = np.empty(n, dtype=np.uint64)
        want[ranks.astype(np.int64)] = np.arange(n, dtype=np.uint64)
        got = np.fromiter((L.idx_rank_slot(n, k, r) for r in range(n)), dtype=np.uint64, count=n)
        assert np.array_equal(got, want), (k, n)
    assert L.idx_rank_slot(5, 1, 0) == 2**64 - 1
    assert L.idx_rank_slot(5, 66, 0) == 2**64 - 1
    assert L.idx_rank_slot(5, 2, 5) == 2**64 - 1


def test_build_permutation_large_sampled():
    L = idx.lib()
    rng = np.random.default_rng(9)
    for k in (2, 9, 17, 33):
        n = int(rng.integers(1 << 20, 1 << 21))
        want = oracle.eytzinger_ranks(n, k)
        for t in rng.integers(0, n, size=2000).tolist() + [0, n - 1]:
            assert L.idx_slot_rank(n, k, t) == want[t]

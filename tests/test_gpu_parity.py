"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, bit-exact.

Sizes span several sort tiles (4096 keys) and lookup tiles with ragged
tails; edge cases cover empty and tiny sets, complete/perfect tree
boundaries (k^m - 1, k^m, k^m + 1), duplicate keys, all-equal keys, extreme
key values and inverted ranges.
"""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import rows_host, to_dev, to_host

pytestmark = pytest.mark.gpu

idx = pytest.importorskip("paper_2506_01576_amd")

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

MISS = 0xFFFFFFFF


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def key_set(seed, n, bits, kind="unique"):
    rng = np.random.default_rng(seed)
    dt = np.uint64 if bits == 64 else np.uint32
    if kind == "unique":
        keys, _ = gen.unique_keys(seed, n, bits, 63 if bits == 64 else 32)
    elif kind == "dup":
        keys = rng.integers(0, max(1, n // 3), size=n, dtype=np.uint64).astype(dt)
    elif kind == "equal":
        keys = np.full(n, 12345, dtype=dt)
    elif kind == "small":  # only the low byte varies: upper digit passes are skipped
        keys = rng.integers(0, 256, size=n, dtype=np.uint64).astype(dt)
    elif kind == "extreme":  # values near 0 and near the top of the range
        top = np.iinfo(dt).max
        keys = np.concatenate([rng.integers(0, 4, size=n // 2, dtype=np.uint64).astype(dt),
                               (top - rng.integers(0, 4, size=n - n // 2, dtype=np.uint64)).astype(dt)])
        rng.shuffle(keys)
    else:
        raise ValueError(kind)
    rows = (rng.permutation(n).astype(np.uint64) * 3 + 7).astype(np.uint32)  # distinct, never MISS
    return keys.astype(dt), rows


def queries_for(seed, keys, m, bits):
    rng = np.random.default_rng(seed + 1000)
    dt = keys.dtype
    top = int(np.iinfo(dt).max)
    parts = [rng.integers(0, top, size=m // 2, dtype=np.uint64, endpoint=True).astype(dt)]
    if len(keys):
        parts.append(keys[rng.integers(0, len(keys), size=m - m // 2)])
        lo, hi = int(keys.min()), int(keys.max())
        ext = [0, top, lo, hi, max(lo - 1, 0), min(hi + 1, top), max(hi - 1, 0), min(lo + 1, top)]
    else:
        parts.append(rng.integers(0, top, size=m - m // 2, dtype=np.uint64, endpoint=True).astype(dt))
        ext = [0, top]
    parts.append(np.array(ext, dtype=np.uint64).astype(dt))
    return np.concatenate(parts)


def build(keys, rows, layout, k=9, aos=False):
    return idx.Index(to_dev(keys), to_dev(rows), layout=layout, k=k, aos=aos)


# ------------------------------------------------------------------ build ---

SORT_SIZES = [0, 1, 2, 3, 63, 64, 65, 4095, 4096, 4097, 12289, 100003]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("kind", ["unique", "dup", "equal", "small", "extreme"])
def test_sort_parity(bits, kind):
    """The BS layout is the stable (key, rowid) sort."""
    for n in SORT_SIZES:
        keys, rows = key_set(n * 7 + bits, n, bits, kind)
        say(f"sort bits={bits} kind={kind} n={n}")
        with build(keys, rows, "bs") as ix:
            gk, gr = ix.export()
            ek, er = oracle.stable_sort(keys, rows)
            assert np.array_equal(to_host(gk, bits), ek)
            assert np.array_equal(rows_host(gr), er)
            info = ix.info()
            assert info["unique"] == int(len(np.unique(keys)) == n)


LAYOUT_CASES = [("ebs", 2)] + [("eks", k) for k in (2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 65)]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("aos", [False, True, "padded"])
@pytest.mark.parametrize("layout,k", LAYOUT_CASES)
def test_layout_parity(layout, k, aos, bits):
    """Eytzinger layouts built by the closed-form permutation equal the
    oracle's in-order-walk layout slot for slot."""
    sizes = sorted({0, 1, 2, max(0, k - 2), k - 1, k, k * k - 1, k * k, k * k + 1, 1000, 20011})
    for n in sizes:
        keys, rows = key_set(n + k, n, bits, "dup" if n % 2 else "unique")
        say(f"layout {layout} k={k} aos={aos} bits={bits} n={n}")
        with build(keys, rows, layout, k, aos) as ix:
            gk, gr = ix.export()
            sk, sr = oracle.stable_sort(keys, rows)
            ek, er = oracle.eytzinger_layout(sk, sr, k, one_based=(layout == "ebs"))
            assert np.array_equal(to_host(gk, bits), ek)
            assert np.array_equal(rows_host(gr), er)


@pytest.mark.parametrize("bits", [32, 64])
def test_relayout_parity(bits):
    """Layouts permuted from an existing sorted-array index (no second sort)
    equal the oracle's layouts; the source index is left intact."""
    for n, kind in ((20011, "unique"), (4097, "dup"), (0, "unique"), (1, "unique")):
        keys, rows = key_set(n + 5, n, bits, kind)
        sk, sr = oracle.stable_sort(keys, rows)
        with build(keys, rows, "bs") as base:
            for layout, k, aos in (("ebs", 2, False), ("eks", 9, False), ("eks", 17, True), ("eks", 4, False),
                                   ("bs", 1, True), ("bs", 1, False)):
                say(f"relayout bits={bits} n={n} {kind} -> {layout} k={k} aos={aos}")
                with base.relayout(layout, k, aos) as ix:
                    gk, gr = ix.export()
                    if layout == "bs":
                        ek, er = sk, sr
                    else:
                        ek, er = oracle.eytzinger_layout(sk, sr, k, one_based=(layout == "ebs"))
                    assert np.array_equal(to_host(gk, bits), ek)
                    assert np.array_equal(rows_host(gr), er)
                    assert ix.info()["unique"] == base.info()["unique"]
                    check_point(ix, keys, rows, bits, seed=n + k, m=4099)
            bk, br = base.export()
            assert np.array_equal(to_host(bk, bits), sk) and np.array_equal(rows_host(br), sr)
        with build(keys, rows, "ebs") as not_sorted:
            with pytest.raises(idx.IdxError):
                not_sorted.relayout("eks", 9)


# ----------------------------------------------------------------- points ---

def check_point(ix, keys, rows, bits, seed, m=30011):
    q = queries_for(seed, keys, m, bits)
    sk, sr = oracle.stable_sort(keys, rows)
    want = oracle.point(sk, sr, q, nthreads=4)
    got = rows_host(ix.point(to_dev(q)))
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, f"{len(bad)} mismatches, first q={q[bad[0]]} got={got[bad[0]]} want={want[bad[0]]}"


POINT_PARAMS = {
    "bs": [{}, {"per_lane": 1}, {"per_lane": 8, "block": 1024}, {"lds_levels": 10, "persistent": 2},
           {"lds_levels": 3, "block": 64}],
    "ebs": [{}, {"per_lane": 1}, {"per_lane": 8, "block": 64}, {"lds_levels": 11, "persistent": 2},
            {"lds_levels": 2}],
    "eks": [{}, {"group": 1}, {"group": 1, "per_lane": 8}, {"per_lane": 1, "block": 1024},
            {"per_lane": 8, "early_exit": 2}, {"lds_levels": 2, "persistent": 1}, {"group": 64},
            {"group": 1, "lds_levels": 2}, {"group": 2}, {"group": 4, "per_lane": 8}, {"group": 8, "per_lane": 1},
            {"group": 16, "lds_levels": 2, "persistent": 2}, {"group": 4, "early_exit": 2, "lds_levels": 1}],
}


def resolve(ix, p):
    """Apply a parameter set, lowering lds_levels to what the tree and LDS
    allow; returns False for a set the index does not support (e.g. a lane
    group narrower than its node without 16-byte aligned nodes)."""
    p = dict(p)
    while True:
        try:
            ix.set_params(**p)
            return True
        except idx.IdxError:
            if p.get("lds_levels", 0) > 0:
                p["lds_levels"] -= 1
            else:
                return False


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("aos", [False, True, "padded"])
@pytest.mark.parametrize("layout,k", [("bs", 1), ("ebs", 2)] + [("eks", k) for k in (3, 4, 5, 8, 9, 16, 17, 32, 33)])
def test_point_parity(layout, k, aos, bits):
    for n, kind in ((20011, "unique"), (20011, "dup"), (4096, "extreme"), (k * k, "unique"), (1, "unique"),
                    (0, "unique")):
        keys, rows = key_set(n * 13 + k, n, bits, kind)
        with build(keys, rows, layout, k, aos) as ix:
            for p in POINT_PARAMS["eks" if layout == "eks" else layout]:
                if not resolve(ix, p):
                    continue
                say(f"point {layout} k={k} aos={aos} bits={bits} n={n} {kind} params={ix.params()}")
                check_point(ix, keys, rows, bits, seed=n + k)
                ix.reset_params()


# ----------------------------------------------------------------- ranges ---

def check_range(ix, keys, rows, bits, seed, m=5003):
    rng = np.random.default_rng(seed)
    dt = keys.dtype
    top = int(np.iinfo(dt).max)
    if len(keys):
        L, U, _ = gen.ranges(seed, keys, m, 1, 64)
        # wide ranges: many matches per level, where each lane hands its scan to the whole wave
        if len(keys) > 65:
            Lw, Uw, _ = gen.ranges(seed + 1, keys, 301, 65, min(len(keys), 8192))
            L, U = np.concatenate([L, Lw]), np.concatenate([U, Uw])
    else:
        L = np.zeros(m, dtype=dt)
        U = np.zeros(m, dtype=dt)
    # plus arbitrary bounds: random, inverted, unbounded above / below
    R1 = rng.integers(0, top, size=(2, 500), dtype=np.uint64, endpoint=True).astype(dt)
    extra_lo = np.concatenate([R1.min(axis=0), R1.max(axis=0), np.array([0, 0, top, 5], dtype=dt)])
    extra_hi = np.concatenate([R1.max(axis=0), R1.min(axis=0), np.array([top, 0, top, 4], dtype=dt)])
    L = np.concatenate([L, extra_lo]).astype(dt)
    U = np.concatenate([U, extra_hi]).astype(dt)
    sk, sr = oracle.stable_sort(keys, rows)
    want_off, want = oracle.range_lookup(sk, sr, L, U, nthreads=4)
    off, got = ix.range(to_dev(L), to_dev(U))
    off = off.cpu().numpy().view(np.uint64)
    assert np.array_equal(off, want_off)
    assert np.array_equal(rows_host(got), want)
    # count-only and a too-small capacity
    off2, none = ix.range(to_dev(L), to_dev(U), count_only=True)
    assert none is None and np.array_equal(off2.cpu().numpy().view(np.uint64), want_off)
    if want_off[-1] > 0:
        with pytest.raises(idx.IdxError) as ei:
            ix.range(to_dev(L), to_dev(U), capacity=int(want_off[-1]) - 1)
        assert ei.value.status == idx.IDX_ERR_CAPACITY


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("aos", [False, True, "padded"])
@pytest.mark.parametrize("layout,k", [("bs", 1), ("ebs", 2)] + [("eks", k) for k in (3, 5, 8, 9, 17, 33)])
def test_range_parity(layout, k, aos, bits):
    for n, kind in ((20011, "unique"), (20011, "dup"), (3000, "extreme"), (k * k + 1, "unique"), (1, "unique"),
                    (0, "unique")):
        keys, rows = key_set(n * 17 + k, n, bits, kind)
        say(f"range {layout} k={k} aos={aos} bits={bits} n={n} {kind}")
        with build(keys, rows, layout, k, aos) as ix:
            check_range(ix, keys, rows, bits, seed=n + 3 * k)
            if layout != "bs" and n > 1000:
                # the default gathers by rank; the level scan, with the hybrid
                # hand-over to the wave and with every range scanned by its own
                # lane, gives the same answers
                for mode in (1, 2):
                    ix.set_params(range_scan=mode)
                    check_range(ix, keys, rows, bits, seed=n + 3 * k)
            if n > 1000 and not aos:
                # counts on the batch partitioned by the lower bounds' rank buckets
                ix.set_params(reorder=2)
                check_range(ix, keys, rows, bits, seed=n + 5 * k)


@pytest.mark.parametrize("bits,n,kind", [(64, 1 << 22, "unique"), (32, 1 << 21, "dup")])
def test_partitioned_range_counts_large(bits, n, kind):
    """Range counts through the rank-bucket partition (reorder = 2) at sizes
    with 32 to 128 buckets (coarse and fine scatter passes), every layout (the
    sorted array also in AoS storage): offsets and row IDs equal the oracle's,
    including inverted, unbounded and empty ranges."""
    keys, rows = key_set(71 + bits, n, bits, kind)
    sk, sr = oracle.stable_sort(keys, rows)
    L, U, _ = gen.ranges(72, keys, 1 << 20, 1, 64)
    rng = np.random.default_rng(73)
    dt = keys.dtype
    top = int(np.iinfo(dt).max)
    R1 = rng.integers(0, top, size=(2, 4000), dtype=np.uint64, endpoint=True).astype(dt)
    L = np.concatenate([L, R1.min(axis=0), R1.max(axis=0), np.array([0, top, 0], dtype=dt)])
    U = np.concatenate([U, R1.max(axis=0), R1.min(axis=0), np.array([top, top, 0], dtype=dt)])
    perm = rng.permutation(len(L))
    L, U = L[perm], U[perm]
    want_off, want = oracle.range_lookup(sk, sr, L, U, nthreads=8)
    for layout, k, aos in (("bs", 1, False), ("bs", 1, True), ("ebs", 2, False), ("eks", 9, False)):
        with build(keys, rows, layout, k, aos) as ix:
            ix.set_params(reorder=2)
            say(f"partitioned range counts {layout} aos={aos} bits={bits} n={n} {kind}")
            off, got = ix.range(to_dev(L), to_dev(U))
            assert np.array_equal(off.cpu().numpy().view(np.uint64), want_off), (layout, aos)
            assert np.array_equal(rows_host(got), want), (layout, aos)


def test_range_scan_modes_on_wide_ranges():
    """Ranges of 1 to 8192 matches (every level past the hand-over threshold)
    in both level-scan modes and gathered by rank equal the oracle, EBS and
    EKS."""
    n = 200003
    keys, rows = key_set(5, n, 64, "unique")
    sk, sr = oracle.stable_sort(keys, rows)
    lo, hi, _ = gen.ranges(9, keys, 4000, 1, 8192)
    want_off, want_rows = oracle.range_lookup(sk, sr, lo, hi, nthreads=4)
    for layout, k in (("ebs", 2), ("eks", 9), ("eks", 17)):
        with build(keys, rows, layout, k, False) as ix:
            for mode in (1, 2, 3):
                ix.set_params(range_scan=mode)
                off, rr = ix.range(to_dev(lo), to_dev(hi))
                assert np.array_equal(off.cpu().numpy().view(np.uint64), want_off), (layout, k, mode)
                assert np.array_equal(rows_host(rr), want_rows), (layout, k, mode)


# ------------------------------------------------------------ error paths ---

def test_reserved_rowid_rejected():
    keys = np.arange(100, dtype=np.uint32)
    rows = np.arange(100, dtype=np.uint32)
    rows[57] = MISS
    with pytest.raises(idx.IdxError) as ei:
        build(keys, rows, "eks", 9)
    assert ei.value.status == idx.IDX_ERR_RESERVED_ROWID


def test_bad_params_rejected():
    keys, rows = key_set(1, 5000, 32)
    with build(keys, rows, "eks", 9) as ix:
        before = ix.params()
        for bad in ({"group": 128}, {"group": 3}, {"block": 96}, {"per_lane": 3}, {"lds_levels": 30},
                    {"early_exit": 3}, {"reorder": 4}, {"reorder": 1, "group": 8}, {"range_scan": 4}):
            with pytest.raises(idx.IdxError):
                ix.set_params(**bad)
            assert ix.params() == before
        ix.set_params(group=2)  # 4 u32 pivots per lane
        ix.set_params(group=8)  # one pivot per lane
    with build(keys, rows, "eks", 8) as ix:  # 7 pivots: nodes are not 16-byte aligned
        with pytest.raises(idx.IdxError):
            ix.set_params(group=4)
        ix.set_params(group=8)

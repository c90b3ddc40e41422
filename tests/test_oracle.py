"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the layouts are checked against
the paper's printed worked examples (tests/golden), the closed form the paper
gives for perfect trees, and the search-tree property over the implicit tree
shape of Section 6.2 (which, together with "is a permutation", determines the
layout uniquely); lookups are checked by brute force and by the generator's
answers known by construction.
"""
import itertools

import numpy as np
import pytest

import gen
import oracle
from conftest import read_golden

MISS = oracle.MISS


# ---------------------------------------------------------------- helpers ---

def level_bounds(n, k):
    """[(first_slot, end_slot)] per level of the 0-based k-ary level order."""
    out, start, width = [], 0, k - 1
    while start < n:
        out.append((start, min(n, start + width)))
        start += width
        width *= k
    return out


def slot_levels(n, k):
    lv = np.empty(n, dtype=np.int64)
    for l, (a, b) in enumerate(level_bounds(n, k)):
        lv[a:b] = l
    return lv


def children_start(i, k):
    """Section 6.2: the node starting at slot i has its k children at
    slots i*k + (j+1)*(k-1), j = 0..k-1."""
    return [i * k + (j + 1) * (k - 1) for j in range(k)]


def check_search_tree(ranks, k):
    """The layout is a permutation of 0..n-1 and every key lies strictly
    between the bounds its ancestors impose (walked top-down over the
    Section 6.2 child offsets, independently of the oracle's walk)."""
    n = len(ranks)
    assert sorted(ranks.tolist()) == list(range(n))
    if n == 0:
        return
    stack = [(0, -1, n)]  # node start slot, exclusive lower / upper rank bound
    seen = 0
    while stack:
        i, lo, hi = stack.pop()
        piv = [int(ranks[s]) for s in range(i, min(i + k - 1, n))]
        seen += len(piv)
        assert all(lo < p < hi for p in piv)
        assert piv == sorted(piv)
        bounds = [lo] + piv + [hi]
        for j, c in enumerate(children_start(i, k)):
            if c < n:
                assert j <= len(piv)  # only a full node can have children
                stack.append((c, bounds[j], bounds[j + 1]))
    assert seen == n


# ---------------------------------------------------- paper worked examples ---

def test_fig10_ternary_order():
    g = read_golden("fig10_ternary.txt")
    k = int(g["k"][0][0])
    srt = np.array(g["sorted"][0], dtype=np.uint64)
    want = np.array(g["eytzinger"][0], dtype=np.uint64)
    rows = np.arange(len(srt), dtype=np.uint32)
    keys, _ = oracle.eytzinger_layout(srt, rows, k, one_based=False)
    assert keys.tolist() == want.tolist()
    assert slot_levels(len(srt), k).tolist() == [int(v) for v in g["eytzinger_levels"][0]]
    # level at which each sorted entry is first visited (top table of Fig. 10)
    ranks = oracle.eytzinger_ranks(len(srt), k)
    lv = slot_levels(len(srt), k)
    by_rank = np.empty(len(srt), dtype=np.int64)
    by_rank[ranks] = lv
    assert by_rank.tolist() == [int(v) for v in g["sorted_levels"][0]]


def test_fig11_ternary_lookup_path():
    g = read_golden("fig11_path.txt")
    k = int(g["k"][0][0])
    x = int(g["target"][0][0])
    srt = np.array(read_golden("fig10_ternary.txt")["sorted"][0], dtype=np.uint64)
    keys, _ = oracle.eytzinger_layout(srt, np.arange(len(srt), dtype=np.uint32), k, one_based=False)
    n = len(keys)
    i, path, hit = 0, [], None
    while i < n:
        path.append(i)
        node = [int(keys[s]) for s in range(i, min(i + k - 1, n))]
        if x in node:
            hit = i + node.index(x)
            break
        j = sum(1 for p in node if p < x)
        i = i * k + (j + 1) * (k - 1)
    assert path == [int(v) for v in g["path_offsets"][0]]
    assert [int(keys[s]) for s in (0, 1)] == [int(v) for v in g["root_pivots"][0]]
    assert [int(keys[s]) for s in (2, 3)] == [int(v) for v in g["second_pivots"][0]]
    assert hit == int(g["hit_offset"][0][0])


def test_fig8_binary_eytzinger_range_narrative():
    g = read_golden("fig8_ebs_range.txt")
    L, U = (int(v) for v in g["range"][0])
    srt = np.array(read_golden("fig10_ternary.txt")["sorted"][0], dtype=np.uint64)
    keys, _ = oracle.eytzinger_layout(srt, np.arange(len(srt), dtype=np.uint32), 2, one_based=True)
    for slot, key in g["slot_key"]:
        assert int(keys[int(slot)]) == int(key)
    n = len(srt)
    # within every level the qualifying entries are consecutive, and a scan
    # from the lower-bound path node wastes at most two entries per level
    # (Section 5)
    i, level = 1, 0
    while i <= n:
        a, b = 1 << level, min(n, (2 << level) - 1)
        lev = [int(keys[s]) for s in range(a, b + 1)]
        q = [s for s in range(a, b + 1) if L <= int(keys[s]) <= U]
        if q:
            assert q == list(range(q[0], q[-1] + 1))
            assert q[0] in (i, i + 1)
        assert lev == sorted(lev)
        i = 2 * i + (int(keys[i]) < L)
        level += 1


def test_fig7_complete_binary_tree_n17():
    g = read_golden("fig7_n17.txt")
    n = int(g["n"][0][0])
    full = int(g["full_levels"][0][0])
    bottom = int(g["bottom_entries"][0][0])
    srt = np.arange(100, 100 + n, dtype=np.uint64)
    keys, _ = oracle.eytzinger_layout(srt, np.arange(n, dtype=np.uint32), 2, one_based=True)
    sizes = [len(range(1 << l, min(n, (2 << l) - 1) + 1)) for l in range(full + 1)]
    assert sizes[:full] == [1 << l for l in range(full)]
    assert sizes[full] == bottom
    # the lowest level is left-aligned: its entries are the children of the
    # leftmost node above it, i.e. slot 2^(m-1) has children 2^m and 2^m + 1
    left = 1 << (full - 1)
    assert int(keys[2 * left]) < int(keys[left]) < int(keys[2 * left + 1])
    assert int(keys[2 * left]) == 100  # smallest key
    # in-order traversal (left, node, right) of the 1-based tree is sorted
    order = []

    def walk(s):
        if s > n:
            return
        walk(2 * s)
        order.append(int(keys[s]))
        walk(2 * s + 1)

    walk(1)
    assert order == srt.tolist()


@pytest.mark.parametrize("k", [2, 3, 4, 5, 9, 17])
def test_perfect_tree_closed_form(k):
    """Sections 4 and 6.1: for a perfect tree of m levels (n = k^m - 1) the
    entry at level-order slot t comes from sorted position
    k^(m-l-1) * (1 + i + floor(i/(k-1))) - 1, with l the level of t and i its
    position within that level (for k = 2: 2^(m-l-1) * (1 + 2i) - 1)."""
    for m in range(1, 12 if k == 2 else 5):
        n = k ** m - 1
        if n > 300000:
            break
        ranks = oracle.eytzinger_ranks(n, k)
        t = np.arange(n)
        lv = slot_levels(n, k)
        i = t - (k ** lv - 1)
        p = k ** (m - lv - 1) * (1 + i + i // (k - 1)) - 1
        assert np.array_equal(ranks.astype(np.int64), p)


# -------------------------------------------- search-tree property (unique) ---

@pytest.mark.parametrize("k", [2, 3, 4, 5, 8, 9, 16, 17, 32, 33])
def test_layout_is_the_search_tree_small(k):
    for n in itertools.chain(range(0, 130), [k - 2, k - 1, k, k * k - 1, k * k, k * k + 1, 257, 1000]):
        if n < 0:
            continue
        check_search_tree(oracle.eytzinger_ranks(n, k), k)


def test_layout_is_the_search_tree_large():
    rng = np.random.default_rng(5)
    for k in (2, 9, 17):
        for n in rng.integers(1, 1 << 17, size=3).tolist() + [(1 << 16) - 1, 1 << 16]:
            ranks = oracle.eytzinger_ranks(n, k)
            assert np.array_equal(np.sort(ranks), np.arange(n, dtype=np.uint64))
            # every level ascending and every node's pivots ascending
            for a, b in level_bounds(n, k):
                assert np.all(np.diff(ranks[a:b].astype(np.int64)) > 0)
            # the search-tree bounds, one level at a time (vectorised): the
            # interval of a node is inherited by its slots; pivot j of a node
            # caps child j from above and child j+1 from below (Section 6.2)
            lo = np.full(n, -1, dtype=np.int64)
            hi = np.full(n, n, dtype=np.int64)
            for a, b in level_bounds(n, k):
                s = np.arange(a, b)
                r = ranks[a:b].astype(np.int64)
                assert np.all((lo[a:b] < r) & (r < hi[a:b]))
                node, j = s // (k - 1), s % (k - 1)
                lo_node, hi_node = lo[a:b].copy(), hi[a:b].copy()
                for child, val, which in ((node * k + 1 + j, r, "hi"), (node * k + 2 + j, r, "lo"),
                                          (node * k + 1, lo_node, "lo"), (node * k + k, hi_node, "hi")):
                    for w in range(k - 1):
                        cs = child * (k - 1) + w
                        ok = cs < n
                        if which == "hi":
                            hi[cs[ok]] = val[ok]
                        else:
                            lo[cs[ok]] = val[ok]


def test_layout_brute_force_tiny():
    """For tiny n, exactly one permutation satisfies the search-tree property
    on the complete tree shape -- and it is the oracle's."""
    for k in (2, 3, 4):
        for n in range(0, 7):
            ok = []
            for perm in itertools.permutations(range(n)):
                try:
                    check_search_tree(np.array(perm, dtype=np.uint64), k)
                    ok.append(perm)
                except AssertionError:
                    pass
            assert len(ok) == 1
            assert list(ok[0]) == oracle.eytzinger_ranks(n, k).tolist()


# ------------------------------------------------------------------ lookups ---

def brute_sort(keys, rows):
    """Insertion sort: obviously stable."""
    out = []
    for kv in zip(keys.tolist(), rows.tolist()):
        p = len(out)
        while p > 0 and out[p - 1][0] > kv[0]:
            p -= 1
        out.insert(p, kv)
    return [a for a, _ in out], [b for _, b in out]


def test_stable_sort_brute_force():
    rng = np.random.default_rng(1)
    for n in list(range(0, 40)) + [257]:
        keys = rng.integers(0, max(1, n // 3), size=n).astype(np.uint64)
        rows = rng.permutation(n).astype(np.uint32)
        k, r = oracle.stable_sort(keys, rows)
        bk, br = brute_sort(keys, rows)
        assert k.tolist() == bk and r.tolist() == br


def test_stable_sort_library():
    rng = np.random.default_rng(2)
    for dt, hi in ((np.uint32, 1 << 32), (np.uint64, 1 << 63)):
        keys = rng.integers(0, hi, size=200003, dtype=np.uint64).astype(dt)
        keys[::7] = keys[3]  # plenty of ties
        rows = rng.permutation(len(keys)).astype(np.uint32)
        k, r = oracle.stable_sort(keys, rows)
        o = np.argsort(keys, kind="stable")
        assert k.dtype == dt
        assert np.array_equal(k, keys[o]) and np.array_equal(r, rows[o])


def test_point_brute_force():
    rng = np.random.default_rng(3)
    for n in range(0, 30):
        keys = rng.integers(0, 20, size=n).astype(np.uint64)
        rows = rng.permutation(n).astype(np.uint32) + 5
        q = rng.integers(0, 22, size=50).astype(np.uint64)
        K, R = oracle.stable_sort(keys, rows)
        got = oracle.point(K, R, q)
        for x, g in zip(q.tolist(), got.tolist()):
            # first occurrence in (stable) sorted order = first in input order
            hits = [int(r) for kk, r in zip(keys.tolist(), rows.tolist()) if kk == x]
            assert g == (hits[0] if hits else MISS)


@pytest.mark.parametrize("key_bits,w", [(32, 32), (64, 63)])
def test_point_generator_answers(key_bits, w):
    """The generator knows every answer by construction (query f(i) -> i)."""
    n, m = 1 << 16, 1 << 20
    keys, rows = gen.unique_keys(11, n, key_bits, w)
    q, expect = gen.point_queries(11, n, m, 0.5, key_bits, w)
    K, R = oracle.stable_sort(keys, rows)
    got = oracle.point(K, R, q, nthreads=4)
    assert np.array_equal(got, expect)
    assert (expect == MISS).sum() == m // 2


def test_range_brute_force():
    rng = np.random.default_rng(4)
    for n in range(0, 25):
        keys = rng.integers(0, 15, size=n).astype(np.uint64)
        rows = rng.permutation(n).astype(np.uint32)
        L = rng.integers(0, 17, size=40).astype(np.uint64)
        U = rng.integers(0, 17, size=40).astype(np.uint64)
        K, R = oracle.stable_sort(keys, rows)
        off, out = oracle.range_lookup(K, R, L, U)
        assert off[0] == 0 and len(out) == off[-1]
        for q in range(len(L)):
            want = sorted([(int(kk), i, int(r)) for i, (kk, r) in enumerate(zip(keys.tolist(), rows.tolist()))
                           if L[q] <= kk <= U[q]])
            assert out[off[q]:off[q + 1]].tolist() == [r for _, _, r in want]


def test_range_generator_counts():
    n, m = 1 << 14, 1 << 12
    keys, rows = gen.unique_keys(12, n, 64, 63)
    L, U, c = gen.ranges(12, keys, m, 1, 256)
    K, R = oracle.stable_sort(keys, rows)
    off, out = oracle.range_lookup(K, R, L, U)
    assert np.array_equal(np.diff(off), c.astype(np.uint64))
    # rowids of a range are in key order
    seg = out[off[5]:off[6]]
    assert np.all(np.diff(keys[seg].astype(np.int64)) > 0)


def test_edge_cases():
    e64 = np.zeros(0, dtype=np.uint64)
    e32 = np.zeros(0, dtype=np.uint32)
    K, R = oracle.stable_sort(e64, e32)
    assert len(K) == 0
    q = np.array([0, 1, 2**64 - 1], dtype=np.uint64)
    assert oracle.point(K, R, q).tolist() == [MISS] * 3
    off, out = oracle.range_lookup(K, R, q, q)
    assert off.tolist() == [0, 0, 0, 0] and len(out) == 0
    K, R = oracle.stable_sort(np.array([7], dtype=np.uint64), np.array([3], dtype=np.uint32))
    assert oracle.point(K, R, np.array([6, 7, 8], dtype=np.uint64)).tolist() == [MISS, 3, MISS]
    # inverted and extreme bounds
    off, out = oracle.range_lookup(K, R, np.array([8, 0, 7], dtype=np.uint64),
                                   np.array([6, 2**64 - 1, 7], dtype=np.uint64))
    assert off.tolist() == [0, 0, 1, 2] and out.tolist() == [3, 3]
    assert oracle.eytzinger_ranks(0, 2).tolist() == []
    assert oracle.eytzinger_ranks(1, 9).tolist() == [0]
    with pytest.raises(ValueError):
        oracle.eytzinger_ranks(5, 1)

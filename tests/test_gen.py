"""Properties of the seeded input generators (shared by both sides)."""
import math

import numpy as np
import pytest

import gen
from conftest import read_golden


@pytest.mark.parametrize("w", [2, 3, 8, 13, 16])
def test_bijection_is_a_permutation(w):
    keys, _ = gen.unique_keys(7, 1 << w, 32, w)
    assert np.array_equal(np.sort(keys), np.arange(1 << w, dtype=np.uint32))


def test_perm_cycle_walk():
    L = gen.lib()
    for N in (1, 2, 3, 5, 1000, 4097):
        vals = sorted(L.gen_perm(123, N, x) for x in range(N))
        assert vals == list(range(N))


@pytest.mark.parametrize("key_bits,w", [(32, 32), (64, 63), (64, 64)])
def test_unique_keys_and_queries(key_bits, w):
    n, m = 5000, 20000
    keys, rows = gen.unique_keys(3, n, key_bits, w)
    assert len(np.unique(keys)) == n and np.array_equal(rows, np.arange(n, dtype=np.uint32))
    if w < 64:
        assert int(keys.max()) < (1 << w)
    q, e = gen.point_queries(3, n, m, 0.8, key_bits, w)
    member = np.isin(q, keys)
    assert member.sum() == round(0.8 * m)
    assert np.array_equal(member, e != gen.MISS)
    assert np.array_equal(keys[e[member]], q[member])
    # determinism
    q2, _ = gen.point_queries(3, n, m, 0.8, key_bits, w)
    assert np.array_equal(q, q2)


def _expected_distinct(s, N, M, chunk=1 << 24):
    """E[#distinct] = sum_i 1 - (1 - p_i)^M for bounded Zipf p_i ~ i^-s."""
    H = 0.0
    for a in range(1, N + 1, chunk):
        i = np.arange(a, min(N, a + chunk - 1) + 1, dtype=np.float64)
        H += float(np.sum(i ** -s))
    E = 0.0
    for a in range(1, N + 1, chunk):
        i = np.arange(a, min(N, a + chunk - 1) + 1, dtype=np.float64)
        p = i ** -s / H
        E += float(np.sum(-np.expm1(M * np.log1p(-p))))
    return E


def test_zipf_distinct_matches_paper():
    """Section 8.9 prints the number of distinct keys touched by 2^25 Zipf
    lookups over 2^28 keys; the sampler reproduces the bounded-Zipf
    expectation and lands within 0.5% of the printed counts."""
    g = read_golden("zipf_distinct.txt")
    N = int(g["build_keys"][0][0])
    M = int(g["lookups"][0][0])
    for s_txt, printed in g["exponent_distinct"]:
        s, printed = float(s_txt), int(printed)
        want = _expected_distinct(s, N, M)
        got = len(np.unique(gen.zipf_ranks(99, s, N, M)))
        assert abs(got - want) < 6 * math.sqrt(want) + 5
        assert abs(got - printed) / printed < 0.005
        r = gen.zipf_ranks(99, s, 1000, 1000)
        assert r.min() >= 1 and r.max() <= 1000


def test_zipf_queries_shape():
    n, m = 1 << 12, 1 << 14
    keys, _ = gen.unique_keys(4, n, 64, 63)
    q, e = gen.zipf_queries(4, 1.1, n, m, 0.1, 64, 63)
    hit = e != gen.MISS
    assert (~hit).sum() == round(0.1 * m)
    assert np.array_equal(keys[e[hit]], q[hit])
    assert not np.isin(q[~hit], keys).any()
    # explicit key set: hits come from it
    q2, e2 = gen.zipf_queries(4, 1.1, n, m, 0.1, 64, 63, keys=keys[::-1].copy())
    hit2 = e2 != gen.MISS
    assert np.array_equal(keys[::-1][e2[hit2]], q2[hit2])


def test_lognormal_keys():
    n = 1 << 16
    keys, rows = gen.lognormal_keys(21, n)
    assert len(np.unique(keys)) == n
    assert int(keys.max()) <= (1 << 63) - 1
    assert np.array_equal(rows, np.arange(n, dtype=np.uint32))
    mu, sg = gen.lognormal_params(21)
    assert mu.min() >= 20 and mu.max() <= 50 and sg.min() >= 0.5 and sg.max() <= 2
    k2, _ = gen.lognormal_keys(21, n)
    assert np.array_equal(keys, k2)
    # spread over many orders of magnitude
    lg = np.log(keys.astype(np.float64) + 1)
    assert lg.min() < 25 and lg.max() > 43


def test_log_uniform_and_ranges():
    v = gen.log_uniform(5, 0, 64, 1 << 22, 20000)
    assert v.min() >= 64 and v.max() <= 1 << 22
    med = float(np.median(np.log2(v.astype(np.float64))))
    assert abs(med - 14.0) < 0.2
    keys, _ = gen.unique_keys(8, 3000, 32)
    lo, hi, c = gen.ranges(8, keys, 500, 1, 256)
    s = np.sort(keys)
    assert np.array_equal(np.searchsorted(s, hi, "right") - np.searchsorted(s, lo, "left"), c)

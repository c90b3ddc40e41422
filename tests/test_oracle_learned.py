"""Pins of the oracle's learned-model functions: the gradient and Hessian it
reports are checked against central finite differences of its loss, and
against numpy's least-squares solver (where the gradient must vanish); the
root feature and leaf assignment against their defining properties."""
import struct

import numpy as np
import pytest

import gen
import oracle


def _leaf_problem(seed, n=3000, L=7):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0, 1e6, size=n)
    leaf = np.sort(rng.integers(0, L, size=n)).astype(np.uint32)
    y = 3.5e-4 * d + rng.normal(0, 20, size=n) + 100 * leaf
    params = rng.normal(0, 1, size=2 * L) * np.tile([1e-4, 10.0], L)
    return d, y, leaf, params, L


def test_leaf_gradient_finite_differences():
    d, y, leaf, params, L = _leaf_problem(1)
    loss, grad, hess = oracle.leaf_grad(d, y, leaf, params, L)
    for j in range(2 * L):
        h = 1e-7 if j % 2 == 0 else 1e-3
        p1, p2 = params.copy(), params.copy()
        p1[j] += h
        p2[j] -= h
        fd = (oracle.leaf_grad(d, y, leaf, p1, L)[0][j // 2] - oracle.leaf_grad(d, y, leaf, p2, L)[0][j // 2]) / (2 * h)
        assert grad[j // 2, j % 2] == pytest.approx(fd, rel=1e-5, abs=1e-3)
    # Hessian = derivative of the gradient
    for l in range(L):
        for j in range(2):
            h = 1e-7 if j == 0 else 1e-3
            p1, p2 = params.copy(), params.copy()
            p1[2 * l + j] += h
            p2[2 * l + j] -= h
            g1 = oracle.leaf_grad(d, y, leaf, p1, L)[1][l]
            g2 = oracle.leaf_grad(d, y, leaf, p2, L)[1][l]
            col = (g1 - g2) / (2 * h)
            # hess layout: (dd, d1, 11)
            if j == 0:
                assert col[0] == pytest.approx(hess[l, 0], rel=1e-6)
                assert col[1] == pytest.approx(hess[l, 1], rel=1e-6)
            else:
                assert col[0] == pytest.approx(hess[l, 1], rel=1e-6)
                assert col[1] == pytest.approx(hess[l, 2], rel=1e-6)


def test_leaf_gradient_vanishes_at_least_squares():
    d, y, leaf, _, L = _leaf_problem(2)
    params = np.zeros(2 * L)
    for l in range(L):
        sel = leaf == l
        A = np.stack([d[sel], np.ones(sel.sum())], axis=1)
        sol, *_ = np.linalg.lstsq(A, y[sel], rcond=None)
        params[2 * l], params[2 * l + 1] = sol
    loss, grad, hess = oracle.leaf_grad(d, y, leaf, params, L)
    scale = np.abs(d * y).sum()
    assert np.all(np.abs(grad) < 1e-9 * scale)
    # and any perturbation increases the loss
    loss2, _, _ = oracle.leaf_grad(d, y, leaf, params * (1 + 1e-6), L)
    assert np.all(loss2 >= loss - 1e-6 * loss)


def test_root_gradient():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, 5000)
    t = 4096 * x ** 1.3
    A = np.stack([x, np.ones_like(x)], axis=1)
    sol, *_ = np.linalg.lstsq(A, t, rcond=None)
    loss, grad, hess = oracle.root_grad(x, t, sol)
    assert np.all(np.abs(grad) < 1e-8 * np.abs(x * t).sum())
    p = np.array([2000.0, -3.0])
    loss, grad, _ = oracle.root_grad(x, t, p)
    for j in range(2):
        h = 1e-4
        p1, p2 = p.copy(), p.copy()
        p1[j] += h
        p2[j] -= h
        fd = (oracle.root_grad(x, t, p1)[0] - oracle.root_grad(x, t, p2)[0]) / (2 * h)
        assert grad[j] == pytest.approx(fd, rel=1e-6)
    assert hess[2] == pytest.approx(2 * len(x))


def test_key_feature_properties():
    f = oracle.key_feature
    assert f(0, 1) == 0.0 and f(0, 2) == 0.0
    assert f(2**64 - 1, 1) == 1.0  # rounds to 2^64
    assert f(2**63, 2) == pytest.approx(0x5F000000 / 2**31)  # float(2^63) has bits 0x5F000000
    assert f(1, 2) == pytest.approx(0x3F800000 / 2**31)
    keys, _ = gen.unique_keys(4, 200000, 64, 63)
    ks = np.sort(keys)
    for mode in (1, 2):
        vals = np.array([f(int(k), mode) for k in ks[::97]])
        assert np.all(np.diff(vals) >= 0) and vals.min() >= 0 and vals.max() <= 1


@pytest.mark.parametrize("mode", [1, 2])
def test_leaf_assignment_monotone(mode):
    keys, _ = gen.lognormal_keys(5, 1 << 15)
    ks = np.sort(keys)
    for a0, a1, L in ((0.0, 4096.0, 4096), (-10.0, 9000.0, 4096), (3.0, 0.0, 16), (0.0, 1e9, 1)):
        leaf, x = oracle.assign_leaves(ks, mode, a0, a1, L)
        assert np.all(np.diff(leaf.astype(np.int64)) >= 0)
        assert leaf.max() < L
        d, y, base, size = oracle.leaf_frame(ks, leaf, L)
        assert size.sum() == len(ks) and np.all(y >= 0) and np.all(d >= 0)
        # each leaf's first key has local feature 0 and local target 0
        first = base[size > 0].astype(np.int64)
        assert np.all(d[first] == 0) and np.all(y[first] == 0)


# ------------------------------------------------------------ spline root

def test_spline_bins_rule():
    """The largest power of two <= 65536 with at least 64 keys per bin."""
    assert [oracle.spline_bins(n) for n in (1, 127, 128, 255, 256, 64 * 4096, 64 * 65536, 1 << 40)] == [
        1, 1, 2, 2, 4, 4096, 65536, 65536]


def _double_code(x):
    """The log-like bin feature read off the IEEE-754 double encoding of x
    (exact for x < 2^53 and for x with at most 53 significant bits): the
    unbiased exponent above 58 bits of fraction."""
    if x == 0:
        return 0
    bits = struct.unpack("<Q", struct.pack("<d", float(x)))[0]
    assert int(float(x)) == x
    return (((bits >> 52) - 1023) << 58) | ((bits & ((1 << 52) - 1)) << 6)


def test_spline_log_feature_is_the_double_encoding():
    """f_lo of a one-key root is the bin feature of that key; for LOG it must
    equal the exponent and fraction bits of the key as an IEEE double."""
    rng = np.random.default_rng(3)
    xs = [0, 1, 2, 3, 5, 1000, (1 << 52) + 1, (1 << 53) - 1, 1 << 63, ((1 << 53) - 1) << 11]
    xs += [int(v) for v in rng.integers(1, 1 << 53, 200, dtype=np.uint64)]
    xs += [int(v) << int(e) for v, e in zip(rng.integers(1, 1 << 53, 100, dtype=np.uint64), rng.integers(0, 11, 100))]
    for x in xs:
        r = oracle.spline_root(np.array([x], dtype=np.uint64), 4, 2)
        assert r["f_lo"] == _double_code(x), x
        assert oracle.spline_root(np.array([x], dtype=np.uint64), 4, 1)["f_lo"] == x


def _brute_spline(sk, L, bfeat, queries, domain):
    """The spline root on a small key domain: bins of every key of the domain
    by scanning, bin boundaries and ranks by counting, then the bin records."""
    n = len(sk)
    B = 1
    while B < 65536 and B * 2 * 64 <= n:
        B *= 2
    u = (lambda x: x) if bfeat == 1 else _double_code
    f_lo = u(int(sk[0]))
    span = u(int(sk[-1])) - f_lo
    sh = next(t for t in range(65) if t == 64 or (span >> t) < B)
    nb = 1 if sh == 64 else (span >> sh) + 1

    def bin_of(x):
        v = u(x)
        if v <= f_lo or sh == 64:
            return 0
        return min(nb - 1, (v - f_lo) >> sh)

    bins = [bin_of(x) for x in range(domain)]
    lower = {}
    for x, b in enumerate(bins):
        for c in range(1, b + 1):
            lower.setdefault(c, x)
    rank = [sum(1 for k in sk if bin_of(int(k)) < b) for b in range(nb + 1)]
    out = []
    for q in queries:
        q = int(q)
        b = bin_of(q)
        f0, f1 = rank[b] * L // n, rank[b + 1] * L // n
        if rank[b + 1] == rank[b] or f1 == f0:
            out.append(min(f0, L - 1))
            continue
        anchor = int(sk[rank[b]])
        w = (1 << 64) - 1 - anchor if b + 1 == nb else lower[b + 1] - 1 - anchor
        k = 0
        while (w >> k) >= 1 << 32:
            k += 1
        mul = min((1 << 32) - 1, ((f1 - f0) << 32) // ((w >> k) + 1))
        d = max(q - anchor, 0)
        out.append(min(L - 1, f0 + (((d >> k) * mul) >> 32)))
    return np.array(out, dtype=np.uint32), nb


@pytest.mark.parametrize("bfeat", [1, 2])
@pytest.mark.parametrize("case", ["uniform", "clusters", "tiny", "equal"])
def test_spline_leaves_match_brute_force(bfeat, case):
    rng = np.random.default_rng(11)
    domain = 1 << 12
    if case == "uniform":
        sk = np.sort(rng.integers(0, domain, 3000))
    elif case == "clusters":
        sk = np.sort(np.concatenate([rng.integers(3, 40, 900), rng.integers(700, 760, 1500),
                                     rng.integers(3000, 4095, 600)]))
    elif case == "tiny":
        sk = np.sort(rng.integers(1, domain, 9))
    else:
        sk = np.full(500, 1234)
    sk = sk.astype(np.uint64)
    for L in (1, 5, 64, 333):
        root = oracle.spline_root(sk, L, bfeat)
        want, nb = _brute_spline(sk, L, bfeat, range(domain), domain)
        assert root["nb"] == nb
        assert np.array_equal(oracle.spline_leaves(root, np.arange(domain, dtype=np.uint64)), want)


@pytest.mark.parametrize("bfeat", [1, 2])
def test_spline_partition_invariants(bfeat):
    """On lognormal-mixture keys (n = 2^18) and uniform keys: the leaf is
    non-decreasing over build keys and over arbitrary keys between them; each
    bin's keys stay inside the leaves it owns, [floor(r_b L / n),
    floor(r_(b+1) L / n)), so the leaf of the key at rank i is at most
    floor(i L / n) + the bins it shares; and the largest leaf is within a small
    factor of n / L where the bins resolve the distribution."""
    for kind in ("lognormal", "uniform"):
        if kind == "lognormal":
            keys, _ = gen.lognormal_keys(7, 1 << 18)
        else:
            keys, _ = gen.unique_keys(7, 1 << 18, 64, 63)
        sk = np.sort(keys)
        n = len(sk)
        for L in (1 << 10, 1 << 12):
            root = oracle.spline_root(sk, L, bfeat)
            leaf = oracle.spline_leaves(root, sk)
            assert leaf[0] == 0 and int(leaf.max()) <= L - 1
            assert np.all(np.diff(leaf.astype(np.int64)) >= 0)
            rng = np.random.default_rng(L)
            q = np.sort(np.concatenate([sk - np.uint64(1), sk + np.uint64(1), rng.integers(0, 1 << 63, 5000,
                                                                                          dtype=np.uint64),
                                        np.array([0, (1 << 64) - 1], dtype=np.uint64)]))
            ql = oracle.spline_leaves(root, q)
            assert np.all(np.diff(ql.astype(np.int64)) >= 0)
            # rank-proportional: the first key of leaf l has rank within one
            # bin's keys of l n / L
            sizes = np.bincount(leaf, minlength=L)
            starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
            ideal = np.arange(L) * n / L
            if kind == "uniform" or bfeat == 2:
                assert sizes.max() <= 4 * n / L, (kind, bfeat, L, sizes.max())
                assert np.max(np.abs(starts[sizes > 0] - ideal[sizes > 0])) <= 4 * n / L

"""Pins of the oracle's learned-model functions: the gradient and Hessian it
reports are checked against central finite differences of its loss, and
against numpy's least-squares solver (where the gradient must vanish); the
root feature and leaf assignment against their defining properties."""
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

def test_spline_segments_rule():
    """The largest power of two G <= 4096 with G * 64 <= n and G * 8 <= L."""
    big = 1 << 30
    assert [oracle.spline_segments(n, big) for n in (1, 127, 128, 255, 256, 64 * 4096, 1 << 40)] == [1, 1, 2, 2, 4,
                                                                                                      4096, 4096]
    assert [oracle.spline_segments(big, L) for L in (1, 15, 16, 1000, 8 * 4096, 1 << 22)] == [1, 1, 2, 64, 4096,
                                                                                              4096]


def test_spline_leaves_pins():
    """Knot keys land on the first leaf of their segment, the key list maps
    monotonically onto [0, L), keys below the first knot go to leaf 0 and keys
    above the last to L - 1, and evenly spaced keys fill every leaf with
    n / L keys up to rounding."""
    n, L = 1 << 16, 1000
    sk = np.arange(1, n + 1, dtype=np.uint64) * np.uint64(977)
    G = oracle.spline_segments(n, L)
    leaf = oracle.spline_leaves(sk, L, G)
    assert leaf[0] == 0 and leaf[-1] == L - 1
    assert np.all(np.diff(leaf.astype(np.int64)) >= 0)
    sizes = np.bincount(leaf, minlength=L)
    # each segment holds n / G keys over floor or ceil of L / G (>= 8) leaves
    per = n / L
    assert sizes.min() >= per * (1 - 1 / 8) - 1 and sizes.max() <= per * (1 + 1 / 8) + 1
    knot_ranks = (np.arange(G + 1, dtype=np.uint64) * np.uint64(n - 1)) // np.uint64(G)
    first = (np.arange(G, dtype=np.uint64) * np.uint64(L)) // np.uint64(G)
    assert np.array_equal(leaf[knot_ranks[:-1]], first.astype(np.uint32))
    out = oracle.spline_leaves(sk, L, G, np.array([0, 976, sk[-1] + 1, (1 << 64) - 1], dtype=np.uint64))
    assert list(out) == [0, 0, L - 1, L - 1]


def test_spline_leaves_match_brute_force():
    """Against the definition evaluated with numpy's float32 arithmetic, key
    by key, on clustered keys with repeated knots."""
    rng = np.random.default_rng(5)
    sk = np.sort(np.concatenate([rng.integers(0, 1000, 3000), rng.integers(10 ** 12, 10 ** 12 + 50, 2000),
                                 rng.integers(1 << 60, 1 << 61, 3000)]).astype(np.uint64))
    n, L = len(sk), 333
    G = oracle.spline_segments(n, L)
    got = oracle.spline_leaves(sk, L, G)
    knots = sk[(np.arange(G + 1, dtype=np.uint64) * np.uint64(n - 1)) // np.uint64(G)]
    want = np.empty(n, dtype=np.uint32)
    for i, k in enumerate(sk):
        j = int(np.searchsorted(knots, k, side="right")) - 1
        if j >= G:
            want[i] = L - 1
            continue
        f0, f1 = (j * L) // G, ((j + 1) * L) // G
        if f1 == f0:
            want[i] = min(f0, L - 1)
            continue
        gap = int(knots[j + 1]) - int(knots[j])
        s = np.float32(f1 - f0) / np.float32(gap)
        f = np.float32(np.float32(int(k) - int(knots[j])) * s)
        want[i] = f0 + (int(f) if f < np.float32(f1 - f0) else f1 - f0 - 1)
    assert np.array_equal(got, want)

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

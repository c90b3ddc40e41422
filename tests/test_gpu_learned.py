"""GPU tests of the learned rank model: lookups through the model are
bit-exact against the oracle; the training kernels' loss, gradient and
Hessian sums match the oracle's double-precision definitions; training lands
on the least-squares fit; the model narrows the search far below plain
binary search."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import rows_host, to_dev, to_host

pytestmark = pytest.mark.gpu

idx = pytest.importorskip("paper_2506_01576_amd")

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

AUTO, LINEAR, LOG, SPLINE = idx.IDX_FEATURE_AUTO, idx.IDX_FEATURE_LINEAR, idx.IDX_FEATURE_LOG, idx.IDX_FEATURE_SPLINE


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def make(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform32":
        keys, _ = gen.unique_keys(seed, n, 32)
    elif kind == "uniform64":
        keys, _ = gen.unique_keys(seed, n, 64, 63)
    elif kind == "lognormal":
        keys, _ = gen.lognormal_keys(seed, n)
    elif kind == "dup":
        keys = rng.integers(0, max(1, n // 5), size=n, dtype=np.uint64)
    else:
        raise ValueError(kind)
    rows = (rng.permutation(n).astype(np.uint64) * 5 + 3).astype(np.uint32)
    return keys, rows


def oracle_leaves(sk, st, L):
    """The oracle's leaf of every sorted key under the trained root described
    by the model statistics st (linear root or spline)."""
    if st["feature"] == SPLINE:
        root = oracle.spline_root(sk, L, st["bin_feature"])
        assert root["nb"] == st["segments"]
        return oracle.spline_leaves(root, sk)
    return oracle.assign_leaves(sk, st["feature"], st["root_a0"], st["root_a1"], L)[0]


def queries(keys, m, seed):
    rng = np.random.default_rng(seed)
    dt = keys.dtype
    top = int(np.iinfo(dt).max)
    lo, hi = int(keys.min()), int(keys.max())
    q = np.concatenate([keys[rng.integers(0, len(keys), m // 2)],
                        rng.integers(0, top, size=m // 4, dtype=np.uint64, endpoint=True).astype(dt),
                        (keys[rng.integers(0, len(keys), m // 4)].astype(np.uint64) + 1).astype(dt),
                        np.array([0, top, lo, hi, max(lo - 1, 0), min(hi + 1, top)], dtype=np.uint64).astype(dt)])
    return q.astype(dt)


@pytest.mark.parametrize("aos", [False, True, "padded"])
@pytest.mark.parametrize("kind", ["uniform32", "uniform64", "lognormal", "dup"])
@pytest.mark.parametrize("leaves,epochs,feature", [(1, 1, AUTO), (7, 2, LINEAR), (4096, 2, AUTO), (4096, 1, LOG),
                                                   (65536, 2, AUTO), (4096, 2, SPLINE), (100, 1, SPLINE)])
def test_learned_lookup_parity(kind, leaves, epochs, feature, aos):
    """The model on the sorted array in each storage (SoA, AoS, line-padded
    AoS): points, ranges and the answers without the model equal the oracle's."""
    n = 50021
    keys, rows = make(kind, n, seed=leaves + epochs)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 20011, seed=7)
    want = oracle.point(sk, sr, q, nthreads=4)
    bits = keys.dtype.itemsize * 8
    say(f"learned {kind} leaves={leaves} epochs={epochs} feature={feature} aos={aos}")
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as ix:
        st = ix.learn(leaves, epochs, feature)
        assert st["leaves"] == leaves and st["mean_window"] >= 1 and st["max_window"] <= n + 1
        for R in (1, 4, 8):
            ix.set_params(per_lane=R)
            got = rows_host(ix.point(to_dev(q)))
            bad = np.nonzero(got != want)[0]
            assert len(bad) == 0, f"R={R}: {len(bad)} mismatches, first q={q[bad[0]]}"
        # the bound invariant: every build key's rank lies inside its leaf's
        # window, shown by looking up all n build keys (a window that missed
        # a key's lower-bound rank would answer a miss or another row ID)
        all_want = oracle.point(sk, sr, keys, nthreads=4)
        all_got = rows_host(ix.point(to_dev(keys)))
        bad = np.nonzero(all_got != all_want)[0]
        assert len(bad) == 0, f"{len(bad)} build keys not found through the model, first {keys[bad[0]]}"
        # ranges through the model
        L, U, _ = gen.ranges(3, keys, 3001, 1, 64)
        L = np.concatenate([L, q[:500]]).astype(keys.dtype)
        U = np.concatenate([U, np.maximum(q[:500], q[500:1000])]).astype(keys.dtype)
        woff, wrows = oracle.range_lookup(sk, sr, L, U, nthreads=4)
        off, rr = ix.range(to_dev(L), to_dev(U))
        assert np.array_equal(off.cpu().numpy().view(np.uint64), woff)
        assert np.array_equal(rows_host(rr), wrows)
        # dropping the model gives the same answers through plain search
        ix.set_params(model=2)
        assert np.array_equal(rows_host(ix.point(to_dev(q))), want)
        ix.set_params(model=0)
        ix.unlearn()
        assert np.array_equal(rows_host(ix.point(to_dev(q))), want)


def test_learned_tiny_sets():
    for n in (1, 2, 3, 17):
        keys, rows = make("uniform64", n, seed=n)
        sk, sr = oracle.stable_sort(keys, rows)
        q = queries(keys, 64, seed=n)
        for aos in (False, "padded"):
            with idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as ix:
                ix.learn(16, 2, AUTO)
                assert np.array_equal(rows_host(ix.point(to_dev(q))), oracle.point(sk, sr, q))
                assert np.array_equal(rows_host(ix.point(to_dev(keys))), oracle.point(sk, sr, keys))


@pytest.mark.parametrize("aos", [True, "padded"])
def test_learned_aos_same_model_as_soa(aos):
    """Training reads the keys through the layout's accessor: the model on an
    AoS copy of the sorted array is the SoA model up to the order of FP64
    atomic additions (same feature, same weights to FP32 rounding, the
    oracle's leaf partition under its own root)."""
    n = 1 << 17
    keys, rows = make("lognormal", n, seed=4)
    sk, _ = oracle.stable_sort(keys, rows)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as a, \
            idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as b:
        sa, sb = a.learn(2048, 2), b.learn(2048, 2)
        assert sa["feature"] == sb["feature"]
        assert sb["root_a1"] == pytest.approx(sa["root_a1"], rel=1e-5)
        assert sb["mean_window"] == pytest.approx(sa["mean_window"], rel=1e-2)
        tb = b.learn_export().cpu().numpy().view(np.uint8).reshape(2048, 32)
        leaf = oracle_leaves(sk, sb, 2048)
        _, _, base, size = oracle.leaf_frame(sk, leaf, 2048)
        assert np.array_equal(tb[:, 8:12].copy().view(np.uint32).ravel(), base.astype(np.uint32))
        assert np.array_equal(tb[:, 12:16].copy().view(np.uint32).ravel(), size.astype(np.uint32))


def test_learn_rejects_other_layouts():
    keys, rows = make("uniform32", 1000, seed=1)
    with idx.Index(to_dev(keys), to_dev(rows), layout="eks", k=9) as ix:
        with pytest.raises(idx.IdxError):
            ix.learn(64)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        for bad in ((0, 2, AUTO), ((1 << 26) + 1, 2, AUTO), (64, 0, AUTO), (64, 2, 4)):
            with pytest.raises(idx.IdxError):
                ix.learn(*bad)


def _sums_from_oracle_root(x, t, a0, a1):
    loss, grad, hess = oracle.root_grad(x.astype(np.float64), t, np.array([a1, a0], dtype=np.float64))
    # N, Sx, Sxx, Sr, Srx, Srr
    return np.array([hess[2] / 2, hess[1] / 2, hess[0] / 2, grad[1] / 2, grad[0] / 2, loss])


@pytest.mark.parametrize("kind,mode", [("lognormal", LOG), ("uniform64", LINEAR), ("uniform32", LOG)])
def test_training_kernel_sums_match_oracle(kind, mode):
    n, L = 1 << 16, 64
    keys, rows = make(kind, n, seed=11)
    sk, _ = oracle.stable_sort(keys, rows)
    leaf0, x0 = oracle.assign_leaves(sk, mode, 0.0, 1.0, 1)
    t = np.arange(n, dtype=np.float64) * L / n
    A = np.stack([x0.astype(np.float64), np.ones(n)], axis=1)
    (a1, a0), *_ = np.linalg.lstsq(A, t, rcond=None)
    a0, a1 = float(np.float32(a0 + 0.37)), float(np.float32(max(a1, 0.0) * 1.01))
    leaf, x = oracle.assign_leaves(sk, mode, a0, a1, L)
    d, y, base, size = oracle.leaf_frame(sk, leaf, L)
    rng = np.random.default_rng(5)
    leaf_ab = np.zeros(2 * L, dtype=np.float32)
    for l in range(L):
        sel = leaf == l
        if sel.sum() >= 2:
            (b1, b0), *_ = np.linalg.lstsq(np.stack([d[sel], np.ones(sel.sum())], 1), y[sel], rcond=None)
            leaf_ab[2 * l], leaf_ab[2 * l + 1] = np.float32(b0 + rng.normal(0, 3)), np.float32(max(b1, 0) * 1.02)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        racc, lacc = ix.learn_eval(mode, (a0, a1), L, torch.from_numpy(leaf_ab).cuda())
    racc = np.array(racc)
    lacc = lacc.cpu().numpy()
    # the integer decisions (which leaf each key falls in) agree exactly
    assert np.array_equal(lacc[:, 0].astype(np.int64), np.bincount(leaf, minlength=L))
    # root: feature sums exact up to summation order; residual sums within the
    # FP32 rounding of the forward pass (|dr| <= 2 ulp of the larger operand)
    want = _sums_from_oracle_root(x, t, a0, a1)
    eps = 2.0 ** -23
    mag = np.abs(a1 * x.astype(np.float64)) + abs(a0) + np.abs(t)
    r = a1 * x.astype(np.float64) + a0 - t
    tol = np.array([0, 1e-9 * want[1], 1e-9 * want[2], 3 * eps * mag.sum(),
                    3 * eps * (mag * x).sum(), 6 * eps * (np.abs(r) * mag).sum() + 1e-9 * want[5]]) + 1e-6
    assert np.all(np.abs(racc - want) <= tol), (racc, want, tol)
    # leaves: oracle definition of loss / gradient / Hessian in FP64
    params = np.empty(2 * L)
    params[0::2] = leaf_ab[1::2]  # slope
    params[1::2] = leaf_ab[0::2]  # intercept
    loss, grad, hess = oracle.leaf_grad(d, y, leaf, params, L)
    magl = np.abs(params[2 * leaf] * d) + np.abs(params[2 * leaf + 1]) + np.abs(y)
    rl = params[2 * leaf] * d + params[2 * leaf + 1] - y
    tol_r = 3 * eps * np.bincount(leaf, weights=magl, minlength=L) + 1e-6
    tol_rx = 3 * eps * np.bincount(leaf, weights=magl * d, minlength=L) + 1e-6
    tol_rr = 6 * eps * np.bincount(leaf, weights=np.abs(rl) * magl, minlength=L) + 1e-9 * loss + 1e-6
    assert np.allclose(lacc[:, 2], hess[:, 0] / 2, rtol=1e-9, atol=1e-6)
    assert np.allclose(lacc[:, 1], hess[:, 1] / 2, rtol=1e-9, atol=1e-6)
    assert np.all(np.abs(lacc[:, 3] - grad[:, 1] / 2) <= tol_r)
    assert np.all(np.abs(lacc[:, 4] - grad[:, 0] / 2) <= tol_rx)
    assert np.all(np.abs(lacc[:, 5] - loss) <= tol_rr)


def test_training_reaches_least_squares():
    n, L = 1 << 18, 256
    keys, rows = make("lognormal", n, seed=21)
    sk, _ = oracle.stable_sort(keys, rows)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        st = ix.learn(L, 2, LOG)
        table = ix.learn_export().cpu().numpy()
    a0, a1 = st["root_a0"], st["root_a1"]
    leaf, x = oracle.assign_leaves(sk, LOG, a0, a1, 1)
    t = np.arange(n, dtype=np.float64) * L / n
    (w1, w0), *_ = np.linalg.lstsq(np.stack([x.astype(np.float64), np.ones(n)], 1), t, rcond=None)
    # the FP32 parameters equal the FP64 least-squares fit up to FP32 rounding
    # amplified by the fit's conditioning
    assert a1 == pytest.approx(w1, rel=2e-4)
    assert abs(a0 - w0) <= 2e-4 * (abs(w1) + abs(w0))
    leaf, _ = oracle.assign_leaves(sk, LOG, a0, a1, L)
    d, y, base, size = oracle.leaf_frame(sk, leaf, L)
    rec = table.view(np.uint8).reshape(L, 32)
    base_g = rec[:, 8:12].copy().view(np.uint32).ravel()
    size_g = rec[:, 12:16].copy().view(np.uint32).ravel()
    b0 = rec[:, 16:20].copy().view(np.float32).ravel()
    b1 = rec[:, 20:24].copy().view(np.float32).ravel()
    assert np.array_equal(base_g, base.astype(np.uint32)) and np.array_equal(size_g, size.astype(np.uint32))
    for l in np.nonzero(size >= 64)[0][:40]:
        sel = leaf == l
        (c1, c0), *_ = np.linalg.lstsq(np.stack([d[sel], np.ones(sel.sum())], 1), y[sel], rcond=None)
        span = d[sel].max()
        # predictions agree to a small fraction of the leaf size over the leaf
        assert abs((b1[l] - c1) * span) + abs(b0[l] - c0) <= 1e-3 * size[l] + 0.5


def test_model_narrows_the_search():
    """What the trained model gains over the search without it: the window a
    lookup searches shrinks from n keys to a few hundred, so binary search
    takes ~log2(window) instead of log2(n) steps, and lookups get faster."""
    n, m = 1 << 24, 1 << 24
    keys, rows = gen.unique_keys(31, n, 64, 63)
    q, expect = gen.point_queries(31, n, m, 1.0, 64, 63)
    dq, de = to_dev(q), to_dev(expect)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        out = torch.empty(m, dtype=torch.int32, device="cuda")

        def timed():
            ix.point(dq, out)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                ix.point(dq, out)
            b.record()
            b.synchronize()
            assert torch.equal(out, de)
            return a.elapsed_time(b) / 3

        t_plain = timed()
        st = ix.learn(1 << 16, 2, AUTO)
        t_model = timed()
    steps_plain = np.log2(n)
    steps_model = np.log2(st["mean_window"])
    say(f"plain {t_plain:.3f} ms, learned {t_model:.3f} ms, mean window {st['mean_window']:.1f}, "
        f"steps {steps_plain:.1f} -> {steps_model:.1f}")
    assert steps_model < steps_plain - 10
    assert t_model < t_plain


@pytest.mark.parametrize("kind", ["uniform64", "lognormal", "dup", "uniform32"])
@pytest.mark.parametrize("leaves", [1, 64, 5000, 1 << 15])
@pytest.mark.parametrize("aos", [False, True])
def test_spline_root_partition_matches_oracle(kind, leaves, aos):
    """The spline root's leaf partition (base rank and size of every leaf)
    equals the oracle's evaluation of the same definition over the bin feature
    the trainer kept, with the same number of bins; lookups stay exact."""
    n = 200003
    keys, rows = make(kind, n, seed=leaves)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 20000, leaves)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as ix:
        st = ix.learn(leaves, 2, SPLINE)
        assert st["feature"] == SPLINE and st["bin_feature"] in (LINEAR, LOG)
        table = ix.learn_export().cpu().numpy().view(np.uint8).reshape(leaves, 32)
        got = rows_host(ix.point(to_dev(q)))
    leaf = oracle_leaves(sk, st, leaves)
    _, _, base, size = oracle.leaf_frame(sk, leaf, leaves)
    assert np.array_equal(table[:, 12:16].copy().view(np.uint32).ravel(), size.astype(np.uint32))
    assert np.array_equal(table[:, 8:12].copy().view(np.uint32).ravel(), base.astype(np.uint32))
    assert np.array_equal(got, oracle.point(sk, sr, q, nthreads=4))


def test_spline_root_beyond_2p24_leaves():
    """A spline root with more than 2^24 leaves (the first-leaf field's upper
    bits): the leaf sizes and bases equal the oracle's evaluation of the same
    definition, and points (every build key, misses) and ranges through the
    model, with and without leaf lines, equal the oracle's answers."""
    n, leaves = 1 << 20, (1 << 25) + 3
    keys, rows = make("lognormal", n, seed=25)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 1 << 16, 26)
    L, U, _ = gen.ranges(27, keys, 4001, 1, 64)
    woff, wrows = oracle.range_lookup(sk, sr, L, U, nthreads=4)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        st = ix.learn(leaves, 1, SPLINE)
        words = ix.learn_export().view(torch.int32).reshape(leaves, 8)
        base_d, size_d = words[:, 2].cpu().numpy().view(np.uint32), words[:, 3].cpu().numpy().view(np.uint32)
        del words
        leaf = oracle_leaves(sk, st, leaves)
        assert int(leaf.max()) >= 1 << 24  # keys reach leaves beyond 2^24
        _, _, base, size = oracle.leaf_frame(sk, leaf, leaves)
        assert np.array_equal(size_d, size.astype(np.uint32))
        assert np.array_equal(base_d, base.astype(np.uint32))
        for lines in (2, 1):
            ix.set_params(leaf_lines=lines)
            assert np.array_equal(rows_host(ix.point(to_dev(q))), oracle.point(sk, sr, q, nthreads=4))
            assert np.array_equal(rows_host(ix.point(to_dev(keys))), oracle.point(sk, sr, keys, nthreads=4))
            off, rr = ix.range(to_dev(L), to_dev(U))
            assert np.array_equal(off.cpu().numpy().view(np.uint64), woff)
            assert np.array_equal(rows_host(rr), wrows)


def test_spline_root_gain_on_clustered_keys():
    """On the 64-cluster lognormal mixture a linear root leaves most leaves
    empty and a few huge; the spline root spreads the keys by rank, so the
    mean search window shrinks by far (the model's gain over the plain
    linear root), and AUTO keeps the spline."""
    n = 1 << 20
    keys, rows = make("lognormal", n, seed=3)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        lin = min(ix.learn(n // 64, 2, LINEAR)["mean_window"], ix.learn(n // 64, 2, LOG)["mean_window"])
        spl = ix.learn(n // 64, 2, SPLINE)["mean_window"]
        auto = ix.learn(n // 64, 2, AUTO)
    say(f"lognormal mean window: best linear root {lin:.1f}, spline {spl:.1f}, auto {auto['feature']}")
    assert spl * 10 < lin
    assert auto["feature"] == SPLINE and auto["mean_window"] == spl


def test_auto_keeps_linear_root_on_uniform_keys():
    """On uniform keys a linear root already gives the spline's windows, so
    AUTO keeps the root without the bin record (a tie keeps the linear root)."""
    n = 1 << 20
    keys, rows = make("uniform64", n, seed=4)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        lin = ix.learn(n // 64, 2, LINEAR)["mean_window"]
        spl = ix.learn(n // 64, 2, SPLINE)["mean_window"]
        auto = ix.learn(n // 64, 2, AUTO)
    say(f"uniform mean window: linear {lin:.2f}, spline {spl:.2f}, auto {auto['feature']}")
    assert np.log2(1 + lin) <= np.log2(1 + spl) + 1
    assert auto["feature"] == LINEAR and auto["segments"] == 0


@pytest.mark.parametrize("aos", [False, True])
@pytest.mark.parametrize("rounds", [1, 2])
def test_window_rounds_parity(aos, rounds):
    """Both short-window scan modes (whole window at once, or its first line
    first) give the oracle's answers for the learned form and plain BS, on
    uniform and duplicate-heavy keys; an unknown mode is refused."""
    for kind in ("uniform64", "dup"):
        n = 70001
        keys, rows = make(kind, n, seed=rounds + 10)
        sk, sr = oracle.stable_sort(keys, rows)
        q = queries(keys, 30000, 17 + rounds)
        want = oracle.point(sk, sr, q, nthreads=4)
        with idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as ix:
            ix.set_params(window_rounds=rounds, model=2)
            assert np.array_equal(rows_host(ix.point(to_dev(q))), want)
            ix.learn(n // 16, 2)
            for per_lane in (4, 8):
                ix.set_params(window_rounds=rounds, model=0, per_lane=per_lane)
                assert ix.params()["window_rounds"] == rounds
                assert np.array_equal(rows_host(ix.point(to_dev(q))), want)
            with pytest.raises(idx.IdxError):
                ix.set_params(window_rounds=3)


@pytest.mark.parametrize("aos", [False, True, "padded"])
@pytest.mark.parametrize("kind", ["uniform32", "uniform64", "lognormal", "dup"])
@pytest.mark.parametrize("per_leaf", [0.25, 3, 8, 40])
def test_leaf_lines_parity(kind, per_leaf, aos):
    """Lookups through the leaf lines (one 128-byte line per leaf holding its
    first keys; past them a larger leaf's rest is searched in the sorted
    array): point lookups of every build key and of misses, range counts and
    row IDs equal the oracle's in every storage and at every lookup count per
    lane; the lines follow a retrained model; leaf_lines = 2 returns to the
    window search."""
    n = 50021
    keys, rows = make(kind, n, seed=int(per_leaf * 4) + 1)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 20011, seed=int(per_leaf * 4) + 2)
    want = oracle.point(sk, sr, q, nthreads=4)
    all_want = oracle.point(sk, sr, keys, nthreads=4)
    L, U, _ = gen.ranges(5, keys, 3001, 1, 64)
    L = np.concatenate([L, q[:500]]).astype(keys.dtype)
    U = np.concatenate([U, np.maximum(q[:500], q[500:1000])]).astype(keys.dtype)
    woff, wrows = oracle.range_lookup(sk, sr, L, U, nthreads=4)
    cap = 10 if keys.dtype.itemsize == 8 else 15
    say(f"leaf lines {kind} per_leaf={per_leaf} aos={aos}")
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as ix:
        leaves = max(1, int(n / per_leaf))
        ix.learn(leaves, 2)
        sizes = ix.learn_export().cpu().numpy().view(np.uint8).reshape(leaves, 32)[:, 12:16].copy().view(np.uint32)
        say(f"  leaves {leaves}: within a line {int((sizes <= cap).sum())}, larger {int((sizes > cap).sum())}")
        if per_leaf == 8:  # both kinds of leaf
            assert (sizes <= cap).any() and (sizes > cap).any()
        # lookups per lane pair; partitioned batches (answers placed back or
        # written in place); locally sorted tiles (one lane per line);
        # workgroup sizes and persistent grids
        for R, reorder, block, persistent in [(1, 0, 256, 0), (2, 0, 256, 0), (4, 0, 256, 0), (8, 0, 256, 0),
                                              (4, 0, 64, 0), (4, 0, 1024, 0), (2, 0, 256, 3), (1, 1, 256, 0),
                                              (4, 1, 128, 0), (4, 2, 256, 0), (4, 3, 256, 0), (2, 3, 128, 2)]:
            ix.set_params(per_lane=R, leaf_lines=1, reorder=reorder, block=block, persistent=persistent)
            got = rows_host(ix.point(to_dev(q)))
            bad = np.nonzero(got != want)[0]
            assert len(bad) == 0, f"R={R} reorder={reorder} block={block}: {len(bad)} mismatches, first q={q[bad[0]]}"
        ix.set_params(per_lane=4, leaf_lines=1)
        assert ix.params()["leaf_lines"] == 1
        all_got = rows_host(ix.point(to_dev(keys)))
        bad = np.nonzero(all_got != all_want)[0]
        assert len(bad) == 0, f"{len(bad)} build keys not found through the lines, first {keys[bad[0]]}"
        off, rr = ix.range(to_dev(L), to_dev(U))
        assert np.array_equal(off.cpu().numpy().view(np.uint64), woff)
        assert np.array_equal(rows_host(rr), wrows)
        # a retrained model gets new lines
        ix.learn(max(1, leaves // 3), 2)
        assert np.array_equal(rows_host(ix.point(to_dev(q))), want)
        assert np.array_equal(rows_host(ix.point(to_dev(keys))), all_want)
        ix.set_params(leaf_lines=2)
        assert np.array_equal(rows_host(ix.point(to_dev(q))), want)
        off, rr = ix.range(to_dev(L), to_dev(U))
        assert np.array_equal(off.cpu().numpy().view(np.uint64), woff)
        with pytest.raises(idx.IdxError):
            ix.set_params(leaf_lines=3)


def test_leaf_lines_tiny_sets_and_max_leaves():
    """Leaf lines on sets of 1 to 17 keys, and a model with the largest leaf
    count (2^24 leaves over 2^18 keys: almost every line empty)."""
    for n in (1, 2, 3, 17):
        keys, rows = make("uniform64", n, seed=n + 40)
        sk, sr = oracle.stable_sort(keys, rows)
        q = queries(keys, 64, seed=n)
        with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
            ix.learn(16, 2, AUTO)
            for reorder in (0, 1):
                ix.set_params(leaf_lines=1, reorder=reorder)
                assert np.array_equal(rows_host(ix.point(to_dev(q))), oracle.point(sk, sr, q))
                assert np.array_equal(rows_host(ix.point(to_dev(keys))), oracle.point(sk, sr, keys))
    n = 1 << 18
    keys, rows = make("uniform32", n, seed=77)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 1 << 16, seed=78)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        ix.set_params(leaf_lines=1)  # the lines are written by the training call
        ix.learn(1 << 24, 1, AUTO)
        assert np.array_equal(rows_host(ix.point(to_dev(q))), oracle.point(sk, sr, q, nthreads=4))
        assert np.array_equal(rows_host(ix.point(to_dev(keys))), oracle.point(sk, sr, keys, nthreads=4))


def test_leaf_lines_after_retraining():
    """Re-training a model with leaf lines reuses the previous lines' buffer
    when the leaf count is the same, and takes a new one otherwise: every
    lookup equals the oracle's after each training, after dropping the model
    and training again, and for ranges through the reused lines."""
    n = 200003
    keys, rows = make("lognormal", n, seed=91)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 50000, seed=92)
    want, want_keys = oracle.point(sk, sr, q), oracle.point(sk, sr, keys)
    lo, hi, _ = gen.ranges(93, keys, 4000, 1, 40)
    want_off, want_rows = oracle.range_lookup(sk, sr, lo, hi)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        ix.set_params(leaf_lines=1)
        for step, L in enumerate((n // 4, n // 4, n // 2, n // 2, 4096)):
            if step == 3:
                ix.unlearn()
            ix.learn(L, 2, AUTO)
            say(f"re-training step {step}: {L} leaves")
            assert np.array_equal(rows_host(ix.point(to_dev(q))), want), (step, L)
            assert np.array_equal(rows_host(ix.point(to_dev(keys))), want_keys), (step, L)
            off, got = ix.range(to_dev(lo), to_dev(hi))
            assert np.array_equal(off.cpu().numpy().view(np.uint64), want_off), (step, L)
            assert np.array_equal(rows_host(got), want_rows), (step, L)

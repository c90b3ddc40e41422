"""GPU parity on the skew and duplicate workloads (Sections 8.9 and 8.11):
Zipf-popular and sorted point batches through every form and lookup
reordering mode, and equality ranges over keys replicated up to hundreds of
times (each level then holds many matches, so the Eytzinger scans hand over
to whole waves)."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import rows_host, to_dev

pytestmark = pytest.mark.gpu

idx = pytest.importorskip("paper_2506_01576_amd")

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


FORMS = [("bs", 1, {}), ("bs", 1, {"reorder": 2}), ("ebs", 2, {}), ("ebs", 2, {"reorder": 1}),
         ("eks", 9, {"group": 1}), ("eks", 9, {"group": 8}), ("eks", 9, {"group": 4}),
         ("eks", 17, {"group": 1, "reorder": 2}), ("learned", 1, {}), ("learned", 1, {"reorder": 1})]


def make(keys, rows, layout, k):
    if layout == "learned":
        ix = idx.Index(to_dev(keys), to_dev(rows), layout="bs")
        ix.learn(max(1, len(keys) // 32), 2)
        return ix
    return idx.Index(to_dev(keys), to_dev(rows), layout=layout, k=k)


@pytest.mark.parametrize("case", ["zipf1.25", "zipf2", "sorted"])
def test_skewed_and_sorted_points(case):
    n, m = (1 << 20) + 7, (1 << 18) + 3
    seed = gen.BASE_SEED + 60
    keys, rows = gen.unique_keys(seed, n, 64, 63)
    if case == "sorted":
        q, e = gen.point_queries(seed, n, m, 0.8, 64, 63)
        order = np.argsort(q, kind="stable")
        q, e = q[order], e[order]
    else:
        q, e = gen.zipf_queries(seed, 1.25 if case == "zipf1.25" else 2.0, n, m, 0.1, 64, 63)
    sk, sr = oracle.stable_sort(keys, rows)
    sample = np.random.default_rng(1).integers(0, m, 2048)
    want_s = oracle.point(sk, sr, q[sample], nthreads=4)
    hit = e != 0xFFFFFFFF
    for layout, k, params in FORMS:
        with make(keys, rows, layout, k) as ix:
            ix.set_params(**params)
            say(f"{case} {layout} k={k} {params}")
            got = rows_host(ix.point(to_dev(q)))
            assert np.array_equal(got[hit], e[hit])
            assert np.array_equal(got[sample], want_s)


@pytest.mark.parametrize("r", [1, 7, 64, 300])
def test_replicated_equality_ranges(r):
    distinct = 2000
    seed = gen.BASE_SEED + 61
    vals, _ = gen.unique_keys(seed + r, distinct, 64, 63)
    rng = np.random.default_rng(r)
    keys = np.repeat(vals, r)
    perm = rng.permutation(len(keys))
    keys = keys[perm]
    rows = (perm.astype(np.uint64) * 3 + 1).astype(np.uint32)
    q = np.concatenate([vals, vals[rng.integers(0, distinct, 3000)], rng.integers(0, 1 << 63, 500, dtype=np.uint64)])
    sk, sr = oracle.stable_sort(keys, rows)
    woff, wrows = oracle.range_lookup(sk, sr, q, q, nthreads=4)
    wpt = oracle.point(sk, sr, q, nthreads=4)
    for layout, k, params in [f for f in FORMS if "reorder" not in f[2]] + [("eks", 33, {"group": 1})]:
        with make(keys, rows, layout, k) as ix:
            ix.set_params(**params)
            say(f"replicas r={r} {layout} k={k} {params}")
            off, rr = ix.range(to_dev(q), to_dev(q))
            assert np.array_equal(off.cpu().numpy().view(np.uint64), woff)
            assert np.array_equal(rows_host(rr), wrows)
            # a point lookup returns the first replica in input order
            assert np.array_equal(rows_host(ix.point(to_dev(q))), wpt)

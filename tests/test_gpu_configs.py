"""Parity at the benchmark configurations' full sizes, in the launch
configurations the benchmark times (the tuned table).  Where the oracle
cannot answer every query in seconds, all answers are checked against the
generator's answers (known by construction) and a sample against the
oracle's plain definition."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import rows_host, to_dev

pytestmark = pytest.mark.gpu

idx = pytest.importorskip("paper_2506_01576_amd")

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2506_01576_amd import autotune  # noqa: E402

MISS = 0xFFFFFFFF


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_small_u32_full():
    """2^16 unique u32 keys, 2^20 lookups with 50% misses: every answer
    against the oracle, for every tuned form."""
    n, m = 1 << 16, 1 << 20
    seed = gen.BASE_SEED
    keys, rows = gen.unique_keys(seed, n, 32)
    q, expect = gen.point_queries(seed, n, m, 0.5, 32)
    sk, sr = oracle.stable_sort(keys, rows)
    want = oracle.point(sk, sr, q, nthreads=8)
    assert np.array_equal(want, expect)
    dq = to_dev(q)
    with idx.Index(to_dev(keys), to_dev(rows), "bs") as base:
        for layout in ("bs", "ebs", "eks"):
            lay, k, aos, params = autotune.choose(n, 32, layout)
            ix = base if (lay == "bs" and not aos) else base.relayout(lay, k, aos)
            ix.set_params(**params)
            say(f"small u32 {lay} k={k} aos={aos} {params}")
            assert np.array_equal(rows_host(ix.point(dq)), want)
            if ix is not base:
                ix.close()
            else:
                ix.reset_params()
        base.learn(1024, 2)
        assert np.array_equal(rows_host(base.point(dq)), want)


@pytest.fixture(scope="module")
def big_u64():
    n, m = 1 << 26, 1 << 27
    seed = gen.BASE_SEED + 1
    keys, rows = gen.unique_keys(seed, n, 64, 63)
    q, expect = gen.point_queries(seed, n, m, 1.0, 64, 63)
    return keys, rows, q, expect


def test_full_scale_u64_points(big_u64):
    """n = 2^26 u64, 2^27 uniform hits: all answers equal the generator's
    (query f(i) -> rowid i) for BS, EBS, EKS and learned in their tuned
    launch configurations; 4096 sampled answers equal the oracle's."""
    keys, rows, q, expect = big_u64
    n = len(keys)
    dq, de = to_dev(q), to_dev(expect)
    rng = np.random.default_rng(1)
    sample = rng.integers(0, len(q), 4096)
    sk, sr = oracle.stable_sort(keys, rows)
    want_s = oracle.point(sk, sr, q[sample], nthreads=8)
    out = torch.empty(len(q), dtype=torch.int32, device="cuda")
    with idx.Index(to_dev(keys), to_dev(rows), "bs") as base:
        for layout in ("bs", "ebs", "eks", "learned"):
            lay, k, aos, params = autotune.choose(n, 64, layout)
            say(f"full u64 {lay} k={k} aos={aos} {params}")
            if lay == "learned":
                base.learn(params.pop("leaves", 1 << 20), 2)
                ix = base
                params["model"] = 0
            else:
                ix = base if (lay == "bs" and not aos) else base.relayout(lay, k, aos)
                params["model"] = 2
            ix.set_params(**{kk: v for kk, v in params.items() if kk != "leaves"})
            ix.point(dq, out)
            torch.cuda.synchronize()
            assert torch.equal(out, de)
            assert np.array_equal(rows_host(out[torch.from_numpy(sample).cuda()]), want_s)
            if ix is not base:
                ix.close()


def test_full_scale_u64_ranges(big_u64):
    """2^24 ranges of 16 consecutive keys: every count is 16; sampled
    queries' rowids equal the oracle's, in key order."""
    keys, rows, _, _ = big_u64
    mr = 1 << 24
    lo, hi, c = gen.ranges(gen.BASE_SEED + 1, keys, mr, 16, 16)
    sk, sr = oracle.stable_sort(keys, rows)
    rng = np.random.default_rng(2)
    sample = rng.integers(0, mr, 2048)
    woff, wrows = oracle.range_lookup(sk, sr, lo[sample], hi[sample], nthreads=8)
    dlo, dhi = to_dev(lo), to_dev(hi)
    with idx.Index(to_dev(keys), to_dev(rows), "bs") as base:
        for layout in ("bs", "eks", "learned"):
            lay, k, aos, params = autotune.choose(len(keys), 64, layout)
            if lay == "learned":
                base.learn(params.get("leaves", 1 << 20), 2)
                ix = base
            else:
                ix = base if (lay == "bs" and not aos) else base.relayout(lay, k, aos)
                if lay == "bs":
                    base.set_params(model=2)
            say(f"full ranges {lay} k={k}")
            off, rr = ix.range(dlo, dhi, capacity=mr * 16)
            offh = off.cpu().numpy().view(np.uint64)
            assert np.all(np.diff(offh) == 16)
            rrh = rows_host(rr)
            for j, s in enumerate(sample[:256]):
                assert np.array_equal(rrh[offh[s]:offh[s + 1]], wrows[woff[j]:woff[j + 1]])
            if ix is not base:
                ix.close()


def test_lognormal_zipf_learned_vs_eks():
    """2^28 unique u64 keys from the 64-cluster lognormal mixture; 2^27 lookups,
    Zipf(1.1) hits plus 10% uniform misses.  The learned model (4096 leaves)
    and EKS k=16 both answer every hit with the generator's rowid and agree on
    every miss; 64 sampled misses are confirmed absent by a linear scan."""
    n, m = 1 << 28, 1 << 27
    seed = gen.BASE_SEED + 3
    keys, rows = gen.lognormal_keys(seed, n)
    q, expect = gen.zipf_queries(seed, 1.1, n, m, 0.1, 64, 63, keys=keys)
    dq = to_dev(q)
    de = to_dev(expect)
    hit = de != -1
    with idx.Index(to_dev(keys), to_dev(rows), "bs") as base:
        st = base.learn(4096, 2)
        say(f"lognormal learned: {st}")
        a = base.point(dq)
        with base.relayout("eks", 16) as eks:
            b = eks.point(dq)
        torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(a[hit], de[hit])
    miss_idx = torch.nonzero(~hit).flatten()[:64].cpu().numpy()
    for j in miss_idx:
        present = bool((keys == q[j]).any())
        assert (rows_host(a[j:j + 1])[0] == MISS) == (not present)


def test_batched_1024_indexes():
    """1024 uneven u32 indexes (n log-uniform in [2^6, 2^20]) in their tuned
    batch forms, point batches log-uniform in [1, 2^14], 80% hits: the one
    launch equals the generator's answers and the per-index launch loop."""
    count = 1024
    seed = gen.BASE_SEED + 2
    sizes = gen.log_uniform(seed, 11, 1 << 6, 1 << 20, count)
    qcounts = gen.log_uniform(seed, 12, 1, 1 << 14, count)
    idxs, qs, ex = [], [], []
    for j in range(count):
        n = int(sizes[j])
        kh, rh = gen.unique_keys(seed * 7 + j, n, 32)
        qh, eh = gen.point_queries(seed * 7 + j, n, int(qcounts[j]), 0.8, 32)
        idxs.append(autotune.build_form(to_dev(kh), to_dev(rh), autotune.batch_form(n, 32)))
        qs.append(qh)
        ex.append(eh)
    off = np.zeros(count + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(x) for x in qs])
    dq, de, doff = to_dev(np.concatenate(qs)), to_dev(np.concatenate(ex)), to_dev(off)
    with idx.Batch(idxs) as bt:
        got = bt.point(dq, doff)
        g2 = bt.point(dq, doff, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(got, de) and torch.equal(g2, de)
    loop = torch.empty_like(got)
    for j, ix in enumerate(idxs):
        a, b = int(off[j]), int(off[j + 1])
        if b > a:
            ix.point(dq[a:b], loop[a:b])
    torch.cuda.synchronize()
    assert torch.equal(loop, de)
    for ix in idxs:
        ix.close()

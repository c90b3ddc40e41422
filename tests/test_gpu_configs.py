"""Parity at the benchmark configurations' full sizes, in the launch
configurations the benchmark times (the tuned table).  Where the oracle
cannot answer every query in seconds, all answers are checked against the
generator's answers (known by construction) and a sample against the
oracle's plain definition."""
import os
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

from paper_2506_01576_amd import autotune  # noqa: E402

MISS = 0xFFFFFFFF
# host threads for the oracle at full sizes: the GPU machine's CPU share
CPU_THREADS = max(1, min(16, os.cpu_count() or 1))


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
    """2^24 ranges of 16 consecutive keys: every count is 16 and every row ID
    of every range equals the oracle's, in key order (the oracle's first
    rank of each range, then its 16 stable-sorted row IDs from there)."""
    keys, rows, _, _ = big_u64
    mr = 1 << 24
    lo, hi, c = gen.ranges(gen.BASE_SEED + 1, keys, mr, 16, 16)
    sk, sr = oracle.stable_sort(keys, rows)
    first, cnt = oracle.range_count(sk, lo, hi, nthreads=CPU_THREADS)
    assert np.all(cnt == 16)
    want = sr[first[:, None] + np.arange(16, dtype=np.uint64)[None, :]].reshape(-1)
    del first, cnt
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
            bad = np.nonzero(rrh != want)[0]
            assert len(bad) == 0, f"{lay}: {len(bad)} row IDs differ, first in range {bad[0] // 16}"
            del rrh, rr, off
            if ix is not base:
                ix.close()


def test_lognormal_zipf_learned_vs_eks():
    """2^28 unique u64 keys from the 64-cluster lognormal mixture; 2^27 lookups,
    Zipf(1.1) hits plus 10% uniform misses.  Every answer of the learned model
    (4096 leaves, and the tuned 2^22 leaves) and of EKS k=16 equals the
    oracle's (lower bound and equality on the oracle's stable sort of all
    2^28 keys), hits and misses alike; the hits also equal the generator's."""
    n, m = 1 << 28, 1 << 27
    seed = gen.BASE_SEED + 3
    keys, rows = gen.lognormal_keys(seed, n)
    q, expect = gen.zipf_queries(seed, 1.1, n, m, 0.1, 64, 63, keys=keys)
    say("lognormal: oracle sort and lookups")
    sk, sr = oracle.stable_sort(keys, rows)
    want = oracle.point(sk, sr, q, nthreads=CPU_THREADS)
    del sk, sr
    hit_h = expect != MISS
    assert np.array_equal(want[hit_h], expect[hit_h])
    dq = to_dev(q)
    with idx.Index(to_dev(keys), to_dev(rows), "bs") as base:
        for leaves in (4096, 1 << 22):
            st = base.learn(leaves, 2)
            say(f"lognormal learned: {st}")
            got = rows_host(base.point(dq))
            bad = np.nonzero(got != want)[0]
            assert len(bad) == 0, f"learned {leaves}: {len(bad)} answers differ, first query {q[bad[0]]}"
        base.unlearn()
        with base.relayout("eks", 16) as eks:
            got = rows_host(eks.point(dq))
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, f"EKS k=16: {len(bad)} answers differ"


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


def combined_keys(seed, j, n):
    """Keys of index j of the combined workload: uniform in [0, 2^63) for even
    j, the 64-cluster lognormal mixture for odd j."""
    if j % 2 == 0:
        return gen.unique_keys(seed * 1009 + j, n, 64, 63)
    return gen.lognormal_keys(seed * 1009 + j, n)


@pytest.mark.timeout(900)
def test_combined_full_shape():
    """The combined configuration at its full shape: 1024 u64 indexes with n
    log-uniform in [2^16, 2^24] (half uniform, half lognormal keys), their
    models trained by one batched launch sequence, and a mixed stream of 2^26
    lookups (70% points with 10% misses, 30% ranges of 1-256 matches) in one
    persistent launch pair.  Every answer of 32 indexes spread over the size
    range equals the oracle's; every answer of all 1024 equals the same
    stream through plain EKS (k = 17)."""
    count, m_total = 1024, 1 << 26
    seed = gen.BASE_SEED + 4
    sizes = gen.log_uniform(seed, 1, 1 << 16, 1 << 24, count).astype(np.int64)
    per = np.full(count, m_total // count, dtype=np.int64)
    ixs, los, his, kinds = [], [], [], []
    for j in range(count):
        kh, rh = combined_keys(seed, j, int(sizes[j]))
        dk = to_dev(kh)
        ixs.append(idx.Index(dk, to_dev(rh), "bs"))
        lo, hi, kd = gen.mixed_queries_device(seed * 7 + j, dk, int(per[j]))
        los.append(lo)
        his.append(hi)
        kinds.append(kd)
        del dk, kh, rh
    lo, hi, kind = torch.cat(los), torch.cat(his), torch.cat(kinds)
    del los, his, kinds
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum(per)
    doff = torch.from_numpy(off).cuda()
    say(f"combined: {count} indexes, {int(sizes.sum())} keys, {int(kind.sum())} ranges")
    idx.learn_batch(ixs, [max(1, int(n) // 64) for n in sizes], 2)
    with idx.Batch(ixs) as bt:
        p_l, o_l, r_l = bt.mixed(lo, hi, kind, doff)
    eks = [ix.relayout("eks", 17) for ix in ixs]
    with idx.Batch(eks) as bt:
        p_e, o_e, r_e = bt.mixed(lo, hi, kind, doff)
    for e in eks:
        e.close()
    torch.cuda.synchronize()
    say(f"combined: {len(r_l)} matched row IDs")
    assert torch.equal(p_l, p_e) and torch.equal(o_l, o_e) and torch.equal(r_l, r_e)
    del p_e, o_e, r_e
    # 32 indexes evenly spread over the size order, against the oracle
    order = np.argsort(sizes, kind="stable")
    sample = sorted(set(order[np.linspace(0, count - 1, 32).round().astype(int)].tolist()))
    offs_all = o_l.cpu().numpy().view(np.uint64)
    for j in sample:
        kh, rh = combined_keys(seed, j, int(sizes[j]))
        sk, sr = oracle.stable_sort(kh, rh)
        a, b = int(off[j]), int(off[j + 1])
        kd = kind[a:b].cpu().numpy()
        lh = to_host(lo[a:b], 64)
        hh = to_host(hi[a:b], 64)
        pts, rgs = np.nonzero(kd == 0)[0], np.nonzero(kd == 1)[0]
        want_p = np.full(b - a, MISS, dtype=np.uint32)
        want_p[pts] = oracle.point(sk, sr, lh[pts], nthreads=CPU_THREADS)
        assert np.array_equal(rows_host(p_l[a:b]), want_p), f"index {j}: points"
        wo, wr = oracle.range_lookup(sk, sr, lh[rgs], hh[rgs], nthreads=CPU_THREADS)
        counts = np.zeros(b - a, dtype=np.uint64)
        counts[rgs] = np.diff(wo)
        assert np.array_equal(np.diff(offs_all[a:b + 1]), counts), f"index {j}: range counts"
        s0, s1 = int(offs_all[a]), int(offs_all[b])
        assert np.array_equal(rows_host(r_l[s0:s1]), wr), f"index {j}: range row IDs"
    for ix in ixs:
        ix.close()

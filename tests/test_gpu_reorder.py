"""GPU parity of lookup reordering: the tile-local sort (reorder=1) and the
batch partitioned by rank bucket (reorder=2) give, element by element, the
oracle's answers in the caller's order, for every form, key width and
launch shape, including empty, tiny and ragged batches and sets."""
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


def key_set(seed, n, bits, dup):
    dt = np.uint64 if bits == 64 else np.uint32
    if dup:
        rng = np.random.default_rng(seed)
        keys = rng.integers(0, max(1, n // 4), size=n, dtype=np.uint64).astype(dt)
        rows = (rng.permutation(n).astype(np.uint64) * 5 + 1).astype(np.uint32)
        return keys, rows
    return gen.unique_keys(seed, n, bits, 63 if bits == 64 else 32)


def queries(seed, keys, m, bits):
    rng = np.random.default_rng(seed)
    dt = keys.dtype
    top = int(np.iinfo(dt).max)
    half = m // 2
    miss = rng.integers(0, top, size=half, dtype=np.uint64, endpoint=True).astype(dt)
    hit = keys[rng.integers(0, len(keys), size=m - half)] if len(keys) else miss[:0]
    q = np.concatenate([miss, hit, np.array([0, top], dtype=dt)])[:m] if m else np.zeros(0, dtype=dt)
    rng.shuffle(q)
    return q


# (layout, k, aos, params); "learned" trains a model on the sorted array
FORMS = [
    ("bs", 1, False, {}),
    ("bs", 1, False, {"lds_levels": 10, "persistent": 2, "block": 1024}),
    ("bs", 1, True, {"per_lane": 8}),
    ("ebs", 2, False, {"per_lane": 8}),
    ("ebs", 2, False, {"lds_levels": 8, "persistent": 2, "per_lane": 1}),
    ("eks", 9, False, {"group": 1}),
    ("eks", 9, False, {"group": 1, "lds_levels": 3, "persistent": 2, "block": 1024}),
    ("eks", 17, "padded", {"group": 1, "per_lane": 8, "block": 1024}),
    ("eks", 5, True, {"group": 1, "per_lane": 2}),
    ("eks", 9, False, {"group": 8}),
    ("eks", 9, False, {"group": 4}),
    ("learned", 1, False, {}),
    ("learned", 1, False, {"per_lane": 8, "block": 1024, "persistent": 2}),
]


def make(keys, rows, layout, k, aos):
    if layout == "learned":
        ix = idx.Index(to_dev(keys), to_dev(rows), layout="bs")
        if len(keys):
            ix.learn(max(1, len(keys) // 64), 2)
        return ix
    return idx.Index(to_dev(keys), to_dev(rows), layout=layout, k=k, aos=aos)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("reorder", [1, 2, 3])
@pytest.mark.parametrize("form", range(len(FORMS)))
def test_reorder_parity(form, reorder, bits):
    layout, k, aos, params = FORMS[form]
    if reorder == 1 and params.get("group", 1) > 1:
        # the tile-local sort needs one lookup per lane
        keys, rows = key_set(7, 1000, bits, False)
        with make(keys, rows, layout, k, aos) as ix:
            with pytest.raises(idx.IdxError):
                ix.set_params(reorder=1, **params)
        return
    for n, dup, m in ((20011, False, 100003), (20011, True, 30011), (5, False, 4097), (1, False, 65),
                      (0, False, 1000), (3000, False, 0), (3000, False, 1)):
        keys, rows = key_set(n * 31 + bits + k, n, bits, dup)
        q = queries(n + m + form, keys, m, bits)
        sk, sr = oracle.stable_sort(keys, rows)
        want = oracle.point(sk, sr, q, nthreads=4)
        with make(keys, rows, layout, k, aos) as ix:
            try:
                ix.set_params(reorder=reorder, **params)
            except idx.IdxError:
                ix.set_params(reorder=reorder, **{kk: v for kk, v in params.items() if kk != "lds_levels"})
            say(f"reorder={reorder} {layout} k={k} aos={aos} bits={bits} n={n} dup={dup} m={m} {ix.params()}")
            got = rows_host(ix.point(to_dev(q))) if m else np.zeros(0, dtype=np.uint32)
            bad = np.nonzero(got != want)[0]
            assert len(bad) == 0, f"{len(bad)} mismatches, first q={q[bad[0]]} got={got[bad[0]]} want={want[bad[0]]}"


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("layout,k,aos", [("bs", 1, False), ("ebs", 2, False), ("eks", 9, False),
                                          ("eks", 17, "padded"), ("learned", 1, False)])
def test_partitioned_many_buckets(layout, k, aos, bits):
    """n = 2^21 + 5 keys (tens of rank buckets), 2^20 + 3 lookups (17
    partition tiles, ragged): every answer equals the generator's (hits)
    and the sentinel (misses); 4096 sampled answers equal the oracle's."""
    n, m = (1 << 21) + 5, (1 << 20) + 3
    seed = gen.BASE_SEED + 40 + bits
    w = 63 if bits == 64 else 32
    keys, rows = gen.unique_keys(seed, n, bits, w)
    q, expect = gen.point_queries(seed, n, m, 0.75, bits, w)
    sk, sr = oracle.stable_sort(keys, rows)
    rng = np.random.default_rng(3)
    sample = rng.integers(0, m, 4096)
    want_s = oracle.point(sk, sr, q[sample], nthreads=8)
    with make(keys, rows, layout, k, aos) as ix:
        for params in ({"reorder": 2}, {"reorder": 2, "persistent": 2, "block": 1024, "per_lane": 4},
                       {"reorder": 3}):
            ix.set_params(**params)
            say(f"partitioned {layout} k={k} aos={aos} bits={bits} {ix.params()}")
            got = ix.point(to_dev(q))
            torch.cuda.synchronize()
            assert torch.equal(got, to_dev(expect))
            assert np.array_equal(rows_host(got)[sample], want_s)
            # a second call reuses the cached splitters
            got2 = ix.point(to_dev(q[: m // 3]))
            assert torch.equal(got2, to_dev(expect[: m // 3]))


@pytest.mark.parametrize("m", [(1 << 17) + 5, (1 << 22) + 7])
def test_partitioned_scatter_paths(m):
    """n = 2^24 + 3 keys (512 rank buckets: 64 coarse x 8 fine).  With 2^17
    lookups every partition tile spans all coarse buckets, so the fine pass
    places entries directly; with 2^22 a tile spans few of them and every
    pass stages its rounds in LDS.  Both must give the generator's answers."""
    n = (1 << 24) + 3
    seed = gen.BASE_SEED + 47
    keys, rows = gen.unique_keys(seed, n, 64, 63)
    q, expect = gen.point_queries(seed, n, m, 0.8, 64, 63)
    sk, sr = oracle.stable_sort(keys, rows)
    sample = np.random.default_rng(m).integers(0, m, 2048)
    want_s = oracle.point(sk, sr, q[sample], nthreads=8)
    for layout, k in (("bs", 1), ("ebs", 2)):
        with idx.Index(to_dev(keys), to_dev(rows), layout=layout, k=k) as ix:
            for reorder in (2, 3):
                ix.set_params(reorder=reorder)
                say(f"partitioned paths {layout} n={n} m={m} reorder={reorder}")
                got = ix.point(to_dev(q))
                torch.cuda.synchronize()
                assert torch.equal(got, to_dev(expect))
                assert np.array_equal(rows_host(got)[sample], want_s)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("aos", [False, True])
def test_partitioned_duplicates_many_buckets(bits, aos):
    """The sorted array's partitioned search starts inside each lookup's
    bucket; with every key repeated about 8 times, equal splitters border
    many buckets.  n = 2^21 + 3 keys, 2^20 + 7 lookups (half hits, some
    below and above every key): every answer equals the oracle's (the first
    row ID of the key in stable order)."""
    n, m = (1 << 21) + 3, (1 << 20) + 7
    keys, rows = key_set(90 + bits, n, bits, True)
    keys = (keys // 2 + 3).astype(keys.dtype)  # about 8 copies of each value
    q = queries(91 + bits, keys, m, bits)
    q[:3] = np.array([0, 1, 2], dtype=q.dtype)  # below every key
    sk, sr = oracle.stable_sort(keys, rows)
    want = oracle.point(sk, sr, q, nthreads=8)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs", aos=aos) as ix:
        for params in ({"reorder": 2}, {"reorder": 2, "per_lane": 8}, {"reorder": 3}):
            ix.set_params(**params)
            say(f"partitioned duplicates bits={bits} aos={aos} {params}")
            got = rows_host(ix.point(to_dev(q)))
            bad = np.nonzero(got != want)[0]
            assert len(bad) == 0, f"{len(bad)} mismatches, first q={q[bad[0]]} got={got[bad[0]]} want={want[bad[0]]}"

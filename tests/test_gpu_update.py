"""GPU parity of the read-mostly update path: an index merged with a batch
of new pairs equals the index built from all pairs (old first), slot for
slot, and answers like the oracle; a saved and loaded handle equals the
original, learned model included."""
import sys

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import rows_host, to_dev, to_host

pytestmark = pytest.mark.gpu

idx = pytest.importorskip("paper_2506_01576_amd")

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

MISS = 0xFFFFFFFF


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def pairs(seed, n, bits, dup):
    rng = np.random.default_rng(seed)
    dt = np.uint64 if bits == 64 else np.uint32
    if dup:
        keys = rng.integers(0, max(1, n // 3), size=n, dtype=np.uint64).astype(dt)
    else:
        keys, _ = gen.unique_keys(seed, n, bits, 63 if bits == 64 else 32)
    rows = (rng.permutation(n).astype(np.uint64) * 2 + seed % 2).astype(np.uint32)
    return keys.astype(dt), rows


def queries(keys, m, seed, bits):
    rng = np.random.default_rng(seed)
    dt = np.uint64 if bits == 64 else np.uint32
    top = int(np.iinfo(dt).max)
    rnd = rng.integers(0, top, size=m // 2, dtype=np.uint64, endpoint=True).astype(dt)
    hit = keys[rng.integers(0, len(keys), m - m // 2)] if len(keys) else rnd[:0]
    return np.concatenate([rnd, hit]).astype(dt)


TARGETS = [("bs", 1, False), ("ebs", 2, False), ("eks", 9, False), ("eks", 17, "padded"), ("bs", 1, True)]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("dup", [False, True])
def test_merge_equals_build_of_all_pairs(bits, dup):
    for n_old, n_new in ((20011, 5003), (0, 4097), (3000, 0), (1, 1), (65536, 65536)):
        ka, ra = pairs(11 + n_old, n_old, bits, dup)
        kb, rb = pairs(12 + n_new, n_new, bits, dup)
        if len(ka) and len(kb) and bits == 64:
            kb[: len(kb) // 4] = ka[: len(kb) // 4][: len(kb) // 4]  # equal keys across old and new
        allk, allr = np.concatenate([ka, kb]), np.concatenate([ra, rb])
        sk, sr = oracle.stable_sort(allk, allr)
        q = queries(allk, 8000, n_old + n_new, bits)
        want = oracle.point(sk, sr, q, nthreads=4)
        with idx.Index(to_dev(ka), to_dev(ra), layout="bs") as old:
            for layout, k, aos in TARGETS:
                say(f"merge bits={bits} dup={dup} n_old={n_old} n_new={n_new} -> {layout} k={k} aos={aos}")
                with old.merge(to_dev(kb), to_dev(rb), layout, k, aos) as mg, \
                        idx.Index(to_dev(allk), to_dev(allr), layout=layout, k=k, aos=aos) as built:
                    gk, gr = mg.export()
                    bk, br = built.export()
                    assert np.array_equal(to_host(gk, bits), to_host(bk, bits))
                    assert np.array_equal(rows_host(gr), rows_host(br))
                    assert mg.info()["unique"] == built.info()["unique"]
                    assert np.array_equal(rows_host(mg.point(to_dev(q))), want)
            # the old index is unchanged
            ok, orow = old.export()
            ek, er = oracle.stable_sort(ka, ra)
            assert np.array_equal(to_host(ok, bits), ek) and np.array_equal(rows_host(orow), er)


def test_merge_rejects():
    ka, ra = pairs(3, 1000, 64, False)
    kb, rb = pairs(4, 100, 64, False)
    rb[7] = MISS
    with idx.Index(to_dev(ka), to_dev(ra), layout="bs") as old:
        with pytest.raises(idx.IdxError) as ei:
            old.merge(to_dev(kb), to_dev(rb))
        assert ei.value.status == idx.IDX_ERR_RESERVED_ROWID
        with old.relayout("eks", 9) as e:
            with pytest.raises(idx.IdxError):
                e.merge(to_dev(kb), to_dev(rb))


@pytest.mark.parametrize("bits", [32, 64])
def test_save_load_roundtrip(bits):
    keys, rows = pairs(21, 50021, bits, False)
    sk, sr = oracle.stable_sort(keys, rows)
    q = queries(keys, 10000, 5, bits)
    want = oracle.point(sk, sr, q, nthreads=4)
    for layout, k, aos in TARGETS + [("learned", 1, False), ("learned", 1, True)]:
        lay = "bs" if layout == "learned" else layout
        with idx.Index(to_dev(keys), to_dev(rows), layout=lay, k=k, aos=aos) as ix:
            if layout == "learned":
                ix.learn(1024, 2)
            blob = ix.save()
            say(f"save/load bits={bits} {layout} k={k} aos={aos}: {len(blob)} bytes")
            with idx.Index.load(blob) as back:
                assert back.info() == ix.info() or {kk: v for kk, v in back.info().items() if not kk.startswith("build")} \
                    == {kk: v for kk, v in ix.info().items() if not kk.startswith("build")}
                a_k, a_r = ix.export()
                b_k, b_r = back.export()
                assert np.array_equal(to_host(a_k, bits), to_host(b_k, bits))
                assert np.array_equal(rows_host(a_r), rows_host(b_r))
                assert np.array_equal(rows_host(back.point(to_dev(q))), want)
                if layout == "learned":
                    assert back.learn_stats() == ix.learn_stats()
                    assert torch.equal(back.learn_export(), ix.learn_export())
    # bytes that are not a blob
    with pytest.raises(idx.IdxError):
        idx.Index.load(b"not an index blob at all" * 8)
    with idx.Index(to_dev(keys), to_dev(rows), layout="bs") as ix:
        blob = ix.save()
        with pytest.raises(idx.IdxError):
            idx.Index.load(blob[:-4])

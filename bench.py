#!/usr/bin/env python3
"""Benchmark: point lookups/s on a static index of n = 2^26 unique uint64 keys.

Workload (the full-scale configuration): n = 2^26 keys uniform in [0, 2^63),
unique by construction, rowid = insertion position; 2^27 point lookups, all
hits, uniform over the build keys, in random order (the paper's default
lookup workload, Section 8.1, at this size); 2^24 range lookups covering 16
consecutive keys each.  All inputs are resident in HBM before timing.

A step is one pass of the hot path over the batch: sort (BS build), the
Eytzinger permutations (EBS and the tuned EKS), point lookups on BS, EBS and
EKS, range lookups on BS and EKS.  `value` is the point-lookup throughput of
the fastest form, from HIP events around its kernel inside the timed steps;
every other phase is reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "point lookups/s at n=2^26 (BS vs EKS vs learned, bit-exact); % of HBM roofline"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
ONCHIP_BYTES = 256 << 20  # Infinity Cache (MALL); the per-XCD L2 is far smaller and not counted
GRANULE = 64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# Algorithmic bytes per point lookup (the per-unit figure of the roofline):
# 8 B query + 4 B result streamed, plus every tree level that cannot stay on
# chip (cumulative top-down footprint above ONCHIP_BYTES) costs the bytes of
# the node read there, rounded up to 64-byte granules, weighted by the share
# of lookups that reach the level; plus one granule for the row ID (SoA).
# --------------------------------------------------------------------------

def levels_eytzinger(n: int, k: int):
    out, start, width = [], 0, k - 1
    while start < n:
        out.append((start, min(n, start + width)))
        start += width
        width *= k
    return out


def algo_bytes(form: str, n: int, k: int, key_bytes: int, early_exit: bool = True, window: float = 0.0,
               leaves: int = 0, aos=False, onchip: int = ONCHIP_BYTES, lines: bool = False,
               over: float = 0.0) -> dict:
    ONCHIP_BYTES = onchip  # noqa: N806 (the capacity this estimate assumes)
    stream = key_bytes + 4
    uncached = 0.0
    rowid = GRANULE if n * (key_bytes + 4) > onchip else 0
    if form == "learned" and lines:
        # leaf lines: the 128-byte line of the query's leaf (its keys, then
        # their row IDs: both granules), counted if the lines exceed on-chip
        # capacity; the share `over` of lookups in leaves too large for a
        # line also searches the leaf's window as below
        big = algo_bytes(form, n, k, key_bytes, early_exit, window, leaves, aos, onchip)
        inline = 2 * GRANULE if leaves * 128 > ONCHIP_BYTES else 0
        tree = inline + over * (big["tree"] + big["rowid"])
        req = (1.0 if inline else 0.0) + over * (big["tree"] + big["rowid"]) / GRANULE
        return {"stream": stream, "tree": round(tree, 1), "rowid": 0, "total": round(stream + tree, 1),
                "random_lines": round(req, 3), "over": round(over, 5)}
    if form == "learned":
        # leaf record (32 B each; counted only if the table exceeds on-chip
        # capacity) + binary search over the mean window: one granule per
        # step until the remaining interval fits one granule; with the array
        # of structures each slot holds the row ID too (no separate granule)
        if leaves * 32 > ONCHIP_BYTES:
            uncached += GRANULE
        slot = key_bytes if not aos else (16 if aos == "padded" else key_bytes + 4)
        if aos:
            rowid = 0
        span = max(window, 1.0) * slot
        uncached += GRANULE * max(0.0, math.ceil(math.log2(max(span / GRANULE, 1.0))))
        if span > 0:
            uncached += GRANULE  # the final granule holding the answer
    elif form == "bs":
        length, depth, cum = n, 0, 0
        while length > 1:
            half = length >> 1
            granules_so_far = min(2 ** (depth + 1), (n * key_bytes + GRANULE - 1) // GRANULE)
            cum = granules_so_far * GRANULE
            if cum > ONCHIP_BYTES and length * key_bytes > GRANULE:
                uncached += GRANULE
            length -= half
            depth += 1
    else:
        kk = 2 if form == "ebs" else k
        cum = 0
        for lvl, (a, b) in enumerate(levels_eytzinger(n, kk)):
            cum += (b - a) * key_bytes
            node_bytes = (kk - 1) * key_bytes
            node_g = math.ceil(node_bytes / GRANULE) * GRANULE
            reach = (n - a) / n if (early_exit and form == "eks") else (1.0 if b - a == (kk - 1) * kk ** lvl
                                                                             else (b - a) / ((kk - 1) * kk ** lvl))
            if cum > ONCHIP_BYTES:
                uncached += reach * node_g
    return {"stream": stream, "tree": uncached, "rowid": rowid, "total": stream + uncached + rowid}


# Algorithmic bytes per range lookup of `width` matches: the two bounds in,
# the offset and the row IDs out, the descent of the lower bound as for a
# point lookup, one more granule where the upper bound's search ends (its
# path shares the rest), and the granules holding the matches' row IDs where
# the layout stores them (sampled at random ranks: consecutive ranks lie in
# one run on the sorted array, on a few levels of an Eytzinger layout).
def line_overflow(ix, leaves: int, cap: int) -> float:
    """Share of the build keys (so of uniform hit lookups) that lie past the
    first `cap` keys of their leaf, whose lookups search the rest of the leaf
    beyond its line, from the exported leaf table (word 3 of each 32-byte
    record is the leaf's size)."""
    import torch

    sizes = ix.learn_export().view(torch.int32).reshape(leaves, 8)[:, 3].to(torch.int64)
    tot = int(sizes.sum())
    return float((sizes - cap).clamp(min=0).sum()) / tot if tot else 0.0


def algo_bytes_range(form: str, n: int, k: int, key_bytes: int, width: int, rank_slot=None, window: float = 0.0,
                     leaves: int = 0, aos=False, samples: int = 2048, lines: bool = False, over: float = 0.0) -> dict:
    import numpy as np

    pt = algo_bytes(form, n, k, key_bytes, early_exit=False, window=window, leaves=leaves, aos=aos, lines=lines,
                    over=over)
    rng = np.random.default_rng(1)
    starts = rng.integers(0, n - width + 1, size=samples)
    total = 0
    for r0 in starts.tolist():
        addrs = set()
        for r in range(r0, r0 + width):
            if form in ("bs", "learned") and not aos:
                a = 4 * r
            elif form == "learned":
                a = (16 if aos == "padded" else key_bytes + 4) * r + key_bytes
            elif form == "ebs":
                a = 4 * (1 + rank_slot(n, 2, r))
            else:
                a = 4 * rank_slot(n, k, r)
            addrs.add(a // GRANULE)
        total += len(addrs)
    rowid_g = total / samples
    stream = 2 * key_bytes + 8 + 4 * width
    # the upper bound's search: one more granule where its path leaves the
    # lower bound's; through leaf lines, its own line
    tree = 2 * pt["tree"] if lines else pt["tree"] + GRANULE
    rowid = rowid_g * GRANULE
    return {"stream": stream, "tree": tree, "rowid": round(rowid, 1), "rowid_granules": round(rowid_g, 3),
            "total": round(stream + tree + rowid, 1)}


def source_sha() -> str:
    """Hash of every kernel source: traffic counters are only reported while
    they were taken on exactly these sources."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_01576_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key: str):
    """HBM bytes per launch of `kernel_key` from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_point_lookup.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith(kernel_key + " "):
                for kv in line.split()[1:]:
                    k, _, v = kv.partition("=")
                    rec[k] = v
    if not rec or rec.get("source_sha") != source_sha():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_batched(args, idx, gen, np, torch, dev, log, table):
    """Many uneven indexes in one persistent launch: `batch_indexes` uint32
    indexes with n log-uniform in [2^6, 2^22], each with a point batch of
    log-uniform size in [1, 2^16], 80% hits; the form of each index comes from
    the tuned per-size-class table.  The one-launch rate (eager and replayed
    from a HIP graph) is compared with a loop of one launch per index."""
    from paper_2506_01576_amd import autotune

    count = args.batch_indexes
    seed = gen.BASE_SEED + 2
    t0 = time.time()
    sizes = gen.log_uniform(seed, 1, 1 << 6, 1 << 22, count)
    qcounts = gen.log_uniform(seed, 2, 1, 1 << 16, count)
    idxs, qs, ex, forms_used = [], [], [], {}
    for j in range(count):
        n = int(sizes[j])
        kh, rh = gen.unique_keys(seed * 100003 + j, n, 32)
        qh, eh = gen.point_queries(seed * 100003 + j, n, int(qcounts[j]), 0.8, 32)
        form = autotune.batch_form(n, 32, table)
        forms_used[str(form)] = forms_used.get(str(form), 0) + 1
        ix = autotune.build_form(torch.from_numpy(kh.view(np.int32)).to(dev),
                                 torch.from_numpy(rh.view(np.int32)).to(dev), form)
        idxs.append(ix)
        qs.append(qh)
        ex.append(eh)
    dq = torch.from_numpy(np.concatenate(qs).view(np.int32)).to(dev)
    de = torch.from_numpy(np.concatenate(ex).view(np.int32)).to(dev)
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(q) for q in qs])
    doff = torch.from_numpy(off).to(dev)
    out = torch.empty(len(dq), dtype=torch.int32, device=dev)
    total = int(off[-1])
    log(f"batched: built {count} indexes ({int(sizes.sum())} keys), {total} queries in {time.time() - t0:.1f}s")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    # roofline of the one-launch kernel: per lookup the algorithmic bytes of
    # its index's form (4 B query + 4 B answer, plus the granules of levels,
    # leaf records, windows and row IDs that cannot stay in one XCD's 4 MiB
    # L2: the launch walks many indexes at once, so the shared 256 MiB
    # Infinity Cache is not counted as on-chip here), weighted by the lookups
    # each index receives
    algo_total = 0.0
    for j, ix in enumerate(idxs):
        lay, kk, per_leaf, _ = autotune._form(autotune.batch_form(int(sizes[j]), 32, table))
        nj = int(sizes[j])
        if per_leaf:
            st = ix.learn_stats()
            ab = algo_bytes("learned", nj, 1, 4, window=st["mean_window"], leaves=st["leaves"], onchip=4 << 20)
        else:
            ab = algo_bytes(lay, nj, kk, 4, onchip=4 << 20)
        algo_total += ab["total"] * int(qcounts[j])
    res = {"indexes": count, "keys": int(sizes.sum()), "queries": total, "forms_by_count": forms_used,
           "algorithmic_bytes_per_lookup": round(algo_total / max(total, 1), 1)}
    with idx.Batch(idxs) as bt:
        ms_eager = timed(lambda: bt.point(dq, doff, out), 10)
        exact_eager = bool(torch.equal(out, de))
        out.fill_(-1)
        ms_graph = timed(lambda: bt.point(dq, doff, out, graph=True), 10)
        exact_graph = bool(torch.equal(out, de))

    def loop():
        for j, ix in enumerate(idxs):
            a, b = int(off[j]), int(off[j + 1])
            if b > a:
                ix.point(dq[a:b], out[a:b])

    out.fill_(-1)
    ms_loop = timed(loop, 2)
    exact_loop = bool(torch.equal(out, de))
    ach = algo_total / (min(ms_eager, ms_graph) / 1e3) / 1e9
    res["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": "k_batch_point",
                       "onchip_bytes_assumed": 4 << 20}
    res.update({"ms_one_launch": round(ms_eager, 4), "ms_graph_replay": round(ms_graph, 4),
                "ms_per_index_loop": round(ms_loop, 4),
                "lookups_per_s_one_launch": total / ms_eager * 1e3,
                "lookups_per_s_graph_replay": total / ms_graph * 1e3,
                "lookups_per_s_per_index_loop": total / ms_loop * 1e3,
                "speedup_vs_loop": ms_loop / min(ms_eager, ms_graph),
                "bit_exact": exact_eager and exact_graph and exact_loop})
    log(f"batched: one launch {ms_eager:.3f} ms, graph {ms_graph:.3f} ms, loop {ms_loop:.3f} ms")
    for ix in idxs:
        ix.close()
    return res


def run_skewed(args, idx, gen, np, torch, dev, log):
    """The learned-model configuration: n = 2^log2n_skew unique uint64 keys from
    the 64-cluster lognormal mixture, 2^27 lookups: Zipf(1.1)-popular hits
    plus 10% uniform misses.  The learned form with 4096 leaves (the
    configuration's model), with 2^22 leaves and with leaf lines, against EKS
    with 16 keys per node (k = 17) and k = 16; all must agree, hits must
    return the generator's rowids."""
    n, m = 1 << args.log2n_skew, 1 << 27
    seed = gen.BASE_SEED + 3
    t0 = time.time()
    kh, rh = gen.lognormal_keys(seed, n)
    qh, eh = gen.zipf_queries(seed, 1.1, n, m, 0.1, 64, 63, keys=kh)
    keys = torch.from_numpy(kh.view(np.int64)).to(dev)
    rows = torch.from_numpy(rh.view(np.int32)).to(dev)
    q = torch.from_numpy(qh.view(np.int64)).to(dev)
    expect = torch.from_numpy(eh.view(np.int32)).to(dev)
    del kh, rh, qh, eh
    hit = expect != -1
    out = torch.empty(m, dtype=torch.int32, device=dev)
    log(f"skewed: {n} lognormal keys, {m} Zipf(1.1) lookups generated in {time.time() - t0:.1f}s")

    def timed(ix, reps=3):
        ix.point(q, out)
        torch.cuda.synchronize()
        res = out.clone()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            ix.point(q, out)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), res

    forms, answers = {}, {}
    base = idx.Index(keys, rows, layout="bs")
    # the 4096-leaf model; 2^22 leaves (window search), the scan in two
    # rounds and in one (skewed batches keep many windows cached); leaf
    # lines with about four keys per leaf (spline root)
    cands = [("learned_4096", 4096, False, {"per_lane": 8}),
             ("learned_2^22_soa_r4", 1 << 22, False, {"per_lane": 4}),
             ("learned_2^22_soa_r4_1round", 1 << 22, False, {"per_lane": 4, "window_rounds": 1}),
             ("learned_lines", min(1 << 26, n // 4), False, {"per_lane": 4, "block": 128, "leaf_lines": 1})]
    for name, L, aos, params in cands:
        arr = base if not aos else base.relayout("bs", 1, aos)
        arr.set_params(model=0, **params)  # leaf lines, when used, are written by the training call
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        st = arr.learn(L, 2)
        b.record()
        b.synchronize()
        ms, res = timed(arr)
        forms[name] = {"leaves": L, "aos": aos, "ms": round(ms, 4), "lookups_per_s": m / ms * 1e3,
                       "train_ms": round(a.elapsed_time(b), 3), "mean_window": st["mean_window"],
                       "max_window": st["max_window"],
                       "root": {1: "linear", 2: "log", 3: "spline"}[st["feature"]] +
                       (f"({st['segments']} {'log' if st['bin_feature'] == 2 else 'linear'} bins)"
                        if st["feature"] == 3 else "")}
        answers[name] = res
        if arr is not base:
            arr.close()
        else:
            arr.unlearn()
            arr.reset_params()
    for name, k, params in (("eks_k17", 17, {"group": 1, "per_lane": 4, "lds_levels": 3, "persistent": 2,
                                             "block": 1024}),
                            ("eks_k16", 16, {})):
        with base.relayout("eks", k) as e:
            try:
                e.set_params(**params)
            except idx.IdxError:
                e.reset_params()
            ms, res = timed(e)
            forms[name] = {"k": k, "params": e.params(), "ms": round(ms, 4), "lookups_per_s": m / ms * 1e3}
            answers[name] = res
    base.close()
    ref = answers["eks_k17"]
    agree = all(bool(torch.equal(v, ref)) for v in answers.values())
    hits_exact = bool(torch.equal(ref[hit], expect[hit]))
    best_l = min((v["ms"] for k2, v in forms.items() if k2.startswith("learned")))
    best_e = min((v["ms"] for k2, v in forms.items() if k2.startswith("eks")))
    log("skewed: " + ", ".join(f"{k2} {v['ms']:.3f} ms" for k2, v in forms.items()) + f"; agree={agree} hits={hits_exact}")
    return {"n": n, "queries": m, "workload": "lognormal mixture keys, Zipf(1.1) hits + 10% uniform misses",
            "forms": forms, "all_forms_agree": agree, "hits_equal_generator": hits_exact,
            "learned_vs_eks": best_e / best_l}


def run_study(args, idx, gen, np, torch, dev, log):
    """Skew and duplicates (Sections 8.9 and 8.11), n = 2^26 uint64 keys.
    Skew: 2^27 lookups drawn Zipf(s) over the build keys (s = 0 is uniform)
    and the uniform batch sorted ascending, through each form.  Duplicates:
    2^24 keys, each distinct value replicated r times, and 2^24 equality
    ranges [x, x] (every replica in key order, the paper's treatment of point
    lookups on duplicated keys).  Every answer is checked against the
    generator's answers (known by construction)."""
    from paper_2506_01576_amd import autotune

    res = {"skew": {}, "duplicates": {}}
    n, m = 1 << 26, 1 << 27
    seed = gen.BASE_SEED + 1
    kh, rh = gen.unique_keys(seed, n, 64, 63)
    keys = torch.from_numpy(kh.view(np.int64)).to(dev)
    rows = torch.from_numpy(rh.view(np.int32)).to(dev)
    del kh, rh
    base = idx.Index(keys, rows, layout="bs")
    forms = {}
    for layout in ("bs", "ebs", "eks"):
        lay, k, aos, params = autotune.choose(n, 64, layout)
        ix = base.relayout(lay, k, aos)
        ix.set_params(**params)
        forms[layout.upper() if layout != "eks" else f"EKS(k={k},single)"] = ix
    g8 = base.relayout("eks", 9)
    g8.set_params(group=8, per_lane=2)
    forms["EKS(k=9,group8)"] = g8
    v4 = base.relayout("eks", 9)
    v4.set_params(group=4, per_lane=4)
    forms["EKS(k=9,vgroup4)"] = v4
    # the window search form (2^22 leaves, about 16 keys each) ...
    ln = base.relayout("bs", 1, False)
    ln.set_params(model=0, per_lane=4, leaf_lines=2)
    ln.learn(1 << 22, 2)
    forms["LEARNED"] = ln
    # ... and the tuned form (leaf lines), trained with its parameters set so
    # that the training writes its lines
    _, _, laos, lp = autotune.choose(n, 64, "learned")
    lp = dict(lp)
    lines_leaves = lp.pop("leaves", 1 << 24)
    ll = base.relayout("bs", 1, laos)
    ll.set_params(**lp)
    ll.learn(lines_leaves, 2)
    forms["LEARNED(lines)" if lp.get("leaf_lines") == 1 else "LEARNED(tuned)"] = ll
    out = torch.empty(m, dtype=torch.int32, device=dev)

    def timed(ix, q, reps=3):
        ix.point(q, out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            ix.point(q, out)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    cases = [(f"zipf_{s_}", s_) for s_ in (0.0, 0.5, 1.0, 1.25, 1.5, 2.0)] + [("sorted", None)]
    for name, s_ in cases:
        if s_ is None or s_ == 0.0:
            qh, eh = gen.point_queries(seed, n, m, 1.0, 64, 63)
        else:
            qh, eh = gen.zipf_queries(seed, s_, n, m, 0.0, 64, 63)
        q = torch.from_numpy(qh.view(np.int64)).to(dev)
        e = torch.from_numpy(eh.view(np.int32)).to(dev)
        if s_ is None:
            q, order = torch.sort(q)
            e = e[order]
        row = {"distinct_fraction": float(torch.unique(q).numel()) / m}
        for fname, ix in forms.items():
            ms = timed(ix, q)
            ok = bool(torch.equal(out, e))
            row[fname] = {"ms": round(ms, 4), "lookups_per_s": m / ms * 1e3, "exact": ok}
        # the learned form reading each window in one round (cached windows)
        ln.set_params(**dict(ln.params(), window_rounds=1))
        ms = timed(ln, q)
        row["LEARNED(1 round)"] = {"ms": round(ms, 4), "lookups_per_s": m / ms * 1e3,
                                   "exact": bool(torch.equal(out, e))}
        ln.set_params(**dict(ln.params(), window_rounds=2))
        res["skew"][name] = row
        log(f"study skew {name}: " + ", ".join(f"{f} {v['ms']:.2f}" for f, v in row.items() if isinstance(v, dict)))
        del q, e
    for ix in forms.values():
        ix.close()
    base.close()
    del keys, rows
    torch.cuda.empty_cache()

    # duplicates: equality ranges over replicated keys
    nd = 1 << 24
    for r in (1, 4, 16, 64, 256):
        md = min(1 << 24, (1 << 28) // r)  # at most 2^28 row IDs out
        distinct = nd // r
        vh, _ = gen.unique_keys(seed + r, distinct, 64, 63)
        kh = np.repeat(vh, r)
        rng = np.random.default_rng(r)
        perm = rng.permutation(nd)
        kh = kh[perm]
        rh = perm.astype(np.uint32)
        qh = vh[rng.integers(0, distinct, md)]
        dk = torch.from_numpy(kh.view(np.int64)).to(dev)
        dr = torch.from_numpy(rh.view(np.int32)).to(dev)
        dq = torch.from_numpy(qh.view(np.int64)).to(dev)
        # by construction: value v's replicas carry the row IDs v*r .. v*r+r-1
        # at input positions pos[row]; a stable order lists them by position
        pos = np.argsort(perm)
        sample = rng.integers(0, md, 256)
        want = {}
        for s2 in sample.tolist():
            v = int(np.nonzero(vh == qh[s2])[0][0])
            ids = np.arange(v * r, v * r + r, dtype=np.int64)
            want[s2] = ids[np.argsort(pos[ids], kind="stable")].astype(np.uint32)
        row = {}
        with idx.Index(dk, dr, layout="bs") as b2:
            hs = {"BS": b2, "EBS": b2.relayout("ebs", 2), "EKS(k=9,single)": b2.relayout("eks", 9),
                  "EKS(k=17,single)": b2.relayout("eks", 17)}
            lb = b2.relayout("bs", 1, False)
            lb.learn(max(1, nd // 16), 2)
            hs["LEARNED"] = lb
            for fname, ix in hs.items():
                ix.range(dq, dq, capacity=md * r)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                off, rr = ix.range(dq, dq, capacity=md * r)
                b.record()
                b.synchronize()
                ms = a.elapsed_time(b)
                offh = off.cpu().numpy().view(np.uint64)
                ok = bool(np.all(np.diff(offh) == r))
                for s2 in sample.tolist():
                    got = rr[int(offh[s2]):int(offh[s2 + 1])].cpu().numpy().view(np.uint32)
                    ok &= bool(np.array_equal(got, want[s2]))
                row[fname] = {"ms": round(ms, 4), "lookups_per_s": md / ms * 1e3, "rowids_per_s": md * r / ms * 1e3,
                              "exact": ok}
                del off, rr
            for fname, ix in hs.items():
                if ix is not b2:
                    ix.close()
        res["duplicates"][f"r{r}"] = row
        log(f"study dup r={r}: " + ", ".join(f"{f} {v['ms']:.2f}" for f, v in row.items()))
        del dk, dr, dq
        torch.cuda.empty_cache()
    return res


def run_update(args, idx, gen, np, torch, dev, log):
    """The read-mostly update path (Section 8.5): an index of 2^26 uint64
    keys takes a batch of 2^20 new pairs by merging (sort the batch, merge,
    lay out) against rebuilding from all pairs; the merged and rebuilt
    layouts must be identical.  Also the size and the time of saving and
    loading the merged handle."""
    n, m = 1 << 26, 1 << 20
    seed = gen.BASE_SEED + 1
    kh, rh = gen.unique_keys(seed, n + m, 64, 63)
    keys = torch.from_numpy(kh[:n].view(np.int64)).to(dev)
    rows = torch.from_numpy(rh[:n].view(np.int32)).to(dev)
    nk = torch.from_numpy(kh[n:].view(np.int64)).to(dev)
    nr = torch.from_numpy(rh[n:].view(np.int32)).to(dev)
    allk = torch.from_numpy(kh.view(np.int64)).to(dev)
    allr = torch.from_numpy(rh.view(np.int32)).to(dev)
    del kh, rh
    res = {"n": n, "new": m}

    def wall(fn, reps=3):
        fn().close()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            h = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
            h.close()
        return float(np.median(ts))

    with idx.Index(keys, rows, layout="bs") as old:
        for layout, k in (("bs", 1), ("eks", 9)):
            ms_merge = wall(lambda: old.merge(nk, nr, layout, k))
            ms_build = wall(lambda: idx.Index(allk, allr, layout=layout, k=k))
            with old.merge(nk, nr, layout, k) as a, idx.Index(allk, allr, layout=layout, k=k) as b:
                ak, ar = a.export()
                bk, br = b.export()
                same = bool(torch.equal(ak, bk) and torch.equal(ar, br))
                t0 = time.perf_counter()
                blob = a.save()
                ms_save = (time.perf_counter() - t0) * 1e3
                t0 = time.perf_counter()
                c = idx.Index.load(blob)
                torch.cuda.synchronize()
                ms_load = (time.perf_counter() - t0) * 1e3
                ck, cr = c.export()
                same_loaded = bool(torch.equal(ck, ak) and torch.equal(cr, ar))
                c.close()
            res[layout] = {"merge_ms": round(ms_merge, 3), "rebuild_ms": round(ms_build, 3),
                           "merge_equals_rebuild": same, "blob_bytes": len(blob), "save_ms": round(ms_save, 1),
                           "load_ms": round(ms_load, 1), "load_equals": same_loaded}
            log(f"update {layout}: merge {ms_merge:.2f} ms, rebuild {ms_build:.2f} ms, equal={same}; "
                f"save {ms_save:.0f} ms load {ms_load:.0f} ms ({len(blob) >> 20} MiB)")
    return res


def run_combined(args, idx, gen, np, torch, dev, log):
    """Many learned indexes with a mixed stream: `combined_indexes` uint64
    indexes with n log-uniform in [2^16, 2^24], half with uniform keys and
    half with lognormal-mixture keys; their models are trained by one batched
    launch sequence (against a loop of per-index training); then a stream of
    2^26 * indexes / 1024 lookups -- 70% point lookups with 10% misses, 30%
    ranges of 1-256 matches -- runs through the batch in the learned form and
    in plain EKS (k = 17, 16 keys per node); both must agree, and sampled
    every hit and every range's match count of every index equals the
    generator's answer (known by construction)."""
    count = args.combined_indexes
    seed = gen.BASE_SEED + 4
    t0 = time.time()
    sizes = gen.log_uniform(seed, 1, 1 << 16, 1 << 24, count)
    m_total = max(count, (1 << 26) * count // 1024)
    per = np.full(count, m_total // count, dtype=np.int64)
    per[: m_total - int(per.sum())] += 1
    def keyset(j):
        n = int(sizes[j])
        if j % 2 == 0:
            return gen.unique_keys(seed * 1009 + j, n, 64, 63)
        return gen.lognormal_keys(seed * 1009 + j, n)

    # indexes, and per index a seeded mixed stream drawn on the device from
    # its keys (torch's sort and generator: input preparation only)
    ixs, los, his, kinds, exps, cnts = [], [], [], [], [], []
    for j in range(count):
        kh, rh = keyset(j)
        dk = torch.from_numpy(kh.view(np.int64)).to(dev)
        dr = torch.from_numpy(rh.view(np.int32)).to(dev)
        ixs.append(idx.Index(dk, dr, layout="bs"))
        lo, hi, kd, ex, ct = gen.mixed_queries_device(seed * 7 + j, dk, int(per[j]), rows=dr)
        los.append(lo)
        his.append(hi)
        kinds.append(kd)
        exps.append(ex)
        cnts.append(ct)
        del dk, dr, kh, rh
    torch.cuda.synchronize()
    keys_total = int(sum(ix.n for ix in ixs))
    log(f"combined: built {count} indexes ({keys_total} keys) and their streams in {time.time() - t0:.1f}s")
    lo, hi, kind = torch.cat(los), torch.cat(his), torch.cat(kinds)
    expect, counts = torch.cat(exps), torch.cat(cnts)
    del los, his, kinds, exps, cnts
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum(per)
    doff = torch.from_numpy(off).to(dev)
    n_ranges = int(kind.sum().item())
    res = {"indexes": count, "keys": keys_total, "queries": m_total, "ranges": n_ranges,
           "workload": "uint64 keys, n log-uniform in [2^16, 2^24], half uniform in [0, 2^63), half 64-cluster "
                       "lognormal; 70% point lookups (10% misses), 30% ranges of 1-256 matches"}

    leaves = [max(1, ix.n // 64) for ix in ixs]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for ix, L in zip(ixs, leaves):
        ix.learn(L, 2)
    torch.cuda.synchronize()
    ms_loop = (time.perf_counter() - t1) * 1e3
    t1 = time.perf_counter()
    stats = idx.learn_batch(ixs, leaves, 2)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t1) * 1e3
    res.update({"train_batched_ms": round(ms_batch, 3), "train_per_index_loop_ms": round(ms_loop, 3),
                "train_keys_per_s": keys_total / ms_batch * 1e3,
                "mean_window": float(np.average([s["mean_window"] for s in stats], weights=sizes))})
    log(f"combined: batched training {ms_batch:.1f} ms, per-index loop {ms_loop:.1f} ms")

    def timed_mixed(bt, reps=3):
        out = bt.mixed(lo, hi, kind, doff)
        cap = int(out[1][-1].item())
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            bt.mixed(lo, hi, kind, doff, capacity=cap)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), out

    with idx.Batch(ixs) as bt:
        ms_learned, got_l = timed_mixed(bt)
    eks = [ix.relayout("eks", 17) for ix in ixs]
    with idx.Batch(eks) as bt:
        ms_eks, got_e = timed_mixed(bt)
    agree = all(bool(torch.equal(a, b)) for a, b in zip(got_l, got_e))
    for e in eks:
        e.close()
    # every hit and every range's size against the generator's answers
    hits = expect != -1
    gen_exact = bool(torch.equal(got_l[0][hits], expect[hits]))
    gen_exact &= bool(torch.equal(got_l[1][1:] - got_l[1][:-1], counts))
    del expect, counts, hits
    matches = int(got_l[1][-1].item())
    res.update({"matches": matches, "mixed_learned_ms": round(ms_learned, 4), "mixed_eks17_ms": round(ms_eks, 4),
                "lookups_per_s_learned": m_total / ms_learned * 1e3, "lookups_per_s_eks17": m_total / ms_eks * 1e3,
                "learned_vs_eks": ms_eks / ms_learned, "learned_equals_eks": agree,
                "hits_and_range_counts_equal_generator": gen_exact})
    log(f"combined: mixed stream learned {ms_learned:.3f} ms, EKS {ms_eks:.3f} ms, agree={agree} "
        f"generator answers={gen_exact}")
    for ix in ixs:
        ix.close()
    return res


def run_small(idx, gen, np, torch, dev, log):
    """The small configuration: n = 2^16 unique uint32 keys uniform in
    [0, 2^32), rowid = insertion position; 2^20 point lookups, half hits
    (uniform over the keys) and half misses (uniform over the complement),
    shuffled.  Each layout in its tuned form, checked against the generator's
    answers; median of 10 launches."""
    from paper_2506_01576_amd import autotune

    n, m = 1 << 16, 1 << 20
    seed = gen.BASE_SEED
    kh, rh = gen.unique_keys(seed, n, 32)
    qh, eh = gen.point_queries(seed, n, m, 0.5, 32)
    keys = torch.from_numpy(kh.view(np.int32)).to(dev)
    rows = torch.from_numpy(rh.view(np.int32)).to(dev)
    q = torch.from_numpy(qh.view(np.int32)).to(dev)
    expect = torch.from_numpy(eh.view(np.int32)).to(dev)
    out = torch.empty(m, dtype=torch.int32, device=dev)
    res = {"workload": "n=2^16 unique uint32 keys, 2^20 point lookups (50% hits, 50% misses)", "forms": {}}
    with idx.Index(keys, rows, layout="bs") as base:
        for layout in ("bs", "ebs", "eks", "learned"):
            lay, k, aos, params = autotune.choose(n, 32, layout)
            if lay == "learned":
                ix = base.relayout("bs", 1, aos) if aos else base
                ix.learn(params.pop("leaves", max(1, n // 16)), 2)
                params["model"] = 0
            else:
                ix = base if (lay == "bs" and not aos) else base.relayout(lay, k, aos)
                params["model"] = 2
            ix.set_params(**params)
            ix.point(q, out)
            torch.cuda.synchronize()
            ok = bool(torch.equal(out, expect))
            ts = []
            for _ in range(10):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                ix.point(q, out)
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b))
            ms = float(np.median(ts))
            res["forms"][layout] = {"layout": lay, "k": k, "aos": aos, "params": ix.params(), "ms": round(ms, 4),
                                    "lookups_per_s": m / ms * 1e3, "bit_exact": ok}
            log(f"small u32 {layout}: {ms:.4f} ms ({m / ms / 1e6:.0f} M/s) exact={ok}")
            if ix is not base:
                ix.close()
            else:
                ix.unlearn()
                ix.reset_params()
    best = max(res["forms"], key=lambda f: res["forms"][f]["lookups_per_s"])
    res["best"] = best
    res["lookups_per_s"] = res["forms"][best]["lookups_per_s"]
    res["bit_exact"] = all(v["bit_exact"] for v in res["forms"].values())
    return res


def run_range_scan(idx, np, torch, dev, keys, rows, sorted_rows, log):
    """Hybrid coalesced against single-lane level scanning of EBS range
    lookups (Section 5.1; the paper's Fig. 17 experiment at this index size),
    and the library's default, the gather by rank: the n = 2^26 index in EBS
    layout, 2^18 ranges covering exactly c keys for c = 2^4 .. 2^14; the same
    ranges in every mode, every offset and row ID checked against the ranks
    the ranges were drawn at."""
    m = 1 << 18
    n = len(keys)
    ordered = torch.sort(keys, stable=True).values
    g = torch.Generator(device=dev)
    g.manual_seed(0x2506)
    res = {"layout": "ebs", "n": n, "ranges": m, "rows": []}
    with idx.Index(keys, rows, layout="bs") as base, base.relayout("ebs", 2) as ix:
        for lc in (4, 6, 8, 10, 12, 14):
            c = 1 << lc
            r = torch.randint(0, n - c + 1, (m,), generator=g, device=dev)
            lo, hi = ordered[r], ordered[r + c - 1]
            row = {"hits": c}
            for mode, name in ((1, "hybrid"), (2, "single"), (3, "rank_gather")):
                ix.set_params(range_scan=mode)
                reps = 3 if c <= 1024 else 1
                off, rr = ix.range(lo, hi, capacity=m * c)
                torch.cuda.synchronize()
                ok = bool(torch.equal(off, torch.arange(m + 1, device=dev, dtype=torch.int64) * c))
                step = max(1, (1 << 24) // c)
                for c0 in range(0, m, step):
                    c1 = min(m, c0 + step)
                    pos = (r[c0:c1, None] + torch.arange(c, device=dev)[None, :]).reshape(-1)
                    ok &= bool(torch.equal(rr[c0 * c:c1 * c], sorted_rows[pos]))
                del off, rr
                ts = []
                for _ in range(reps):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    off, rr = ix.range(lo, hi, capacity=m * c)
                    b.record()
                    b.synchronize()
                    ts.append(a.elapsed_time(b))
                    del off, rr
                ms = float(np.median(ts))
                row[name] = {"ms": round(ms, 4), "ranges_per_s": m / ms * 1e3, "rowids_per_s": m * c / ms * 1e3,
                             "bit_exact": ok}
            row["hybrid_speedup"] = row["single"]["ms"] / row["hybrid"]["ms"]
            res["rows"].append(row)
            log(f"range scan c={c}: hybrid {row['hybrid']['ms']:.3f} ms, single {row['single']['ms']:.3f} ms "
                f"({row['hybrid_speedup']:.2f}x), rank gather {row['rank_gather']['ms']:.3f} ms "
                f"exact={all(row[k]['bit_exact'] for k in ('hybrid', 'single', 'rank_gather'))}")
            torch.cuda.empty_cache()
    res["bit_exact"] = all(rw[k]["bit_exact"] for rw in res["rows"] for k in ("hybrid", "single", "rank_gather"))
    return res


# --------------------------------------------------------------------------


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--log2n", type=int, default=26)
    ap.add_argument("--log2m", type=int, default=27)
    ap.add_argument("--log2ranges", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="leave the learned form out")
    ap.add_argument("--no-batched", action="store_true", help="leave the many-index batched workload out")
    ap.add_argument("--batch-indexes", type=int, default=8192)
    ap.add_argument("--no-combined", action="store_true", help="leave the combined learned/mixed workload out")
    ap.add_argument("--no-skewed", action="store_true", help="leave the lognormal / Zipf learned-vs-EKS workload out")
    ap.add_argument("--no-update", action="store_true", help="leave the merge / save / load measurement out")
    ap.add_argument("--study", action="store_true",
                    help="also run the skew (Zipf, sorted) and duplicate-key studies (a few minutes)")
    ap.add_argument("--log2n-skew", type=int, default=28, help="keys in the lognormal / Zipf workload (log2)")
    ap.add_argument("--combined-indexes", type=int, default=1024,
                    help="indexes in the combined workload (1024 = the full configuration; the query count scales "
                         "with it, 2^26 at 1024)")
    ap.add_argument("--sweep", action="store_true",
                    help="re-measure every candidate form (autotuner) instead of using the tuned table")
    ap.add_argument("--write-table", action="store_true", help="with --sweep: store the winners in the tuned table")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24, help="lookups in the CPU oracle sample")
    ap.add_argument("--no-small", action="store_true", help="leave the 2^16-key uint32 configuration out")
    ap.add_argument("--no-k-sweep", action="store_true", help="leave the EKS fan-out sweep out")
    ap.add_argument("--no-range-scan", action="store_true",
                    help="leave the hybrid against single-lane range-scan measurement out")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB device copy (known bytes) to scale hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this index build and its lookups run on a single MI355X; "
              "multi-GPU runs are not part of this benchmark (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2506_01576_amd as idx

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n, m, mr = 1 << args.log2n, 1 << args.log2m, 1 << args.log2ranges
    seed = gen.BASE_SEED + 1
    W = 63

    t0 = time.time()
    keys_h, rows_h = gen.unique_keys(seed, n, 64, W)
    q_h, expect_h = gen.point_queries(seed, n, m, 1.0, 64, W)
    log(f"generated keys/queries in {time.time() - t0:.1f}s")
    t0 = time.time()
    lo_h, hi_h, _, rank_h = gen.ranges(seed, keys_h, mr, 16, 16, with_ranks=True)
    log(f"generated ranges in {time.time() - t0:.1f}s")

    def up(a):
        return torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a.view(np.int32)).to(dev)

    keys, rows, q, expect = up(keys_h), up(rows_h), up(q_h), up(expect_h)
    lo, hi = up(lo_h), up(hi_h)
    range_first = torch.from_numpy(rank_h.view(np.int64)).to(dev)
    del q_h, lo_h, hi_h, rank_h
    out = torch.empty(m, dtype=torch.int32, device=dev)
    # the build set's row IDs in ascending key order (torch's stable sort:
    # input preparation for the generator-known range answers)
    sorted_rows = rows[torch.sort(keys, stable=True).indices]
    torch.cuda.synchronize()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    flush_buf = None

    def time_point(ix, reps=3, check=False, cold=False):
        """Median event time of one point launch over the batch; cold: each
        timed launch follows a 1 GiB write that evicts L2 and the 256 MiB
        Infinity Cache."""
        nonlocal flush_buf
        ix.point(q, out)
        ok = None
        if check:
            torch.cuda.synchronize()
            ok = bool(torch.equal(out, expect))
        if cold and flush_buf is None:
            flush_buf = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        ts = []
        for rep in range(reps):
            if cold:
                flush_buf.fill_(rep)
            a = ev()
            ix.point(q, out)
            b = ev()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), ok

    if args.calibrate:
        src = torch.empty(1 << 27, dtype=torch.int64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        log("calibration copy: 1073741824 bytes read, 1073741824 bytes written")
        del src, dst

    # ------------------------------------------- forms: tuned table or sweep
    from paper_2506_01576_amd import autotune

    base = idx.Index(keys, rows, layout="bs")
    sweep = []
    best_by_layout = {}
    if args.sweep:
        sweep, best_by_layout = autotune.tune(base, q, expect, reps=3, log=log)
        if args.write_table:
            autotune.save_table(autotune.record_best(autotune.load_table(), 64, n, best_by_layout))
    for layout in ("bs", "ebs", "eks"):
        if layout in best_by_layout:
            continue
        lay, k, aos, params = autotune.choose(n, 64, layout)
        ix = base if (lay == "bs" and not aos) else base.relayout(lay, k, aos)
        ix.set_params(**params)
        ms, ok = time_point(ix, reps=10, check=True)
        ms_cold, _ = time_point(ix, reps=10, cold=True)
        best_by_layout[layout] = {"layout": lay, "k": k, "aos": aos, "params": ix.params(), "ms": round(ms, 4),
                                  "ms_cold": round(ms_cold, 4), "lookups_per_s": m / ms * 1e3, "bit_exact": ok}
        log(f"tuned {lay} k={k} aos={aos} {params}: {ms:.3f} ms exact={ok}")
        if ix is not base:
            ix.close()
        else:
            ix.reset_params()
    # learned form: the sorted array plus a trained rank model (leaves tuned)
    lrec = None
    if not args.no_learned:
        if args.sweep:
            cands = [(L, {"per_lane": r}, False) for L in (1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 21,
                                                           1 << 22) for r in (4, 8)]
            cands += [(1 << 20, {"per_lane": 8, "reorder": 1}, False), (1 << 20, {"per_lane": 4, "reorder": 2}, False)]
            # the array of structures: the window scan reads each key with its row ID
            cands += [(L, {"per_lane": r}, a) for a in ("padded", True) for L in (1 << 21, 1 << 22) for r in (2, 4, 8)]
            # leaf lines: a line per leaf of at most a few keys on average
            cands += [(L, {"per_lane": r, "leaf_lines": 1}, a) for a in (False, True) for L in (1 << 23, 1 << 24)
                      for r in (1, 2, 4)]
        else:
            _, _, laos, lp = autotune.choose(n, 64, "learned")
            cands = [(lp.get("leaves", 1 << 16), {kk: v for kk, v in lp.items() if kk != "leaves"}, laos)]
        trained = None
        arrays = {False: base}
        for L, lparams, la in cands:
            if la not in arrays:
                arrays[la] = base.relayout("bs", 1, la)
            arr = arrays[la]
            if trained != (L, la):
                st = arr.learn(L, 2)
                trained = (L, la)
            arr.set_params(**{**lparams, "model": 0})
            r, ro = arr.params()["per_lane"], arr.params()["reorder"]
            ms, ok = time_point(arr, reps=3 if args.sweep else 10, check=True)
            rec = {"layout": "learned", "k": 1, "aos": la, "params": dict(arr.params(), leaves=L), "ms": round(ms, 4),
                   "lookups_per_s": m / ms * 1e3, "bit_exact": ok, "mean_window": st["mean_window"],
                   "max_window": st["max_window"]}
            if arr.params()["leaf_lines"] == 1:
                rec["line_overflow"] = line_overflow(arr, L, 10)
            if not args.sweep:
                rec["ms_cold"] = round(time_point(arr, reps=10, cold=True)[0], 4)
            if args.sweep:
                sweep.append(rec)
            log(f"learned leaves={L} R={r} reorder={ro} aos={la} lines={arr.params()['leaf_lines'] == 1}: "
                f"{ms:.3f} ms exact={ok} mean window {st['mean_window']:.1f}")
            if ok and (lrec is None or ms < lrec["ms"]):
                lrec = rec
        for la, arr in arrays.items():
            if arr is not base:
                arr.close()
        base.unlearn()
        base.reset_params()
        if args.sweep and args.write_table and lrec:
            autotune.save_table(autotune.record_best(autotune.load_table(), 64, n, {**best_by_layout,
                                                                                    "learned": lrec}))

    checked = sweep + [r for r in best_by_layout.values() if r not in sweep] + ([lrec] if lrec else [])
    if not all(r["bit_exact"] for r in checked):
        log("WARNING: some forms were not bit-exact")

    def form_name(r):
        if r["layout"] == "learned":
            return f"LEARNED(leaves={r['params']['leaves']}{',' + ('aos' if r['aos'] is True else str(r['aos'])) if r['aos'] else ''})"
        if r["layout"] != "eks":
            return r["layout"].upper()
        mode = "single" if r["params"]["group"] == 1 else f"group{r['params']['group']}"
        return f"EKS(k={r['k']},{mode}{',aos' if r['aos'] else ''}{',lds' if r['params']['lds_levels'] else ''})"

    forms = [(form_name(best_by_layout[l]), best_by_layout[l]) for l in ("bs", "ebs", "eks")]
    if lrec:
        forms.append((form_name(lrec), lrec))
    base.close()

    def lookup_params(rec):
        p = {kk: v for kk, v in rec["params"].items() if kk != "leaves"}
        p["model"] = 0 if rec["layout"] == "learned" else 2
        return p

    # ---------------------------------------------------------------- steps
    # every form writes its own output buffer, so the outputs of the last
    # timed step can be checked after the timed region
    outs = {name: torch.empty(m, dtype=torch.int32, device=dev) for name, _ in forms}
    last_ranges = {}

    def one_step(record, keep=False):
        t = {}
        a = ev()
        bs = idx.Index(keys, rows, layout="bs")
        b = ev()
        hs = {forms[0][0]: bs if not forms[0][1]["aos"] else bs.relayout("bs", 1, forms[0][1]["aos"])}
        marks = [("build_sort", a, b)]
        for name, rec in forms[1:]:
            if rec["layout"] == "learned":
                # the model attaches to the sorted array itself (copied into
                # the array of structures first when the form uses it)
                a = ev()
                arr = bs if not rec["aos"] else bs.relayout("bs", 1, rec["aos"])
                arr.set_params(**lookup_params(rec))  # leaf lines, when used, are written by the training call
                arr.learn(rec["params"]["leaves"], 2)
                b = ev()
                hs[name] = arr
                marks.append((f"train_{name}", a, b))
                continue
            a = ev()
            hs[name] = bs.relayout(rec["layout"], rec["k"], rec["aos"])
            b = ev()
            marks.append((f"build_permute_{name}", a, b))
        for name, rec in forms:
            hs[name].set_params(**lookup_params(rec))
            a = ev()
            hs[name].point(q, outs[name])
            b = ev()
            marks.append((f"point_{name}", a, b))
        range_forms = [forms[0], forms[2]] + ([forms[3]] if len(forms) > 3 else [])
        for name, rec in range_forms:
            hs[name].set_params(**lookup_params(rec))
            a = ev()
            off, rr = hs[name].range(lo, hi, capacity=mr * 16)
            b = ev()
            marks.append((f"range_{name}", a, b))
            if keep:
                last_ranges[name] = (off, rr)
            del off, rr
        torch.cuda.synchronize()
        for nm, a, b in marks:
            t[nm] = a.elapsed_time(b)
        for h in hs.values():
            h.close()
        record.append(t)

    warm = []
    for _ in range(args.warmup):
        one_step(warm)
    torch.cuda.synchronize()
    rec_steps = []
    t_start = time.perf_counter()
    for st in range(args.steps):
        one_step(rec_steps, keep=st == args.steps - 1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall / args.steps * 1e3

    # bit-exactness of the last timed step's outputs: every point answer
    # against the generator's (query f(i) -> row ID i); every range's offsets
    # (16 keys each) and row IDs (ranks r .. r + 15 of the generator's draw)
    step_exact = {f"point_{name}": bool(torch.equal(outs[name], expect)) for name, _ in forms}
    want_off = torch.arange(mr + 1, device=dev, dtype=torch.int64) * 16
    for name, (off, rr) in last_ranges.items():
        ok = bool(torch.equal(off, want_off))
        for c0 in range(0, mr, 1 << 22):  # 2^22 ranges (2^26 row IDs) at a time
            c1 = min(mr, c0 + (1 << 22))
            pos = (range_first[c0:c1, None] + torch.arange(16, device=dev)[None, :]).reshape(-1)
            ok &= bool(torch.equal(rr[c0 * 16:c1 * 16], sorted_rows[pos]))
        step_exact[f"range_{name}"] = ok
    last_ranges.clear()
    del outs
    failed = [k for k, v in step_exact.items() if not v]
    if failed:
        log(f"ERROR: outputs of the timed steps differ from the generator's answers: {failed}")

    mean = {k: float(np.mean([r[k] for r in rec_steps])) for k in rec_steps[0]}
    point_rates = {name: m / mean[f"point_{name}"] * 1e3 for name, _ in forms}
    exact_forms = [name for name, _ in forms if step_exact[f"point_{name}"]] or [name for name, _ in forms]
    headline = max(exact_forms, key=point_rates.get)
    hrec = dict(forms)[headline]
    value = point_rates[headline]

    # ------------------------------------------------------------ roofline
    ab = algo_bytes(hrec["layout"], n, hrec["k"], 8, early_exit=hrec["params"].get("early_exit", 1) == 1,
                    window=hrec.get("mean_window", 0.0), leaves=hrec["params"].get("leaves", 0),
                    aos=hrec["aos"] if hrec["layout"] == "learned" else False,
                    lines=hrec["params"].get("leaf_lines") == 1, over=hrec.get("line_overflow", 0.0))
    t_kernel = mean[f"point_{headline}"] / 1e3
    achieved = ab["total"] * m / t_kernel / 1e9
    hp = hrec["params"]
    kernel_key = (f"point_{hrec['layout']}_k{hrec['k']}_{'soa' if not hrec['aos'] else hrec['aos'] if hrec['aos'] != True else 'aos'}"
                  f"_g{hp['group']}_r{hp['per_lane']}_l{hp['lds_levels']}_p{hp['persistent']}_b{hp['block']}"
                  f"{'_lines' if hp.get('leaf_lines') == 1 else ''}")
    traffic = read_traffic(kernel_key)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (round(traffic / 1e9 / t_kernel, 1) if traffic else None),
                "kernel": kernel_key, "algorithmic_bytes_per_lookup": ab,
                "launch_ms": round(mean[f"point_{headline}"], 4)}

    # ---------------------------------------- roofline of the range phases
    # each form's whole range call (count, scan, fill) over 2^log2ranges
    # ranges of 16 keys, against the algorithmic bytes per range
    range_roofline = {}
    for name, rec in forms:
        if f"range_{name}" not in mean:
            continue
        lay = rec["layout"]
        rb = algo_bytes_range(lay, n, rec["k"], 8, 16, rank_slot=idx.lib().idx_rank_slot,
                              window=rec.get("mean_window", 0.0), leaves=rec["params"].get("leaves", 0),
                              aos=rec["aos"] if lay == "learned" else False,
                              lines=rec["params"].get("leaf_lines") == 1, over=rec.get("line_overflow", 0.0))
        t = mean[f"range_{name}"] / 1e3
        ach = rb["total"] * mr / t / 1e9
        range_roofline[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_range": rb,
                                "range_call_ms": round(mean[f"range_{name}"], 4)}

    # ------------------------------------------------------ random-access probe
    probe = {}
    try:
        buf = torch.empty(1 << 29, dtype=torch.int64, device=dev)  # 4 GiB, far above the on-chip caches
        for group in (1, 8):
            lanes, steps = 256 * 4096, 32
            idx.probe_random(buf, group, lanes, steps)
            a = ev()
            loads = idx.probe_random(buf, group, lanes, steps)
            b = ev()
            b.synchronize()
            ms = a.elapsed_time(b)
            granules = loads / group
            probe[f"group{group}"] = {"granule_bytes": 8 * group, "granules_per_s": granules / ms * 1e3,
                                      "useful_GB_s": loads * 8 / ms / 1e6}
        del buf
    except Exception as e:  # pragma: no cover - measurement only
        probe["error"] = str(e)
    # the random-access roofline (the paper's Fig. 9 probe design): the probe's
    # rate of independent random requests that miss the caches, A_rand,
    # divided by the lookup's algorithmic granules beyond on-chip capacity, D
    if "group1" in probe:
        a_rand = probe["group1"]["granules_per_s"]
        # (through leaf lines: the random 128-byte lines a lookup reads)
        d_gran = ab["random_lines"] if "random_lines" in ab else (ab["tree"] + ab["rowid"]) / GRANULE
        bound = a_rand / d_gran if d_gran > 0 else None
        roofline["random_access"] = {"a_rand_per_s": a_rand, "granules_per_lookup": d_gran,
                                     "bound_lookups_per_s": bound,
                                     "frac": (value / bound) if bound else None}

    # ------------------------------------------------ small configuration
    small = None if args.no_small else run_small(idx, gen, np, torch, dev, log)

    # ------------------------- EKS fan-out sweep: permutation build and lookups
    ksweep = []
    if not args.no_k_sweep:
        with idx.Index(keys, rows, layout="bs") as kb:
            for k in (4, 8, 16, 32, 5, 9, 17, 33):
                a = ev()
                ix = kb.relayout("eks", k)
                b = ev()
                b.synchronize()
                build_ms = a.elapsed_time(b)
                ms, ok = time_point(ix, reps=3, check=True)
                p_ = ix.params()
                ksweep.append({"k": k, "keys_per_node": k - 1, "build_permute_ms": round(build_ms, 4),
                               "ms": round(ms, 4), "lookups_per_s": m / ms * 1e3, "bit_exact": ok,
                               "group": p_["group"], "per_lane": p_["per_lane"]})
                log(f"k sweep k={k}: permute {build_ms:.3f} ms, lookups {ms:.3f} ms ({m / ms / 1e6:.1f} G/s) "
                    f"exact={ok}")
                ix.close()

    # ------------- hybrid against single-lane level scan over growing hit counts
    scan_row = None
    if not args.no_range_scan:
        scan_row = run_range_scan(idx, np, torch, dev, keys, rows, sorted_rows, log)

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # the host threads this job may use: the machine's CPU share (its thread
        # budget, OMP_NUM_THREADS), not every core the machine reports
        nproc = os.cpu_count() or 1
        share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
        cores = max(1, min(share, nproc))
        ms_ = min(args.cpu_sample, m)
        t0 = time.perf_counter()
        sk, sr = oracle.stable_sort(keys_h, rows_h)
        t_sort = time.perf_counter() - t0
        qs = q.cpu().numpy().view(np.uint64)[:ms_].copy()
        t0 = time.perf_counter()
        got = oracle.point(sk, sr, qs, nthreads=cores)
        t_pt = time.perf_counter() - t0
        cpu_exact = bool(np.array_equal(got, expect_h[:ms_]))
        m1 = ms_ // 8  # the same lookups on one thread
        t0 = time.perf_counter()
        got1 = oracle.point(sk, sr, qs[:m1], nthreads=1)
        t_1 = time.perf_counter() - t0
        cpu_exact = cpu_exact and bool(np.array_equal(got1, expect_h[:m1]))
        cpu = {"value": ms_ / t_pt, "unit": "lookups/s", "cores": cores, "kind": "oracle",
               "value_1thread": m1 / t_1, "nproc": nproc, "affinity_cpus": len(os.sched_getaffinity(0)),
               "sample": f"first {ms_} of the {m} queries against the full n={n} build sorted by the oracle's "
                         f"stable sort ({t_sort:.1f} s, 1 thread); lower_bound + equality per query, "
                         f"{cores} threads; answers equal the generator's: {cpu_exact}"}

    # -------------------------------------------------- batched many-index launch
    batched = None
    if not args.no_batched:
        del out, q, expect
        torch.cuda.empty_cache()
        from paper_2506_01576_amd import autotune as _at
        table = _at.load_table()
        batch_records = None
        if args.sweep:
            batch_sweep, batch_records = _at.tune_batch(gen, 32, log=log)
            table = _at.record_batch(table, 32, batch_sweep)
        batched = run_batched(args, idx, gen, np, torch, dev, log, table)
        if args.sweep:
            batched["class_sweep"] = batch_records
    skewed = None
    if not args.no_skewed:
        torch.cuda.empty_cache()
        skewed = run_skewed(args, idx, gen, np, torch, dev, log)
        torch.cuda.empty_cache()
    update = None
    if not args.no_update:
        torch.cuda.empty_cache()
        update = run_update(args, idx, gen, np, torch, dev, log)
    study = None
    if args.study:
        torch.cuda.empty_cache()
        study = run_study(args, idx, gen, np, torch, dev, log)
    combined = None
    if not args.no_combined:
        torch.cuda.empty_cache()
        combined = run_combined(args, idx, gen, np, torch, dev, log)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "lookups/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"static index, n=2^{args.log2n} unique uint64 keys uniform in [0,2^63), "
                               f"uint32 rowids; 2^{args.log2m} uniform hit point lookups; "
                               f"2^{args.log2ranges} ranges of 16",
                   "form": headline, "layout": hrec["layout"], "k": hrec["k"], "params": hrec["params"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": {name: {"lookups_per_s": point_rates[name], "ms": round(mean[f"point_{name}"], 4),
                         "ms_isolated_warm": rec.get("ms"), "ms_isolated_cold": rec.get("ms_cold"),
                         "layout": rec["layout"], "k": rec["k"], "aos": rec["aos"], "params": rec["params"],
                         **({"mean_window": rec["mean_window"], "max_window": rec["max_window"]}
                            if "mean_window" in rec else {})} for name, rec in forms},
        "phases_ms": {k: round(v, 4) for k, v in mean.items()},
        "range_lookups_per_s": {k[6:]: mr / v * 1e3 for k, v in mean.items() if k.startswith("range_")},
        "range_roofline": range_roofline,
        "bit_exact": (all(r["bit_exact"] for r in checked) and all(step_exact.values())
                      and all(r["bit_exact"] for r in ksweep) and (small is None or small["bit_exact"])
                      and (scan_row is None or scan_row["bit_exact"])),
        "bit_exact_timed_step": step_exact,
        "small": small,
        "k_sweep": ksweep,
        "range_scan": scan_row,
        "random_access": probe,
        "batched": batched,
        "combined": combined,
        "skewed": skewed,
        "study": study,
        "update": update,
        "sweep": [{kk: r[kk] for kk in ("layout", "k", "aos", "params", "ms", "lookups_per_s", "bit_exact")}
                  for r in sweep],
    }
    print(json.dumps(line), flush=True)
    if not line["bit_exact"]:
        sys.exit(1)


if __name__ == "__main__":
    main()

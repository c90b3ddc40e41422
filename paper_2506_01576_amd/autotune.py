"""Autotuner for point lookups: measures candidate forms (layout, fan-out k,
storage, lane grouping, lookups per lane, LDS-pinned levels, persistent grid)
on the device and keeps the fastest per key width and size class in a table.

This generalises the paper's tuning sweeps (Sections 8.2-8.3) and its
composite strategy (Section 10: Eytzinger binary search while the index fits
the cache, k-ary search beyond) into a measured table.  Host-side
orchestration only: every candidate runs through the library's kernels and is
checked bit-exact against a reference answer before it can win.
"""
from __future__ import annotations

import json
import math
import os

import torch

from ._binding import IdxError, Index

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")

# size classes by log2(n): [lo, hi]
SIZE_CLASSES = [(0, 12), (13, 16), (17, 20), (21, 23), (24, 25), (26, 28), (29, 32)]


def size_class(n: int):
    lg = max(0, math.ceil(math.log2(max(n, 1))))
    for lo, hi in SIZE_CLASSES:
        if lo <= lg <= hi:
            return lo, hi
    return SIZE_CLASSES[-1]


def candidates(key_bits: int, n: int):
    """Forms worth measuring for a set of n keys of width key_bits."""
    kb = key_bits // 8
    out = [("bs", 1, False, {}), ("bs", 1, False, {"per_lane": 8}),
           ("ebs", 2, False, {}), ("ebs", 2, False, {"per_lane": 8})]
    lds_ok = n >= 1 << 12
    if lds_ok:
        out.append(("bs", 1, False, {"lds_levels": 12, "persistent": 2, "block": 1024}))
        out.append(("ebs", 2, False, {"lds_levels": 12, "persistent": 2, "block": 1024}))
    for k in (4, 5, 8, 9, 16, 17, 32, 33):
        g = k - 1
        node = g * kb
        out.append(("eks", k, False, {"group": 1 << (g - 1).bit_length(), "per_lane": 4}))
        if g <= 32:
            out.append(("eks", k, False, {"group": 1, "per_lane": 4}))
        v = 16 // kb
        if g % v == 0 and g // v >= 2:
            vg = 1 << ((g // v) - 1).bit_length()
            out.append(("eks", k, False, {"group": vg, "per_lane": 4}))
        if k in (5, 9, 17, 33) and node % 16 == 0 and g <= 32:
            for aos in (False, "padded"):
                # top levels that fit 64 KiB of LDS
                lev, slots = 0, 0
                while (slots + g * k ** lev) * kb <= 64 * 1024:
                    slots += g * k ** lev
                    lev += 1
                if lev and lds_ok:
                    out.append(("eks", k, aos, {"group": 1, "per_lane": 4, "lds_levels": lev, "persistent": 2,
                                                "block": 1024}))
            out.append(("eks", k, "padded", {"group": 1, "per_lane": 4}))
    # lookup reordering (Section 7.4): the tile-local sort, and the batch
    # partitioned by rank bucket, which pays once the index is far larger
    # than one XCD's L2
    out.append(("bs", 1, False, {"reorder": 1, "per_lane": 4, "block": 1024}))
    out.append(("ebs", 2, False, {"reorder": 1, "per_lane": 8, "block": 512}))
    if n >= 1 << 20:
        out.append(("bs", 1, False, {"reorder": 2, "per_lane": 4}))
        out.append(("bs", 1, False, {"reorder": 2, "per_lane": 8}))
        # partitioned and pinned: the top levels from LDS, the rest from L2
        out.append(("bs", 1, False, {"reorder": 2, "per_lane": 4, "lds_levels": 12, "persistent": 2,
                                     "block": 1024}))
        out.append(("ebs", 2, False, {"reorder": 2, "per_lane": 4, "lds_levels": 12, "persistent": 2,
                                      "block": 1024}))
        out.append(("ebs", 2, False, {"reorder": 2, "per_lane": 8}))
        out.append(("ebs", 2, False, {"reorder": 2, "per_lane": 4}))
        out.append(("eks", 9, False, {"group": 1, "per_lane": 4, "reorder": 2}))
        # the partition with each answer written straight to its position
        out.append(("bs", 1, False, {"reorder": 3, "per_lane": 4}))
        out.append(("ebs", 2, False, {"reorder": 3, "per_lane": 4}))
        out.append(("eks", 17, "padded", {"group": 1, "per_lane": 4, "reorder": 2}))
    return out


def learned_candidates(n: int):
    """Learned forms worth measuring: (leaves, lookup parameters, storage).
    Leaf lines pay off when most leaves fit a line (a few keys per leaf on
    average)."""
    out = {}
    for per_leaf in (64, 16, 8):
        L = max(1, min(1 << 22, n // per_leaf))
        for r in (4, 8):
            for aos in (False, True):
                out[(L, r, 0, 0, aos)] = (L, {"per_lane": r}, aos)
    for per_leaf in (4, 2):
        L = max(1, min(1 << 24, n // per_leaf))
        for r in (2, 4):
            for block in (128, 256):
                for aos in (False, True):
                    out[(L, r, 1, block, aos)] = (L, {"per_lane": r, "leaf_lines": 1, "block": block}, aos)
    return [out[k] for k in sorted(out, key=lambda c: (c[0], c[1], c[2], c[3], str(c[4])))]


def tune_learned(base: Index, q: torch.Tensor, expect: torch.Tensor, cands=None, reps: int = 3, log=None):
    """Train the rank model on `base`'s sorted array (and on its packed
    array-of-structures copy) for every candidate leaf count and time the
    model lookups; returns (records, best record)."""
    cands = cands if cands is not None else learned_candidates(base.n)
    out = torch.empty(len(q), dtype=torch.int32, device=q.device)
    arrays, records, best, trained = {False: base}, [], None, {}
    try:
        for L, params, aos in cands:
            if aos not in arrays:
                arrays[aos] = base.relayout("bs", 1, aos)
            arr = arrays[aos]
            if trained.get(aos) != L:
                st = arr.learn(L, 2)
                trained[aos] = L
            arr.set_params(**params, model=0)
            ms = _time_point(arr, q, out, reps)
            exact = bool(torch.equal(out, expect))
            rec = {"layout": "learned", "k": 1, "aos": aos, "params": dict(arr.params(), leaves=L),
                   "ms": round(ms, 4), "lookups_per_s": len(q) / ms * 1e3, "bit_exact": exact,
                   "mean_window": st["mean_window"]}
            records.append(rec)
            if log:
                log(f"tune learned leaves={L} {params} aos={aos}: {ms:.3f} ms {rec['lookups_per_s'] / 1e9:.2f} G/s "
                    f"exact={exact}")
            if exact and (best is None or ms < best["ms"]):
                best = rec
    finally:
        for aos, arr in arrays.items():
            if arr is not base:
                arr.close()
        base.unlearn()
        base.reset_params()
    return records, best


def _time_point(ix: Index, q: torch.Tensor, out: torch.Tensor, reps: int) -> float:
    stream = torch.cuda.current_stream()
    ix.point(q, out)
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ix.point(q, out)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(base: Index, q: torch.Tensor, expect: torch.Tensor, cands=None, reps: int = 3, log=None):
    """Measure every candidate form built from the sorted index `base` on the
    queries `q`; a candidate whose answers differ from `expect` is recorded
    but can never win.  Returns (records, best record per layout)."""
    cands = cands if cands is not None else candidates(base.key_bits, base.n)
    out = torch.empty(len(q), dtype=torch.int32, device=q.device)
    records, best = [], {}
    for layout, k, aos, params in cands:
        ix = base if (layout == "bs" and not aos) else base.relayout(layout, k, aos)
        try:
            try:
                ix.set_params(**params)
            except IdxError:
                continue
            ms = _time_point(ix, q, out, reps)
            exact = bool(torch.equal(out, expect))
            rec = {"layout": layout, "k": k, "aos": aos, "params": ix.params(), "ms": round(ms, 4),
                   "lookups_per_s": len(q) / ms * 1e3, "bit_exact": exact}
            records.append(rec)
            if log:
                log(f"tune {layout} k={k} aos={aos} {params}: {ms:.3f} ms {rec['lookups_per_s'] / 1e9:.2f} G/s "
                    f"exact={exact}")
            if exact and (layout not in best or ms < best[layout]["ms"]):
                best[layout] = rec
        finally:
            if ix is not base:
                ix.close()
            else:
                ix.reset_params()
    return records, best


def load_table(path: str = TABLE_PATH) -> dict:
    if not os.path.exists(path):
        return {"device": "gfx950", "entries": []}
    with open(path) as f:
        return json.load(f)


def save_table(table: dict, path: str = TABLE_PATH):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")


def record_best(table: dict, key_bits: int, n: int, best: dict):
    lo, hi = size_class(n)
    table["entries"] = [e for e in table["entries"]
                        if not (e["key_bits"] == key_bits and e["log2n_lo"] == lo and e["layout"] in best)]
    for layout, rec in best.items():
        table["entries"].append({"key_bits": key_bits, "log2n_lo": lo, "log2n_hi": hi, "layout": layout,
                                 "k": rec["k"], "aos": rec["aos"], "params": rec["params"],
                                 "measured_n": n, "lookups_per_s": rec["lookups_per_s"]})
    return table


def choose(n: int, key_bits: int, layout: str | None = None, table: dict | None = None):
    """Best known form for n keys of width key_bits (optionally of one
    layout): (layout, k, aos, params).  Falls back to the library defaults and
    to the size class nearest in log2(n)."""
    table = table if table is not None else load_table()
    lg = max(0, math.ceil(math.log2(max(n, 1))))
    ents = [e for e in table.get("entries", []) if e["key_bits"] == key_bits
            and (layout is None or e["layout"] == layout)]
    if not ents:
        lay = layout or "eks"
        if lay == "learned":
            return lay, 1, False, {"leaves": max(1, min(1 << 22, n // 16))}
        return lay, {"bs": 1, "ebs": 2, "eks": 9}[lay], False, {}

    def dist(e):
        if e["log2n_lo"] <= lg <= e["log2n_hi"]:
            return 0
        return min(abs(lg - e["log2n_lo"]), abs(lg - e["log2n_hi"]))

    ents.sort(key=lambda e: (dist(e), -e["lookups_per_s"]))
    e = ents[0]
    return e["layout"], e["k"], e["aos"], dict(e["params"])


# --------------------------------------------------------------- batched
# Forms the batched launch supports: (layout, k, learned keys per leaf or 0,
# lookup parameters the batch takes from each member: "group" = EKS lanes
# per lookup (1 = whole node per lane; >= k-1 = one pivot per lane; fewer =
# one 16-byte chunk per lane), "lds_levels" = top levels pinned in LDS, cut to
# what the member's size allows).
BATCH_FORMS = [
    ("bs", 1, 0, {}), ("bs", 1, 0, {"lds_levels": 10}),
    ("ebs", 2, 0, {}), ("ebs", 2, 0, {"lds_levels": 10}),
    ("eks", 5, 0, {"group": 1}), ("eks", 5, 0, {"group": 4}), ("eks", 5, 0, {"group": 1, "lds_levels": 4}),
    ("eks", 9, 0, {"group": 1}), ("eks", 9, 0, {"group": 8}), ("eks", 9, 0, {"group": 2}),
    ("eks", 9, 0, {"group": 1, "lds_levels": 3}),
    ("eks", 17, 0, {"group": 1}), ("eks", 17, 0, {"group": 16}), ("eks", 17, 0, {"group": 4}),
    ("eks", 17, 0, {"group": 1, "lds_levels": 2}),
    ("bs", 1, 64, {}), ("bs", 1, 16, {}),
]
BATCH_CLASSES = [(6, 8), (9, 11), (12, 14), (15, 17), (18, 20), (21, 22)]


def _form(form):
    """(layout, k, keys per leaf, params) from a table or list entry (older
    three-field entries carry no parameters)."""
    if isinstance(form, dict):
        return form["layout"], form["k"], form["keys_per_leaf"], dict(form.get("params", {}))
    if len(form) == 3:
        return form[0], form[1], form[2], {}
    return form[0], form[1], form[2], dict(form[3])


def build_form(keys: torch.Tensor, rows: torch.Tensor, form) -> Index:
    """Build one index in a batch form and set the lookup parameters the
    batch takes from it; pinned levels are cut to what the index allows."""
    layout, k, per_leaf, params = _form(form)
    ix = Index(keys, rows, layout=layout, k=k)
    if per_leaf:
        ix.learn(max(1, len(keys) // per_leaf), 2)
    if params:
        lev = params.get("lds_levels", 0)
        while True:
            try:
                ix.set_params(**{**params, "lds_levels": lev})
                break
            except IdxError:
                if lev == 0:
                    ix.close()
                    raise
                lev -= 1
    return ix


def tune_batch(gen_module, key_bits: int = 32, per_class: int = 64, queries_per_index: int = 1 << 14,
               seed: int = 7, forms=None, log=None):
    """For every size class, time the batched launch over `per_class`
    indexes built in each candidate form (layout, k, model, lanes per lookup,
    pinned levels); returns ({class_lo: best record}, all records).  A form
    whose answers differ from the generator's can never win."""
    from ._binding import Batch
    import numpy as np

    best, records = {}, []
    dev = torch.device("cuda")
    forms = forms if forms is not None else BATCH_FORMS
    for lo, hi in BATCH_CLASSES:
        sizes = gen_module.log_uniform(seed + lo, 3, 1 << lo, 1 << hi, per_class)
        sets, qs, ex = [], [], []
        for j, n in enumerate(sizes.tolist()):
            kh, rh = gen_module.unique_keys(seed * 1000 + lo * 100 + j, int(n), key_bits)
            qh, eh = gen_module.point_queries(seed * 1000 + lo * 100 + j, int(n), queries_per_index, 0.8, key_bits)
            sets.append((kh, rh))
            qs.append(qh)
            ex.append(eh)
        view = np.int32 if key_bits == 32 else np.int64
        dq = torch.from_numpy(np.concatenate(qs).view(view)).to(dev)
        de = torch.from_numpy(np.concatenate(ex).view(np.int32)).to(dev)
        off = np.zeros(per_class + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(q) for q in qs])
        doff = torch.from_numpy(off).to(dev)
        out = torch.empty(len(dq), dtype=torch.int32, device=dev)
        for form in forms:
            layout, k, per_leaf, params = _form(form)
            idxs = [build_form(torch.from_numpy(kh.view(view)).to(dev), torch.from_numpy(rh.view(np.int32)).to(dev),
                               form) for kh, rh in sets]
            used = idxs[0].params()
            with Batch(idxs) as bt:
                out.fill_(-1)
                bt.point(dq, doff, out)
                torch.cuda.synchronize()
                exact = bool(torch.equal(out, de))
                # median over 5 samples of 10 back-to-back launches each
                ts = []
                for _ in range(5):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    for _ in range(10):
                        bt.point(dq, doff, out)
                    b.record()
                    b.synchronize()
                    ts.append(a.elapsed_time(b) / 10)
                ms = sorted(ts)[len(ts) // 2]
            for ix in idxs:
                ix.close()
            rec = {"log2n_lo": lo, "log2n_hi": hi, "layout": layout, "k": k, "keys_per_leaf": per_leaf,
                   "params": {f: used[f] for f in ("group", "lds_levels") if f in params},
                   "ms": round(ms, 4), "lookups_per_s": len(dq) / ms * 1e3, "bit_exact": exact}
            records.append(rec)
            if log:
                log(f"batch class 2^{lo}-2^{hi} {layout} k={k} leaf={per_leaf} {params}: {ms:.4f} ms "
                    f"{rec['lookups_per_s'] / 1e9:.2f} G/s exact={exact}")
            if exact and (lo not in best or ms < best[lo]["ms"]):
                best[lo] = rec
    return best, records


def batch_class_of(n: int):
    """The batch size class (lo, hi) of an index of n keys."""
    lg = max(0, math.ceil(math.log2(max(n, 1))))
    for lo, hi in BATCH_CLASSES:
        if lg <= hi:
            return lo, hi
    return BATCH_CLASSES[-1]


def tune_batch_joint(gen_module, key_bits: int = 32, count: int = 1024, seed: int = 11, forms=None, table=None,
                     log=None):
    """Coordinate descent over the size classes on one representative batch:
    `count` indexes with n log-uniform in [2^6, 2^22] and query batches
    log-uniform in [1, 2^16] with 80% hits (the many-index configuration
    scaled down), all served by one launch, so each class is timed under the
    cache pressure of the others.  Every index starts in its class's current
    form (the table's, else the per-class measurement's); class by class,
    largest first, each candidate form is built for that class's indexes and
    the whole launch is timed (median of 5 samples of 10 launches); the
    fastest bit-exact form is kept before the next class.  Returns
    ({class_lo: best record}, all records)."""
    from ._binding import Batch
    import numpy as np

    forms = forms if forms is not None else BATCH_FORMS
    table = table if table is not None else load_table()
    dev = torch.device("cuda")
    view = np.int32 if key_bits == 32 else np.int64
    sizes = gen_module.log_uniform(seed, 1, 1 << 6, 1 << 22, count)
    qcounts = gen_module.log_uniform(seed, 2, 1, 1 << 16, count)
    keys, rows, qs, ex = [], [], [], []
    for j in range(count):
        kh, rh = gen_module.unique_keys(seed * 100003 + j, int(sizes[j]), key_bits)
        qh, eh = gen_module.point_queries(seed * 100003 + j, int(sizes[j]), int(qcounts[j]), 0.8, key_bits)
        keys.append(torch.from_numpy(kh.view(view)).to(dev))
        rows.append(torch.from_numpy(rh.view(np.int32)).to(dev))
        qs.append(qh)
        ex.append(eh)
    dq = torch.from_numpy(np.concatenate(qs).view(view)).to(dev)
    de = torch.from_numpy(np.concatenate(ex).view(np.int32)).to(dev)
    off = np.zeros(count + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(q) for q in qs])
    doff = torch.from_numpy(off).to(dev)
    out = torch.empty(len(dq), dtype=torch.int32, device=dev)
    cls = [batch_class_of(int(n))[0] for n in sizes]
    current = {lo: batch_form(1 << lo, key_bits, table) for lo, _ in BATCH_CLASSES}
    idxs = [build_form(keys[j], rows[j], current[cls[j]]) for j in range(count)]

    def timed():
        with Batch(idxs) as bt:
            out.fill_(-1)
            bt.point(dq, doff, out)
            torch.cuda.synchronize()
            exact = bool(torch.equal(out, de))
            ts = []
            for _ in range(5):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(10):
                    bt.point(dq, doff, out)
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b) / 10)
        return sorted(ts)[len(ts) // 2], exact

    best, records = {}, []
    try:
        for lo, hi in reversed(BATCH_CLASSES):
            members = [j for j in range(count) if cls[j] == lo]
            if not members:
                continue
            for form in forms:
                layout, k, per_leaf, params = _form(form)
                for j in members:
                    idxs[j].close()
                    idxs[j] = build_form(keys[j], rows[j], form)
                used = idxs[members[0]].params()
                ms, exact = timed()
                rec = {"log2n_lo": lo, "log2n_hi": hi, "layout": layout, "k": k, "keys_per_leaf": per_leaf,
                       "params": {f: used[f] for f in ("group", "lds_levels") if f in params},
                       "ms": round(ms, 4), "lookups_per_s": len(dq) / ms * 1e3, "bit_exact": exact,
                       "members": len(members), "lookups_in_class": int(sum(int(qcounts[j]) for j in members))}
                records.append(rec)
                if log:
                    log(f"batch joint class 2^{lo}-2^{hi} ({len(members)} indexes) {layout} k={k} leaf={per_leaf} "
                        f"{params}: whole launch {ms:.4f} ms exact={exact}")
                if exact and (lo not in best or ms < best[lo]["ms"]):
                    best[lo] = rec
            win = best[lo]
            current[lo] = (win["layout"], win["k"], win["keys_per_leaf"], win["params"])
            for j in members:
                idxs[j].close()
                idxs[j] = build_form(keys[j], rows[j], current[lo])
    finally:
        for ix in idxs:
            ix.close()
    return best, records


def record_batch(table: dict, key_bits: int, best: dict):
    table["batch"] = [e for e in table.get("batch", []) if e["key_bits"] != key_bits]
    for lo, rec in sorted(best.items()):
        table["batch"].append({"key_bits": key_bits, **rec})
    return table


def batch_form(n: int, key_bits: int, table: dict | None = None):
    """(layout, k, keys per leaf, params) for an index of n keys in a batch."""
    table = table if table is not None else load_table()
    lg = max(0, math.ceil(math.log2(max(n, 1))))
    ents = [e for e in table.get("batch", []) if e["key_bits"] == key_bits]
    if not ents:
        return ("ebs", 2, 0, {}) if lg <= 16 else ("eks", 9, 0, {})

    def dist(e):
        if e["log2n_lo"] <= lg <= e["log2n_hi"]:
            return 0
        return min(abs(lg - e["log2n_lo"]), abs(lg - e["log2n_hi"]))

    return _form(min(ents, key=dist))


# --------------------------------------------------------------- command line
def _main(argv=None):
    """python -m paper_2506_01576_amd.autotune [--point] [--batch] [--bits 32,64]
    [--log2n 12,16,...] [--log2m 24] [--write]: measure the candidate forms on
    the GPU (seeded synthetic keys, uniform unique; half of the point lookups
    miss) and, with --write, store the winners in the tuned table."""
    import argparse
    import sys
    import time

    import numpy as np

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import gen

    ap = argparse.ArgumentParser(prog="python -m paper_2506_01576_amd.autotune")
    ap.add_argument("--point", action="store_true", help="single-index forms per size class")
    ap.add_argument("--learned-only", action="store_true",
                    help="with --point: measure only the learned forms (other entries are kept)")
    ap.add_argument("--batch", action="store_true", help="batched-launch forms per size class")
    ap.add_argument("--batch-joint", action="store_true",
                    help="batched-launch forms per size class, timed inside one representative many-index launch")
    ap.add_argument("--bits", default="32,64")
    ap.add_argument("--log2n", default="12,16,20,23,25,26,29",
                    help="one measured size per class (log2 of the key count)")
    ap.add_argument("--log2m", type=int, default=24, help="point lookups per measurement (log2)")
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--out", default=TABLE_PATH, help="table file read and written (default: the package's table)")
    args = ap.parse_args(argv)
    t_start = time.time()

    def log(msg):
        print(f"[{time.time() - t_start:7.1f}s] {msg}", flush=True)

    dev = torch.device("cuda")
    table = load_table(args.out if os.path.exists(args.out) else TABLE_PATH)
    for bits in [int(b) for b in args.bits.split(",")]:
        view = np.int32 if bits == 32 else np.int64
        if args.point:
            for lg in [int(x) for x in args.log2n.split(",")]:
                n, m = 1 << lg, 1 << args.log2m
                seed = 0x2506_01576 + 100 + lg
                kh, rh = gen.unique_keys(seed, n, bits)
                qh, eh = gen.point_queries(seed, n, m, 0.5, bits)
                keys = torch.from_numpy(kh.view(view)).to(dev)
                rows = torch.from_numpy(rh.view(np.int32)).to(dev)
                q = torch.from_numpy(qh.view(view)).to(dev)
                expect = torch.from_numpy(eh.view(np.int32)).to(dev)
                del kh, rh, qh, eh
                log(f"point: {bits}-bit keys, n = 2^{lg}, {m} lookups")
                with Index(keys, rows, layout="bs") as base:
                    best = {} if args.learned_only else tune(base, q, expect, log=log)[1]
                    _, lbest = tune_learned(base, q, expect, log=log)
                if lbest:
                    best["learned"] = lbest
                for lay, rec in sorted(best.items()):
                    log(f"point {bits}-bit 2^{lg} best {lay}: k={rec['k']} aos={rec['aos']} "
                        f"{rec['lookups_per_s'] / 1e9:.2f} G/s")
                table = record_best(table, bits, n, best)
                del keys, rows, q, expect
                torch.cuda.empty_cache()
                if args.write:
                    save_table(table, args.out)
        if args.batch or args.batch_joint:
            if args.batch_joint:
                best, _ = tune_batch_joint(gen, bits, table=table, log=log)
            else:
                best, _ = tune_batch(gen, bits, log=log)
            table = record_batch(table, bits, best)
            for lo, rec in sorted(best.items()):
                log(f"batch {bits}-bit class 2^{lo}: {rec['layout']} k={rec['k']} leaf={rec['keys_per_leaf']} "
                    f"{rec['params']} {rec['lookups_per_s'] / 1e9:.2f} G/s")
            if args.write:
                save_table(table, args.out)
    log("done")


if __name__ == "__main__":
    _main()

"""Host logic of the autotuner: table lookups by size class and key width,
the batch forms with their lookup parameters, and the candidate lists (no
GPU: the measurements themselves run in the GPU tests and the benchmark)."""
import json

import pytest

from paper_2506_01576_amd import autotune


def test_size_classes_cover_every_size():
    for lg in range(0, 33):
        lo, hi = autotune.size_class(1 << lg)
        assert lo <= lg <= hi


def test_table_has_every_class_for_both_key_widths():
    table = autotune.load_table()
    for bits in (32, 64):
        for lo, hi in autotune.SIZE_CLASSES:
            layouts = {e["layout"] for e in table["entries"] if e["key_bits"] == bits and e["log2n_lo"] == lo}
            assert layouts == {"bs", "ebs", "eks", "learned"}, (bits, lo)
    for lo, hi in autotune.BATCH_CLASSES:
        assert any(e["key_bits"] == 32 and e["log2n_lo"] == lo for e in table["batch"]), lo


def test_choose_returns_measured_entries():
    table = autotune.load_table()
    for bits, n in ((32, 1 << 16), (64, 1 << 26), (64, 1 << 29), (32, 1000)):
        for layout in ("bs", "ebs", "eks", "learned"):
            lay, k, aos, params = autotune.choose(n, bits, layout, table)
            assert lay == layout
            ents = [e for e in table["entries"] if e["key_bits"] == bits and e["layout"] == layout
                    and e["log2n_lo"] <= max(0, (n - 1).bit_length()) <= e["log2n_hi"]]
            assert ents and ents[0]["k"] == k and ents[0]["aos"] == aos


def test_choose_falls_back_without_a_table():
    empty = {"entries": []}
    assert autotune.choose(1 << 20, 64, "eks", empty)[:2] == ("eks", 9)
    lay, k, aos, p = autotune.choose(1 << 20, 64, "learned", empty)
    assert lay == "learned" and p["leaves"] == (1 << 20) // 16


def test_batch_form_carries_parameters():
    table = {"batch": [{"key_bits": 32, "log2n_lo": 6, "log2n_hi": 8, "layout": "ebs", "k": 2, "keys_per_leaf": 0,
                        "params": {"lds_levels": 7}},
                       {"key_bits": 32, "log2n_lo": 9, "log2n_hi": 11, "layout": "eks", "k": 9, "keys_per_leaf": 0},
                       {"key_bits": 32, "log2n_lo": 12, "log2n_hi": 22, "layout": "bs", "k": 1,
                        "keys_per_leaf": 16, "params": {}}]}
    assert autotune.batch_form(100, 32, table) == ("ebs", 2, 0, {"lds_levels": 7})
    assert autotune.batch_form(1000, 32, table) == ("eks", 9, 0, {})  # an entry without parameters
    assert autotune.batch_form(1 << 20, 32, table) == ("bs", 1, 16, {})
    assert autotune.batch_form(1 << 30, 32, table) == ("bs", 1, 16, {})  # nearest class
    assert autotune.batch_form(100, 64, {"batch": []}) == ("ebs", 2, 0, {})


def test_candidate_lists():
    c = autotune.candidates(64, 1 << 26)
    assert ("eks", 9, False, {"group": 1, "per_lane": 4}) in c
    assert any(p.get("reorder") == 2 and p.get("lds_levels") for _, _, _, p in c)
    assert not any(p.get("reorder") == 2 for _, _, _, p in autotune.candidates(32, 1 << 12))
    lc = autotune.learned_candidates(1 << 20)
    assert (1 << 16, {"per_lane": 4}, False) in lc
    assert all(1 <= L <= 1 << 22 for L, p, _ in lc if not p.get("leaf_lines"))
    assert (1 << 18, {"per_lane": 2, "leaf_lines": 1, "block": 128}, True) in lc
    assert all(L <= 1 << 24 for L, _, _ in lc)
    forms = [autotune._form(f) for f in autotune.BATCH_FORMS]
    assert any(p.get("group", 1) > 1 for _, _, _, p in forms)
    assert any(p.get("lds_levels") for _, _, _, p in forms)


def test_table_is_valid_json_with_exact_records():
    with open(autotune.TABLE_PATH) as f:
        table = json.load(f)
    assert table["device"] == "gfx950"
    for e in table["entries"]:
        assert e["lookups_per_s"] > 0 and e["measured_n"] >= 1
    for e in table["batch"]:
        assert e["bit_exact"] is True


def test_record_best_replaces_only_the_measured_layouts():
    table = {"device": "gfx950", "entries": []}
    rec = {"k": 1, "aos": False, "params": {"per_lane": 4}, "lookups_per_s": 1e9}
    table = autotune.record_best(table, 64, 1 << 26, {"bs": rec, "learned": dict(rec, params={"leaves": 4})})
    table = autotune.record_best(table, 64, 1 << 26, {"learned": dict(rec, params={"leaves": 8}, lookups_per_s=2e9)})
    lay = sorted(e["layout"] for e in table["entries"])
    assert lay == ["bs", "learned"]
    assert autotune.choose(1 << 26, 64, "learned", table=table)[3] == {"leaves": 8}

"""Host logic of the batch autotuner: the pick rule, the table it writes for
each precision, and the table shipped next to the package (CPU only)."""
import json
import os

import pytest

import paper_2603_07038_amd as etm
from paper_2603_07038_amd import tune


def test_pick_takes_the_longest_chunk_among_the_tied():
    # (layout, chunk) -> us per step; 2 % of 100 is the tie band
    res = {(1, 2): 100.0, (1, 6): 101.5, (1, 12): 101.9, (1, 24): 102.5, (2, 12): 101.0, (2, 16): 101.9}
    assert tune.pick(res) == (2, 16)
    # runs before row segments at the same chunk
    assert tune.pick({(2, 8): 100.0, (1, 8): 101.0, (1, 4): 99.5}) == (1, 8)
    # nothing tied: the fastest
    assert tune.pick({(0, 2): 90.0, (0, 4): 100.0, (0, 24): 120.0}) == (0, 2)


def _fake_time_class(c, steps, precision):
    res = {}
    layouts = (1, 2) if precision == etm.ETM_PREC_MIXED else (0,)
    for lay in layouts:
        for kc in tune.CANDIDATES:
            res[(lay, kc)] = 100.0 + abs(kc - (4 + c % 3)) * 5.0 + (3.0 if lay == 2 else 0.0)
    return res, 4, 2 ** c


def test_table_merge_per_precision(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "time_class", _fake_time_class)
    out = tmp_path / "t.json"
    tune.main(["--out", str(out), "--classes", "15-17", "--precision", "mixed"])
    t = json.loads(out.read_text())
    # class 15: 4 alone within 2 %; 16: 4 and 6 tie, the longer wins; 17: 6
    assert t["kchunk"] == {"15": 4, "16": 6, "17": 6}
    assert set(t["layout"].values()) == {1}
    assert "timings_us" in t and "kchunk_fp64" not in t
    mixed = dict(t)
    # an FP64 run records its timings and keeps the mixed maps
    tune.main(["--out", str(out), "--classes", "15-16", "--precision", "fp64"])
    t = json.loads(out.read_text())
    for k in ("kchunk", "layout", "timings_us"):
        assert t[k] == mixed[k]
    assert set(t["timings_fp64_us"]) == {"15", "16"} and "kchunk_fp64" not in t
    assert all(key.startswith("tile/") for key in t["timings_fp64_us"]["15"])
    # its picks only on request
    tune.main(["--out", str(out), "--classes", "15-16", "--precision", "fp64", "--fp64-map"])
    t = json.loads(out.read_text())
    assert set(t["kchunk_fp64"]) == {"15", "16"}
    assert all(v in tune.CANDIDATES for v in t["kchunk_fp64"].values())
    assert t["kchunk"] == mixed["kchunk"]


def test_shipped_table_is_well_formed():
    with open(tune.DEFAULT_TABLE) as f:
        t = json.load(f)
    assert set(t["kchunk"]) == {str(c) for c in range(15, 25)}
    assert all(v in tune.CANDIDATES for v in t["kchunk"].values())
    assert set(t["layout"]) == set(t["kchunk"]) and set(t["layout"].values()) <= {1, 2}
    # FP64 classes take the library's automatic chunk (no map shipped)
    assert "kchunk_fp64" not in t
    for c, row in t["timings_us"].items():
        lay, kc = (1 if t["layout"][c] == 1 else 2), t["kchunk"][c]
        best = min(row.values())
        key = f"{'runs' if lay == 1 else 'rows'}/{kc}"
        assert row[key] <= (1.0 + tune.TIE) * best + 1e-9, (c, key)

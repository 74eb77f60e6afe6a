"""The committed tuning file and its conversion to mr_tune_entry records.

The tuning is a measurement (candidate launch parameters timed by the
runtime on an MI355X), so there is no reference value to pin it to; these
checks pin its form: every map kind's buckets tile [0, 2^62) without gaps,
every field lies in the set mr_tune_set accepts, each bucket keeps the
fastest measured candidate when it saves at least 3% over the defaults and
the defaults otherwise, and every candidate of the grid was measured.
"""
import json

import pytest

from paper_1309_0215_amd import _lib as L
from paper_1309_0215_amd import autotune as A
from paper_1309_0215_amd import tune_entries

DOC = json.load(open(A.TUNING_PATH))


def test_buckets_tile_the_size_axis():
    for kind, buckets in (("words", A.WORD_BUCKETS), ("u32", A.U32_BUCKETS)):
        es = [e for e in DOC["entries"] if e["kind"] == kind]
        assert [(e["bytes_lo"], e["bytes_hi"]) for e in es] == buckets
        assert es[0]["bytes_lo"] == 0 and es[-1]["bytes_hi"] == 1 << 62
        assert all(a["bytes_hi"] == b["bytes_lo"] for a, b in zip(es, es[1:]))


def test_fields_are_in_range():
    for e in DOC["entries"]:
        assert set(e) <= {"kind", "bytes_lo", "bytes_hi", "lds_slots", "max_load_pct", "map_grid_pct", "lds_array_bytes"}
        assert e.get("lds_slots", 0) in (0, 256, 1024, 2048, 4096)
        assert 0 <= e.get("max_load_pct", 0) <= 95
        assert 0 <= e.get("map_grid_pct", 0) <= 100
        assert 0 <= e.get("lds_array_bytes", 0) <= 65536


def test_each_bucket_keeps_its_best_measured_setting():
    cands = {"words": A.WORD_CANDIDATES, "u32": A.U32_CANDIDATES}
    for e, m in zip(DOC["entries"], DOC["measurements"]):
        assert (e["kind"], e["bytes_lo"], e["bytes_hi"]) == (m["kind"], m["bytes_lo"], m["bytes_hi"])
        rows = m["all"]
        assert len(rows) == len(cands[e["kind"]]) and all(r["ms"] > 0 for r in rows)
        assert [{k: v for k, v in r.items() if k != "ms"} for r in rows] == cands[e["kind"]]
        best = min(rows, key=lambda r: r["ms"])
        params = {k: v for k, v in e.items() if k not in ("kind", "bytes_lo", "bytes_hi")}
        if best["ms"] <= (1 - A.MIN_GAIN) * m["default_ms"]:
            assert params == {k: v for k, v in best.items() if k != "ms"}
        else:
            assert params == {}


def test_entry_records():
    arr = tune_entries(DOC["entries"])
    for rec, e in zip(arr, DOC["entries"]):
        assert rec.kind == {"words": L.MAP_WORDS, "u32": L.MAP_U32_KEYS}[e["kind"]]
        assert (rec.bytes_lo, rec.bytes_hi) == (e["bytes_lo"], e["bytes_hi"])
        assert rec.lds_slots == e.get("lds_slots", 0) and rec.max_load_pct == e.get("max_load_pct", 0)
        assert rec.map_grid_pct == e.get("map_grid_pct", 0) and rec.lds_array_bytes == e.get("lds_array_bytes", 0)
    with pytest.raises(KeyError):
        tune_entries([dict(kind="rgb", bytes_lo=0, bytes_hi=1)])

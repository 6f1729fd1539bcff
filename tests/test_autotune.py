"""The autotuner's table logic (no GPU needed: the knobs are process-wide settings of the library)."""
import json

import pytest

from paper_1911_02675_amd import autotune, lsq


def test_bucket_is_largest_not_above_d():
    assert autotune.bucket(1) == "64"
    assert autotune.bucket(64) == "64"
    assert autotune.bucket(255) == "64"
    assert autotune.bucket(256) == "256"
    assert autotune.bucket(5000) == "1024"


def test_choose_and_apply_from_table(tmp_path):
    entry = {"fused_groups_per_cu": {"f32": {"64": 4, "256": 8, "1024": 16}, "f64": {"64": 2}},
             "batched_slots": 192}
    assert autotune.choose(entry, "f32", 300) == {"fused_groups_per_cu": 8, "batched_slots": 192}
    assert autotune.choose(entry, "f64", 4096) == {"fused_groups_per_cu": 2, "batched_slots": 192}
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"gfxTEST": entry}))
    try:
        assert autotune.apply("f32", 2048, arch="gfxTEST", path=str(p)) == {"fused_groups_per_cu": 16,
                                                                             "batched_slots": 192}
        assert autotune.apply("f32", 2048, arch="gfxOTHER", path=str(p)) == {}
    finally:
        lsq.tune("fused_groups_per_cu", 8)
        lsq.tune("batched_slots", 0)


def test_bad_knob_values_rejected():
    with pytest.raises(lsq.LsqError):
        lsq.tune("fused_groups_per_cu", 0)
    with pytest.raises(lsq.LsqError):
        lsq.tune("no_such_knob", 1)

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


def test_choose_all_knobs_and_fold_threshold():
    entry = {"fused_groups_per_cu": {"f32": {"1024": 2}},
             "srht": {"f32": {"1024": {"srht_passa_wgs": 65536, "srht_passb_wgs": 4096, "fold8_rows": 96,
                                       "stream_rows": 160},
                              "256": {"srht_passa_wgs": 32768, "srht_passb_wgs": 8192, "fold8_rows": 48,
                                      "stream_rows": 192}},
                      "f64": {"1024": {"srht_passa_wgs": 262144, "srht_passb_wgs": 4096, "fold8_rows": 80,
                                       "stream_rows": 128}}},
             "gauss_wgs": 2048, "gauss_planes_wgs": 512, "gram_wgs": {"256": 1024, "1024": 4096}}
    assert autotune.choose(entry, "f32", 1024) == {"fused_groups_per_cu": 2, "srht_passa_wgs": 65536,
                                                   "srht_passb_wgs": 4096, "srht_fold8_rows_f32": 96,
                                                   "srht_fold8_rows_f64": 80, "srht_stream_rows_f32": 160,
                                                   "srht_stream_rows_f64": 128, "gauss_wgs": 2048,
                                                   "gauss_planes_wgs": 512, "gram_wgs": 4096}
    assert autotune.choose(entry, "f64", 1024)["srht_passa_wgs"] == 262144
    # d = 300 takes the 256 bucket; a bucket without SRHT entries takes the nearest measured one
    v = autotune.choose(entry, "f32", 300)
    assert v["srht_fold8_rows_f32"] == 48 and v["srht_stream_rows_f32"] == 192 and v["gram_wgs"] == 1024
    assert autotune.choose(entry, "f32", 64)["srht_passa_wgs"] == 32768
    # the 8-point form from the smallest count where it stays faster
    t4 = {32: 1.0, 48: 1.0, 64: 1.0, 96: 1.0}
    assert autotune._fold_threshold(t4, {32: 0.9, 48: 1.1, 64: 0.9, 96: 0.8}) == 64
    assert autotune._fold_threshold(t4, {32: 1.2, 48: 1.1, 64: 1.1, 96: 1.1}) == 97
    assert autotune._fold_threshold(t4, {32: 0.5, 48: 0.5, 64: 0.5, 96: 0.5}) == 32


def test_bad_knob_values_rejected():
    with pytest.raises(lsq.LsqError):
        lsq.tune("fused_groups_per_cu", 0)
    with pytest.raises(lsq.LsqError):
        lsq.tune("no_such_knob", 1)
    for key, bad in (("srht_fold8_rows_f32", 0), ("srht_stream_rows_f64", 0), ("srht_passb_wgs", 100), ("gauss_wgs", 1 << 20),
                     ("gram_wgs", 10), ("srht_passa_wgs", -1), ("gauss_planes_wgs", 4),
                     ("gauss_planes_min_d", 0), ("gauss_chunk_rows", -1)):
        with pytest.raises(lsq.LsqError):
            lsq.tune(key, bad)
    for key, v in autotune.DEFAULTS.items():
        lsq.tune(key, v)

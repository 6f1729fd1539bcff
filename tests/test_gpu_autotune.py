"""The autotuner measures on the GPU and writes a table entry the library accepts."""
import json

import pytest

pytestmark = pytest.mark.gpu


def test_autotune_quick(tmp_path):
    from paper_1911_02675_amd import autotune, lsq
    p = str(tmp_path / "table.json")
    entry = autotune.tune(quick=True, path=p)
    print(json.dumps(entry["measured"]), flush=True)
    tab = json.load(open(p))
    assert autotune.arch_name() in tab
    for dt in ("f32", "f64"):
        for b in autotune.D_BUCKETS:
            assert entry["fused_groups_per_cu"][dt][str(b)] in autotune.GPC_CANDIDATES
    assert entry["batched_slots"] in autotune.SLOT_CANDIDATES
    for dt in ("f32", "f64"):
        for b, v in entry["srht"][dt].items():
            assert v["srht_passa_wgs"] in autotune.PASSA_CANDIDATES
            assert v["srht_passb_wgs"] in autotune.PASSB_CANDIDATES
            for key in ("fold8_rows", "stream_rows"):
                assert v[key] in autotune.FOLD_ROWS or v[key] == max(autotune.FOLD_ROWS) + 1
    assert entry["gauss_wgs"] in autotune.GAUSS_CANDIDATES
    assert entry["gauss_planes_wgs"] in autotune.PLANES_CANDIDATES
    assert all(v in autotune.GRAM_CANDIDATES for v in entry["gram_wgs"].values())
    try:
        vals = autotune.apply("f32", 512, path=p)
        assert set(vals) == {"fused_groups_per_cu", "batched_slots", "batched_gang_unit", "srht_passa_wgs", "srht_passb_wgs",
                             "srht_fold8_rows_f32", "srht_fold8_rows_f64", "srht_stream_rows_f32",
                             "srht_stream_rows_f64", "gauss_wgs", "gauss_planes_wgs", "gram_wgs"}
    finally:
        for k, v in autotune.DEFAULTS.items():
            lsq.tune(k, v)

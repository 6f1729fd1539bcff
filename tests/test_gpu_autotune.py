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
    try:
        vals = autotune.apply("f32", 512, path=p)
        assert set(vals) == {"fused_groups_per_cu", "batched_slots"}
    finally:
        lsq.tune("fused_groups_per_cu", 8)
        lsq.tune("batched_slots", 0)

"""Autotuner for liblsq's launch parameters.

    python -m paper_1911_02675_amd.autotune [--quick] [--out PATH]   measure on this GPU, write the table
    from paper_1911_02675_amd import autotune; autotune.apply()        set the library's knobs from it

Two knobs are measured (see lsq_tune in include/lsq.h):
  fused_groups_per_cu  workgroups per compute unit of the fused A^T(A p) pass, per storage dtype and
                       bucket of d (the pass is HBM-bound; the best oversubscription depends on the
                       row width and on how many rows a workgroup streams);
  batched_slots        workgroups of the persistent batched kernel (each streams one problem; fewer
                       than one per compute unit can win when the largest problems set the makespan).

The table is JSON keyed by the GPU's architecture name (gcnArchName), so a table measured on one
chip is never applied to another:
  {"gfx950:sramecc+:xnack-": {"fused_groups_per_cu": {"f32": {"64": 8, ...}, "f64": {...}},
                              "batched_slots": 192, "measured": {...raw timings...}}}
apply(dtype, d) picks the entry of the bucket that contains d (the largest bucket not above d).
The default table path is tune_table.json next to this file; LSQ_TUNE_TABLE overrides it.
"""
import argparse
import json
import os
import time

from . import lsq

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tune_table.json")
D_BUCKETS = (64, 256, 1024)
GPC_CANDIDATES = (2, 4, 8, 16)
SLOT_CANDIDATES = (128, 192, 256)


def table_path():
    return os.environ.get("LSQ_TUNE_TABLE", DEFAULT_TABLE)


def arch_name():
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName


def load_table(path=None):
    path = path or table_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def bucket(d):
    """The tuned bucket for d: the largest bucket not above d (the smallest for tiny d)."""
    b = D_BUCKETS[0]
    for v in D_BUCKETS:
        if d >= v:
            b = v
    return str(b)


def choose(entry, dtype="f32", d=1024):
    """Knob values for (dtype, d) from one architecture's entry of the table."""
    out = {}
    g = entry.get("fused_groups_per_cu", {}).get(dtype, {})
    if g:
        out["fused_groups_per_cu"] = int(g.get(bucket(d), next(iter(g.values()))))
    if "batched_slots" in entry:
        out["batched_slots"] = int(entry["batched_slots"])
    return out


def apply(dtype="f32", d=1024, arch=None, path=None):
    """Set the library's knobs from the table for this GPU; returns the values set ({} when the table
    has no entry for the architecture)."""
    tab = load_table(path)
    arch = arch or arch_name()
    if arch not in tab:
        return {}
    vals = choose(tab[arch], dtype, d)
    for k, v in vals.items():
        lsq.tune(k, v)
    return vals


# ------------------------------------------------------------------------------------------------
# measurement
# ------------------------------------------------------------------------------------------------
def _time_fused(ctx, A, y, reps):
    import torch
    d = A.shape[1]
    v = torch.randn(d, dtype=torch.float64, device="cuda")
    w = torch.empty(d, dtype=torch.float64, device="cuda")
    s = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.fused_pass(A, y, v, w, s)  # warm-up
    ctx.fused_pass_timing(reset=True)
    for _ in range(reps):
        ctx.fused_pass(A, y, v, w, s)
    _, avg_ms, _ = ctx.fused_pass_timing()
    return avg_ms


def measure_fused(ctx, quick=False):
    """GB/s of the fused pass for each (dtype, d bucket, workgroups per CU)."""
    import torch
    res = {}
    target = (1 << 28) if quick else (1 << 30)  # bytes of A per measurement
    reps = 3 if quick else 10
    for dtype, tdt, size in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        res[dtype] = {}
        for d in D_BUCKETS:
            n = max(1 << 12, target // (size * d))
            A = torch.randn(n, d, dtype=tdt, device="cuda")
            y = torch.randn(n, dtype=torch.float64, device="cuda")
            row = {}
            for g in GPC_CANDIDATES:
                lsq.tune("fused_groups_per_cu", g)
                ms = _time_fused(ctx, A, y, reps)
                row[str(g)] = round(n * d * size / (ms * 1e-3) / 1e9, 1)
            res[dtype][str(d)] = row
            del A, y
    lsq.tune("fused_groups_per_cu", 8)
    return res


def measure_batched(ctx, quick=False):
    """Solves/s of the batched form on a batch with the c4 shape distribution, per slot count."""
    import numpy as np
    import torch
    rng = np.random.default_rng(77)
    count = 64 if quick else 256
    As, ys, xs, descs = [], [], [], []
    for i in range(count):
        n = int(rng.integers(4096, 65537))
        d = int(rng.integers(16, 257))
        A = torch.randn(n, d, dtype=torch.float32, device="cuda")
        As.append(A)
        ys.append(torch.randn(n, dtype=torch.float64, device="cuda"))
        xs.append(torch.zeros(d, dtype=torch.float64, device="cuda"))
        descs.append(lsq.sketch_desc("sjlt", 4 * d, seed=1000 + i, s=4))
    res = {}
    for slots in SLOT_CANDIDATES:
        lsq.tune("batched_slots", slots)
        best = None
        for _ in range(3):
            for x in xs:
                x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            ctx.pcg_solve_batched(As, ys, descs, xs, tol=1e-10, max_iter=300, mixed=1, max_refine=10,
                                  raise_on_error=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
        res[str(slots)] = round(count / best, 1)
    lsq.tune("batched_slots", 0)
    return res


def tune(quick=False, path=None):
    """Measure, write the architecture's entry of the table, return it."""
    ctx = lsq.Context()
    try:
        fused = measure_fused(ctx, quick)
        batched = measure_batched(ctx, quick)
    finally:
        ctx.close()
    entry = {"fused_groups_per_cu": {dt: {b: int(max(row, key=row.get)) for b, row in per.items()}
                                     for dt, per in fused.items()},
             "batched_slots": int(max(batched, key=batched.get)),
             "measured": {"fused_gbs": fused, "batched_solves_per_s": batched, "quick": quick}}
    path = path or table_path()
    tab = load_table(path)
    tab[arch_name()] = entry
    with open(path, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller matrices and batch")
    ap.add_argument("--out", default=None, help="table path (default: tune_table.json in the package)")
    a = ap.parse_args()
    entry = tune(a.quick, a.out)
    print(json.dumps(entry, indent=1))


if __name__ == "__main__":
    main()

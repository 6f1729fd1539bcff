"""Autotuner for liblsq's launch parameters.

    python -m paper_1911_02675_amd.autotune [--quick] [--out PATH]   measure on this GPU, write the table
    from paper_1911_02675_amd import autotune; autotune.apply()        set the library's knobs from it

Knobs measured (see lsq_tune in include/lsq.h), each as the fastest of a few candidates:
  fused_groups_per_cu  workgroups per compute unit of the fused A^T(A p) pass, per storage dtype and
                       bucket of d (the pass is HBM-bound; the best oversubscription depends on the
                       row width and on how many rows a workgroup streams);
  batched_slots        workgroups of the persistent batched kernel (each streams one problem; fewer
                       than one per compute unit can win when the largest problems set the makespan);
  batched_gang_unit    elements of n d per workgroup of a gang (problems above it are solved by 2-4
                       workgroups together), timed jointly with batched_slots;
  srht_passa_wgs       workgroups of the SRHT's first pass, per transform precision and d bucket (timed
                       at m = 4d, where the second pass is small);
  srht_passb_wgs       workgroups of the LDS-staged second pass (timed at m = 40 d);
  srht_fold8_rows_*    from how many selected rows per 256-row bucket the staged second pass folds by
                       the 8-point transform instead of the 4-point one (both timed at 32..256 rows per
                       bucket; the threshold is the smallest count from which the 8-point form stays
                       faster);
  srht_stream_rows_*   from how many rows per bucket the streamed second pass (16-point fold) replaces
                       the staged one (the 8-point staged form against the streamed one at 32..256 rows);
  gauss_wgs            workgroups of the Gaussian sketch (FP64 form, n = 2^20, d = 512, m = 2048);
  gram_wgs             workgroups of the CholeskyQR Gram kernel, per d bucket (the factor of an m = 40 d
                       sketch).

The table is JSON keyed by the GPU's architecture name (gcnArchName), so a table measured on one
chip is never applied to another:
  {"gfx950:sramecc+:xnack-": {"fused_groups_per_cu": {"f32": {"64": 8, ...}, "f64": {...}},
                              "batched_slots": 192,
                              "srht": {"f32": {"256": {"srht_passa_wgs": ..., "srht_passb_wgs": ...,
                                                       "fold8_rows": ..., "stream_rows": ...}, "1024": {...}}, "f64": {...}},
                              "gauss_wgs": 1024, "gram_wgs": {"256": ..., "1024": ...},
                              "measured": {...raw timings...}}}
apply(dtype, d) picks the entry of the bucket that contains d (the largest bucket not above d; the
nearest measured bucket for the SRHT and Gram knobs, which are measured at fewer widths).
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
GANG_CANDIDATES = (0, 6 << 20, 8 << 20, 10 << 20)
PASSA_CANDIDATES = (1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18)
PASSB_CANDIDATES = (4096, 8192, 16384)
FOLD_ROWS = (32, 48, 64, 96, 128, 160, 192, 256)
GAUSS_CANDIDATES = (512, 1024, 2048, 4096)
PLANES_CANDIDATES = (256, 512, 768, 1024)
GRAM_CANDIDATES = (1024, 2048, 4096)
# library defaults, restored after measuring
DEFAULTS = {"fused_groups_per_cu": 8, "batched_slots": 0, "batched_gang_unit": 8 << 20, "srht_passa_wgs": 0, "srht_passb_wgs": 8192,
            "srht_fold8_rows_f32": 64, "srht_fold8_rows_f64": 128,
            "srht_stream_rows_f32": 192, "srht_stream_rows_f64": 192, "gauss_wgs": 1024, "gauss_planes_wgs": 512,
            "gram_wgs": 2048}


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


def _by_bucket(tab, d):
    """The entry of a {bucket: value} map for d: its bucket, else the nearest bucket measured."""
    if not tab:
        return None
    b = bucket(d)
    if b in tab:
        return tab[b]
    return tab[min(tab, key=lambda k: abs(int(k) - int(b)))]


def choose(entry, dtype="f32", d=1024):
    """Knob values for (dtype, d) from one architecture's entry of the table: dtype is the storage type of A
    and the precision of the SRHT transform ("f32" for the precision form, "f64" for the plain one)."""
    out = {}
    g = entry.get("fused_groups_per_cu", {}).get(dtype, {})
    if g:
        out["fused_groups_per_cu"] = int(g.get(bucket(d), next(iter(g.values()))))
    if "batched_slots" in entry:
        out["batched_slots"] = int(entry["batched_slots"])
    if "batched_gang_unit" in entry:
        out["batched_gang_unit"] = int(entry["batched_gang_unit"])
    srht = entry.get("srht", {})
    sr = _by_bucket(srht.get(dtype, {}), d)
    if sr:
        out["srht_passa_wgs"] = int(sr["srht_passa_wgs"])
        out["srht_passb_wgs"] = int(sr["srht_passb_wgs"])
    # the fold threshold is held per transform precision: both, since a solve may change its transform
    for prec in ("f32", "f64"):
        sp = _by_bucket(srht.get(prec, {}), d)
        for key in ("fold8_rows", "stream_rows"):
            if sp and key in sp:
                out["srht_" + key + "_" + prec] = int(sp[key])
    if "gauss_wgs" in entry:
        out["gauss_wgs"] = int(entry["gauss_wgs"])
    if "gauss_planes_wgs" in entry:
        out["gauss_planes_wgs"] = int(entry["gauss_planes_wgs"])
    gw = _by_bucket(entry.get("gram_wgs", {}), d)
    if gw:
        out["gram_wgs"] = int(gw)
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
    for slots, unit in [(sl, u) for sl in SLOT_CANDIDATES for u in GANG_CANDIDATES]:
        lsq.tune("batched_slots", slots)
        lsq.tune("batched_gang_unit", unit)
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
        res[f"{slots}/{unit}"] = round(count / best, 1)
    lsq.tune("batched_slots", 0)
    lsq.tune("batched_gang_unit", DEFAULTS["batched_gang_unit"])
    return res


def _time_ms(fn, reps):
    """Fastest of `reps` runs of fn (after one warm-up), from torch events on the current stream."""
    import torch
    fn()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1)
        best = t if best is None else min(best, t)
    return best


def _fold_threshold(t_narrow, t_wide):
    """The smallest rows-per-bucket count from which the wider fold is faster at every larger count
    measured (one past the largest when it never wins)."""
    rows = sorted(t_narrow)
    thr = rows[-1] + 1
    for r in reversed(rows):
        if t_wide[r] < t_narrow[r]:
            thr = r
        else:
            break
    return thr


def measure_srht(ctx, quick=False):
    """Sketch times (ms) for the SRHT knobs, per transform precision and d bucket."""
    import torch
    shapes = {"1024": ((1 << 19) if quick else (1 << 22), 1024), "256": ((1 << 18) if quick else (1 << 21), 256)}
    reps = 2 if quick else 3
    res = {}
    for dt, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        res[dt] = {}
        for b, (n, d) in shapes.items():
            A = torch.randn(n, d, dtype=tdt, device="cuda")
            y = torch.zeros(n, dtype=torch.float64, device="cuda")
            N = 1 << (n - 1).bit_length()
            rec = {"n": n, "d": d, "passa": {}, "passb": {}, "fold4": {}, "fold8": {}, "stream16": {}}

            def sk(m):
                SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
                desc = lsq.sketch_desc("srht", m, seed=3, compute=dt)
                return lambda: ctx.sketch(A, y, desc, SA)
            m_small = 4 * d
            for w in PASSA_CANDIDATES:
                lsq.tune("srht_passa_wgs", w)
                rec["passa"][str(w)] = round(_time_ms(sk(m_small), reps), 4)
            lsq.tune("srht_passa_wgs", 0)
            m_big = min(40 * d, N // 2)
            for w in PASSB_CANDIDATES:
                lsq.tune("srht_passb_wgs", w)
                rec["passb"][str(w)] = round(_time_ms(sk(m_big), reps), 4)
            lsq.tune("srht_passb_wgs", 8192)
            try:
                for rows in FOLD_ROWS:
                    m = rows * 256
                    if m > N or m > 65536:
                        continue
                    for mode, key in ((3, "fold4"), (4, "fold8"), (6, "stream16")):
                        ctx.set_option("srht_passb", mode)
                        rec[key][str(rows)] = round(_time_ms(sk(m), reps), 4)
            finally:
                ctx.set_option("srht_passb", 0)
            res[dt][b] = rec
            del A, y
            torch.cuda.empty_cache()
    return res


def measure_gauss(ctx, quick=False):
    """FP64 Gaussian sketch time (ms) per workgroup target."""
    import torch
    n, d, m = ((1 << 17) if quick else (1 << 20)), 512, 2048
    A = torch.randn(n, d, dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
    desc = lsq.sketch_desc("gaussian", m, seed=3)
    res = {}
    for w in GAUSS_CANDIDATES:
        lsq.tune("gauss_wgs", w)
        res[str(w)] = round(_time_ms(lambda: ctx.sketch(A, y, desc, SA), 2), 4)
    lsq.tune("gauss_wgs", 1024)
    return res


def measure_gauss_planes(ctx, quick=False):
    """BF16 Gaussian sketch (planes form) time (ms) per workgroup target (its split of n), at the
    precision form's shape n = 2^22, d = 1024, m = 4 d (n = 2^19 when quick)."""
    import torch
    n, d, m = ((1 << 19) if quick else (1 << 22)), 1024, 4096
    A = torch.randn(n, d, dtype=torch.float32, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
    desc = lsq.sketch_desc("gaussian", m, seed=3, compute="bf16")
    res = {}
    for w in PLANES_CANDIDATES:
        lsq.tune("gauss_planes_wgs", w)
        res[str(w)] = round(_time_ms(lambda: ctx.sketch(A, y, desc, SA), 2), 4)
    lsq.tune("gauss_planes_wgs", DEFAULTS["gauss_planes_wgs"])
    del A
    torch.cuda.empty_cache()
    return res


def measure_gram(ctx, quick=False):
    """Factor time (ms) of an m = 40 d sketch per Gram workgroup target, per d bucket."""
    import torch
    res = {}
    for d in ((256,) if quick else (256, 1024)):
        m = 40 * d
        SA = torch.randn(m, d, dtype=torch.float64, device="cuda")
        R = torch.empty((d, d), dtype=torch.float64, device="cuda")
        W = torch.empty((d, d), dtype=torch.float64, device="cuda")
        row = {}
        for w in GRAM_CANDIDATES:
            lsq.tune("gram_wgs", w)
            row[str(w)] = round(_time_ms(lambda: ctx.factor(SA, R, W), 3), 4)
        res[str(d)] = row
    lsq.tune("gram_wgs", 2048)
    return res


def _argmin(row):
    return int(min(row, key=lambda k: (row[k], int(k))))


def tune(quick=False, path=None):
    """Measure, write the architecture's entry of the table, return it."""
    ctx = lsq.Context()
    try:
        fused = measure_fused(ctx, quick)
        batched = measure_batched(ctx, quick)
        srht = measure_srht(ctx, quick)
        gauss = measure_gauss(ctx, quick)
        planes = measure_gauss_planes(ctx, quick)
        gram = measure_gram(ctx, quick)
    finally:
        ctx.close()
        for k, v in DEFAULTS.items():
            lsq.tune(k, v)
    entry = {"fused_groups_per_cu": {dt: {b: int(max(row, key=row.get)) for b, row in per.items()}
                                     for dt, per in fused.items()},
             "batched_slots": int(max(batched, key=batched.get).split("/")[0]),
             "batched_gang_unit": int(max(batched, key=batched.get).split("/")[1]),
             "srht": {dt: {b: {"srht_passa_wgs": _argmin(rec["passa"]), "srht_passb_wgs": _argmin(rec["passb"]),
                               "fold8_rows": _fold_threshold({int(k): v for k, v in rec["fold4"].items()},
                                                             {int(k): v for k, v in rec["fold8"].items()}),
                               "stream_rows": _fold_threshold({int(k): v for k, v in rec["fold8"].items()},
                                                              {int(k): v for k, v in rec["stream16"].items()})}
                          for b, rec in per.items()} for dt, per in srht.items()},
             "gauss_wgs": _argmin(gauss),
             "gauss_planes_wgs": _argmin(planes),
             "gram_wgs": {b: _argmin(row) for b, row in gram.items()},
             "measured": {"fused_gbs": fused, "batched_solves_per_s": batched, "srht_ms": srht,
                          "gauss_ms": gauss, "gauss_planes_ms": planes, "gram_ms": gram, "quick": quick}}
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

"""Time-to-solve of sketch-preconditioned least squares on one MI355X, plain FP64 vs mixed precision.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--kappa 1e6] [--sketch srht] [--m 4096]

Workload: n = 2^22 rows, d = 1024 columns, A = U diag(s) V^T with geometric singular values
(condition number --kappa), noise sigma = 0.01, planted so that the exact minimiser is known
(synth.make_planted).  A step is one complete solve to relative A-norm error 1e-10: sketch S A,
Householder factor of S A, PCG (plain FP64 form: A in FP64; mixed form: A in FP32 with an FP32
SRHT, FP64 factor, FP64 residuals and iterative refinement).  Inputs are resident in HBM before the
timed region.  One JSON line is printed; `value` is the mixed-form time-to-solve in seconds.

The roofline block reports the dominant kernel (the fused A^T(A p) pass of the mixed form): its
algorithmic bytes per launch (n d 4 bytes of FP32 A) over its average launch time, measured with HIP
events recorded around every launch on the library's stream inside the timed region.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FUSED_PROFILE = os.path.join(ROOT, "profiles", "k_fused_f32_n4194304_d1024.md")
FUSED_SOURCE = os.path.join(ROOT, "paper_1911_02675_amd", "csrc", "iter.hip")


def counter_traffic(n, d, head, gpc=None):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    record (scaled by the calibration recorded with it), or None when the record does not cover this
    workload or the kernel source has changed since the counters were taken."""
    import hashlib
    if head != "mixed" or (n, d) != (1 << 22, 1024) or not os.path.exists(FUSED_PROFILE):
        return None
    rec = None
    for line in open(FUSED_PROFILE):
        if line.startswith("traffic_json:"):
            rec = json.loads(line.split(":", 1)[1])
    if not rec:
        return None
    if hashlib.sha256(open(FUSED_SOURCE, "rb").read()).hexdigest() != rec.get("source_sha256"):
        return None
    if gpc is not None and rec.get("fused_groups_per_cu") != gpc:
        return None
    return rec["traffic_bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--d", type=int, default=1024)
    ap.add_argument("--m", default="auto",
                    help="sketch size, or 'auto': the Section 6 cost model with this GPU's measured sketch, "
                         "factor and pass times (paper_1911_02675_amd/msize.py), chosen per form before timing")
    ap.add_argument("--kappa", type=float, default=1e6)
    ap.add_argument("--sigma", type=float, default=0.01)
    ap.add_argument("--sketch", default="srht", choices=["srht", "sjlt", "gaussian"])
    ap.add_argument("--s", type=int, default=4, help="SJLT nonzeros per column")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=3001)
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 16)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="before the solves, convert 2^28 FP32 values to FP64 once (1 GiB read, 2 GiB "
                         "written): a kernel of known traffic for scaling rocprofv3 byte counters")
    ap.add_argument("--sweep", choices=["c2", "c4", "c5", "msize", "gauss"], default=None,
                    help="c2: n=2^20 d=512 kappa=1e4, {SRHT, SJLT s=1,2,4,8, Gaussian} x m={2d,4d,8d}; "
                         "c4: 512 uneven problems, batched form vs a per-problem loop; "
                         "c5: refreshed IHS / Polyak-IHS statistics over 32 sketch seeds vs closed forms; "
                         "gauss: the Gaussian sketch alone at the c2, c5 and c3 shapes; "
                         "one JSON line per run")
    ap.add_argument("--gauss-cases", default="", help="gauss: comma list of case indices to run (default all)")
    ap.add_argument("--count", type=int, default=512, help="c4: number of problems")
    ap.add_argument("--slots", default="0", help="c4: comma list of batched workgroup counts to time "
                                                 "(0 = one per compute unit)")
    ap.add_argument("--gang-units", default="",
                    help="c4: comma list of batched gang sizes (elements of n d per workgroup; 0 = no gangs) "
                         "to time at every slot count (default: the library's)")
    ap.add_argument("--no-loop", action="store_true", help="c4: skip the per-problem loop")
    ap.add_argument("--seeds", type=int, default=32, help="c5: sketch seeds per configuration")
    ap.add_argument("--c5-methods", default="ihs,fcg,fixed,pcg",
                    help="c5: comma list of ihs (refreshed IHS and Polyak-IHS), fcg (IPCG and GCC), fixed "
                         "(fixed-sketch IHS and Polyak-IHS, Theorem 3.2 parameters), pcg (fixed sketch)")
    ap.add_argument("--c5-kinds", default="srht,gaussian", help="c5: sketches to run")
    return ap.parse_args()


def sweep_c2(a):
    """Plain FP64 PCG at n = 2^20, d = 512, kappa = 1e4, sigma = 0.01 for every sketch and sketch size:
    sketch ms, factor ms, iterations, fused-pass GB/s and the error against the exact minimiser."""
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted
    n, d = 1 << 20, 512
    P = make_planted(n, d, 1e4, sigma=0.01, seed=2001)
    A = torch.from_numpy(P["A64"]).cuda()
    y = torch.from_numpy(P["y64"]).cuda()
    xs = torch.from_numpy(P["x_star"]).cuda()
    ax = torch.linalg.norm(A @ xs)
    ctx = lsq.Context()
    kinds = [("srht", 1), ("sjlt", 1), ("sjlt", 2), ("sjlt", 4), ("sjlt", 8), ("gaussian", 1)]
    for kind, s in kinds:
        for m in (2 * d, 4 * d, 8 * d):
            desc = lsq.sketch_desc(kind, m, seed=7, s=s)
            x = torch.zeros(d, dtype=torch.float64, device="cuda")
            ctx.pcg_solve(A, y, desc, x, tol=a.tol, max_iter=300)  # warm-up (workspace, code objects)
            ctx.fused_pass_timing(reset=True)
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = ctx.pcg_solve(A, y, desc, x, tol=a.tol, max_iter=300)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            _, fms, _ = ctx.fused_pass_timing()
            e = float(torch.linalg.norm(A @ (x - xs)) / ax)
            print(json.dumps({"sweep": "c2", "n": n, "d": d, "kappa": 1e4, "sketch": kind, "s": s, "m": m,
                              "time_s": round(dt, 5), "sketch_ms": round(info.t_sketch_ms, 3),
                              "factor_ms": round(info.t_factor_ms, 3), "iter_ms": round(info.t_iter_ms, 3),
                              "iters": info.iters, "fused_ms": round(fms, 4),
                              "fused_gbs": round(n * d * 8 / (fms * 1e-3) / 1e9, 1) if fms > 0 else None,
                              "rel_a_norm_error": e}), flush=True)
    ctx.close()


def sweep_gauss(a):
    """The Gaussian sketch alone (counter-based normals fused into the matrix-core GEMM) at the shapes of
    the workloads that use it: n = 2^20, d = 512, m in {2d, 4d, 8d} (FP64, plain form), n = 2^21, d = 256,
    m = 4d (FP64, refreshed IHS), n = 2^22, d = 1024, m = 4d (BF16 S times a three-term BF16 split of
    FP32 A, the precision form; and the FP64 form on FP64 A at that shape).  Time per sketch from torch events on the library's stream (median of
    `steps` after `warmup`), matrix-core work 2 m n d (x 3 split terms for BF16) against the dense peak
    (FP64 78.6 TF/s, BF16 2.5 PF/s)."""
    import torch

    from paper_1911_02675_amd import lsq
    cases = [(1 << 20, 512, 1024, "f64"), (1 << 20, 512, 2048, "f64"), (1 << 20, 512, 4096, "f64"),
             (1 << 21, 256, 1024, "f64"), (1 << 22, 1024, 4096, "bf16"), (1 << 22, 1024, 4096, "f64")]
    if a.gauss_cases:
        keep = {int(c) for c in a.gauss_cases.split(",")}
        cases = [c for i, c in enumerate(cases) if i in keep]
    ctx = lsq.Context()
    g = torch.Generator(device="cuda").manual_seed(5)
    for n, d, m, comp in cases:
        dt = torch.float32 if comp == "bf16" else torch.float64
        A = torch.randn((n, d), dtype=dt, device="cuda", generator=g)
        y = torch.zeros(n, dtype=torch.float64, device="cuda")
        SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
        desc = lsq.sketch_desc("gaussian", m, seed=7, compute=comp)
        for _ in range(max(a.warmup, 1)):
            ctx.sketch(A, y, desc, SA)
        times = []
        for _ in range(max(a.steps, 1)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.sketch(A, y, desc, SA)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        terms = 3 if comp == "bf16" else 1
        peak = 2500.0 if comp == "bf16" else 78.6
        tf = terms * 2.0 * m * n * d / (ms * 1e-3) / 1e12
        print(json.dumps({"sweep": "gauss", "n": n, "d": d, "m": m, "compute": comp, "ms": round(ms, 3),
                          "mfma_tflops": round(tf, 1), "peak_tflops": peak, "frac": round(tf / peak, 4),
                          "product_tflops": round(2.0 * m * n * d / (ms * 1e-3) / 1e12, 1)}), flush=True)
        del A, y, SA
        torch.cuda.empty_cache()
    ctx.close()


def gen_c4(count, seed=4001):
    """The batched workload on the device: n_i ~ U{4096..65536} (even), d_i ~ U{16..256},
    log10 kappa_i ~ U[2, 6], sigma = 0.01, geometric singular values, Haar factors.  Planted as in
    synth.make_planted (rows in +- pairs, noise orthogonal to the range of the stored FP32 matrix),
    so x*_i is exact; rows are stored at a stride of roundup(d_i, 4) floats (16-byte rows)."""
    import math

    import torch
    rng = np.random.default_rng(seed)
    ns = 2 * (rng.integers(4096, 65537, count) // 2)
    ds = rng.integers(16, 257, count)
    lk = rng.uniform(2.0, 6.0, count)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = []
    for i in range(count):
        n, d, kappa = int(ns[i]), int(ds[i]), 10.0 ** lk[i]
        h = n // 2
        Z = torch.randn(h, d, dtype=torch.float64, device="cuda", generator=g)
        for _ in range(2):  # orthonormal columns (Cholesky QR, twice)
            L = torch.linalg.cholesky(Z.T @ Z)
            Z = torch.linalg.solve_triangular(L, Z.T.contiguous(), upper=False).T.contiguous()
        V, Rv = torch.linalg.qr(torch.randn(d, d, dtype=torch.float64, device="cuda", generator=g))
        V = V * torch.sign(torch.diagonal(Rv))[None, :]
        sv = kappa ** (-torch.arange(d, dtype=torch.float64, device="cuda") / max(d - 1, 1))
        B = ((Z * sv[None, :]) @ V.T / math.sqrt(2.0)).float()
        D = torch.where(torch.rand(h, dtype=torch.float64, device="cuda", generator=g) < 0.5, -1.0, 1.0)
        lda = (d + 3) // 4 * 4
        buf = torch.zeros(n, lda, dtype=torch.float32, device="cuda")
        buf[:h, :d] = B
        buf[h:, :d] = B * D[:, None].float()
        A = buf[:, :d]
        xs = torch.randn(d, dtype=torch.float64, device="cuda", generator=g)
        w = 0.01 * torch.randn(h, dtype=torch.float64, device="cuda", generator=g)
        y = A.double() @ xs
        y[:h] += w
        y[h:] -= D * w
        out.append(dict(n=n, d=d, kappa=kappa, A=A, buf=buf, y=y, xs=xs))
        del Z, V, B, D
    torch.cuda.synchronize()
    return out


def sweep_c4(a):
    """The batched form (one persistent launch per sweep of all problems) against a loop of
    single-problem solves, FP32 A with FP64 refinement to 1e-10, SJLT m = 4 d_i, s = 4."""
    import torch

    from paper_1911_02675_amd import lsq
    t0 = time.time()
    probs = gen_c4(a.count)
    log(f"[c4] generated {a.count} problems in {time.time() - t0:.1f} s; "
        f"sum n d = {sum(p['n'] * p['d'] for p in probs):.3e}")
    X = torch.zeros(sum(p["d"] for p in probs), dtype=torch.float64, device="cuda")
    xs, off = [], 0
    for p in probs:
        xs.append(X[off:off + p["d"]])
        off += p["d"]
    descs = [lsq.sketch_desc("sjlt", 4 * p["d"], seed=7000 + i, s=4) for i, p in enumerate(probs)]
    As, ys = [p["A"] for p in probs], [p["y"] for p in probs]
    ctx = lsq.Context()

    def errors():
        e = []
        for p, x in zip(probs, xs):
            A64 = p["A"].double()
            e.append(float(torch.linalg.norm(A64 @ (x - p["xs"])) / torch.linalg.norm(A64 @ p["xs"])))
        return e

    def batch():
        X.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, infos = ctx.pcg_solve_batched(As, ys, descs, xs, tol=a.tol, max_iter=300, mixed=1,
                                          max_refine=10, raise_on_error=False)
        torch.cuda.synchronize()
        return time.perf_counter() - t, st, infos

    results = []
    units = [int(v) for v in a.gang_units.split(",")] if a.gang_units else [None]
    for slots, unit in [(sl, u) for sl in (int(v) for v in a.slots.split(",")) for u in units]:
        lsq.tune("batched_slots", slots)
        if unit is not None:
            lsq.tune("batched_gang_unit", unit)
        for _ in range(a.warmup):
            batch()
        times = []
        for _ in range(a.steps):
            dt, st, infos = batch()
            times.append(dt)
        e = errors()
        dt = min(times)
        kern_ms = infos[0].t_total_ms
        # algorithmic HBM bytes of one sweep: every pass over A (PCG iterations and residual passes,
        # the latter also read y), the sketch's s reads of A, and the solution writes
        byt = 0.0
        for p, inf in zip(probs, infos):
            passes = inf.iters + inf.refinements + 1
            byt += passes * p["n"] * p["d"] * 4.0 + (inf.refinements + 1) * p["n"] * 8.0
            byt += 4 * p["n"] * p["d"] * 4.0
        # schedule: per-problem durations from the device clock, per-workgroup bandwidth
        dur = np.array([i.t_sketch_ms + i.t_factor_ms + i.t_iter_ms for i in infos])
        pb = np.array([(i.iters + i.refinements + 1 + 4) * p["n"] * p["d"] * 4.0
                       for p, i in zip(probs, infos)])
        wg_gbs = pb / (dur * 1e-3) / 1e9
        big = int(np.argmax(dur))
        sched = {"max_problem_ms": round(float(dur[big]), 3),
                 "max_problem_n_d": [probs[big]["n"], probs[big]["d"]],
                 "last_start_ms": round(max(i.t_start_ms for i in infos), 3),
                 "wg_gbs_p10_p50_p90": [round(float(v), 1) for v in np.percentile(wg_gbs, [10, 50, 90])],
                 "phase_ms_sum": {"sketch": round(sum(i.t_sketch_ms for i in infos), 2),
                                  "factor": round(sum(i.t_factor_ms for i in infos), 2),
                                  "iterate": round(sum(i.t_iter_ms for i in infos), 2)}}
        rec = {"sweep": "c4", "count": a.count, "slots": slots, "gang_unit": unit, "status": st, "schedule": sched,
               "failed": sum(1 for i in infos if i.status != 0),
               "batch_s": round(dt, 5), "kernel_ms": round(kern_ms, 3),
               "solves_per_s": round(a.count / dt, 1),
               "agg_gbs": round(byt / (kern_ms * 1e-3) / 1e9, 1),
               "hbm_frac": round(byt / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "bytes": byt, "iters_mean": round(float(np.mean([i.iters for i in infos])), 2),
               "iters_max": max(i.iters for i in infos),
               "refinements_mean": round(float(np.mean([i.refinements for i in infos])), 2),
               "max_rel_a_norm_error": max(e)}
        log(f"[c4] slots {slots} gang unit {unit}: {dt * 1e3:.1f} ms per sweep ({a.count / dt:.0f} solves/s), kernel "
            f"{kern_ms:.1f} ms, {rec['agg_gbs']} GB/s, max e_A {max(e):.2e}, failed {rec['failed']}; "
            f"schedule {json.dumps(sched)}")
        results.append(rec)
    lsq.tune("batched_slots", 0)
    lsq.tune("batched_gang_unit", 8 << 20)
    best = min(results, key=lambda r: r["batch_s"])
    loop = None
    if not a.no_loop:
        X.zero_()  # x_0 = 0 (the stop rule is relative to the error of x_0)
        for i in range(min(4, a.count)):  # warm-up: code objects and workspace
            ctx.pcg_solve(As[i], ys[i], descs[i], xs[i], tol=a.tol, max_iter=300, mixed=1, max_refine=10)
        X.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(a.count):
            ctx.pcg_solve(As[i], ys[i], descs[i], xs[i], tol=a.tol, max_iter=300, mixed=1, max_refine=10,
                          raise_on_error=False)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t
        e = errors()
        loop = {"loop_s": round(tl, 4), "loop_solves_per_s": round(a.count / tl, 1),
                "loop_max_rel_a_norm_error": max(e)}
        log(f"[c4] per-problem loop: {tl:.2f} s ({a.count / tl:.0f} solves/s), max e_A {max(e):.2e}")
    ctx.close()
    print(json.dumps({"sweep": "c4", "best": best, "all": results, "loop": loop,
                      "speedup_vs_loop": round(loop["loop_s"] / best["batch_s"], 2) if loop else None}),
          flush=True)


def sweep_c5(a):
    """Refreshed IHS (beta = 0) and Polyak-IHS (beta > 0) with a fresh sketch every iteration, the
    library's step rule mu = theta_1 / theta_2, then flexible CG (IPCG, GCC) on the same sketches, x_0 = 0,
    at n = 2^21, d = 256, kappa = 1e5, sigma = 0.01:
    mean and relative standard error over the sketch seeds of delta_t / delta_0 (delta = ||A (x_t - x*)||^2),
    time per iteration, and fixed-sketch PCG's iterations and time to the error refreshed IHS reached.
    (The comparison with the closed forms is made by the tests, which may use the oracle.)"""
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted
    n, d, T, kappa = 1 << 21, 256, 20, 1e5
    t0 = time.time()
    P = make_planted(n, d, kappa, sigma=0.01, seed=5001)
    A = torch.from_numpy(P["A64"]).cuda()
    y = torch.from_numpy(P["y64"]).cuda()
    xs = torch.from_numpy(P["x_star"]).cuda()
    del P
    log(f"[c5] planted problem in {time.time() - t0:.1f} s")
    ctx = lsq.Context()
    trace = torch.zeros(T + 1, dtype=torch.float64, device="cuda")
    for kind in [k for k in a.c5_kinds.split(",") if k]:
        for m in (512, 1024):
            ihs_mean_T = None
            methods = a.c5_methods.split(",")
            for beta in ((0.0, 0.05, 0.1, 0.5) if "ihs" in methods else ()):
                ratios, it_ms, mu = [], [], None
                for r in range(a.seeds):
                    x = torch.zeros(d, dtype=torch.float64, device="cuda")
                    desc = lsq.sketch_desc(kind, m, seed=7000000 + 5000 + r, t=0)
                    info = ctx.ihs_solve(A, y, desc, x, iters=T, beta=beta, refresh=1, mu_rule=0, x_ref=xs,
                                         err_trace=trace)
                    e = host_np(trace)
                    ratios.append((e / e[0]) ** 2)
                    it_ms.append((info.t_sketch_ms + info.t_factor_ms + info.t_iter_ms) / T)
                    mu = info.mu
                R = np.array(ratios)
                mean = R.mean(axis=0)
                se = R.std(axis=0, ddof=1) / np.sqrt(len(R)) / np.maximum(mean, 1e-300)
                if beta == 0.0:
                    ihs_mean_T = float(mean[-1])
                rec = {"sweep": "c5", "kind": kind, "n": n, "d": d, "kappa": kappa, "m": m, "beta": beta,
                       "mu": mu, "seeds": a.seeds, "T": T,
                       "ratio_mean": [float(v) for v in mean], "ratio_rel_se": [float(v) for v in se],
                       "ms_per_iter": float(np.median(it_ms))}
                log(f"[c5] {kind} m={m} beta={beta}: mu {mu:.5f}, delta_T/delta_0 mean {mean[-1]:.3e} "
                    f"(rel se {se[-1]:.3f}), {rec['ms_per_iter']:.2f} ms/iter")
                print(json.dumps(rec), flush=True)
            # flexible CG with the same refreshed sketches: IPCG (window 1) and GCC (every direction)
            for name, window in ((("ipcg", 1), ("gcc", T)) if "fcg" in methods else ()):
                ratios, it_ms = [], []
                for r in range(a.seeds):
                    x = torch.zeros(d, dtype=torch.float64, device="cuda")
                    desc = lsq.sketch_desc(kind, m, seed=7000000 + 5000 + r, t=0)
                    info = ctx.fcg_solve(A, y, desc, x, iters=T, window=window, refresh=1, x_ref=xs,
                                         err_trace=trace)
                    e = host_np(trace)
                    ratios.append((e / e[0]) ** 2)
                    it_ms.append((info.t_sketch_ms + info.t_factor_ms + info.t_iter_ms) / T)
                R = np.array(ratios)
                mean = R.mean(axis=0)
                se = R.std(axis=0, ddof=1) / np.sqrt(len(R)) / np.maximum(mean, 1e-300)
                rec = {"sweep": "c5", "kind": kind, "n": n, "d": d, "kappa": kappa, "m": m, "method": name,
                       "window": window, "seeds": a.seeds, "T": T,
                       "ratio_mean": [float(v) for v in mean], "ratio_rel_se": [float(v) for v in se],
                       "ms_per_iter": float(np.median(it_ms))}
                if kind == "gaussian":
                    # Corollary 4.2: E delta_t / E delta_0 <= (1 - theta_1^2 / theta_2)^t
                    t1 = m / (m - d - 1.0)
                    t2 = m * m * (m - 1.0) / ((m - d) * (m - d - 1.0) * (m - d - 3.0))
                    rec["bound"] = [float((1.0 - t1 * t1 / t2) ** t) for t in range(T + 1)]
                log(f"[c5] {name.upper()} {kind} m={m}: delta_T/delta_0 mean {mean[-1]:.3e} "
                    f"(rel se {se[-1]:.3f}), {rec['ms_per_iter']:.2f} ms/iter")
                print(json.dumps(rec), flush=True)
            # fixed sketch (refresh = 0): IHS and Polyak-IHS with the Theorem 3.2 parameters (rho = d/m)
            for name, rule in ((("fixed_ihs", 2), ("fixed_polyak", 3)) if "fixed" in methods else ()):
                ratios, it_ms, mu = [], [], None
                for r in range(a.seeds):
                    x = torch.zeros(d, dtype=torch.float64, device="cuda")
                    desc = lsq.sketch_desc(kind, m, seed=7000000 + 5000 + r, t=0)
                    info = ctx.ihs_solve(A, y, desc, x, iters=T, refresh=0, mu_rule=rule, x_ref=xs,
                                         err_trace=trace)
                    e = host_np(trace)
                    ratios.append((e / e[0]) ** 2)
                    it_ms.append(info.t_iter_ms / T)
                    mu = info.mu
                R = np.array(ratios)
                mean = R.mean(axis=0)
                se = R.std(axis=0, ddof=1) / np.sqrt(len(R)) / np.maximum(mean, 1e-300)
                rho = d / m
                rate = 4 * rho / (1 + rho) ** 2 if rule == 2 else rho
                rec = {"sweep": "c5", "kind": kind, "n": n, "d": d, "kappa": kappa, "m": m, "method": name,
                       "mu": mu, "beta": 0.0 if rule == 2 else rho, "seeds": a.seeds, "T": T,
                       "ratio_mean": [float(v) for v in mean], "ratio_rel_se": [float(v) for v in se],
                       "theorem_3_2_rate": rate, "ms_per_iter_excl_sketch": float(np.median(it_ms))}
                log(f"[c5] {name} {kind} m={m}: mu {mu:.5f}, delta_T/delta_0 mean {mean[-1]:.3e} "
                    f"(rate^T {rate ** T:.3e}), {rec['ms_per_iter_excl_sketch']:.3f} ms/iter after one sketch")
                print(json.dumps(rec), flush=True)
            # fixed-sketch PCG: iterations (and time) to the error refreshed IHS reached in T steps
            if "pcg" not in methods or ihs_mean_T is None:
                continue
            target = float(np.sqrt(ihs_mean_T))
            x = torch.zeros(d, dtype=torch.float64, device="cuda")
            ptrace = torch.zeros(201, dtype=torch.float64, device="cuda")
            desc = lsq.sketch_desc(kind, m, seed=7000000 + 5000, t=0)
            _, info = ctx.pcg_solve(A, y, desc, x, tol=1e-300, max_iter=200, stop_rule=1, x_ref=xs,
                                    err_trace=ptrace)
            pe = host_np(ptrace)
            k = int(np.argmax(pe <= target)) if np.any(pe <= target) else None
            per_it = info.t_iter_ms / max(info.iters, 1)
            rec = {"sweep": "c5", "kind": kind, "m": m, "pcg_fixed_sketch": True,
                   "target_rel_a_norm_error": target, "iters_to_target": k,
                   "time_to_target_ms": (info.t_sketch_ms + info.t_factor_ms + k * per_it) if k else None,
                   "ihs_time_ms": float(np.median(it_ms)) * T,
                   "pcg_error_trace": [float(v) for v in pe[: (k or 40) + 1]]}
            log(f"[c5] PCG fixed {kind} m={m}: {k} iterations to e_A {target:.2e} "
                f"({rec['time_to_target_ms']} ms) vs refreshed IHS {rec['ihs_time_ms']:.1f} ms")
            print(json.dumps(rec), flush=True)
    ctx.close()


def sweep_msize(a):
    """Sketch-size chooser (Section 6) on the benchmark workload: for each form, the measured sketch and
    factor times at every candidate m, the predicted time-to-solve (measured costs + T(m) passes), the
    chooser's pick, the paper's m*, and the measured time-to-solve of full solves at every candidate."""
    import torch

    from paper_1911_02675_amd import autotune, lsq, msize
    from synth import make_planted
    forms = [f for f in a.forms.split(",") if f]
    t0 = time.time()
    P = make_planted(a.n, a.d, a.kappa, sigma=a.sigma, seed=a.seed, want64=True, want32="mixed" in forms)
    log(f"[msize] planted problem in {time.time() - t0:.1f} s")
    A64 = torch.from_numpy(P["A64"]).cuda()
    y64 = torch.from_numpy(P["y64"]).cuda()
    A32 = torch.from_numpy(P["A32"]).cuda() if "mixed" in forms else None
    y32 = torch.from_numpy(P["y32"]).cuda() if "mixed" in forms else None
    del P
    ctx = lsq.Context()
    for form in forms:
        autotune.apply("f64" if form == "fp64" else "f32", a.d)
        A, y = (A64, y64) if form == "fp64" else (A32, y32)
        comp = "f64" if form == "fp64" or a.sketch != "srht" else "f32"
        extra = 2.0 if form == "fp64" else 3.0  # verification / refinement residual passes
        meas, t_pass, pick, _ = msize.calibrate(ctx, A, y, a.sketch, compute=comp, s=a.s, seed=a.seed, tol=a.tol,
                                                extra_passes=extra)
        _, pred = msize.choose(meas, t_pass, a.d, a.tol, extra)
        measured = {}
        for m in sorted(meas):
            best = None
            for _ in range(a.steps + a.warmup):
                x = torch.zeros(a.d, dtype=torch.float64, device="cuda")
                desc = lsq.sketch_desc(a.sketch, m, seed=a.seed, s=a.s, compute=comp)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st, info = ctx.pcg_solve(A, y, desc, x, tol=a.tol, max_iter=300, mixed=int(form != "fp64"),
                                         max_refine=8, raise_on_error=False)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t1) * 1e3
                best = (dt, info.iters, st) if best is None or dt < best[0] else best
            measured[m] = best
            log(f"[msize] {form} m={m}: sketch {meas[m][0]:.2f} factor {meas[m][1]:.2f} ms, T(m) "
                f"{msize.pcg_iterations(m, a.d, a.tol)}, predicted {pred[m]:.1f} ms, measured {best[0]:.1f} ms "
                f"({best[1]} iterations, status {best[2]})")
        rec = {"sweep": "msize", "form": form, "n": a.n, "d": a.d, "kappa": a.kappa, "sketch": a.sketch,
               "tol": a.tol, "t_pass_ms": t_pass, "chooser_m": pick,
               "paper_m_star": msize.paper_m_star(a.sketch, a.n, a.d, a.tol),
               "rows": [{"m": m, "sketch_ms": meas[m][0], "factor_ms": meas[m][1],
                         "T_model": msize.pcg_iterations(m, a.d, a.tol), "predicted_ms": pred[m],
                         "measured_ms": measured[m][0], "iters": measured[m][1], "status": measured[m][2]}
                        for m in sorted(meas)]}
        best_m = min(measured, key=lambda k: measured[k][0])
        log(f"[msize] {form}: chooser picks m={pick} ({measured[pick][0]:.1f} ms measured); fastest measured "
            f"m={best_m} ({measured[best_m][0]:.1f} ms); paper m* = {rec['paper_m_star']}")
        print(json.dumps(rec), flush=True)
    ctx.close()


def host_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def host_description():
    """CPU model, logical CPUs visible to this process, and RAM of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                ram = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "ram_gib": ram}


def cpu_baseline(A64, m, kind, s, seed, iters, sketch_rows=1 << 16, qr_rows=4096, pass_rows=1 << 19):
    """The CPU oracle as it stands, timed on bounded samples of the workload and scaled by each step's own
    cost law, once with one BLAS thread and once with all of them:
      sketch  the oracle's SRHT of the first `sketch_rows` rows (a full transform of that length, then
              the m selected rows), scaled by N log2 N (N = the padded length);
      factor  the oracle's Householder QR of the first `qr_rows` rows of that sketch, scaled by the flop
              count 2 m d^2 - 2 d^3 / 3;
      pass    one oracle PCG step (A p, A^T q, the triangular solves) on the first `pass_rows` rows,
              scaled linearly to n, times the GPU solve's passes (its iterations + the first gradient).
    Gaussian and SJLT sketches are scaled linearly in n."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import householder, sketch
    from oracle.pcg import apply_hs_inv

    n, d = A64.shape
    N = 1
    while N < n:
        N *= 2
    rs = min(n, sketch_rows)
    Ns = 1
    while Ns < rs:
        Ns *= 2
    ms = min(m, Ns)
    sk_scale = (N * np.log2(N)) / (Ns * np.log2(Ns)) if kind == "srht" else n / rs
    sk_scale *= m / ms
    qr_m = min(qr_rows, ms)
    flops = lambda mm: 2.0 * mm * d * d - 2.0 * d ** 3 / 3.0
    qr_scale = flops(m) / flops(qr_m)
    pr = min(n, pass_rows)
    p = np.random.default_rng(0).standard_normal(d)

    def run():
        t0 = time.perf_counter()
        SA = sketch.sketch(A64[:rs], kind, ms, seed, 0, s)
        t_sk = time.perf_counter() - t0
        t0 = time.perf_counter()
        R = householder.householder_qr(SA[:qr_m])
        t_qr = time.perf_counter() - t0
        t0 = time.perf_counter()
        q = A64[:pr] @ p
        Hp = A64[:pr].T @ q
        apply_hs_inv(R, Hp)
        t_it = time.perf_counter() - t0
        comp = {"sketch_s": t_sk * sk_scale, "factor_s": t_qr * qr_scale, "pass_s": t_it * n / pr}
        total = comp["sketch_s"] + comp["factor_s"] + (iters + 1) * comp["pass_s"]
        return total, comp, t_sk + t_qr + t_it

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        one, comp1, spent1 = run()
    allc, compa, spenta = run()
    rnd = lambda c: {k: round(v, 3) for k, v in c.items()}
    return {
        "value": round(allc, 3), "unit": "s", "cores": threads, "kind": "oracle",
        "sample": (f"oracle {kind} sketch of the first {rs} rows with m={ms} (scaled x{sk_scale:.0f}: "
                   f"{'N log N' if kind == 'srht' else 'n'}{' and m' if ms < m else ''}), its Householder QR of the first {qr_m} "
                   f"rows of that sketch (scaled x{qr_scale:.1f} by 2md^2 - 2d^3/3 to m={m}), one oracle PCG "
                   f"step on the first {pr} rows (scaled x{n / pr:.0f}) times {iters + 1} passes; "
                   f"{spenta:.1f} s of CPU time on {threads} threads, {spent1:.1f} s on one"),
        "components_s": rnd(compa),
        "single_thread": {"value": round(one, 3), "cores": 1, "components_s": rnd(comp1)},
        "host": host_description(),
    }


def main():
    a = parse()
    if a.sweep == "c2":
        sweep_c2(a)
        return
    if a.sweep == "c4":
        sweep_c4(a)
        return
    if a.sweep == "c5":
        sweep_c5(a)
        return
    if a.sweep == "msize":
        sweep_msize(a)
        return
    if a.sweep == "gauss":
        sweep_gauss(a)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); multi-GPU sharding is not "
              "built: see the design notes on row-block sharding.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1911_02675_amd import lsq
    from synth import make_planted

    from paper_1911_02675_amd import autotune, msize
    forms = [f for f in a.forms.split(",") if f]
    log(f"[bench] generating planted problem n={a.n} d={a.d} kappa={a.kappa:g}")
    t0 = time.time()
    P = make_planted(a.n, a.d, a.kappa, sigma=a.sigma, seed=a.seed, want64=True,
                     want32="mixed" in forms)
    log(f"[bench] generated in {time.time() - t0:.1f} s; uploading")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A64 = torch.from_numpy(P["A64"]).to(dev)
    y64 = torch.from_numpy(P["y64"]).to(dev)
    xs = torch.from_numpy(P["x_star"]).to(dev)
    A32 = y32 = None
    if "mixed" in forms:
        A32 = torch.from_numpy(P["A32"]).to(dev)
        y32 = torch.from_numpy(P["y32"]).to(dev)
    torch.cuda.synchronize()
    if a.calibration_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = src.double()
        torch.cuda.synchronize()
        del src, dst
    ctx = lsq.Context()
    ax = torch.linalg.norm(A64 @ xs)

    m_form, m_model, comp_form = {}, {}, {}

    def solve(form):
        x = torch.zeros(a.d, dtype=torch.float64, device=dev)
        # not converged is reported, not raised
        if form == "fp64":
            desc = lsq.sketch_desc(a.sketch, m_form[form], seed=a.seed, s=a.s, compute="f64")
            st, info = ctx.pcg_solve(A64, y64, desc, x, tol=a.tol, max_iter=200, raise_on_error=False)
        else:
            desc = lsq.sketch_desc(a.sketch, m_form[form], seed=a.seed, s=a.s, compute=comp_form[form])
            st, info = ctx.pcg_solve(A32, y32, desc, x, tol=a.tol, max_iter=200, mixed=1, max_refine=8,
                                     raise_on_error=False)
        if st not in (lsq.LSQ_OK, lsq.LSQ_ERR_NOT_CONVERGED):
            raise lsq.LsqError(st, "solve failed")
        return x, info

    res = {}
    tuned = {}
    for form in forms:
        # launch parameters from the autotuner's table for this GPU (defaults when it has no entry)
        tuned[form] = autotune.apply("f64" if form == "fp64" else "f32", a.d)
        comp_form[form] = "f64" if form == "fp64" or a.sketch != "srht" else "f32"
        Af, yf = (A64, y64) if form == "fp64" else (A32, y32)
        if a.m == "auto":
            # sketch size from the Section 6 cost model with costs measured here by the library's chooser
            # (outside the timed region); the precision form's transform: FP32, unless the factor's diagonal
            # spread (about kappa / 25) exceeds 1e6, where the FP32 transform weakens the preconditioner
            # (the library would otherwise retake the sketch in FP64 inside the solve)
            extra = 2.0 if form == "fp64" else 3.0
            meas, t_pass, m_best, tab = msize.calibrate(ctx, Af, yf, a.sketch, compute=comp_form[form], s=a.s,
                                                        seed=a.seed, tol=a.tol, extra_passes=extra)
            spread = {r["m"]: r["r_spread"] for r in tab}[m_best]
            if form != "fp64" and comp_form[form] == "f32" and spread > 1e6:
                comp_form[form] = "f64"
                meas, t_pass, m_best, tab = msize.calibrate(ctx, Af, yf, a.sketch, compute="f64", s=a.s,
                                                            seed=a.seed, tol=a.tol, extra_passes=extra)
            m_form[form] = m_best
            m_model[form] = [{"m": r["m"], "sketch_ms": round(r["t_sketch_ms"], 3),
                              "factor_ms": round(r["t_factor_ms"], 3), "T": r["iters"],
                              "predicted_ms": round(r["predicted_ms"], 2), "r_spread": float(f"{r['r_spread']:.3g}")}
                             for r in tab]
            log(f"[bench] {form}: sketch size m={m_form[form]} ({comp_form[form]} transform) chosen by the cost model "
                f"(pass {t_pass:.3f} ms, diag(R) spread {spread:.2e})")
        else:
            m_form[form] = int(a.m)
        for _ in range(a.warmup):
            solve(form)
        ctx.fused_pass_timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(a.steps):
            x, info = solve(form)
            infos.append(info.as_dict())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        _, fused_ms, launches = ctx.fused_pass_timing()
        Aref = A64 if form == "fp64" else A32.double()
        e = float(torch.linalg.norm(Aref @ (x - xs)) / ax)
        if form != "fp64":
            del Aref
        bytes_per_pass = a.n * a.d * (8 if form == "fp64" else 4)
        res[form] = dict(s=dt, err=e, info=infos[-1], fused_ms=fused_ms, launches=launches,
                         fused_gbs=bytes_per_pass / (fused_ms * 1e-3) / 1e9 if fused_ms > 0 else None,
                         bytes_per_pass=bytes_per_pass)
        log(f"[bench] {form}: m={m_form[form]} {dt * 1e3:.1f} ms/solve  e_A={e:.2e}  status={info.status}  iters={info.iters} "
            f"refine={info.refinements} sketch={info.t_sketch_ms:.1f} factor={info.t_factor_ms:.1f} "
            f"iter={info.t_iter_ms:.1f} ms  fused {fused_ms:.3f} ms/launch "
            f"({res[form]['fused_gbs']:.0f} GB/s)")
    # the measured read ceiling over the largest operand (the bare streaming read of lsq_read_bandwidth)
    read_peak = ctx.read_bandwidth(A32 if A32 is not None else A64, reps=3)
    # and the read + write ceiling (bare streaming copy of 4 GiB of the same matrix)
    src = (A32 if A32 is not None else A64).view(-1)[: (1 << 30) // (A32 if A32 is not None else A64).element_size() * 4]
    dst = torch.empty_like(src)
    copy_peak = ctx.copy_bandwidth(src, dst, reps=3)
    del src, dst
    log(f"[bench] measured read ceiling {read_peak:.0f} GB/s, read + write ceiling {copy_peak:.0f} GB/s")
    ctx.close()
    # the SRHT's two passes at those ceilings: pass A reads A and writes the intermediate T (N rows of the
    # transform's precision), pass B reads T once
    sketch_floor = None
    if a.sketch == "srht":
        sketch_floor = {}
        nN = 1 << (a.n - 1).bit_length()
        for form in res:
            ab = a.n * a.d * (8 if form == "fp64" else 4)
            tb = nN * a.d * (8 if comp_form[form] == "f64" else 4)
            floor = ((ab + tb) / copy_peak + tb / read_peak) / 1e6
            meas = res[form]["info"]["t_sketch_ms"]
            sketch_floor[form] = {"pass_a_bytes": ab + tb, "pass_b_bytes": tb, "floor_ms": round(floor, 3),
                                  "measured_ms": round(meas, 3), "frac": round(floor / meas, 4)}

    head = "mixed" if "mixed" in res else forms[0]
    h = res[head]
    cpu = None
    if not a.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(P["A64"], m_form[head], a.sketch, a.s, a.seed, h["info"]["iters"],
                           sketch_rows=a.cpu_sample_rows)
    out = {
        "metric": "time-to-solve (s) + HBM GB/s, n=2^22 d=1024 to 1e-10; mixed vs FP64",
        "value": round(h["s"], 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(h["s"] * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage + f64" if head == "mixed" else "f64",
        "data": "synthetic (planted, exact minimiser known)",
        "config": {"workload": f"least squares n={a.n} d={a.d} kappa={a.kappa:g} sigma={a.sigma} "
                               f"{a.sketch} m={m_form[head]} tol={a.tol:g}",
                   "n": a.n, "d": a.d, "m": m_form[head], "m_by_form": m_form,
                   "m_rule": ("Section 6 cost model, measured costs (lsq_choose_sketch_size)" if a.m == "auto"
                              else "fixed"),
                   "transform_by_form": comp_form,
                   "m_model": m_model or None, "kappa": a.kappa, "sketch": a.sketch,
                   "parallelism": "single GPU", "tuned": tuned},
        "rel_a_norm_error": h["err"],
        "fp64": ({"time_s": round(res["fp64"]["s"], 5), "rel_a_norm_error": res["fp64"]["err"],
                  "status": res["fp64"]["info"]["status"],
                  "iters": res["fp64"]["info"]["iters"], "refinements": res["fp64"]["info"]["refinements"],
                  "fused_gbs": round(res["fp64"]["fused_gbs"], 1),
                  "phases_ms": {k: round(res["fp64"]["info"][k], 3) for k in
                                ("t_sketch_ms", "t_factor_ms", "t_iter_ms")}}
                 if "fp64" in res else None),
        "mixed": ({"time_s": round(res["mixed"]["s"], 5), "rel_a_norm_error": res["mixed"]["err"],
                   "status": res["mixed"]["info"]["status"],
                   "iters": res["mixed"]["info"]["iters"], "refinements": res["mixed"]["info"]["refinements"],
                   "fused_gbs": round(res["mixed"]["fused_gbs"], 1),
                   "phases_ms": {k: round(res["mixed"]["info"][k], 3) for k in
                                 ("t_sketch_ms", "t_factor_ms", "t_iter_ms")}}
                  if "mixed" in res else None),
        "speedup_mixed_vs_fp64": (round(res["fp64"]["s"] / res["mixed"]["s"], 3)
                                  if "fp64" in res and "mixed" in res else None),
        "roofline": {"bound": "hbm", "achieved": round(h["fused_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(h["fused_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(a.n, a.d, head,
                                                tuned.get(head, {}).get("fused_groups_per_cu", 8)),
                     "measured_read_peak": round(read_peak, 1),
                     "measured_copy_peak": round(copy_peak, 1),
                     "frac_of_measured": round(h["fused_gbs"] / read_peak, 4),
                     "kernel": "k_fused (A^T(A p), one pass)",
                     "bytes_per_launch": h["bytes_per_pass"], "avg_launch_ms": round(h["fused_ms"], 4),
                     "launches": h["launches"]},
        "sketch_floor": sketch_floor,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Sketch-size chooser (Section 6): the paper's optimized sketch sizes, and the same cost model refined
with costs measured on this GPU.

Section 6 writes the cost of PCG to an (eps, delta)-accurate solution as
    C(m) = C_sketch(m) + C_factor(m) + T(m) C_pass,   T(m) = ceil(log(4/eps) / log(1/rho)),
with rho = d/m for the fixed-sketch PCG bound delta_t/delta_0 <= 4 rho^t (Section 3.1), and minimises
it in flop counts:
  * Gaussian (Theorem 6.2): C(m) = m d^2 + n d log(1/eps) / log(m/d), for which the theorem gives
        m* = d exp(W0((n / d^2) log(1/eps)))          (W0: principal branch of Lambert's W);
    the exact minimiser of that C(m) is d exp(2 W0(sqrt(K)/2)) with K = (n/d^2) log(1/eps)
    (`m_opt_gaussian`; the theorem's stationarity condition drops a factor log(m/d));
  * SRHT (Theorem 6.1, constants dropped): if sqrt(log(1/eps)) < log(n/d^2),
        m* = e^{sqrt(log(1/eps))} d log d,  else  m* = (n/d) max(log d, log(1/eps) / log(n/d^2)).
The paper leaves a hardware-specific version as future work; `choose` does it by replacing the flop
counts with times measured on this GPU (`calibrate`: the library's sketch and factor at each candidate
m, and one fused pass) and keeping the iteration count T(m).  Here eps = tol^2, since tol bounds the
relative A-norm error and delta is its square.
"""
import math

FACTOR_M_MAX = 65536  # largest m the factorization accepts


def lambert_w0(a):
    """Principal branch W0(a) for a >= 0 (W e^W = a) by Halley's iteration from a log-based start."""
    a = float(a)
    if a < 0.0:
        raise ValueError("lambert_w0 is implemented for a >= 0")
    if a == 0.0:
        return 0.0
    w = math.log1p(a) if a < 3.0 else math.log(a) - math.log(math.log(a))
    for _ in range(64):
        ew = math.exp(w)
        f = w * ew - a
        wn = w - f / (ew * (w + 1.0) - (w + 2.0) * f / (2.0 * w + 2.0))
        if abs(wn - w) <= 4e-16 * max(1.0, abs(wn)):
            return wn
        w = wn
    return w


def pcg_iterations(m, d, tol):
    """T(m) = ceil(log(4 / eps) / log(m / d)) with eps = tol^2 (Section 6 with rho = d/m)."""
    if m <= d:
        return math.inf
    return math.ceil(math.log(4.0 / (tol * tol)) / math.log(m / d))


def m_star_gaussian(n, d, tol):
    """Theorem 6.2 (needs n > d^2): m* = d exp(W0((n/d^2) log(1/eps)))."""
    eps = tol * tol
    return d * math.exp(lambert_w0(n / (d * d) * math.log(1.0 / eps)))


def m_opt_gaussian(n, d, tol):
    """The exact minimiser of the cost Theorem 6.2 starts from, C(m) = m d^2 + n d log(1/eps) / log(m/d):
    with alpha = m/d its derivative vanishes where alpha (log alpha)^2 = K, K = (n/d^2) log(1/eps), i.e.
    log alpha = 2 W0(sqrt(K) / 2).  (The theorem's closed form solves alpha log alpha = K instead.)"""
    eps = tol * tol
    K = n / (d * d) * math.log(1.0 / eps)
    return d * math.exp(2.0 * lambert_w0(0.5 * math.sqrt(K)))


def m_star_srht(n, d, tol):
    """Theorem 6.1 with the constants dropped (needs n > d^2)."""
    eps = tol * tol
    le = math.log(1.0 / eps)
    if math.sqrt(le) < math.log(n / (d * d)):
        return math.exp(math.sqrt(le)) * d * math.log(d)
    return (n / d) * max(math.log(d), le / math.log(n / (d * d)))


def paper_m_star(kind, n, d, tol):
    """The paper's prescription (Gaussian: Theorem 6.2, SRHT: Theorem 6.1); None when it does not apply
    (n <= d^2, or an embedding without a theorem)."""
    if n <= d * d:
        return None
    if kind == "gaussian":
        return m_star_gaussian(n, d, tol)
    if kind == "srht":
        return m_star_srht(n, d, tol)
    return None


def candidates(n, d, kind):
    """Sketch sizes the chooser considers: 1.5d .. 64d, within the factorization's limit, m <= N for the
    SRHT and m <= 16384 for the SJLT."""
    N = 1 << max(0, (n - 1).bit_length())
    hi = FACTOR_M_MAX
    if kind == "srht":
        hi = min(hi, N)
    if kind == "sjlt":
        hi = min(hi, 16384)
    out = []
    for f in (1.5, 2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32, 40, 48, 64):
        m = int(round(f * d / 64.0)) * 64 if d >= 64 else int(round(f * d))
        if d < m <= hi and m not in out:
            out.append(m)
    return out


def predict(meas, t_pass, d, tol, extra_passes=0.0):
    """Predicted time-to-solve (ms) per candidate m: measured sketch + factor, plus T(m) + extra passes
    at the measured time of one pass.  meas: {m: (t_sketch_ms, t_factor_ms)}."""
    return {m: ts + tf + (pcg_iterations(m, d, tol) + extra_passes) * t_pass for m, (ts, tf) in meas.items()}


def choose(meas, t_pass, d, tol, extra_passes=0.0):
    """The candidate with the smallest predicted time, and the predictions."""
    pred = predict(meas, t_pass, d, tol, extra_passes)
    return min(pred, key=lambda m: (pred[m], m)), pred


def calibrate(ctx, A, y, kind, compute="f64", s=4, seed=1, ms=None, reps=2):
    """Measure the library's sketch and factor times (ms) at each candidate m and the time of one fused
    pass, on the caller's matrix (torch CUDA tensors A, y).  Returns (meas, t_pass_ms)."""
    import torch

    from . import lsq
    n, d = A.shape
    ms = ms or candidates(n, d, kind)
    ev0, ev1, ev2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    stream = torch.cuda.current_stream()
    meas = {}
    for m in ms:
        SA = torch.empty((m, d), dtype=torch.float64, device="cuda")
        R = torch.empty((d, d), dtype=torch.float64, device="cuda")
        W = torch.empty((d, d), dtype=torch.float64, device="cuda")
        best = None
        for _ in range(reps + 1):
            desc = lsq.sketch_desc(kind, m, seed=seed, s=s, compute=compute)
            ev0.record(stream)
            ctx.sketch(A, y, desc, SA)
            ev1.record(stream)
            ctx.factor(SA, R, W)
            ev2.record(stream)
            ev2.synchronize()
            cur = (ev0.elapsed_time(ev1), ev1.elapsed_time(ev2))
            best = cur if best is None else (min(best[0], cur[0]), min(best[1], cur[1]))
        meas[m] = best
        del SA, R, W
    v = torch.randn(d, dtype=torch.float64, device="cuda")
    w = torch.empty(d, dtype=torch.float64, device="cuda")
    sc = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.fused_pass(A, y, v, w, sc)
    ctx.fused_pass_timing(reset=True)
    for _ in range(3):
        ctx.fused_pass(A, y, v, w, sc)
    _, t_pass, _ = ctx.fused_pass_timing()
    return meas, float(t_pass)


def table(meas, t_pass, d, tol, extra_passes=0.0):
    """Rows (m, sketch ms, factor ms, T(m), predicted ms) for reports."""
    pred = predict(meas, t_pass, d, tol, extra_passes)
    return [(m, meas[m][0], meas[m][1], pcg_iterations(m, d, tol), pred[m]) for m in sorted(meas)]


__all__ = ["lambert_w0", "pcg_iterations", "m_star_gaussian", "m_opt_gaussian", "m_star_srht", "paper_m_star", "candidates",
           "predict", "choose", "calibrate", "table"]

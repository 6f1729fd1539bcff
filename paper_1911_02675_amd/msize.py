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


def calibrate(ctx, A, y, kind, compute="f64", s=4, seed=1, tol=1e-10, extra_passes=0.0, reps=2):
    """The library's chooser (lsq_choose_sketch_size: the sketch, factor and one fused pass timed on this GPU
    at every candidate m, on the caller's torch CUDA tensors A, y).  Returns (meas, t_pass_ms, m_best, table)
    with meas = {m: (t_sketch_ms, t_factor_ms)} for `choose` / `predict` and table the library's rows."""
    from . import lsq
    desc = lsq.sketch_desc(kind, 0, seed=seed, s=s, compute=compute)
    m_best, table, t_pass = ctx.choose_sketch_size(A, y, desc, tol=tol, extra_passes=extra_passes, reps=reps)
    meas = {r["m"]: (r["t_sketch_ms"], r["t_factor_ms"]) for r in table}
    return meas, float(t_pass), m_best, table


def table(meas, t_pass, d, tol, extra_passes=0.0):
    """Rows (m, sketch ms, factor ms, T(m), predicted ms) of the cost model, by increasing m."""
    pred = predict(meas, t_pass, d, tol, extra_passes)
    return [(m, meas[m][0], meas[m][1], pcg_iterations(m, d, tol), pred[m]) for m in sorted(meas)]

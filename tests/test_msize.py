"""The sketch-size chooser (Section 6) on the CPU: Lambert's W against scipy, Theorem 6.2's m* against a
direct minimisation of the paper's cost, the iteration count of the PCG bound, and the chooser's
argmin against brute force on synthetic cost tables."""
import math

import numpy as np
import pytest

from paper_1911_02675_amd import msize


def test_lambert_w0_against_scipy():
    from scipy.special import lambertw
    for a in np.concatenate([[0.0], np.logspace(-10, 12, 200)]):
        w = msize.lambert_w0(a)
        ref = float(lambertw(a, 0).real)
        assert abs(w - ref) <= 1e-13 * max(1.0, abs(ref)), a
        assert abs(w * math.exp(w) - a) <= 1e-12 * max(1.0, a)


@pytest.mark.parametrize("n,d,tol", [(10 ** 7, 50, 1e-4), (1 << 22, 256, 1e-10), (1 << 20, 64, 1e-8)])
def test_gaussian_sketch_size_against_the_cost(n, d, tol):
    eps = tol * tol
    K = n / (d * d) * math.log(1 / eps)
    cost = lambda m: m * d * d + n * d * math.log(1 / eps) / math.log(m / d)
    ms = np.exp(np.linspace(math.log(d * 1.01), math.log(d * 1e6), 400001))
    best = ms[np.argmin([cost(m) for m in ms])]
    # the exact minimiser of the cost function of Theorem 6.2
    assert abs(msize.m_opt_gaussian(n, d, tol) - best) <= 1e-3 * best
    # the theorem's closed form as printed: alpha log alpha = K with alpha = m*/d
    alpha = msize.m_star_gaussian(n, d, tol) / d
    assert abs(alpha * math.log(alpha) - K) <= 1e-10 * K
    # it over-sizes the sketch, at a cost within the theorem's order
    assert msize.m_star_gaussian(n, d, tol) > best
    assert cost(msize.m_star_gaussian(n, d, tol)) <= 4 * cost(best)


def test_srht_m_star_regimes():
    # sqrt(log(1/eps)) < log(n/d^2): e^{sqrt(log 1/eps)} d log d
    n, d, tol = 10 ** 9, 32, 1e-2
    le = math.log(1 / tol ** 2)
    assert math.sqrt(le) < math.log(n / d ** 2)
    assert math.isclose(msize.m_star_srht(n, d, tol), math.exp(math.sqrt(le)) * d * math.log(d))
    n, d, tol = 1 << 22, 1024, 1e-10
    le = math.log(1 / tol ** 2)
    assert math.sqrt(le) >= math.log(n / d ** 2)
    assert math.isclose(msize.m_star_srht(n, d, tol), (n / d) * max(math.log(d), le / math.log(n / d ** 2)))
    assert msize.paper_m_star("srht", 1000, 64, 1e-6) is None  # n <= d^2
    assert msize.paper_m_star("sjlt", 1 << 22, 64, 1e-6) is None


def test_pcg_iterations_formula():
    # 4 rho^T <= eps with rho = d/m: the smallest such T
    for m, d, tol in ((4096, 1024, 1e-10), (2048, 1024, 1e-10), (8192, 1024, 1e-8), (300, 64, 1e-6)):
        T = msize.pcg_iterations(m, d, tol)
        assert 4 * (d / m) ** T <= tol * tol * (1 + 1e-12)
        assert 4 * (d / m) ** (T - 1) > tol * tol
    assert msize.pcg_iterations(64, 64, 1e-6) == math.inf


def test_choose_matches_brute_force():
    rng = np.random.default_rng(3)
    d, tol = 512, 1e-10
    for _ in range(20):
        ms = msize.candidates(1 << 20, d, "srht")
        meas = {m: (float(rng.uniform(1, 5)) + 1e-3 * m * rng.uniform(0, 2),
                    float(rng.uniform(0.5, 2)) + 1e-3 * m * rng.uniform(0, 2)) for m in ms}
        t_pass = float(rng.uniform(0.2, 5))
        m, pred = msize.choose(meas, t_pass, d, tol, extra_passes=2)
        brute = min(ms, key=lambda k: meas[k][0] + meas[k][1] + (msize.pcg_iterations(k, d, tol) + 2) * t_pass)
        assert m == brute
        assert set(pred) == set(ms)


def test_candidates_respect_limits():
    assert all(1024 < m <= 65536 for m in msize.candidates(1 << 22, 1024, "srht"))
    assert max(msize.candidates(1 << 22, 1024, "srht")) == 65536  # the factorization's limit
    assert max(msize.candidates(1 << 22, 2048, "srht")) == 65536
    assert max(msize.candidates(1 << 22, 1024, "sjlt")) == 16384
    assert all(m <= 4096 for m in msize.candidates(4096, 1024, "srht"))  # m <= N for the SRHT
    assert msize.candidates(1 << 22, 1024, "srht")[0] == 1536

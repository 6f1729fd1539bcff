"""Pins of the oracle's PCG and IHS/Polyak-IHS against the paper's results:
  Theorem 3.1   PCG attains the polynomial lower bound and beats fixed-sketch IHS at every step
  Section 3.1   the extreme-eigenvalue bound 4 ((sqrt l1 - sqrt ld)/(sqrt l1 + sqrt ld))^{2t}
  CG theory     termination in at most d steps; H_S = H gives one step
  Theorem 3.3   (its proof) the per-instance fixed-sketch IHS error through eig(C_S)
  Theorem 4.1   refreshed Gaussian IHS: E delta_t / delta_0 = (1 - theta_1^2/theta_2)^t
  Theorem 4.3   (its proof) the moment recursion of refreshed Polyak-IHS; no gain from momentum
"""
import numpy as np

from oracle import draws, sketch, theory
from oracle.householder import householder_qr
from oracle.ihs import ihs
from oracle.pcg import pcg, sketch_factor
from oracle.solve import a_norm_error, lstsq_householder
from synth import make_problem


def _delta(A, x, xs):
    return 0.5 * float(np.sum((A @ (x - xs)) ** 2))


def _setup(n, d, kappa, seed):
    P = make_problem(n, d, kappa, seed=seed)
    xs = lstsq_householder(P["A"], P["y"])
    return P, xs


def test_pcg_attains_theorem_3_1_lower_bound():
    n, d, m = 256, 6, 12
    P, xs = _setup(n, d, 1e2, 7)
    A = P["A"]
    S = draws.gaussian_matrix(3, 0, m, n)
    R = householder_qr(S @ A)
    C = theory.c_s(P["U"], S)
    Delta0 = P["U"].T @ A @ (np.zeros(d) - xs)
    _, its = pcg(A, P["y"], R, fixed_iters=4)
    for t in range(5):
        lb = theory.pcg_optimal_error(C, Delta0, t)
        assert abs(_delta(A, its[t], xs) - lb) <= 1e-7 * _delta(A, its[0], xs)
    # any step size of fixed-sketch IHS is no better
    for mu in (0.3, 0.7, 1.0):
        ex = theory.fixed_ihs_exact(C, Delta0, mu, 4)
        for t in range(5):
            assert _delta(A, its[t], xs) <= ex[t] * (1 + 1e-9) + 1e-300


def test_pcg_extreme_eigenvalue_bound_and_termination():
    n, d, m = 2048, 24, 96
    P, xs = _setup(n, d, 1e4, 8)
    A = P["A"]
    for kind in ("gaussian", "srht", "sjlt"):
        if kind == "gaussian":
            S = draws.gaussian_matrix(5, 0, m, n)
        elif kind == "srht":
            S = sketch.srht_matrix(n, m, 5)
        else:
            S = sketch.sjlt_matrix(n, m, 2, 5)
        R = householder_qr(S @ A)
        assert np.allclose(R, sketch_factor(A, kind, m, 5, s=2), rtol=1e-10, atol=1e-14)
        bound = theory.pcg_bound(theory.c_s(P["U"], S), 12)
        _, its = pcg(A, P["y"], R, fixed_iters=d)
        d0 = _delta(A, its[0], xs)
        for t in range(13):
            assert _delta(A, its[t], xs) / d0 <= bound[t] * (1 + 1e-8) + 1e-24
        assert a_norm_error(A, its[d], xs) < 1e-10  # at most d steps


def test_pcg_one_step_when_sketch_is_exact():
    # SRHT with m = N has S^T S = I, so H_S = H and PCG is done after one step
    n, d = 512, 10
    P, xs = _setup(n, d, 1e5, 9)
    R = sketch_factor(P["A"], "srht", 512, 1)
    _, its = pcg(P["A"], P["y"], R, fixed_iters=1)
    assert a_norm_error(P["A"], its[1], xs) < 1e-11


def test_pcg_stop_rule_reaches_tolerance():
    n, d, m = 4096, 64, 256
    P, xs = _setup(n, d, 1e3, 10)
    x, its = pcg(P["A"], P["y"], sketch_factor(P["A"], "srht", m, 2), tol=1e-10)
    assert a_norm_error(P["A"], x, xs) <= 1e-10
    assert 10 <= len(its) - 1 <= 60


def test_fixed_ihs_matches_per_instance_formula():
    n, d, m = 512, 8, 40
    P, xs = _setup(n, d, 1e3, 11)
    A = P["A"]
    mu = 0.8
    its = ihs(A, P["y"], "gaussian", m, seed=4, mu=mu, iters=6, refresh=False)
    S = draws.gaussian_matrix(4, 0, m, n)
    ex = theory.fixed_ihs_exact(theory.c_s(P["U"], S), P["U"].T @ A @ (-xs), mu, 6)
    for t in range(7):
        assert abs(_delta(A, its[t], xs) - ex[t]) <= 1e-9 * ex[0]


def test_refreshed_gaussian_ihs_closed_form():
    n, d, m, T, reps = 1024, 16, 64, 10, 32
    P, xs = _setup(n, d, 1e5, 12)
    A = P["A"]
    t1, t2 = theory.theta_gaussian(m, d)
    mu = theory.optimal_step(t1, t2)
    pred = theory.refreshed_ihs_expected(t1, t2, mu, T)
    assert np.isclose(pred[1], 1 - t1 * t1 / t2)
    ratios = np.array([[_delta(A, x, xs) for x in ihs(A, P["y"], "gaussian", m, seed=100 + r, mu=mu, iters=T)]
                       for r in range(reps)])
    ratios /= ratios[:, :1]
    logs = np.log(ratios[:, 1:])
    mean = ratios[:, 1:].mean(axis=0)
    se = ratios[:, 1:].std(axis=0) / np.sqrt(reps) / mean
    assert np.all(np.abs(np.log(mean / pred[1:])) <= np.maximum(np.log(1.25), 4 * se))
    assert np.all(logs.mean(axis=0) < 0)
    # the closed form also separates step sizes: a step 1.5x too long is predicted (and seen) worse
    worse = theory.refreshed_ihs_expected(t1, t2, 1.5 * mu, T)
    assert np.all(worse[1:] > pred[1:])


def test_refreshed_polyak_recursion_and_no_acceleration():
    n, d, m, T, reps = 1024, 16, 48, 8, 48
    P, xs = _setup(n, d, 1e4, 13)
    A = P["A"]
    t1, t2 = theory.theta_gaussian(m, d)
    mu = theory.optimal_step(t1, t2)
    ihs_pred = theory.refreshed_ihs_expected(t1, t2, mu, T)
    for beta in (0.1, 0.5):
        pred = theory.polyak_expected(t1, t2, mu, beta, T)
        assert np.all(pred[1:] >= ihs_pred[1:] * (1 - 1e-12))  # momentum does not help
        sims = np.array([[_delta(A, x, xs) for x in ihs(A, P["y"], "gaussian", m, seed=500 + r, mu=mu,
                                                        beta=beta, iters=T)] for r in range(reps)])
        sims /= sims[:, :1]
        mean = sims.mean(axis=0)
        se = sims.std(axis=0) / np.sqrt(reps)
        assert np.all(np.abs(mean[1:] - pred[1:]) <= np.maximum(0.2 * pred[1:], 4 * se[1:]))
    # beta = 0 reduces the recursion to the IHS formula exactly
    assert np.allclose(theory.polyak_expected(t1, t2, mu, 0.0, T), ihs_pred)

"""Pins of the fixed-sketch IHS / Polyak-IHS parameters of Theorem 3.2 (rho = d/m):
  Theorem 3.4   mu* = (1 - rho)^2 / (1 + rho) minimises Gamma_t^rho(mu) = E_MP (1 - mu/lambda)^{2t} as
                t grows, with rate 4 rho / (1 + rho)^2 (Marchenko-Pastur density integrated numerically)
  Theorem 3.2   on the Marchenko-Pastur support the IHS contraction is at most sqrt(4 rho/(1+rho)^2),
                and the heavy-ball matrix with mu = (1 - rho)^2, beta = rho has spectral radius at most
                sqrt(rho) (so the asymptotic rate of delta_t is at most rho)
  proof of Thm 3.3   on an instance, fixed-sketch IHS with the rule's step follows the per-instance
                formula through eig(C_S)
"""
import numpy as np
import pytest

from oracle import draws, theory
from oracle.householder import householder_qr
from oracle.ihs import ihs
from oracle.solve import lstsq_householder
from synth import make_problem


def test_mp_density_is_a_probability():
    for rho in (0.1, 0.25, 0.5):
        assert abs(theory.mp_gamma(rho, 0.0, 0) - 1.0) <= 1e-9
        # inverse moments of MP(rho, 1): E 1/lambda = 1/(1 - rho), E 1/lambda^2 = 1/(1 - rho)^3
        lm = theory.mp_gamma(rho, 1.0, 1)  # E (1 - 1/l)^2 = 1 - 2 E l^-1 + E l^-2
        e1 = 1.0 / (1.0 - rho)
        e2 = 1.0 / (1.0 - rho) ** 3
        assert abs(lm - (1.0 - 2.0 * e1 + e2)) <= 1e-8


@pytest.mark.parametrize("rho", [0.25, 0.5])
def test_mp_optimal_step_theorem_3_4(rho):
    d, m = 1, 1.0 / rho
    mu_star, rate, _, _ = theory.fixed_sketch_params(d, m)
    t = 800
    mus = np.linspace(0.5 * mu_star, 1.5 * mu_star, 2001)
    g = np.array([theory.mp_gamma(rho, mu, t) for mu in mus])
    assert abs(mus[int(np.argmin(g))] - mu_star) <= 0.005 * mu_star
    r = theory.mp_gamma(rho, mu_star, t + 1) / theory.mp_gamma(rho, mu_star, t)
    assert abs(r - rate) <= 0.005 * rate


@pytest.mark.parametrize("rho", [0.125, 0.25, 0.5])
def test_theorem_3_2_contractions_on_mp_support(rho):
    mu, rate, mu_p, beta = theory.fixed_sketch_params(1, 1.0 / rho)
    lam = np.linspace((1 - np.sqrt(rho)) ** 2, (1 + np.sqrt(rho)) ** 2, 4001)
    c = np.abs(1.0 - mu / lam)
    assert np.max(c) <= np.sqrt(rate) * (1 + 1e-12)
    assert abs(np.max(c) - np.sqrt(rate)) <= 1e-9  # attained at the edges
    rad = []
    for l in lam:
        M = np.array([[1.0 + beta - mu_p / l, -beta], [1.0, 0.0]])
        rad.append(np.max(np.abs(np.linalg.eigvals(M))))
    # at the support edges the 2 x 2 matrix has a double eigenvalue, whose computed value carries
    # an error of order sqrt(eps)
    assert np.max(rad) <= np.sqrt(beta) * (1 + 1e-6)


def test_fixed_ihs_with_rule_follows_per_instance_formula():
    n, d, m, T = 2048, 16, 64, 10
    P = make_problem(n, d, 1e3, seed=33)
    A, y = P["A"], P["y"]
    xs = lstsq_householder(A, y)
    mu, rate, mu_p, beta = theory.fixed_sketch_params(d, m)
    S = draws.gaussian_matrix(17, 0, m, n)
    C = theory.c_s(P["U"], S)
    Delta0 = P["U"].T @ A @ (np.zeros(d) - xs)
    pred = theory.fixed_ihs_exact(C, Delta0, mu, T)
    its = ihs(A, y, "gaussian", m, seed=17, mu=mu, iters=T, refresh=False)
    got = np.array([0.5 * float(np.sum((A @ (x - xs)) ** 2)) for x in its])
    assert np.allclose(got, pred, rtol=1e-6, atol=1e-12 * got[0])
    # Polyak-IHS with the rule's parameters is faster than the rule's IHS on this instance
    itp = ihs(A, y, "gaussian", m, seed=17, mu=mu_p, beta=beta, iters=T, refresh=False)
    assert 0.5 * float(np.sum((A @ (itp[-1] - xs)) ** 2)) < got[-1]

"""Closed forms from the paper used as pins and as step-size rules.

Oracle module (test infrastructure only).
"""
import numpy as np


def theta_gaussian(m, d):
    """Inverse moments of C_S for a Gaussian embedding (Section 2, from Gupta's lemma):
    theta_1 = m / (m - d - 1),  theta_2 = m^2 (m - 1) / ((m - d)(m - d - 1)(m - d - 3)),  m >= d + 4."""
    if m < d + 4:
        raise ValueError("needs m >= d + 4")
    t1 = m / (m - d - 1)
    t2 = m * m * (m - 1) / ((m - d) * (m - d - 1) * (m - d - 3))
    return t1, t2


def theta_haar(n, d, m):
    """Finite-sample approximations for a Haar embedding with orthonormal rows (Section 2); the same
    trace formulas hold asymptotically for the SRHT:
    theta_1 ~ (n - d)/(m - d),  theta_2 ~ (n - d)(d^2 + m n - 2 d m)/(m - d)^3."""
    t1 = (n - d) / (m - d)
    t2 = (n - d) * (d * d + m * n - 2 * d * m) / (m - d) ** 3
    return t1, t2


def theta1_haar_exact(n, d, m):
    """theta_1 = d^{-1} tr E[C_S^{-1}] for a Haar embedding with orthonormal rows, exactly: C_S = U^T P U
    with P a uniformly random rank-m projection is a d x d matrix-variate beta B(m/2, (n-m)/2), whose
    inverse has mean (n - d - 1)/(m - d - 1) I (m > d + 1).  Section 2's (n - d)/(m - d) is its limit."""
    if m <= d + 1:
        raise ValueError("needs m > d + 1")
    return (n - d - 1) / (m - d - 1)


def theta2_haar_exact(n, d, m):
    """theta_2 = d^{-1} tr E[C_S^{-2}] for a Haar embedding with orthonormal rows, exactly (m > d + 3).
    With the rows of an n x d standard Gaussian Z split into the first m and the other k = n - m,
    X = Z_1^T Z_1 ~ W_d(m, I) and Y = Z_2^T Z_2 ~ W_d(k, I) are independent and C_S has the law of
    (X + Y)^{-1/2} X (X + Y)^{-1/2} (the same matrix-variate beta as in theta1_haar_exact), so
        tr C_S^{-2} = tr (I + X^{-1} Y)^2 = d + 2 tr(X^{-1} Y) + tr(X^{-1} Y X^{-1} Y).
    Averaging over Y first (E[Y M Y] = k(k+1) M + k tr(M) I for symmetric M, from the fourth moments of
    a Gaussian vector) and then over X with the inverse-Wishart moments
        E[X^{-1}] = I / (m-d-1),   E[X^{-2}] = (m-1) I / D,   E[tr(X^{-1}) X^{-1}] = ((m-d-2) d + 2) I / D,
    D = (m-d)(m-d-1)(m-d-3), gives
        theta_2 = 1 + 2k / (m-d-1) + k ((k+1)(m-1) + (m-d-2) d + 2) / D.
    Section 2's (n - d)(d^2 + m n - 2 d m)/(m - d)^3 is its large-size limit."""
    if m <= d + 3:
        raise ValueError("needs m > d + 3")
    k = n - m
    D = (m - d) * (m - d - 1) * (m - d - 3)
    return 1.0 + 2.0 * k / (m - d - 1) + k * ((k + 1) * (m - 1) + (m - d - 2) * d + 2) / D


def srht_thetas_scaled(N, d, m):
    """theta's of the SRHT as scaled here (S = m^{-1/2} R H E, so S S^T = (N/m) I): the Haar values
    for an m x N embedding with orthonormal rows, times (m/N) and (m/N)^2."""
    t1, t2 = theta_haar(N, d, m)
    c = m / N
    return c * t1, c * c * t2


def optimal_step(t1, t2):
    """mu = theta_1 / theta_2, the minimiser of the refreshed-IHS expected error (Theorem 4.1)."""
    return t1 / t2


def refreshed_ihs_expected(t1, t2, mu, T):
    """E delta_t / E delta_0 = prod_j (1 - 2 mu theta_1 + mu^2 theta_2) for constant mu (Theorem 4.1)."""
    c = 1.0 - 2.0 * mu * t1 + mu * mu * t2
    return c ** np.arange(T + 1)


def polyak_expected(t1, t2, mu, beta, T):
    """E delta_t / E delta_0 for refreshed Polyak-IHS with x_{-1} = x_0, from the linear recursion of
    the second moments in the proof of Theorem 4.3: with
        a_t = E delta_{t+1},  b_t = -(beta/2) E<Delta_t, Delta_{t+1}>,  c_t = beta^2 E delta_t,
        eta = (1+beta)^2 - 2 mu theta_1 (1+beta) + mu^2 theta_2,  gamma = 1 + beta - mu theta_1,
    X_{t+1} = [[eta, 2 gamma, 1], [-beta gamma, -beta, 0], [beta^2, 0, 0]] X_t.
    The first step is a plain IHS step, so a_0 = (1 - 2 mu theta_1 + mu^2 theta_2) delta_0,
    b_0 = -beta (1 - mu theta_1) delta_0 and E delta_{t+1} = a_t."""
    eta = (1 + beta) ** 2 - 2 * mu * t1 * (1 + beta) + mu * mu * t2
    gamma = 1 + beta - mu * t1
    M = np.array([[eta, 2 * gamma, 1.0], [-beta * gamma, -beta, 0.0], [beta * beta, 0.0, 0.0]])
    X = np.array([1 - 2 * mu * t1 + mu * mu * t2, -beta * (1 - mu * t1), beta * beta])
    out = [1.0]
    for _ in range(T):
        out.append(X[0])
        X = M @ X
    return np.array(out)


def c_s(U, S):
    """C_S = U^T S^T S U for orthonormal U (n x d) and an explicit S (m x n) (Section 1.3)."""
    SU = S @ U
    return SU.T @ SU


def fixed_ihs_exact(C, Delta0, mu, T):
    """Per-instance IHS error with a fixed sketch (proof of Theorem 3.3):
    delta_t = 1/2 sum_i (1 - mu/lambda_i)^{2t} (v_i^T Delta_0)^2, (lambda_i, v_i) eigenpairs of C_S."""
    lam, V = np.linalg.eigh(C)
    xi2 = (V.T @ Delta0) ** 2
    return np.array([0.5 * np.sum((1 - mu / lam) ** (2 * t) * xi2) for t in range(T + 1)])


def pcg_optimal_error(C, Delta0, t):
    """Theorem 3.1: the smallest delta_t reachable after t steps by any method of the class with the
    fixed sketch, 1/2 min over polynomials Q of degree <= t with Q(0) = 1 of
    sum_i Q(1/lambda_i)^2 xi_i^2, xi_i = <v_i, Delta_0>.  PCG attains it."""
    lam, V = np.linalg.eigh(C)
    xi = V.T @ Delta0
    if t == 0:
        return 0.5 * float(xi @ xi)
    Vand = np.stack([(1.0 / lam) ** k for k in range(1, t + 1)], axis=1)
    c, *_ = np.linalg.lstsq(xi[:, None] * Vand, -xi, rcond=None)
    res = xi + (xi[:, None] * Vand) @ c
    return 0.5 * float(res @ res)


def pcg_bound(C, T):
    """delta_t / delta_0 <= 4 ((sqrt(l1) - sqrt(ld)) / (sqrt(l1) + sqrt(ld)))^{2t} (Section 3.1)."""
    lam = np.linalg.eigvalsh(C)
    q = (np.sqrt(lam[-1]) - np.sqrt(lam[0])) / (np.sqrt(lam[-1]) + np.sqrt(lam[0]))
    return 4.0 * q ** (2 * np.arange(T + 1))


def fixed_sketch_params(d, m):
    """Theorem 3.2 with rho = d/m (the edges (1 -+ sqrt(rho))^2 of the Marchenko-Pastur law that the
    eigenvalues of C_S follow, Section 3.2): the fixed-sketch IHS step mu = (1 - rho)^2 / (1 + rho) with
    delta_t / delta_0 <= (4 rho / (1 + rho)^2)^t, and the Polyak-IHS parameters mu = (1 - rho)^2,
    beta = rho with asymptotic rate rho.  Returns (mu_ihs, rate_ihs, mu_polyak, beta_polyak)."""
    rho = d / m
    return (1.0 - rho) ** 2 / (1.0 + rho), 4.0 * rho / (1.0 + rho) ** 2, (1.0 - rho) ** 2, rho


def mp_gamma(rho, mu, t, nodes=4000):
    """Gamma_t^rho(mu) = E_{lambda ~ MP(rho, 1)} (1 - mu / lambda)^{2t} (Section 3.2) by Gauss-Chebyshev
    quadrature of the second kind on [lambda_-, lambda_+] (the density is sqrt((l+ - l)(l - l-)) /
    (2 pi rho l))."""
    lm, lp = (1.0 - np.sqrt(rho)) ** 2, (1.0 + np.sqrt(rho)) ** 2
    k = np.arange(1, nodes + 1)
    z = np.cos(k * np.pi / (nodes + 1))
    w = np.pi / (nodes + 1) * np.sin(k * np.pi / (nodes + 1)) ** 2  # int sqrt(1-z^2) f(z) dz
    lam = 0.5 * (lp + lm) + 0.5 * (lp - lm) * z
    half = 0.5 * (lp - lm)
    # sqrt((l+ - l)(l - l-)) = half * sqrt(1 - z^2), dl = half dz
    dens = half * half / (2.0 * np.pi * rho * lam)
    with np.errstate(over="ignore"):  # steps far past 2 lambda_- give +inf, which is the right order
        return float(np.sum(w * dens * (1.0 - mu / lam) ** (2 * t)))

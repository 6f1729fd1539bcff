"""Pins of the oracle's explicit sketches: the Hadamard matrix against its definition and scipy's
Sylvester construction, H H = N I, the no-subsampling case S^T S = I, column norms of the SJLT, the
scatter against the dense matrix, and the inverse moments of Gaussian embeddings (Section 2)."""
import numpy as np
import scipy.linalg

from oracle import draws, sketch, theory


def test_fwht_matches_scipy_hadamard_and_hh():
    rng = np.random.default_rng(0)
    for N in (1, 2, 8, 64, 1024):
        X = rng.standard_normal((N, 3))
        H = scipy.linalg.hadamard(N)
        assert np.allclose(sketch.fwht_rows(X), H @ X, atol=1e-11)
        assert np.array_equal(H @ H, N * np.eye(N))
        k, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        assert np.array_equal(sketch.hadamard_entry(k, j), H)


def test_srht_full_sample_is_orthogonal():
    # m = N: R is the identity, S = N^{-1/2} H E and S^T S = I (so H_S = H)
    for n in (32, 29):
        S = sketch.srht_matrix(n, draws.padded_length(n), seed=4)
        assert np.allclose(S.T @ S, np.eye(S.shape[1]), atol=1e-12)


def test_srht_sketch_equals_dense_and_rowwise():
    rng = np.random.default_rng(1)
    for n in (256, 200):
        A = rng.standard_normal((n, 5))
        SA = sketch.srht_sketch(A, 24, seed=9, t=2)
        N = draws.padded_length(n)
        Ap = np.zeros((N, 5))
        Ap[:n] = A
        assert np.allclose(SA, sketch.srht_matrix(n, 24, 9, 2) @ Ap, atol=1e-12)
        pick = sketch.srht_sketch_rows(A, 24, 9, 2, [0, 7, 23], cols=[1, 4])
        assert np.allclose(pick, SA[[0, 7, 23]][:, [1, 4]], atol=1e-12)
    # small-integer A: every sum is exact, so the blocked row form (several blocks and a ragged one,
    # int8 storage) equals the full transform bit for bit before the 1/sqrt(m) scale
    Ai = rng.integers(-3, 4, size=(1000, 6)).astype(np.int8)
    full = sketch.srht_sketch(Ai.astype(np.float64), 40, seed=4, t=1) * np.sqrt(40)
    rows = sketch.srht_sketch_rows(Ai, 40, 4, 1, [0, 13, 39], row_block=96) * np.sqrt(40)
    assert np.array_equal(np.rint(rows), np.rint(full[[0, 13, 39]]))
    assert np.max(np.abs(rows - np.rint(rows))) < 1e-9


def test_sjlt_columns_unit_norm_and_scatter():
    n, m, s = 500, 32, 3
    S = sketch.sjlt_matrix(n, m, s, seed=5)
    assert np.allclose((S * S).sum(axis=0), 1.0, atol=1e-15)
    assert np.all((S != 0).sum(axis=0) == s)
    A = np.random.default_rng(2).standard_normal((n, 4))
    assert np.allclose(sketch.sjlt_sketch(A, m, s, 5), S @ A, atol=1e-12)


def test_embeddings_isotropic_in_expectation():
    # E[S^T S] = I for all three scalings
    n, m, T = 16, 8, 3000
    acc = {k: np.zeros((n, n)) for k in ("srht", "sjlt", "gaussian")}
    for seed in range(T):
        for k in acc:
            if k == "srht":
                S = sketch.srht_matrix(n, m, seed)
            elif k == "sjlt":
                S = sketch.sjlt_matrix(n, m, 2, seed)
            else:
                S = draws.gaussian_matrix(seed, 0, m, n)
            acc[k] += S.T @ S
    for k, v in acc.items():
        assert np.abs(v / T - np.eye(n)).max() < 0.12, k


def test_gaussian_inverse_moments_monte_carlo():
    # Condition 2.1 with Gupta's formulas: d^{-1} tr E[C_S^{-1}] = theta_1, d^{-1} tr E[C_S^{-2}] = theta_2
    n, d, m, T = 64, 4, 24, 4000
    U, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n, d)))
    t1s, t2s = [], []
    for seed in range(T):
        S = draws.gaussian_matrix(seed, 0, m, n)
        Ci = np.linalg.inv(theory.c_s(U, S))
        t1s.append(np.trace(Ci) / d)
        t2s.append(np.trace(Ci @ Ci) / d)
    t1, t2 = theory.theta_gaussian(m, d)
    se1 = np.std(t1s) / np.sqrt(T)
    se2 = np.std(t2s) / np.sqrt(T)
    assert abs(np.mean(t1s) - t1) < 4 * se1
    assert abs(np.mean(t2s) - t2) < 4 * se2
    # and the wrong normalisation (1/n instead of 1/m) would be far off
    assert abs(np.mean(t1s) * m / n - t1) > 20 * se1


def test_round_bf16_pins():
    from oracle.draws import round_bf16
    # exact bfloat16 values are fixed points; halfway cases go to the even significand
    exact = np.array([0.0, 1.0, -2.5, 1.0 + 2.0 ** -7, 3.0 * 2.0 ** -100, 65280.0])
    assert np.array_equal(round_bf16(exact), exact)
    assert round_bf16(1.0 + 2.0 ** -8) == 1.0                        # tie, even below
    assert round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6        # tie, even above
    assert round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert round_bf16(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    x = np.random.default_rng(3).standard_normal(100000) * 10.0 ** np.random.default_rng(4).uniform(-30, 30, 100000)
    r = round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))
    # result has at most 8 significand bits
    m_, e_ = np.frexp(r[r != 0])
    assert np.all(m_ * 2 ** 8 == np.round(m_ * 2 ** 8))


def test_gaussian_sketch_bf16_is_the_rounded_embedding():
    from oracle.draws import gaussian_matrix, round_bf16
    from oracle.sketch import gaussian_sketch, gaussian_sketch_bf16
    rng = np.random.default_rng(9)
    A = rng.standard_normal((300, 7))
    m, seed = 20, 5
    S = gaussian_matrix(seed, 0, m, 300) * np.sqrt(m)
    Sb = round_bf16(S) / np.sqrt(m)
    SA = gaussian_sketch_bf16(A, m, seed, row_block=128)
    assert np.allclose(SA, Sb @ A, rtol=1e-13, atol=1e-13)
    # within one bf16 rounding of the float64 sketch, entry by entry
    bound = 2.0 ** -8 * (np.abs(S) / np.sqrt(m)) @ np.abs(A)
    assert np.all(np.abs(SA - gaussian_sketch(A, m, seed)) <= bound + 1e-13)

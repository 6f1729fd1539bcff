"""Pins of the oracle's random draws against things other than itself: the published Philox
known-answer vectors, numpy's independent Philox4x64-10, exact counting for the multiply-shift
map, and the distributional facts that the embeddings of Section 2 require."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import draws
from oracle.philox import philox4x64_10

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x64_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_philox_matches_numpy_bit_generator():
    key = np.array([0x0123456789ABCDEF, 0xFEDCBA9876543210], dtype=np.uint64)
    for start in (0, 41, 2**40 + 3):
        bg = np.random.Philox(key=key, counter=np.array([start, 0, 0, 0], dtype=np.uint64))
        raw = bg.random_raw(4 * 16).reshape(16, 4)
        # numpy advances the counter before producing a block
        c = np.arange(start + 1, start + 17, dtype=np.uint64)
        mine = np.stack(philox4x64_10(c, 0, 0, 0, key[0], key[1]), axis=1)
        assert np.array_equal(raw, mine)


def test_lemire_map_is_exactly_uniform():
    # brute force over every 12-bit input: each bucket receives exactly floor(2^12 / m) values
    x = np.arange(1 << 12, dtype=np.uint64)
    for m in (1, 3, 7, 100, 255, 1000, 4095):
        h, ok = draws.lemire_map(x, m, width=12)
        counts = np.bincount(h[ok], minlength=m)
        assert counts.shape == (m,)
        assert np.all(counts == (1 << 12) // m)


def test_srht_signs_and_rows_basic():
    N, m = 1 << 12, 256
    e = draws.srht_signs(7, 0, N)
    assert set(np.unique(e)) <= {-1.0, 1.0}
    assert abs(e.sum()) < 4 * np.sqrt(N)
    rows = draws.srht_rows(7, 0, N, m)
    assert rows.shape == (m,) and np.all(np.diff(rows) > 0) and rows[0] >= 0 and rows[-1] < N
    assert not np.array_equal(rows, draws.srht_rows(7, 1, N, m))  # refresh counter changes S


def test_srht_subset_uniform_without_replacement():
    # N = 5, m = 2: all 10 subsets equally likely
    counts = {}
    T = 3000
    for seed in range(T):
        r = tuple(draws.srht_rows(seed, 0, 5, 2))
        counts[r] = counts.get(r, 0) + 1
    assert len(counts) == 10
    obs = np.array(list(counts.values()))
    p = stats.chisquare(obs).pvalue
    assert p > 1e-3


def test_sjlt_draws_distinct_uniform():
    n, m, s = 20000, 64, 4
    tg, sg = draws.sjlt_draws(3, 0, n, m, s)
    assert tg.min() >= 0 and tg.max() < m
    srt = np.sort(tg, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0)  # s distinct targets per row
    assert set(np.unique(sg)) == {-1.0, 1.0}
    p = stats.chisquare(np.bincount(tg.ravel(), minlength=m)).pvalue
    assert p > 1e-3
    assert abs(sg.sum()) < 4 * np.sqrt(sg.size)


def test_sjlt_s_equals_m_takes_every_row():
    tg, _ = draws.sjlt_draws(5, 0, 50, 8, 8)
    assert np.all(np.sort(tg, axis=1) == np.arange(8))


def test_gaussian_normals_distribution():
    g = draws.gaussian_normals(11, 0, np.arange(64)[:, None], np.arange(4096)[None, :]).ravel()
    assert stats.kstest(g, "norm").pvalue > 1e-3
    assert abs(g.mean()) < 4 / np.sqrt(g.size)
    assert abs(g.var() - 1) < 6 * np.sqrt(2 / g.size)
    # cos / sin members of a Box-Muller pair are uncorrelated
    G = g.reshape(64, 4096)
    assert abs(np.corrcoef(G[:, 0::2].ravel(), G[:, 1::2].ravel())[0, 1]) < 0.02


def test_gaussian_random_access_consistent():
    full = draws.gaussian_matrix(2, 3, 16, 40)
    pick = draws.gaussian_normals(2, 3, np.array([5, 9]), np.array([17, 33])) / 4.0
    assert np.array_equal(pick, full[[5, 9], [17, 33]])

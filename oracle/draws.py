"""The random draws of the three embeddings, as pure functions of (seed, t, index).

Oracle module (test infrastructure only).  The GPU library implements the same specification
independently; integer draws (signs, row subsets, SJLT targets) must agree bit for bit, and the
Gaussian entries within a stated floating-point tolerance.

Specification (every draw is a Philox4x64-10 block, key = (seed, 0)):

  SRHT  (Section 2: S = R H E, E random signs, R uniform row subsample without replacement)
        block for padded row j in [0, N):  counter (j, 1, t, 0) -> words (w0, w1, w2, w3)
        sign  e_j = -1 if bit 63 of w0 is set, else +1
        subset: the m rows with the smallest (w1, j) pairs (w1 compared as unsigned 64-bit,
                ties broken by the smaller j); an i.i.d. uniform key per row makes every
                m-subset equally likely.  Selected rows are listed in increasing j.

  SJLT  (Section 2: for every column of S, i.e. every row j of A, s distinct rows of S chosen
        uniformly without replacement, entries +-1/sqrt(s))
        words of row j are read in the order w0..w3 of block (j, 2, t, 0), then of (j, 2, t, 1), ...
        For each word w:  x = w >> 32, P = x * m (64-bit), low = P mod 2^32.
            reject if low < (2^32 mod m)           (Lemire's multiply-shift, exact uniformity)
            h = P >> 32;  reject if h was already taken by row j
            otherwise take target h with sign -1 if bit 0 of w is set, else +1.
        Stop once s targets are taken.  At most MAX_SJLT_WORDS words are read.

  GAUSS (Section 2: i.i.d. N(0, 1/m) entries)
        entry (i, j) of S for i in [0, m), j in [0, n): block (j >> 3, 3, t, i), q = j & 7,
        pair p = q >> 1 uses word w_p:  a = w_p mod 2^32, b = w_p >> 32,
        u1 = (a + 1) 2^-32 in (0, 1],  u2 = b 2^-32 in [0, 1),
        g = sqrt(-2 ln u1) * (cos(2 pi u2) if q even else sin(2 pi u2))        (Box-Muller)
        S_ij = g / sqrt(m).
"""
import numpy as np

from .philox import philox4x64_10

TAG_SRHT = 1
TAG_SJLT = 2
TAG_GAUSS = 3
MAX_SJLT_WORDS = 4096

_U64 = np.uint64


def padded_length(n):
    """N = 2**ceil(log2 n): the SRHT zero-pads A to the next power of two (Section 2, footnote)."""
    N = 1
    while N < n:
        N *= 2
    return N


def srht_words(seed, t, N):
    j = np.arange(N, dtype=np.uint64)
    return philox4x64_10(j, TAG_SRHT, t, 0, seed, 0)


def srht_signs(seed, t, N):
    """Diagonal of E: +-1 for every padded row j in [0, N)."""
    w0, _, _, _ = srht_words(seed, t, N)
    return np.where((w0 >> _U64(63)) == 1, -1.0, 1.0)


def srht_rows(seed, t, N, m):
    """Rows of H E A kept by R: the m rows with the smallest (key, j), listed in increasing j."""
    if not (1 <= m <= N):
        raise ValueError("SRHT needs 1 <= m <= N")
    _, w1, _, _ = srht_words(seed, t, N)
    j = np.arange(N, dtype=np.int64)
    order = np.lexsort((j, w1))  # primary key w1, ties by j
    return np.sort(order[:m])


def lemire_map(x, m, width=32):
    """Multiply-shift map of a `width`-bit integer x onto [0, m), with its rejection rule.
    Returns (h, accepted).  Every h in [0, m) receives exactly floor(2**width / m) accepted x."""
    x = np.asarray(x, dtype=np.uint64)
    P = x * _U64(m)
    low = P & _U64((1 << width) - 1)
    thr = (1 << width) % m
    return (P >> _U64(width)).astype(np.int64), low >= _U64(thr)


def sjlt_draws(seed, t, n, m, s):
    """Targets (n, s) int64 and signs (n, s) float64 of the SJLT, per row j of A, in draw order."""
    if not (1 <= s <= m):
        raise ValueError("SJLT needs 1 <= s <= m")
    targets = np.full((n, s), -1, dtype=np.int64)
    signs = np.zeros((n, s))
    count = np.zeros(n, dtype=np.int64)
    rows = np.arange(n, dtype=np.uint64)
    for c in range(MAX_SJLT_WORDS // 4):
        todo = np.nonzero(count < s)[0]
        if todo.size == 0:
            break
        words = philox4x64_10(rows[todo], TAG_SJLT, t, c, seed, 0)
        for w in words:
            live = count[todo] < s
            h, ok = lemire_map(w >> _U64(32), m)
            dup = (targets[todo] == h[:, None]).any(axis=1)
            take = live & ok & ~dup
            r = todo[take]
            targets[r, count[r]] = h[take]
            signs[r, count[r]] = np.where((w[take] & _U64(1)) == 1, -1.0, 1.0)
            count[r] += 1
    if (count < s).any():
        raise RuntimeError("SJLT draw limit exhausted")
    return targets, signs


def box_muller(a, b, q_odd):
    """Gaussian from two 32-bit words (a, b): the cos branch for even q, the sin branch for odd q."""
    u1 = (np.asarray(a, dtype=np.float64) + 1.0) * 2.0 ** -32
    u2 = np.asarray(b, dtype=np.float64) * 2.0 ** -32
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return np.where(q_odd, r * np.sin(ang), r * np.cos(ang))


def gaussian_normals(seed, t, rows, cols):
    """Standard normals g(i, j) for the given row indices i and column indices j (arrays that
    broadcast); S_ij = g(i, j) / sqrt(m)."""
    rows = np.asarray(rows, dtype=np.uint64)
    cols = np.asarray(cols, dtype=np.uint64)
    rows, cols = np.broadcast_arrays(rows, cols)
    words = philox4x64_10(cols >> _U64(3), TAG_GAUSS, t, rows, seed, 0)
    q = (cols & _U64(7)).astype(np.int64)
    p = q >> 1
    w = np.choose(p, words)
    a = w & _U64(0xFFFFFFFF)
    b = w >> _U64(32)
    return box_muller(a, b, (q & 1) == 1)


def round_bf16(x):
    """Round to bfloat16 (8 significand bits) to nearest, ties to even, via single precision: the
    value is first rounded to float32, then its bit pattern keeps the upper 16 bits after adding
    0x7FFF plus the lowest kept bit.  Returns float64."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    bits = (bits + np.uint64(0x7FFF) + ((bits >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def gaussian_matrix(seed, t, m, n):
    """Dense S (m x n) of the Gaussian embedding, entries N(0, 1/m)."""
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    return gaussian_normals(seed, t, i, j) / np.sqrt(m)

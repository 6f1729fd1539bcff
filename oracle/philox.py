"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3",
SC'11), written from its published definition with plain numpy uint64 arithmetic.

Oracle module (test infrastructure only; see the package docstring).

State: a 4-word counter c = (c0, c1, c2, c3) and a 2-word key k = (k0, k1), all 64-bit.
One round:
    (hi0, lo0) = M0 * c0   (full 128-bit product)
    (hi1, lo1) = M1 * c2
    c' = (hi1 ^ c1 ^ k0,  lo1,  hi0 ^ c3 ^ k1,  lo0)
and between rounds the key is bumped by the Weyl constants (k0 += W0, k1 += W1).  Ten rounds.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo), built from four
    32x32 -> 64 partial products (schoolbook multiplication)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    p00 = a_lo * b_lo
    p01 = a_lo * b_hi
    p10 = a_hi * b_lo
    p11 = a_hi * b_hi
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2**64
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64-10.  Arguments broadcast; returns four uint64 arrays."""
    shape = np.broadcast(c0, c1, c2, c3, k0, k1).shape
    c0, c1, c2, c3, k0, k1 = (np.broadcast_to(np.asarray(v, dtype=np.uint64), shape).copy()
                              for v in (c0, c1, c2, c3, k0, k1))
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo64(M0, c0)
            hi1, lo1 = mulhilo64(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3

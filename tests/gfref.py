"""Independent GF(2^8) arithmetic used only to pin the oracle.

Written from the textbook definition (carry-less polynomial product reduced
modulo x^8 + x^4 + x^3 + x^2 + 1), not from log/antilog tables, so a mistake in
the oracle's tables cannot hide behind the same mistake here.
"""
import numpy as np

POLY = 0x11D


def mul(a, b):
    """Elementwise GF(2^8) product of integer arrays (or scalars)."""
    a = np.asarray(a, dtype=np.uint32)
    b = np.asarray(b, dtype=np.uint32)
    r = np.zeros(np.broadcast(a, b).shape, dtype=np.uint32)
    for bit in range(8):
        r ^= np.where((b >> bit) & 1, a << bit, 0).astype(np.uint32)
    for bit in range(14, 7, -1):
        r ^= np.where((r >> bit) & 1, POLY << (bit - 8), 0).astype(np.uint32)
    return r.astype(np.uint8)


def power(e):
    """g^e with g = 2, by repeated multiplication."""
    r = 1
    for _ in range(e % 255):
        r = int(mul(r, 2))
    return r


def inv(a):
    """Inverse by exhaustive search."""
    a = int(a)
    for b in range(1, 256):
        if int(mul(a, b)) == 1:
            return b
    raise ZeroDivisionError(a)


def matvec_regions(A, X):
    """out[r][p] = XOR_c A[r][c] * X[c][p], straight from the definition."""
    A = np.asarray(A, dtype=np.uint8)
    X = np.asarray(X, dtype=np.uint8)
    out = np.zeros((A.shape[0], X.shape[1]), np.uint8)
    for r in range(A.shape[0]):
        for c in range(A.shape[1]):
            out[r] ^= mul(int(A[r, c]), X[c])
    return out

"""Pins of the oracle's GF(2^8) against an independent textbook multiply."""
import numpy as np

import gfref
import oracle as O


def test_mul_exhaustive_matches_shift_and_reduce():
    a, b = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    want = gfref.mul(a, b)
    got = np.array([[O.mul(i, j) for j in range(256)] for i in range(256)], np.uint8)
    assert np.array_equal(got, want)


def test_generator_is_primitive_and_poly_is_0x11d():
    seen = set()
    for e in range(255):
        seen.add(O.gpow(e))
    assert len(seen) == 255 and 0 not in seen
    assert O.gpow(255) == 1
    # x^8 = x^4 + x^3 + x^2 + 1 modulo the field polynomial
    assert O.gpow(8) == 0x1D == gfref.power(8)


def test_inverse_and_division():
    for a in range(1, 256):
        ia = O.inv(a)
        assert int(gfref.mul(a, ia)) == 1
        assert ia == gfref.inv(a)


def test_matrix_inverse_and_rank():
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 17):
        while True:
            A = rng.integers(0, 256, (n, n), dtype=np.uint8)
            Ai = O.invert(A)
            if Ai is not None:
                break
        eye = np.eye(n, dtype=np.uint8)
        # product with the independent multiply
        prod = np.zeros((n, n), np.uint8)
        for i in range(n):
            for j in range(n):
                prod[i, j] = np.bitwise_xor.reduce(gfref.mul(A[i], Ai[:, j]))
        assert np.array_equal(prod, eye)
        assert O.rank(A) == n
    S = np.array([[1, 2], [2, 4]], np.uint8)  # second row = 2 * first
    assert O.invert(S) is None and O.rank(S) == 1


def test_apply_matches_definition():
    rng = np.random.default_rng(2)
    A = rng.integers(0, 256, (5, 7), dtype=np.uint8)
    A[1, 3] = 0
    A[2, :] = 0
    X = rng.integers(0, 256, (7, 97), dtype=np.uint8)
    assert np.array_equal(O.apply(A, X), gfref.matvec_regions(A, X))
    assert np.array_equal(O.apply(A, X, nthreads=3), gfref.matvec_regions(A, X))

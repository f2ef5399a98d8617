"""Pins of the GF(2^16) oracle (Section 3.3, validity range of the sparse
PM-MSR construction over GF(2^16): k up to 64).

What pins it, other than itself:
* the field against carry-less multiplication with reduction written here
  (a different method from the oracle's exponent/logarithm tables), the
  polynomial's value of x^16, and the order of g;
* the paper's stated validity range: every k in 2..64 at n = d + 1 (the n
  subsets it checks), over GF(2^16) -- where GF(2^8) stops at 39;
* the linearized generator against the product-matrix encoding C = Psi M
  computed symbol by symbol, the systematic form's identity block, and the
  MDS and repair properties by brute force over every node set of small
  codes; a dropped term, a wrong index or a transposed operand in any step
  breaks one of these;
* the specific PM-MSR decoder (Section 4.1's comparison decoder) recovering
  the object from every k-subset, in both forms.
"""
import numpy as np
import pytest

import oracle as O
from oracle import gf16 as F

POLY = 0x1100B


def clmul(a, b):
    """a * b in GF(2^16) by shift-and-add with reduction modulo POLY."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a & 0x10000:
            a ^= POLY
    return r


def test_field_against_carryless_multiplication():
    rng = np.random.default_rng(16)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, 65536, (3000, 2))]
    pairs += [(0, 5), (1, 0xFFFF), (0x8000, 2), (0xFFFF, 0xFFFF), (0x100B, 0x100B)]
    for a, b in pairs:
        assert F.mul(a, b) == clmul(a, b), (a, b)


def test_generator_and_inverses():
    assert F.gpow(16) == POLY & 0xFFFF               # x^16 = x^12 + x^3 + x + 1
    assert F.gpow(65535) == 1
    for p in (3, 5, 17, 257):                         # 65535 = 3 * 5 * 17 * 257
        assert F.gpow(65535 // p) != 1
    rng = np.random.default_rng(17)
    for a in [1, 2, 3, 0xFFFF] + [int(v) for v in rng.integers(1, 65536, 2000)]:
        assert clmul(a, F.inv(a)) == 1


def test_sparse_construction_valid_for_k_2_to_64_in_gf16():
    """Section 3.3: valid for k in {2..64} in GF(2^16), checking the n = d + 1
    possible d x d submatrices of Psi and that Lambda's entries differ."""
    for k in range(2, 65):
        psi, lam = F.msr_sparse_printed(k, 2 * k - 1)
        assert psi is not None, k
        assert F.msr_valid(psi, lam), k


def test_gf8_stops_where_gf16_goes_on():
    """The same construction at k = 40 fails over GF(2^8) and holds over
    GF(2^16) (the reason the paper moves to the larger field)."""
    psi8, lam8 = O.msr_sparse_printed(40, 79)
    assert psi8 is None or not O.msr_valid(psi8, lam8)
    psi16, lam16 = F.msr_sparse_printed(40, 79)
    assert F.msr_valid(psi16, lam16)


@pytest.mark.parametrize("k", [3, 4, 8])
def test_structure_of_psi(k):
    """Phi: identity on the first alpha rows, then Cauchy entries whose
    product with (g^(i + alpha) + g^(j - 1)) is 1 (1-based); Lambda Phi in
    the right half."""
    n = 2 * k - 1
    a = k - 1
    psi, lam = F.msr_sparse_printed(k, n)
    assert np.array_equal(psi[:a, :a], np.eye(a, dtype=np.uint16))
    for i1 in range(a + 1, n + 1):
        for j1 in range(1, a + 1):
            assert clmul(int(psi[i1 - 1, j1 - 1]), F.gpow(i1 + a) ^ F.gpow(j1 - 1)) == 1
        # Lambda_i (g^(i+alpha) + g^alpha) = g^(i+alpha) + 1
        assert clmul(int(lam[i1 - 1]), F.gpow(i1 + a) ^ F.gpow(a)) == F.gpow(i1 + a) ^ 1
        for j in range(a):
            assert psi[i1 - 1, a + j] == clmul(int(lam[i1 - 1]), int(psi[i1 - 1, j]))


@pytest.mark.parametrize("k,n", [(3, 5), (3, 6), (4, 8), (8, 16)])
def test_n_2k_reading_keeps_every_helper_set_invertible(k, n):
    psi, lam = F.msr_sparse(k, n)
    assert psi is not None and F.msr_valid(psi, lam)


@pytest.mark.parametrize("k,n", [(3, 5), (4, 8), (5, 9)])
def test_linearized_generator_is_the_product_matrix_encoding(k, n):
    c = F.Code(k, n, systematic_form=False)
    rng = np.random.default_rng(k * 100 + n)
    X = rng.integers(0, 65536, (c.B, 37), dtype=np.uint16)
    assert np.array_equal(F.apply(c.G, X), F.specific_encode(c.psi, c.L, c.alpha, X))
    # G has at most d nonzeros per row, and the index matrix covers every symbol once per triangle
    assert ((c.G != 0).sum(axis=1) <= c.d).all()


@pytest.mark.parametrize("k,n", [(3, 5), (4, 8)])
def test_systematic_form(k, n):
    c = F.Code(k, n)
    assert np.array_equal(c.Gsys[:c.B], np.eye(c.B, dtype=np.uint16))
    # the systematic code is the linear code of G: G' Z stored = G (G~^-1 Z)
    rng = np.random.default_rng(3)
    X = rng.integers(0, 65536, (c.B, 21), dtype=np.uint16)
    Z = F.apply(F.invert(c.G[:c.B]), X)
    assert np.array_equal(F.apply(c.Gsys, X), F.apply(c.G, Z))


@pytest.mark.parametrize("systematic", [True, False])
def test_every_k_subset_decodes_and_every_helper_set_repairs(systematic):
    k, n = 3, 6
    c = F.Code(k, n, systematic_form=systematic)
    rng = np.random.default_rng(11)
    X = rng.integers(0, 65536, (c.B, 29), dtype=np.uint16)
    out = c.encode(X)
    nodes = {i: c.node_blocks(i, X, out) for i in range(n)}
    for K in O.subsets(n, k):
        Y = np.concatenate([nodes[i] for i in K])
        assert np.array_equal(c.decode(list(K), Y), X), K
    for f in range(n):
        others = [i for i in range(n) if i != f]
        for H in O.subsets(len(others), c.d):
            Hn = [others[i] for i in H]
            assert np.array_equal(c.repair(f, Hn, nodes), nodes[f]), (f, Hn)


def test_k40_code_repairs():
    """A code beyond GF(2^8)'s range (k = 40, n = 79, B = 1560), not
    systematic: node 5 repaired from the other 78 nodes."""
    c = F.Code(40, 79, systematic_form=False, check=False)
    rng = np.random.default_rng(40)
    X = rng.integers(0, 65536, (c.B, 4), dtype=np.uint16)
    out = c.encode(X)
    f = 5
    H = [i for i in range(79) if i != f]
    assert len(H) == c.d
    nodes = {i: c.node_blocks(i, X, out) for i in H + [f]}
    assert np.array_equal(c.repair(f, H, nodes), nodes[f])


@pytest.mark.parametrize("k,n,systematic", [(3, 6, True), (3, 6, False), (4, 8, True), (4, 7, False)])
def test_specific_decode_recovers_every_k_subset(k, n, systematic):
    c = F.Code(k, n, systematic_form=systematic)
    rng = np.random.default_rng(k * 10 + n)
    X = rng.integers(0, 65536, (c.B, 13), dtype=np.uint16)
    out = c.encode(X)
    nodes = {i: c.node_blocks(i, X, out) for i in range(n)}
    for K in O.subsets(n, k):
        Y = np.concatenate([nodes[i] for i in K])
        assert np.array_equal(c.decode_specific(list(K), Y), X), K


def test_specific_decode_k16_node_set():
    """k = 16 (B = 240), systematic: one node set with every kind of node,
    against the linearized decode of the same blocks."""
    c = F.Code(16, 32)
    rng = np.random.default_rng(16)
    X = rng.integers(0, 65536, (c.B, 5), dtype=np.uint16)
    out = c.encode(X)
    K = [0, 3, 9, 14, 15, 16, 17, 20, 22, 24, 25, 26, 28, 29, 30, 31]
    Y = np.concatenate([c.node_blocks(i, X, out) for i in K])
    got = c.decode_specific(K, Y)
    assert np.array_equal(got, X)
    assert np.array_equal(got, c.decode(K, Y))

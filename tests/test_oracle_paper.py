"""Pins of the oracle's constructions against what the paper prints and
against identities the paper states (Sections 3.1-3.3, Table 1)."""
import json
import os

import numpy as np
import pytest

import gfref
import oracle as O
from conftest import GOLDEN


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _pct_zero(A):
    return 100.0 * np.count_nonzero(A == 0) / A.size


def test_table1_sparsity():
    """Table 1: % of zeros of G (non-systematic) and G'' (systematic) at
    n = 2k-1, d = 2k-2.  The paper prints whole numbers, so agree to 0.5."""
    t = _load("table1_sparsity.json")["rows"]
    for k in (4, 8, 16):
        n, d = 2 * k - 1, 2 * k - 2
        van = O.Code(O.MSR, k, d, n, O.VANILLA, systematic_form=False, check=False)
        van_s = O.Code(O.MSR, k, d, n, O.VANILLA, systematic_form=True, check=False)
        spa = O.Code(O.MSR, k, d, n, O.SPARSE, systematic_form=False)
        spa_s = O.Code(O.MSR, k, d, n, O.SPARSE, systematic_form=True)
        got = {"vanilla_nonsystematic": _pct_zero(van.G),
               "sparse_nonsystematic": _pct_zero(spa.G),
               "vanilla_systematic": _pct_zero(van_s.enc),
               "sparse_systematic": _pct_zero(spa_s.enc)}
        for key, val in got.items():
            assert abs(val - t[key][str(k)]) <= 0.5 + 1e-9, (key, k, val)


def test_sparse_validity_range():
    """Section 3.3, validity range of the sparse construction over GF(2^8):
    k = 2..39 pass at n = d + 1, and k = 40, past that range, fails."""
    g = _load("validity_range.json")
    for k in range(g["first_valid_k"], g["last_valid_k"] + 2):
        psi, lam = O.msr_sparse_printed(k, 2 * k - 1)
        ok = psi is not None and O.msr_valid(psi, lam)
        assert ok == (k <= g["last_valid_k"]), k


def test_index_matrix_example_k3():
    g = _load("index_matrix_k3.json")
    L = O.index_msr(g["k"])
    assert np.array_equal(L.T + 1, np.array(g["L_transposed_1based"]))


def test_index_matrices_cover_message_once_per_column():
    """Section 3.1: no row nor column of L repeats a value, and every message
    symbol appears (twice off the diagonal of a symmetric block)."""
    for k in (2, 3, 5, 8):
        L = O.index_msr(k)
        a = k - 1
        assert sorted(set(L.ravel())) == list(range(k * a))
        for j in range(a):
            assert len(set(L[:, j])) == L.shape[0]
        for r in range(L.shape[0]):
            assert len(set(L[r])) == a
    for k, d in ((3, 4), (4, 6), (8, 14)):
        L = O.index_mbr(k, d)
        B = k * d - k * (k - 1) // 2
        vals = L[L >= 0]
        assert sorted(set(vals)) == list(range(B))
        assert np.array_equal(L, L.T)
        for j in range(d):
            col = L[:, j][L[:, j] >= 0]
            assert len(set(col)) == len(col)


def test_vanilla_example_n5_k3():
    g = _load("example_vanilla_n5_k3.json")
    psi, lam = O.msr_vanilla(g["k"], g["n"])
    want_psi = np.array([[gfref.power(e) for e in row] for row in g["Psi_exp"]], np.uint8)
    want_phi = np.array([[gfref.power(e) for e in row] for row in g["Phi_exp"]], np.uint8)
    want_lam = np.array([gfref.power(e) for e in g["Lambda_exp"]], np.uint8)
    assert np.array_equal(psi, want_psi)
    assert np.array_equal(psi[:, :2], want_phi)
    assert np.array_equal(lam, want_lam)


def _expr(s, a):
    return int(eval(s, {"__builtins__": {}}, {"a": a}))


def test_sparse_example_n5_k3():
    g = _load("example_sparse_n5_k3.json")
    a = g["k"] - 1
    psi, lam = O.msr_sparse_printed(g["k"], g["n"])
    for i, row in enumerate(g["Phi"]):
        for j, ent in enumerate(row):
            if ent == "one":
                want = 1
            elif ent == "zero":
                want = 0
            else:
                p, q = (_expr(e, a) for e in ent)
                want = gfref.inv(gfref.power(p) ^ gfref.power(q))
            assert psi[i, j] == want, (i, j)
    for i, (p, q, r, s) in enumerate(g["Lambda"]):
        num = gfref.power(_expr(p, a)) ^ gfref.power(_expr(q, a))
        den = gfref.power(_expr(r, a)) ^ gfref.power(_expr(s, a))
        want = int(gfref.mul(num, gfref.inv(den)))
        assert lam[i] == want, i
        # Psi = [Phi, Lambda Phi]
        assert np.array_equal(psi[i, a:], gfref.mul(want, psi[i, :a]))


CODES = [
    (O.MSR, 3, 4, 5, O.VANILLA), (O.MSR, 3, 4, 6, O.SPARSE), (O.MSR, 4, 6, 8, O.SPARSE),
    (O.MSR, 5, 8, 9, O.SPARSE), (O.MSR, 4, 6, 9, O.VANILLA), (O.MBR, 3, 4, 6, None),
    (O.MBR, 4, 6, 8, None), (O.MBR, 5, 5, 7, None),
]


@pytest.mark.parametrize("kind,k,d,n,cons", CODES)
def test_linearization_identity(kind, k, d, n, cons):
    """Section 3.1: C = Psi M equals Y = G X block for block."""
    c = O.Code(kind, k, d, n, cons if cons is not None else O.SPARSE, systematic_form=False)
    X = np.random.default_rng(k * 100 + n).integers(0, 256, (c.B, 33), dtype=np.uint8)
    C = O.specific_encode(c.psi, c.L, c.alpha, X)
    Y = O.apply(c.G, X)
    assert np.array_equal(C, Y)
    # and with the independent multiply
    assert np.array_equal(Y, gfref.matvec_regions(c.G, X))


@pytest.mark.parametrize("kind,k,d,n,cons", [c for c in CODES if c[0] == O.MSR])
def test_systematic_identity(kind, k, d, n, cons):
    """Section 3.2: G' = G inverse(G~) = [I; G'']."""
    c = O.Code(kind, k, d, n, cons, systematic_form=True)
    assert np.array_equal(c.Gsys[:c.B], np.eye(c.B, dtype=np.uint8))
    # G' G~ = G, checked with the independent multiply
    Gt = c.G[:c.B]
    back = np.zeros_like(c.G)
    for r in range(c.G.shape[0]):
        for col in range(c.B):
            back[r, col] = np.bitwise_xor.reduce(gfref.mul(c.Gsys[r], Gt[:, col]))
    assert np.array_equal(back, c.G)


def test_mbr_systematic_rows_are_uncoded():
    """Section 3.2: PM-MBR is systematic through its Psi; the first k nodes
    hold message symbols uncoded, every symbol at least once."""
    for k, d, n in ((3, 4, 6), (8, 14, 16)):
        c = O.Code(O.MBR, k, d, n)
        assert np.array_equal(c.psi[:k], np.hstack([np.eye(k, dtype=np.uint8),
                                                    np.zeros((k, d - k), np.uint8)]))
        seen = set()
        for t in range(k * d):
            nz = np.nonzero(c.G[t])[0]
            assert len(nz) == 1 and c.G[t, nz[0]] == 1
            seen.add(int(nz[0]))
        assert seen == set(range(c.B))


def test_systematic_generator_independent_of_index_order():
    """Reading of Section 3.1 for alpha >= 3: the order in which message
    symbols are numbered in L does not change G' (G P has the same G')."""
    k = 4
    c = O.Code(O.MSR, k, 6, 8, O.SPARSE)
    perm = np.random.default_rng(5).permutation(c.B)
    L2 = perm[c.L]
    G2 = O.linearize(c.psi, L2, c.alpha, c.B)
    G2s = O.systematic(G2, c.B)
    # renumbering permutes G's columns; G' must be unchanged
    assert np.array_equal(G2s, c.Gsys)


@pytest.mark.parametrize("k", [4, 8, 16])
def test_sparsity_closed_forms(k):
    """Closed forms behind Table 1: vanilla G has 2/k nonzero; sparse G has
    2 alpha^2 (n - alpha + 1) nonzeros; every row of sparse G'' has 2 alpha."""
    a = k - 1
    for n in (2 * k - 1, 2 * k):
        van = O.Code(O.MSR, k, 2 * k - 2, n, O.VANILLA, systematic_form=False, check=False)
        assert np.count_nonzero(van.G) * k == 2 * van.G.size
        spa = O.Code(O.MSR, k, 2 * k - 2, n, O.SPARSE, systematic_form=False)
        assert np.count_nonzero(spa.G) == 2 * a * a * (n - a + 1)
        sps = O.Code(O.MSR, k, 2 * k - 2, n, O.SPARSE, systematic_form=True)
        assert set(np.count_nonzero(sps.enc, axis=1)) == {2 * a}


def test_sparse_repair_rows_read_one_block():
    """Section 3.3, repair paragraph: the repair vector phi_f of the sparse
    code is a unit vector for the first alpha nodes (helpers read one block)
    and dense otherwise."""
    k = 8
    c = O.Code(O.MSR, k, 14, 16, O.SPARSE)
    for f in range(c.n):
        nz = np.count_nonzero(c.helper_row(f))
        assert nz == (1 if f < c.alpha else c.alpha)

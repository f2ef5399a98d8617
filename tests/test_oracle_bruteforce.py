"""Brute-force pins of the oracle on small codes: the properties the paper
requires of a regenerating code (Section 2): any k nodes decode the object,
and a lost node is rebuilt exactly from any d helpers, one block each."""
from itertools import combinations

import numpy as np
import pytest

import oracle as O
from paper_1412_3022_amd import synth


def _encode_all(c, s=64, seed=11):
    X = synth.random_bytes(seed + c.k * 1000 + c.n, c.B * s).reshape(c.B, s)
    out = c.encode(X)
    nodes = {i: c.node_blocks(i, X, out) for i in range(c.n)}
    return X, nodes


SMALL = [
    ("msr-vanilla-cfg1", dict(kind=O.MSR, k=3, d=4, n=6, construction=O.VANILLA, x=np.arange(1, 7))),
    ("msr-vanilla-3-4-5", dict(kind=O.MSR, k=3, d=4, n=5, construction=O.VANILLA)),
    ("msr-sparse-3-4-6", dict(kind=O.MSR, k=3, d=4, n=6, construction=O.SPARSE)),
    ("msr-sparse-4-6-8", dict(kind=O.MSR, k=4, d=6, n=8, construction=O.SPARSE)),
    ("msr-sparse-4-6-7", dict(kind=O.MSR, k=4, d=6, n=7, construction=O.SPARSE)),
    ("msr-sparse-nonsys-3-4-6", dict(kind=O.MSR, k=3, d=4, n=6, construction=O.SPARSE,
                                     systematic_form=False)),
    ("mbr-3-4-6", dict(kind=O.MBR, k=3, d=4, n=6)),
    ("mbr-4-6-8", dict(kind=O.MBR, k=4, d=6, n=8)),
    ("rs-6-3", dict(kind=O.RS, k=3, d=3, n=6)),
]


@pytest.mark.parametrize("name,kw", SMALL, ids=[s[0] for s in SMALL])
def test_every_k_subset_decodes(name, kw):
    c = O.Code(**kw)
    X, nodes = _encode_all(c)
    count = 0
    for K in combinations(range(c.n), c.k):
        Y = np.concatenate([nodes[i] for i in K])
        assert np.array_equal(c.decode(K, Y), X), K
        count += 1
    assert count > 0


@pytest.mark.parametrize("name,kw", SMALL, ids=[s[0] for s in SMALL])
def test_every_node_repairs_from_every_helper_set(name, kw):
    c = O.Code(**kw)
    X, nodes = _encode_all(c)
    pairs = 0
    for f in range(c.n):
        others = [i for i in range(c.n) if i != f]
        for H in combinations(others, c.d):
            rebuilt = c.repair(f, H, nodes)
            assert np.array_equal(rebuilt, nodes[f]), (f, H)
            pairs += 1
    assert pairs == c.n * len(list(combinations(range(c.n - 1), c.d)))


def test_systematic_nodes_hold_the_object():
    c = O.Code(O.MSR, 4, 6, 8, O.SPARSE)
    X, nodes = _encode_all(c)
    for i in range(c.k):
        assert np.array_equal(nodes[i], X[i * c.alpha:(i + 1) * c.alpha])


def test_lambda_distinct_for_config_codes():
    for k in (3, 4, 8, 16):
        c = O.Code(O.MSR, k, 2 * k - 2, 2 * k, O.SPARSE)
        assert len(set(c.lam.tolist())) == c.n


def test_adjusted_last_lambda_values():
    """Regression pin of the project's reading for n = 2k (the adjusted last
    node): the last Lambda is g^t for the smallest t that keeps Lambda
    distinct and every d-subset of Psi containing the last node invertible.
    That gives 0x01 (t = 0) for k = 3, 4, 8 and 0x02 (t = 1) for k = 16;
    the first 2k - 1 values are the printed construction's."""
    for k, want in ((3, 0x01), (4, 0x01), (8, 0x01), (16, 0x02)):
        psi, lam = O.msr_sparse(k, 2 * k)
        _, lam_p = O.msr_sparse_printed(k, 2 * k)
        assert int(lam[-1]) == want, (k, hex(int(lam[-1])))
        assert np.array_equal(lam[:-1], lam_p[:-1]), k
        t = 0
        while O.gpow(t) != want:
            t += 1
        # every smaller exponent collides with a printed Lambda or leaves a
        # singular helper set
        for u in range(t):
            cand = O.gpow(u)
            assert cand in set(int(v) for v in lam[:-1]) or not _last_lambda_valid(k, psi, cand), (k, u)


def _last_lambda_valid(k, psi, lam_last):
    """Whether Psi with its last row rebuilt for Lambda = lam_last keeps every
    d-subset that holds the last node invertible."""
    alpha, n, d = k - 1, 2 * k, 2 * k - 2
    p = psi.copy()
    phi = p[-1, :alpha]
    p[-1, alpha:] = np.array([O.mul(lam_last, int(v)) for v in phi], np.uint8)
    for H in combinations(range(n - 1), d - 1):
        if O.invert(p[list(H) + [n - 1]]) is None:
            return False
    return True


def test_printed_sparse_at_n_equal_2k_has_singular_helper_sets():
    """Reading for n = 2k (the paper checks only n = d + 1): the printed
    construction has helper sets whose Psi_H is singular; the adjusted last
    Lambda removes every one of them."""
    for k in (3, 4):
        n, d = 2 * k, 2 * k - 2
        psi, lam = O.msr_sparse_printed(k, n)
        bad = 0
        for H in combinations(range(n), d):
            if O.invert(psi[list(H)]) is None:
                bad += 1
        assert bad > 0
        psi2, lam2 = O.msr_sparse(k, n)
        assert np.array_equal(psi2[:-1], psi[:-1])
        assert O.all_dsubsets_invertible(psi2, d)
        assert len(set(lam2.tolist())) == n


def test_vanilla_lambda_collision_is_rejected():
    """Vanilla Lambda_i = g^(i alpha) repeats when gcd(alpha, 255) > 1: k = 16
    (alpha = 15) gives only 17 distinct values, so n = 32 is not a valid code."""
    psi, lam = O.msr_vanilla(16, 32)
    assert len(set(lam.tolist())) == 17
    assert not O.msr_valid(psi, lam)
    with pytest.raises(ValueError):
        O.Code(O.MSR, 16, 30, 32, O.VANILLA)


def test_rs_16_8_is_mds():
    c = O.Code(O.RS, 8, 8, 16)
    for K in combinations(range(16), 8):
        assert O.invert(c.G[list(K)]) is not None


@pytest.mark.parametrize("k", [8, 16])
def test_config_codes_repair_everywhere(k):
    """Every (f, H) pair of the sparse n = 2k codes of the configurations."""
    c = O.Code(O.MSR, k, 2 * k - 2, 2 * k, O.SPARSE)
    X, nodes = _encode_all(c, s=16)
    for f in range(c.n):
        others = [i for i in range(c.n) if i != f]
        for H in combinations(others, c.d):
            assert np.array_equal(c.repair(f, H, nodes), nodes[f])


def test_config_codes_decode_sampled():
    """Sampled k-subsets of the k = 8 codes (the k = 3, 4 codes are exhaustive)."""
    st = synth.Stream(77)
    for c in (O.Code(O.MSR, 8, 14, 16, O.SPARSE), O.Code(O.MBR, 8, 14, 16),
              O.Code(O.MSR, 8, 14, 16, O.VANILLA, systematic_form=False)):
        X, nodes = _encode_all(c, s=16)
        for _ in range(25):
            K = st.subset(c.n, c.k)
            Y = np.concatenate([nodes[i] for i in K])
            assert np.array_equal(c.decode(K, Y), X), K


def test_mbr_repair_k8():
    c = O.Code(O.MBR, 8, 14, 16)
    X, nodes = _encode_all(c, s=16)
    for f in (0, 7, 8, 15):
        others = [i for i in range(c.n) if i != f]
        for H in combinations(others, c.d):
            assert np.array_equal(c.repair(f, H, nodes), nodes[f])

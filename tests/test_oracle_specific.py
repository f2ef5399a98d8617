"""Pins of the oracle's specific PM-MSR and PM-MBR decoders (the seminal
paper's data-collector algorithms, Section 2): decoding from every k-subset
returns the encoded object, for both MSR constructions, systematic and not,
and for MBR from the product-matrix encoding C = Psi M itself; a repeated node
(equal lambdas, a singular Phi_DC) is refused."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("k,d,n", [(3, 4, 6), (4, 6, 8), (3, 4, 5)])
@pytest.mark.parametrize("construction", [O.SPARSE, O.VANILLA], ids=["sparse", "vanilla"])
@pytest.mark.parametrize("systematic_form", [True, False], ids=["sys", "nonsys"])
def test_every_k_subset_decodes_to_the_object(k, d, n, construction, systematic_form):
    if construction == O.SPARSE and n < 2 * k - 1:
        pytest.skip("the sparse construction needs n >= 2k - 1")
    o = O.Code(O.MSR, k, d, n, construction, systematic_form)
    rng = np.random.default_rng(k * 100 + n)
    X = rng.integers(0, 256, (o.B, 53), dtype=np.uint8)
    P = o.encode(X)
    nodes = {i: o.node_blocks(i, X, P) for i in range(n)}
    for K in O.subsets(n, k):
        Y = np.concatenate([nodes[i] for i in K])
        got = o.decode_specific(list(K), Y)
        assert got is not None and np.array_equal(got, X), K


def test_k8_random_subsets_and_all_parity():
    o = O.Code(O.MSR, 8, 14, 16, O.SPARSE)
    rng = np.random.default_rng(8)
    X = rng.integers(0, 256, (o.B, 40), dtype=np.uint8)
    P = o.encode(X, nthreads=4)
    nodes = {i: o.node_blocks(i, X, P) for i in range(o.n)}
    subsets = [list(range(8, 16)), list(range(8))] + [sorted(rng.choice(16, 8, replace=False)) for _ in range(6)]
    for K in subsets:
        Y = np.concatenate([nodes[i] for i in K])
        assert np.array_equal(o.decode_specific(K, Y), X), K
        # and the same bytes as the linearized decode
        assert np.array_equal(o.decode(K, Y), X)


def test_order_of_connected_nodes_does_not_matter():
    o = O.Code(O.MSR, 4, 6, 8, O.SPARSE)
    rng = np.random.default_rng(3)
    X = rng.integers(0, 256, (o.B, 17), dtype=np.uint8)
    P = o.encode(X)
    nodes = {i: o.node_blocks(i, X, P) for i in range(o.n)}
    for K in ([7, 2, 5, 0], [5, 7, 0, 2], [1, 3, 6, 4]):
        Y = np.concatenate([nodes[i] for i in K])
        assert np.array_equal(o.decode_specific(K, Y), X)


def test_repeated_node_is_refused():
    o = O.Code(O.MSR, 3, 4, 6, O.SPARSE)
    Y = np.zeros((3 * o.alpha, 8), np.uint8)
    assert o.decode_specific([0, 1, 1], Y) is None


# ---- PM-MBR -----------------------------------------------------------------

@pytest.mark.parametrize("k,d,n", [(2, 3, 4), (3, 4, 6), (4, 6, 8), (4, 4, 6), (3, 5, 7)])
def test_mbr_every_k_subset_inverts_the_product_matrix_encoding(k, d, n):
    # C = Psi M byte by byte (Section 2), without the linearized generator;
    # d = k leaves T empty
    o = O.Code(O.MBR, k, d, n)
    rng = np.random.default_rng(1000 + k * 10 + d)
    X = rng.integers(0, 256, (o.B, 37), dtype=np.uint8)
    C = O.specific_encode(o.psi, o.L, o.alpha, X)
    # systematic through Psi: the first k nodes hold message symbols only
    P = o.encode(X)
    for i in range(n):
        assert np.array_equal(C[i * d:(i + 1) * d], o.node_blocks(i, X, P)), i
    for K in O.subsets(n, k):
        Y = np.concatenate([C[i * d:(i + 1) * d] for i in K])
        got = o.decode_specific(list(K), Y)
        assert got is not None and np.array_equal(got, X), K


def test_mbr_k8_random_subsets_match_the_linearized_decode():
    o = O.Code(O.MBR, 8, 14, 16)
    rng = np.random.default_rng(81)
    X = rng.integers(0, 256, (o.B, 29), dtype=np.uint8)
    P = o.encode(X, nthreads=4)
    nodes = {i: o.node_blocks(i, X, P) for i in range(o.n)}
    subsets = [list(range(8, 16)), list(range(8)), [15, 3, 9, 0, 12, 6, 10, 1]] + \
        [sorted(rng.choice(16, 8, replace=False)) for _ in range(5)]
    for K in subsets:
        Y = np.concatenate([nodes[i] for i in K])
        assert np.array_equal(o.decode_specific(K, Y), X), K
        assert np.array_equal(o.decode(K, Y), X), K


def test_mbr_repeated_node_is_refused():
    o = O.Code(O.MBR, 3, 4, 6)
    Y = np.zeros((3 * o.alpha, 8), np.uint8)
    assert o.decode_specific([0, 4, 4], Y) is None

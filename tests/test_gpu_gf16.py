"""GPU parity of the GF(2^16) codes (Section 3.3: the sparse PM-MSR code over
GF(2^16), valid up to k = 64) through the C ABI, against the GF(2^16) oracle,
symbol for symbol: encode, repair (helper and newcomer), decode, at block
sizes from one symbol to several wave tiles with ragged tails, a code beyond
GF(2^8)'s range (k = 40), a 64 MiB object sampled, and blocks past 4 GiB."""
import numpy as np
import pytest
import torch

from gpu_util import device, out_regions, read, to_regions
from oracle import gf16 as F
from paper_1412_3022_amd import pm, synth

pytestmark = pytest.mark.gpu

SIZES = [2, 6, 2048 + 6, 3 * 2048 + 10, 65536 + 2]   # bytes per block (even)


def _data(rows, s, seed):
    return synth.random_bytes(seed, rows * s).reshape(rows, s).copy()


def _u16(a):
    return np.ascontiguousarray(a).view(np.uint16)


def _encode(c, X, s):
    Xd = to_regions(X)
    out = out_regions(c.enc_rows, s)
    c.encode(Xd, out, s)
    return read(out, s)


def _nodes(o, X, P):
    """Node contents (alpha x s bytes each) from the data and the encode output."""
    Xu, Pu = _u16(X), _u16(P)
    return {i: o.node_blocks(i, Xu, Pu).view(np.uint8) for i in range(o.n)}


CODES = [(4, 8, True), (8, 16, True), (8, 16, False), (8, 15, True)]


@pytest.mark.parametrize("k,n,sys_", CODES)
@pytest.mark.parametrize("s", SIZES)
def test_encode(k, n, sys_, s):
    print("gf16 encode", k, n, sys_, s, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_)
    X = _data(c.B, s, 1600 + k * 10 + s % 97)
    got = _encode(c, X, s)
    assert np.array_equal(_u16(got), o.encode(_u16(X)))


@pytest.mark.parametrize("k,n,sys_", [(4, 8, True), (8, 16, True), (8, 16, False)])
@pytest.mark.parametrize("s", [6, 2048 + 6, 3 * 2048 + 10])
def test_repair(k, n, sys_, s):
    print("gf16 repair", k, n, sys_, s, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_)
    X = _data(c.B, s, 1700 + k + s % 89)
    P = _u16(_encode(c, X, s)).view(np.uint8)
    nodes = _nodes(o, X, P)
    st = synth.Stream(1701 + k)
    for f in sorted({0, c.alpha - 1, c.alpha, n - 1, st.below(n)}):
        H = st.subset(n, c.d, exclude=[f])
        recv = out_regions(c.d, s)
        for j, h in enumerate(H):
            c.repair_helper(f, to_regions(nodes[h]), recv[j:j + 1], s)
        recv_h = read(recv, s)
        want_h = np.stack([F.apply(o.helper_row(f), _u16(nodes[h]))[0] for h in H]).view(np.uint8)
        assert np.array_equal(recv_h, want_h), (f, "helper")
        out = out_regions(c.alpha, s)
        c.repair_newcomer(f, H, to_regions(recv_h), out, s)
        assert np.array_equal(read(out, s), nodes[f]), (f, H)


@pytest.mark.parametrize("k,n,sys_", [(4, 8, True), (4, 8, False), (8, 16, True), (8, 16, False)])
@pytest.mark.parametrize("s", [2, 2048 + 6, 3 * 2048 + 10])
def test_decode(k, n, sys_, s):
    print("gf16 decode", k, n, sys_, s, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_)
    X = _data(c.B, s, 1800 + k + s % 83)
    P = _u16(_encode(c, X, s)).view(np.uint8)
    nodes = _nodes(o, X, P)
    st = synth.Stream(1801 + k)
    sets = [list(range(k)), list(range(n - k, n)), st.subset(n, k)]
    sets.append(list(reversed(st.subset(n, k))))   # node order as given, not sorted
    for K in sets:
        Y = np.concatenate([nodes[i] for i in K])
        out = out_regions(c.B, s)
        c.decode(K, to_regions(Y), out, s)
        assert np.array_equal(read(out, s), X), K


def test_prepare_stages_the_operation():
    c = pm.Code(k=4, d=6, n=8, w=16)
    assert c.prepare(pm.OP_ENCODE) is True           # the bit-sliced kernel, compiled and loaded
    assert c.prepare(pm.OP_DECODE, ids=[7, 5, 3, 1]) is True
    o = F.Code(4, 8)
    s = 4096
    X = _data(c.B, s, 1901)
    assert np.array_equal(_u16(_encode(c, X, s)), o.encode(_u16(X)))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("k,n,sys_", [(4, 8, True), (8, 16, True), (8, 16, False)])
def test_bitsliced_kernels_after_prepare(k, n, sys_):
    """Once prepared, encode, the newcomer and a decode from a half-systematic
    node set run the generated bit-sliced kernels (blocks of at least one
    4 KiB wave tile; a window tile and a byte tail of 1 to 15 symbols):
    every symbol against the oracle."""
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_)
    f = 1
    H = [h for h in range(n) if h != f][:c.d]
    K = list(range(k // 2)) + list(range(n - k // 2, n))
    assert c.prepare(pm.OP_ENCODE) is True
    assert c.prepare(pm.OP_NEWCOMER, failed=f, ids=H) is True
    assert c.prepare(pm.OP_DECODE, ids=K) is True
    for s in (4096, 4096 + 2, 4096 + 30, 3 * 4096 + 1000):
        print("gf16 bit-sliced", k, n, sys_, s, flush=True)
        X = _data(c.B, s, 1950 + k + s % 71)
        P = _encode(c, X, s)
        assert np.array_equal(_u16(P), o.encode(_u16(X))), s
        nodes = _nodes(o, X, P)
        recv = np.stack([F.apply(o.helper_row(f), _u16(nodes[h]))[0] for h in H]).view(np.uint8)
        out = out_regions(c.alpha, s)
        c.repair_newcomer(f, H, to_regions(recv), out, s)
        assert np.array_equal(read(out, s), nodes[f]), s
        Y = np.concatenate([nodes[i] for i in K])
        out = out_regions(c.B, s)
        c.decode(K, to_regions(Y), out, s)
        assert np.array_equal(read(out, s), X), s


@pytest.mark.timeout(300)
def test_split_bitsliced_kernels_after_prepare():
    """The k = 16 systematic encode (240 x 240) and the k = 8 decode from
    the 8 parity nodes (56 x 56 dense) are past one bit-sliced kernel's size:
    prepared, each runs as several generated kernels over consecutive row
    groups, side by side (2 parts each).  Every symbol against the
    oracle at a whole tile, a window tile with a byte tail, and several
    tiles."""
    c16, o16 = pm.Code(k=16, d=30, n=32, w=16), F.Code(16, 32)
    c8, o8 = pm.Code(k=8, d=14, n=16, w=16), F.Code(8, 16)
    K = list(range(8, 16))
    assert c16.prepare(pm.OP_ENCODE) is True
    assert c8.prepare(pm.OP_DECODE, ids=K) is True
    for s in (4096, 4096 + 30, 3 * 4096 + 1002):
        print("gf16 split kernels", s, flush=True)
        X = _data(c16.B, s, 1990 + s % 83)
        assert np.array_equal(_u16(_encode(c16, X, s)), o16.encode(_u16(X))), s
        X8 = _data(c8.B, s, 1991 + s % 79)
        nodes = _nodes(o8, X8, _encode(c8, X8, s))
        out = out_regions(c8.B, s)
        c8.decode(K, to_regions(np.concatenate([nodes[i] for i in K])), out, s)
        assert np.array_equal(read(out, s), X8), s


@pytest.mark.timeout(300)
@pytest.mark.parametrize("k,n,s,f", [(40, 79, 2048 + 14, 41), (64, 127, 1024 + 6, 100)])
def test_beyond_the_byte_field(k, n, s, f):
    """k = 40 (B = 1560; the construction fails over GF(2^8) from here) and
    k = 64 (B = 4032, the top of the paper's range), not systematic: encode
    every row at a ragged size, and repair one node from all the others."""
    print("gf16 beyond GF(2^8)", k, n, s, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=False, w=16)
    o = F.Code(k, n, systematic_form=False, check=False)
    X = _data(c.B, s, 1900 + k)
    P = _encode(c, X, s)
    assert np.array_equal(_u16(P), o.encode(_u16(X)))
    nodes = _nodes(o, X, P)
    H = [i for i in range(n) if i != f]
    recv = out_regions(c.d, s)
    for j, h in enumerate(H):
        c.repair_helper(f, to_regions(nodes[h]), recv[j:j + 1], s)
    out = out_regions(c.alpha, s)
    c.repair_newcomer(f, H, to_regions(read(recv, s)), out, s)
    assert np.array_equal(read(out, s), nodes[f])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("k", [8, 16])
def test_64mib_object_sampled(k):
    """Sparse systematic (8, 14, 16) and (16, 30, 32) over GF(2^16), a 64 MiB
    object (56 blocks of 1 198 400 bytes; 240 of 279 680), in the launches the
    benchmark times (one bit-sliced kernel; two side by side at k = 16):
    sampled symbol positions (the first, around each wave tile edge, the
    last) against the oracle."""
    print("gf16 64MiB", k, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=2 * k, w=16)
    assert c.prepare(pm.OP_ENCODE) is True   # the bit-sliced kernels, as the benchmark runs them
    o = F.Code(k, 2 * k)
    s = synth.block_bytes_for(64 << 20, c.B)
    assert s == {8: 1198400, 16: 279680}[k]
    X = synth.random_bytes_torch(0x16, c.B * s, device()).view(c.B, s)
    out = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=device())
    c.encode(X, out, s)
    torch.cuda.synchronize()
    st = synth.Stream(0x17)
    sym = sorted({0, 1, 1023, 1024, s // 2 - 1} | {st.below(s // 2) for _ in range(300)})
    idx = torch.tensor([2 * p for p in sym] + [2 * p + 1 for p in sym], dtype=torch.int64, device=device())
    xs = X.index_select(1, idx).cpu().numpy()
    got = out.index_select(1, idx).cpu().numpy()
    m = len(sym)
    Xs = (xs[:, :m].astype(np.uint16) | xs[:, m:].astype(np.uint16) << 8)
    want = o.encode(Xs)
    assert np.array_equal(got[:, :m], (want & 0xFF).astype(np.uint8))
    assert np.array_equal(got[:, m:], (want >> 8).astype(np.uint8))


@pytest.mark.timeout(300)
def test_blocks_larger_than_4_gib():
    """Sparse systematic (3, 4, 5) over GF(2^16) with blocks of 4 GiB + 4112
    bytes (6 blocks in, 4 out: 43 GB): symbols on both sides of byte 2^32."""
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 60 * 10**9:
        pytest.skip("needs about 45 GB of free device memory")
    print("gf16 blocks > 4 GiB", flush=True)
    c = pm.Code(k=3, d=4, n=5, w=16)
    o = F.Code(3, 5)
    s = (1 << 32) + 4112
    X = synth.random_bytes_torch(0x4616, c.B * s, device()).view(c.B, s)
    out = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=device())
    out.fill_(0x5A)
    c.encode(X, out, s)
    torch.cuda.synchronize()
    st = synth.Stream(0x4617)
    sym = sorted({0, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, s // 2 - 1} | {st.below(s // 2) for _ in range(100)})
    idx = torch.tensor([2 * p for p in sym] + [2 * p + 1 for p in sym], dtype=torch.int64, device=device())
    xs = X.index_select(1, idx).cpu().numpy()
    got = out.index_select(1, idx).cpu().numpy()
    m = len(sym)
    want = o.encode(xs[:, :m].astype(np.uint16) | xs[:, m:].astype(np.uint16) << 8)
    assert np.array_equal(got[:, :m], (want & 0xFF).astype(np.uint8))
    assert np.array_equal(got[:, m:], (want >> 8).astype(np.uint8))
    del X, out


def test_batches_and_the_server_refuse_gf16_codes():
    """Batched plans and the server take GF(2^8) codes only: a GF(2^16) code
    is refused with PM_EUNSUPPORTED before any work is queued."""
    c = pm.Code(k=4, d=6, n=8, w=16)
    s = 4096
    X = torch.zeros((c.B, s), dtype=torch.uint8, device=device())
    out = torch.zeros((c.enc_rows, s), dtype=torch.uint8, device=device())
    with pytest.raises(pm.PMError) as e:
        pm.Batch([dict(code=c, op="encode", inp=X, out=out, block_bytes=s)], graph=False)
    assert e.value.status == pm.PM_EUNSUPPORTED
    srv = pm.Server(1 << 30, streams=1, max_batch=4, queue_cap=16)
    try:
        with pytest.raises(pm.PMError) as e:
            srv.submit_encode(c, X, s)
        assert e.value.status == pm.PM_EUNSUPPORTED
    finally:
        srv.close()


@pytest.mark.parametrize("k,n,sys_", [(4, 8, True), (4, 8, False), (8, 16, True), (8, 16, False), (16, 32, True)])
@pytest.mark.parametrize("s", [2, 2048 + 6])
def test_specific_decode(k, n, sys_, s):
    """The specific PM-MSR decode over GF(2^16) (Section 4.1's decoder) in
    four or five passes through the workspace: the object back from node
    sets of every kind, against the oracle's specific decoder too."""
    print("gf16 specific decode", k, n, sys_, s, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_)
    X = _data(c.B, s, 2000 + k + s % 79)
    P = _encode(c, X, s)
    nodes = _nodes(o, X, P)
    st = synth.Stream(2001 + k)
    for K in [list(range(k)), list(range(n - k, n)), st.subset(n, k), list(reversed(st.subset(n, k)))]:
        Y = np.concatenate([nodes[i] for i in K])
        out = out_regions(c.B, s)
        c.decode_specific(K, to_regions(Y), out, s)
        got = read(out, s)
        assert np.array_equal(got, X), K
        assert np.array_equal(_u16(got), o.decode_specific(K, _u16(Y))), K


@pytest.mark.timeout(300)
@pytest.mark.parametrize("k,n,sys_", [(40, 79, True), (64, 127, False)])
def test_specific_decode_beyond_the_byte_field(k, n, sys_):
    """k = 40 (systematic, B = 1560) and k = 64 (B = 4032): encode on the
    GPU, then the specific decode (and at k = 40 the linearized one) from
    the last k nodes and from a mixed set gives the object back (round trip; each piece is checked against the
    oracle at smaller k, and the oracle's B x B inversion here would take
    minutes)."""
    print("gf16 specific decode", k, n, sys_, flush=True)
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    s = 1024 + 10
    X = _data(c.B, s, 2100 + k)
    Xd = to_regions(X)
    P = out_regions(c.enc_rows, s)
    c.encode(Xd, P, s)
    Ph = read(P, s)
    a = c.alpha

    def node(i):
        rows = []
        for t in range(i * a, (i + 1) * a):
            # systematic: blocks t < B are data, the others encode rows t - B;
            # otherwise every block t is encode row t
            rows.append(X[t] if sys_ and t < c.B else Ph[t - c.B if sys_ else t])
        return np.stack(rows)

    st = synth.Stream(2101 + k)
    for K in [list(range(n - k, n)), st.subset(n, k)]:
        Y = np.concatenate([node(i) for i in K])
        out = out_regions(c.B, s)
        c.decode_specific(K, to_regions(Y), out, s)
        assert np.array_equal(read(out, s), X), K
        if k == 40:   # the linearized decode too (its B x B inverse takes seconds on the host)
            out = out_regions(c.B, s)
            c.decode(K, to_regions(Y), out, s)
            assert np.array_equal(read(out, s), X), ("linearized", K)

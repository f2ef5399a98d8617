"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Small cases compare every byte; the configurations' full sizes compare
sampled byte positions that the oracle computes one by one.  Output rows are
pre-filled with a guard byte to catch writes past block_bytes."""
from itertools import combinations

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import device, out_regions, read, to_regions
from paper_1412_3022_amd import pm, synth

pytestmark = pytest.mark.gpu

VARIANTS = [(rg, vec) for rg in (4, 8, 16) for vec in (2, 4, 12, 14, 22, 24)] + [(8, 32)]


def _rand(seed, rows, s):
    return synth.random_bytes(seed, rows * s).reshape(rows, s)


def _oracle_for(kw):
    kind = {pm.PM_MSR: O.MSR, pm.PM_MBR: O.MBR, pm.PM_RS: O.RS}[kw.get("kind", pm.PM_MSR)]
    cons = O.VANILLA if kw.get("construction", pm.PM_SPARSE) == pm.PM_VANILLA else O.SPARSE
    x = np.array(kw["x"]) if kw.get("x") is not None else None
    return O.Code(kind, kw["k"], kw["d"], kw["n"], cons, kw.get("systematic", True), x=x)


# --------------------------------------------------------------- engine ---
@pytest.mark.parametrize("rg,vec", VARIANTS)
@pytest.mark.parametrize("s", [1, 15, 16, 17, 100, 1023, 4096, 4097, 12289, 65536 + 13])
def test_apply_random_matrix_every_variant(rg, vec, s):
    print("apply rg=%d vec=%d s=%d" % (rg, vec, s), flush=True)
    rng = np.random.default_rng(s * 31 + rg * 7 + vec)
    rows, cols = 11, 9
    A = rng.integers(0, 256, (rows, cols), dtype=np.uint8)
    A[2] = 0                       # zero row -> zero fill
    A[3] = 0
    A[3, 4] = 1                    # unit row -> copy
    A[5, ::2] = 0                  # partial sparsity
    A[:, 7] = 0                    # unused column
    X = _rand(1000 + s, cols, s)
    want = O.apply(A, X)
    pm.lib()
    pm.pm_set_variant(None, pm.OP_APPLY, rg, vec)
    try:
        xin = to_regions(X, extra=1, offset_rows=1)
        out = out_regions(rows, s, extra=2)
        pm.apply(A, xin, out, s)
        assert np.array_equal(read(out, s), want)
    finally:
        pm.pm_set_variant(None, pm.OP_APPLY, 0, 0)


@pytest.mark.parametrize("shape", [(1, 1), (1, 30), (56, 56), (17, 3), (240, 240), (112, 84)])
def test_apply_dense_shapes(shape):
    rows, cols = shape
    s = 3 * 4096 + 77
    print("apply dense %s s=%d" % (shape, s), flush=True)
    rng = np.random.default_rng(rows * 1000 + cols)
    A = rng.integers(1, 256, (rows, cols), dtype=np.uint8)
    X = _rand(rows + cols, cols, s)
    xin = to_regions(X)
    out = out_regions(rows, s)
    pm.apply(A, xin, out, s)
    assert np.array_equal(read(out, s), O.apply(A, X, nthreads=8))


@pytest.mark.parametrize("shape,dens", [((16, 8), 1.0), ((13, 9), 1.0), ((240, 240), 1.0), ((112, 84), 0.6),
                                        ((56, 56), 0.25), ((100, 37), 1.0)])
@pytest.mark.parametrize("s", [1, 100, 129, 4096, 12289 + 77])
def test_apply_on_the_matrix_cores(shape, dens, s):
    """The matrix-core kernel (variant 40) on dense and sparse matrices,
    padded shapes and every tail case of its 128-byte position blocks."""
    rows, cols = shape
    print("apply mfma %s dens=%.2f s=%d" % (shape, dens, s), flush=True)
    rng = np.random.default_rng(rows * 7919 + cols * 31 + s)
    A = rng.integers(1, 256, (rows, cols), dtype=np.uint8)
    A[rng.random((rows, cols)) >= dens] = 0
    X = _rand(rows + 3 * cols + s, cols, s)
    pm.lib()
    pm.pm_set_variant(None, pm.OP_APPLY, 8, 40)
    try:
        xin = to_regions(X, extra=1, offset_rows=1)
        out = out_regions(rows, s, extra=2)
        pm.apply(A, xin, out, s)
        assert np.array_equal(read(out, s), O.apply(A, X, nthreads=8))
    finally:
        pm.pm_set_variant(None, pm.OP_APPLY, 0, 0)


@pytest.mark.parametrize("shape", [(360, 360), (40, 512)])
@pytest.mark.parametrize("s", [129, 4096 + 77])
def test_matrix_cores_with_more_than_64_kib_of_lds(shape, s):
    """45 and 64 chunks of 8 input blocks: the work-group's operands take
    94 and 132 KiB of LDS (the dynamic limit raised past 64 KiB)."""
    rows, cols = shape
    print("apply mfma %s s=%d" % (shape, s), flush=True)
    rng = np.random.default_rng(rows + cols + s)
    A = rng.integers(1, 256, (rows, cols), dtype=np.uint8)
    X = _rand(rows * 3 + cols + s, cols, s)
    pm.lib()
    pm.pm_set_variant(None, pm.OP_APPLY, 8, 40)
    try:
        xin = to_regions(X, extra=1, offset_rows=1)
        out = out_regions(rows, s, extra=2)
        pm.apply(A, xin, out, s)
        assert np.array_equal(read(out, s), O.apply(A, X, nthreads=8))
    finally:
        pm.pm_set_variant(None, pm.OP_APPLY, 0, 0)


# ----------------------------------------------------------- small codes --
SMALL = [
    dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=list(range(1, 7))),
    dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=4, d=6, n=8, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=4, d=6, n=7, kind=pm.PM_MSR, construction=pm.PM_SPARSE, systematic=False),
    dict(k=3, d=4, n=6, kind=pm.PM_MBR),
    dict(k=4, d=5, n=7, kind=pm.PM_MBR),
    dict(k=3, d=3, n=6, kind=pm.PM_RS),
]


def _gpu_encode(c, X, s):
    xin = to_regions(X, extra=1)
    out = out_regions(c.enc_rows, s)
    c.encode(xin, out, s)
    return read(out, s)


def _nodes(c, X, P):
    nm = c.node_map()
    return {i: np.stack([X[v] if v < c.B else P[v - c.B] for v in nm[i * c.alpha:(i + 1) * c.alpha]])
            for i in range(c.n)}


@pytest.mark.parametrize("kw", SMALL, ids=lambda kw: "%d-%d-%d-%d-%d" % (
    kw["kind"], kw.get("construction", 1), kw["k"], kw["d"], kw["n"]))
@pytest.mark.parametrize("s", [64, 4099])
def test_small_code_roundtrips_on_gpu(kw, s):
    """Encode, every k-subset decode and every (f, H) repair on the GPU,
    checked against the oracle byte for byte."""
    print("small code %s s=%d" % (kw, s), flush=True)
    c = pm.Code(**kw)
    o = _oracle_for(kw)
    X = _rand(7 + s + kw["k"] * 13 + kw["n"], c.B, s)
    P = _gpu_encode(c, X, s)
    assert np.array_equal(P, o.encode(X))
    nodes = _nodes(c, X, P)
    for K in combinations(range(c.n), c.k):
        Y = np.concatenate([nodes[i] for i in K])
        xout = out_regions(c.B, s)
        c.decode(list(K), to_regions(Y), xout, s)
        assert np.array_equal(read(xout, s), X), K
    for f in range(c.n):
        others = [i for i in range(c.n) if i != f]
        hrow = o.helper_row(f)
        for H in combinations(others, c.d):
            recv = np.zeros((c.d, s), np.uint8)
            for j, h in enumerate(H):
                hb = out_regions(1, s)
                c.repair_helper(f, to_regions(nodes[h][:1 if c.kind == pm.PM_RS else c.alpha]), hb, s)
                recv[j] = read(hb, s)[0]
                assert np.array_equal(recv[j], O.apply(hrow, nodes[h])[0])
            rout = out_regions(1 if c.kind == pm.PM_RS else c.alpha, s)
            c.repair_newcomer(f, list(H), to_regions(recv), rout, s)
            assert np.array_equal(read(rout, s), nodes[f]), (f, H)


# ------------------------------------------------------- configurations ---
def _sample_positions(s, seed, count=2048):
    """Scattered positions plus whole 2 KiB wave tiles of the bit-sliced
    kernel: the first, a seeded one in the middle and the last full-width
    window [s16 - 2048, s16) (s16 = s rounded down to 16), so that one wrong
    tile anywhere in those cannot pass; and the last 64 bytes (the byte
    tail)."""
    st = synth.Stream(seed)
    pos = {0, 1, 2, s - 1, s - 2}
    pos |= set(range(max(0, s - 64), s))
    tile = 2048
    s16 = s // 16 * 16
    if s16 >= tile:
        mid = st.below(s16 // tile) * tile
        for t0 in (0, mid, s16 - tile):
            pos |= set(range(t0, t0 + tile))
    while len(pos) < min(s, count + 3 * tile):
        pos.add(st.below(s))
    return np.array(sorted(pos))


def _check_sampled(out_dev, A, X, s, seed):
    torch.cuda.synchronize()
    pos = _sample_positions(s, seed)
    got = out_dev[:, :s].cpu().numpy()[:, pos]
    want = O.apply(A, X[:, pos])
    assert np.array_equal(got, want)


def test_config1_msr_vanilla_k3_full():
    """MSR vanilla (3,4,6), x_i = i+1, 1 MiB object: encode all parity,
    repair node 0 from helpers 1..4, decode from nodes {3,4,5}; every byte."""
    print("config1", flush=True)
    S = 1 << 20
    c = pm.Code(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=list(range(1, 7)))
    o = O.Code(O.MSR, 3, 4, 6, O.VANILLA, True, x=np.arange(1, 7))
    X, s = synth.split_object(S, c.B, synth.CONFIG_SEED + 0)
    assert s == 174784
    P = _gpu_encode(c, X, s)
    assert np.array_equal(P, o.encode(X, nthreads=8))
    nodes = _nodes(c, X, P)
    recv = np.zeros((4, s), np.uint8)
    for j, h in enumerate([1, 2, 3, 4]):
        hb = out_regions(1, s)
        c.repair_helper(0, to_regions(nodes[h]), hb, s)
        recv[j] = read(hb, s)[0]
    rout = out_regions(2, s)
    c.repair_newcomer(0, [1, 2, 3, 4], to_regions(recv), rout, s)
    assert np.array_equal(read(rout, s), nodes[0])
    Y = np.concatenate([nodes[i] for i in (3, 4, 5)])
    xo = out_regions(c.B, s)
    c.decode([3, 4, 5], to_regions(Y), xo, s)
    assert np.array_equal(read(xo, s), X)


CFG2 = [
    ("sparse-sys", dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE)),
    ("vanilla-nonsys", dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA, systematic=False)),
    ("vanilla-sys", dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA)),
    ("rs-16-8", dict(k=8, d=8, n=16, kind=pm.PM_RS)),
]


@pytest.mark.parametrize("name,kw", CFG2, ids=[c[0] for c in CFG2])
def test_config2_encode_64mib_sampled(name, kw):
    print("config2 %s" % name, flush=True)
    c = pm.Code(**kw)
    o = _oracle_for(kw)
    X, s = synth.split_object(64 << 20, c.B, synth.CONFIG_SEED + 1)
    xin = torch.from_numpy(X).to(device())
    out = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=device())
    c.encode(xin, out, s)
    _check_sampled(out, o.enc, X, s, seed=len(name))


def test_headline_in_the_bench_launch_configuration_sampled():
    """The headline as bench.py times it: the 64 MiB configuration-2 object
    (56 x 1198400 B), encode autotuned over every variant on it and then run
    in the chosen one over 8 buffer sets (the bit-sliced kernel once tuned);
    sampled outputs of every set against the oracle, and the two timed
    launch sequences give the same bytes."""
    kw = dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE)
    c = pm.Code(**kw)
    o = _oracle_for(kw)
    X, s = synth.split_object(64 << 20, c.B, synth.CONFIG_SEED + 1)
    assert s == 1198400
    xs = [torch.from_numpy(X).to(device()) for _ in range(2)]
    outs = [torch.empty((c.enc_rows, s), dtype=torch.uint8, device=device()) for _ in range(2)]
    stream = torch.cuda.current_stream().cuda_stream
    st, rg, vec = pm.pm_autotune_encode(c.h, xs[0].data_ptr(), s, outs[0].data_ptr(), s, s, 3, stream)
    assert st == pm.PM_OK
    print("headline variant (%d, %d)" % (rg, vec), flush=True)
    for i in range(6):
        j = i % 2
        outs[j].zero_()
        assert pm.pm_encode(c.h, xs[j].data_ptr(), s, outs[j].data_ptr(), s, s, stream) == pm.PM_OK
    for j in range(2):
        _check_sampled(outs[j], o.enc, X, s, seed=100 + j)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("name,kw", CFG2, ids=[c[0] for c in CFG2])
def test_config2_codes_full_compare_small_object(name, kw):
    """The same codes on an object spanning several tiles and a ragged tail."""
    c = pm.Code(**kw)
    o = _oracle_for(kw)
    X, s = synth.split_object(c.B * 9000 + 37, c.B, 99, align=1)
    assert np.array_equal(_gpu_encode(c, X, s), o.encode(X, nthreads=8))


def test_config3_mbr_k8_full_size():
    """MBR (8,14,16), 64 MiB: systematic encode (sampled), repair of node 0
    (copy-only helpers) and node 8 from the first 14 survivors, decode from a
    seeded random 8-subset (sampled outputs)."""
    print("config3", flush=True)
    c = pm.Code(k=8, d=14, n=16, kind=pm.PM_MBR)
    o = O.Code(O.MBR, 8, 14, 16)
    X, s = synth.split_object(64 << 20, c.B, synth.CONFIG_SEED + 2)
    assert s == 798976
    dev = device()
    xin = torch.from_numpy(X).to(dev)
    P = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=dev)
    c.encode(xin, P, s)
    _check_sampled(P, o.enc, X, s, seed=3)
    nm = c.node_map()

    def node(i):
        rows = [xin[v] if v < c.B else P[v - c.B] for v in nm[i * c.alpha:(i + 1) * c.alpha]]
        return torch.stack(rows)

    for f in (0, 8):
        H = [i for i in range(c.n) if i != f][:c.d]
        recv = torch.empty((c.d, s), dtype=torch.uint8, device=dev)
        for j, h in enumerate(H):
            c.repair_helper(f, node(h), recv[j:j + 1], s)
        rout = torch.empty((c.alpha, s), dtype=torch.uint8, device=dev)
        c.repair_newcomer(f, H, recv, rout, s)
        torch.cuda.synchronize()
        assert torch.equal(rout, node(f)), f
    K = synth.Stream(synth.CONFIG_SEED + 2).subset(c.n, c.k)
    Y = torch.cat([node(i) for i in K])
    xo = torch.empty((c.B, s), dtype=torch.uint8, device=dev)
    c.decode(K, Y, xo, s)
    torch.cuda.synchronize()
    assert torch.equal(xo, xin)


@pytest.mark.parametrize("rg,vec", VARIANTS)
def test_every_variant_encodes_identically(rg, vec):
    c = pm.Code(k=8, d=14, n=16)
    o = O.Code(O.MSR, 8, 14, 16, O.SPARSE)
    X, s = synth.split_object(c.B * 20000 + 5, c.B, 5, align=1)
    c.set_variant(pm.OP_ENCODE, rg, vec)
    assert np.array_equal(_gpu_encode(c, X, s), o.encode(X, nthreads=8))


def test_k16_sparse_encode_repair_decode():
    c = pm.Code(k=16, d=30, n=32)
    o = O.Code(O.MSR, 16, 30, 32, O.SPARSE)
    s = 4096 + 48
    X = _rand(16, c.B, s)
    P = _gpu_encode(c, X, s)
    assert np.array_equal(P, o.encode(X, nthreads=8))
    nodes = _nodes(c, X, P)
    st = synth.Stream(161)
    for f in (0, 14, 15, 31):
        H = st.subset(c.n, c.d, exclude=[f])
        recv = np.stack([O.apply(o.helper_row(f), nodes[h])[0] for h in H])
        rout = out_regions(c.alpha, s)
        c.repair_newcomer(f, H, to_regions(recv), rout, s)
        assert np.array_equal(read(rout, s), nodes[f])
    for _ in range(3):
        K = st.subset(c.n, c.k)
        Y = np.concatenate([nodes[i] for i in K])
        xo = out_regions(c.B, s)
        c.decode(K, to_regions(Y), xo, s)
        assert np.array_equal(read(xo, s), X)


@pytest.mark.parametrize("s", [777, 4096 + 48, 191616])
def test_k16_mixed_decode_on_the_matrix_cores(s):
    """A (16,30,32) decode from 9 systematic and 7 parity nodes (the served
    mix's largest resident object's node set): 135 rows are copies of held
    blocks and 105 are computed, 47 % of their coefficients nonzero.  The
    default path copies the first (copy groups of the table kernel) and
    computes the second on the matrix cores; every byte against the oracle,
    up to that object's 191 616-byte blocks."""
    print("k16 mixed decode s=%d" % s, flush=True)
    c = pm.Code(k=16, d=30, n=32)
    o = O.Code(O.MSR, 16, 30, 32, O.SPARSE)
    K = [0, 6, 7, 9, 10, 11, 12, 13, 15, 16, 17, 20, 21, 23, 25, 29]
    X = _rand(1600 + s % 97, c.B, s)
    P = o.encode(X, nthreads=8)
    Y = np.concatenate([o.node_blocks(i, X, P) for i in K])
    xo = out_regions(c.B, s, extra=1)
    c.decode(K, to_regions(Y, extra=1), xo, s)
    assert np.array_equal(read(xo, s), X)


# ------------------------------------------------- bit-sliced specialization --
BS_CODES = [
    ("msr4", dict(k=4, d=6, n=8)),
    ("msr8", dict(k=8, d=14, n=16)),
    ("mbr8", dict(k=8, d=14, n=16, kind=pm.PM_MBR)),
    ("rs", dict(k=8, d=8, n=16, kind=pm.PM_RS)),
    ("msr3-vanilla-cfg1", dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=list(range(1, 7)))),
]


@pytest.mark.parametrize("name,kw", BS_CODES, ids=[c[0] for c in BS_CODES])
# 100: below one tile (table kernel); 2048: one tile; 2053: byte tail only;
# 2*2048+112: window tile, no byte tail; 4095, 3*2048+17, 40*2048+2047:
# window tile and byte tail.
@pytest.mark.parametrize("s", [100, 2048, 2053, 2 * 2048 + 112, 4095, 3 * 2048 + 17, 40 * 2048 + 2047])
def test_bitslice_encode_matches_oracle(name, kw, s):
    """The hipRTC-specialized bit-sliced kernel (full 2 KiB wave tiles, the
    overlapping window tile and the byte tail) against the oracle byte for
    byte, with guard bytes past s checked."""
    print("bitslice encode %s s=%d" % (name, s), flush=True)
    c = pm.Code(**kw)
    o = _oracle_for(kw)
    c.set_variant(pm.OP_ENCODE, 8, 32)
    X = _rand(s + len(name), c.B, s)
    assert np.array_equal(_gpu_encode(c, X, s), o.encode(X, nthreads=8))


def test_bitslice_decode_and_newcomer_k8():
    print("bitslice decode/newcomer", flush=True)
    c = pm.Code(k=8, d=14, n=16)
    o = O.Code(O.MSR, 8, 14, 16, O.SPARSE)
    for op in (pm.OP_DECODE, pm.OP_NEWCOMER):
        c.set_variant(op, 8, 32)
    s = 5 * 2048 + 300
    X = _rand(77, c.B, s)
    P = o.encode(X, nthreads=8)
    nodes = _nodes(c, X, P)
    st = synth.Stream(88)
    for _ in range(3):
        K = st.subset(c.n, c.k)
        xo = out_regions(c.B, s)
        c.decode(K, to_regions(np.concatenate([nodes[i] for i in K])), xo, s)
        assert np.array_equal(read(xo, s), X)
        f = st.below(c.n)
        H = st.subset(c.n, c.d, exclude=[f])
        recv = np.stack([O.apply(o.helper_row(f), nodes[h])[0] for h in H])
        rout = out_regions(c.alpha, s)
        c.repair_newcomer(f, H, to_regions(recv), rout, s)
        assert np.array_equal(read(rout, s), nodes[f])


def test_default_variant_before_and_after_specialization():
    """Under the default variant an operation runs the table kernel until its
    bit-sliced kernel is compiled (pm_prepare with wait forces that), then the
    bit-sliced kernel: both results equal the oracle's."""
    print("default variant: table then bit-sliced", flush=True)
    c = pm.Code(k=8, d=14, n=16)
    o = O.Code(O.MSR, 8, 14, 16, O.SPARSE)
    s = 9 * 2048 + 77
    X = _rand(4242, c.B, s)
    P = o.encode(X, nthreads=8)
    nodes = _nodes(c, X, P)
    K = [2, 3, 5, 8, 9, 10, 12, 14]
    Y = to_regions(np.concatenate([nodes[i] for i in K]))
    for prepared in (False, True):
        if prepared:
            assert c.prepare(pm.OP_DECODE, ids=K) is True
            assert c.prepare(pm.OP_ENCODE) is True
        xo = out_regions(c.B, s)
        c.decode(K, Y, xo, s)
        assert np.array_equal(read(xo, s), X)
        assert np.array_equal(_gpu_encode(c, X, s), P)


# ------------------------------------------------ specific PM-MSR decoding --
SPECIFIC_CASES = [
    ("cfg1", dict(k=3, d=4, n=6, construction=pm.PM_VANILLA, x=list(range(1, 7))), [3, 4, 5]),
    ("msr4", dict(k=4, d=6, n=8), [7, 2, 5, 0]),
    ("msr4-nonsys", dict(k=4, d=6, n=8, systematic=False), [1, 3, 6, 4]),
    ("msr8-parity", dict(k=8, d=14, n=16), list(range(8, 16))),
    ("msr8-mixed", dict(k=8, d=14, n=16), [0, 3, 5, 8, 9, 11, 13, 15]),
    ("msr16-parity", dict(k=16, d=30, n=32), list(range(16, 32))),
    ("mbr4-parity", dict(k=4, d=6, n=8, kind=pm.PM_MBR), [7, 4, 6, 5]),
    ("mbr4-dk", dict(k=4, d=4, n=6, kind=pm.PM_MBR), [5, 1, 4, 2]),
    ("mbr8-parity", dict(k=8, d=14, n=16, kind=pm.PM_MBR), list(range(8, 16))),
    ("mbr8-mixed", dict(k=8, d=14, n=16, kind=pm.PM_MBR), [0, 1, 2, 6, 10, 12, 13, 15]),
    ("mbr8-sys", dict(k=8, d=14, n=16, kind=pm.PM_MBR), list(range(8))),
]


def _specific_oracle(kw):
    if kw.get("kind") == pm.PM_MBR:
        return O.Code(O.MBR, kw["k"], kw["d"], kw["n"])
    cons = O.VANILLA if kw.get("construction") == pm.PM_VANILLA else O.SPARSE
    x = np.array(kw["x"]) if "x" in kw else None
    return O.Code(O.MSR, kw["k"], kw["d"], kw["n"], cons, kw.get("systematic", True), x=x)


@pytest.mark.parametrize("name,kw,K", SPECIFIC_CASES, ids=[c[0] for c in SPECIFIC_CASES])
@pytest.mark.parametrize("prepared", [False, True], ids=["table", "bitsliced"])
def test_specific_decode_matches_oracle(name, kw, K, prepared):
    """pm_decode_specific (MSR: node times phi products, pair solves, alpha x
    alpha solves, message symbols, systematic re-encoding; MBR: T beside
    copies, then the message symbols; each a region product) returns the
    object, on
    the table kernels and after pm_prepare on the bit-sliced ones; ragged
    block lengths, guard bytes checked."""
    print("specific decode %s prepared=%s" % (name, prepared), flush=True)
    c = pm.Code(**kw)
    o = _specific_oracle(kw)
    if prepared:
        assert c.prepare(pm.OP_DECODE_SPECIFIC, ids=K) is True   # every pass specialized
    for s in (100, 2048 + 19, 3 * 2048 + 16):
        X = _rand(s + 3 * len(K), c.B, s)
        P = o.encode(X, nthreads=8)
        nodes = {i: o.node_blocks(i, X, P) for i in range(c.n)}
        Y = to_regions(np.concatenate([nodes[i] for i in K]), extra=1)
        xo = out_regions(c.B, s)
        c.decode_specific(K, Y, xo, s)
        assert np.array_equal(read(xo, s), X), s


@pytest.mark.timeout(300)
def test_blocks_larger_than_4_gib():
    """Maximum sizes: RS(16,8) encode of 8 blocks of 4 GiB + 4112 bytes
    (34 GB in, 34 GB out), on the table kernel and then on the bit-sliced
    kernel: byte offsets past 2^32 in every address computation.  Sampled
    positions (the start, both sides of 2^32, the end) against the oracle."""
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < 100 * 10**9:
        pytest.skip("needs about 70 GB of free device memory")
    print("blocks > 4 GiB", flush=True)
    c = pm.Code(k=8, d=8, n=16, kind=pm.PM_RS)
    o = _oracle_for(dict(k=8, d=8, n=16, kind=pm.PM_RS))
    s = (1 << 32) + 4112
    X = synth.random_bytes_torch(0x4613, c.B * s, device()).view(c.B, s)
    out = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=device())
    st = synth.Stream(0x4614)
    pos = sorted({0, 1, 2047, (1 << 32) - 16, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, s - 17, s - 16, s - 1} |
                 {st.below(s) for _ in range(200)})
    pos_t = torch.tensor(pos, dtype=torch.int64, device=device())
    Xs = X.index_select(1, pos_t).cpu().numpy()
    want = O.apply(o.enc, Xs)
    for prepared in (False, True):
        if prepared:
            assert c.prepare(pm.OP_ENCODE) is True
        out.fill_(0x5A)
        c.encode(X, out, s)
        torch.cuda.synchronize()
        assert np.array_equal(out.index_select(1, pos_t).cpu().numpy(), want), prepared
    del X, out

"""Host-side checks of the HIP library (no GPU needed): the C ABI loads and
exports every declared entry point, the library's own construction equals
the oracle's byte for byte, and argument errors come back as statuses."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1412_3022_amd import pm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(pm_[a-z_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = pm.lib()
    declared = _declared()
    assert {"pm_code_create", "pm_encode", "pm_repair_helper", "pm_repair_newcomer", "pm_decode"} <= declared
    for name in sorted(declared):
        assert hasattr(L, name), name


CODES = [
    dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=list(range(1, 7))),
    dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=4, d=6, n=8, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=8, d=14, n=15, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=16, d=30, n=32, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA),
    dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA, systematic=False),
    dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE, systematic=False),
    dict(k=3, d=4, n=6, kind=pm.PM_MBR),
    dict(k=8, d=14, n=16, kind=pm.PM_MBR),
    dict(k=5, d=5, n=7, kind=pm.PM_MBR),
    dict(k=8, d=8, n=16, kind=pm.PM_RS),
]


def _oracle_code(kw):
    kind = {pm.PM_MSR: O.MSR, pm.PM_MBR: O.MBR, pm.PM_RS: O.RS}[kw["kind"]]
    cons = O.VANILLA if kw.get("construction", pm.PM_SPARSE) == pm.PM_VANILLA else O.SPARSE
    x = np.array(kw["x"]) if "x" in kw else None
    return O.Code(kind, kw["k"], kw["d"], kw["n"], cons, kw.get("systematic", True), x=x)


@pytest.mark.parametrize("kw", CODES, ids=lambda kw: "%d-%d-%d-%d-%d" % (kw["kind"], kw.get("construction", 1),
                                                                        kw["k"], kw["d"], kw["n"]))
def test_construction_matches_oracle(kw):
    c = pm.Code(**kw)
    o = _oracle_code(kw)
    assert (c.alpha, c.B, c.enc_rows) == (o.alpha, o.B, o.enc.shape[0])
    assert np.array_equal(c.matrix(pm.MAT_PSI), o.psi)
    assert np.array_equal(c.matrix(pm.MAT_G), o.G)
    assert np.array_equal(c.matrix(pm.MAT_GSYS), o.Gsys)
    assert np.array_equal(c.matrix(pm.MAT_ENC), o.enc)
    if kw["kind"] == pm.PM_MSR:
        assert np.array_equal(c.matrix(pm.MAT_LAMBDA)[0], o.lam)
    nm = c.node_map()
    for t, (src, idx) in enumerate(o.node_map):
        assert nm[t] == (idx if src == "x" else c.B + idx)


@pytest.mark.parametrize("kw,status", [
    (dict(k=16, d=30, n=32, kind=pm.PM_MSR, construction=pm.PM_VANILLA), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=13, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=14, n=17, kind=pm.PM_MSR, construction=pm.PM_SPARSE), pm.PM_EUNSUPPORTED),
    (dict(k=40, d=78, n=79, kind=pm.PM_MSR, construction=pm.PM_SPARSE), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=14, n=14, kind=pm.PM_MSR, construction=pm.PM_SPARSE), pm.PM_EINVAL),
    (dict(k=8, d=14, n=300, kind=pm.PM_MSR, construction=pm.PM_VANILLA), pm.PM_EINVAL),
    (dict(k=8, d=7, n=16, kind=pm.PM_MBR), pm.PM_EINVAL),
    (dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE, w=12), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=14, n=16, kind=pm.PM_MBR, w=16), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=8, n=16, kind=pm.PM_RS, w=16), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA, w=16), pm.PM_EUNSUPPORTED),
    (dict(k=8, d=14, n=17, kind=pm.PM_MSR, construction=pm.PM_SPARSE, w=16), pm.PM_EUNSUPPORTED),
    (dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=[1, 2, 3, 4, 5, 5]), pm.PM_EINVAL),
])
def test_create_errors(kw, status):
    st, h = pm.pm_code_create(**kw)
    assert st == status
    assert not h


def test_data_call_argument_errors_need_no_gpu():
    c = pm.Code(k=4, d=6, n=8)
    # NULL / misaligned regions and zero sizes are rejected before any device work
    assert pm.pm_encode(c.h, 0, 64, 0, 64, 64) == pm.PM_EINVAL
    assert pm.pm_encode(c.h, 16, 64, 4096, 64, 0) == pm.PM_EINVAL
    assert pm.pm_encode(c.h, 8, 64, 4096, 64, 64) == pm.PM_EINVAL         # misaligned base
    assert pm.pm_encode(c.h, 4096, 24, 1 << 20, 64, 16) == pm.PM_EINVAL   # ld not a multiple of 16
    assert pm.pm_encode(c.h, 4096, 64, 1 << 20, 64, 128) == pm.PM_EINVAL  # ld < block_bytes
    assert pm.pm_encode(c.h, 4096, 64, 4096 + 64, 64, 64) == pm.PM_EINVAL  # overlap
    assert pm.pm_repair_helper(c.h, 99, 4096, 64, 1 << 20, 64) == pm.PM_EINVAL
    assert pm.pm_repair_newcomer(c.h, 0, [1, 2, 3, 4, 5, 5], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_repair_newcomer(c.h, 0, [0, 2, 3, 4, 5, 6], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_decode(c.h, [0, 1, 2, 2], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_decode(c.h, [0, 1, 2, 9], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_set_variant(c.h, 0, 5, 4) == pm.PM_EINVAL
    assert pm.pm_set_variant(c.h, 0, 8, 3) == pm.PM_EINVAL
    assert pm.pm_set_variant(c.h, 0, 8, 4) == pm.PM_OK
    assert pm.pm_set_variant(c.h, 0, 0, 0) == pm.PM_OK


def test_status_strings():
    for st in range(-6, 1):
        assert pm.status_string(st)


# ---------------------------------------------- init phase / specialization --
def test_prepare_compiles_bitsliced_kernels_without_gpu():
    """pm_prepare builds an operation's matrix and compiles its bit-sliced
    kernel with hipRTC, which needs no GPU; the kernel then counts as ready."""
    c = pm.Code(k=4, d=6, n=8)
    assert c.prepare(pm.OP_ENCODE) is True
    assert c.prepare(pm.OP_HELPER, failed=5) is True
    assert c.prepare(pm.OP_NEWCOMER, failed=5, ids=[0, 1, 2, 3, 4, 6]) is True
    assert c.prepare(pm.OP_DECODE, ids=[1, 4, 6, 7]) is True


def test_default_variant_never_compiles_by_itself():
    """A data call under the default variant must not start a compile: with
    no GPU it fails with PM_EHIP after building the program, and the
    operation still reports no specialized kernel until pm_prepare."""
    c = pm.Code(k=3, d=4, n=6)
    s = 4096
    st = pm.pm_decode(c.h, [0, 2, 5], 1 << 20, s, (1 << 20) + 64 * s, s, s, None)
    assert st == pm.PM_EHIP
    L = pm.lib()
    spec = ctypes.c_int(-1)
    ids = (ctypes.c_uint32 * 3)(0, 2, 5)
    c.set_variant(pm.OP_DECODE, 4, 2)           # explicit table variant: prepare compiles nothing
    assert L.pm_prepare(c.h, pm.OP_DECODE, 0, ids, 0, ctypes.byref(spec)) == pm.PM_OK and spec.value == 0
    c.set_variant(pm.OP_DECODE, 0, 0)
    assert L.pm_prepare(c.h, pm.OP_DECODE, 0, ids, 0, ctypes.byref(spec)) == pm.PM_OK and spec.value == 1


def test_prepare_reports_table_kernel_cases():
    # an explicit table variant never switches to the specialized kernel
    c = pm.Code(k=4, d=6, n=8)
    c.set_variant(pm.OP_ENCODE, 8, 2)
    assert c.prepare(pm.OP_ENCODE) is False
    # a dense k=16 decode (from the 16 parity nodes) is over the size limit
    assert pm.Code(k=16, d=30, n=32).prepare(pm.OP_DECODE, ids=list(range(16, 32))) is False


@pytest.mark.parametrize("op,failed,ids", [
    (pm.OP_DECODE, 0, [1, 1, 2, 3]),        # repeated node
    (pm.OP_NEWCOMER, 5, [0, 1, 2, 3, 4, 5]),  # the failed node as its own helper
    (pm.OP_HELPER, 8, None),               # no such node
    (7, 0, None),                          # no such operation
])
def test_prepare_argument_errors(op, failed, ids):
    c = pm.Code(k=4, d=6, n=8)
    st, spec = pm.pm_prepare(c.h, op, failed, ids)
    assert st == pm.PM_EINVAL and spec == 0


# ------------------------------------------- specific PM-MSR / PM-MBR decode --
SPECIFIC = [
    (dict(k=3, d=4, n=6, construction=pm.PM_VANILLA, x=list(range(1, 7))), (O.MSR, 3, 4, 6, O.VANILLA), [3, 4, 5]),
    (dict(k=4, d=6, n=8), (O.MSR, 4, 6, 8, O.SPARSE), [7, 2, 5, 0]),
    (dict(k=4, d=6, n=8, systematic=False), (O.MSR, 4, 6, 8, O.SPARSE), [1, 3, 6, 4]),
    (dict(k=8, d=14, n=16), (O.MSR, 8, 14, 16, O.SPARSE), list(range(8, 16))),
    (dict(k=16, d=30, n=32), (O.MSR, 16, 30, 32, O.SPARSE), list(range(16, 32))),
]


@pytest.mark.parametrize("kw,ok,K", SPECIFIC, ids=lambda v: None)
def test_specific_decode_factors_multiply_to_the_decode_matrix(kw, ok, K):
    """The library's five sparse factors of the specific decode, multiplied
    with the oracle's field arithmetic, give exactly the oracle's linearized
    decode matrix for the same nodes (every MSR node set uses all k alpha
    received blocks)."""
    c = pm.Code(**kw)
    o = O.Code(*ok[:4], ok[4], kw.get("systematic", True), x=np.array(kw["x"]) if "x" in kw else None)
    F = [c.specific_factor(K, w) for w in range(5)]
    k, a, B = c.k, c.alpha, c.B
    assert F[0].shape == (k * (k - 1), k * a) and F[1].shape == (B, k * (k - 1))
    assert F[2].shape == (2 * a * a, B) and F[3].shape == (B, 2 * a * a)
    # pass 0 reads one node per output block, pass 1 two blocks per output
    assert (np.count_nonzero(F[0], axis=1) <= a).all()
    assert (np.count_nonzero(F[1], axis=1) == 2).all()
    prod = F[0]
    for w in (1, 2, 3):
        prod = O.matmul(F[w], prod)
    if kw.get("systematic", True):
        assert F[4].shape == (B, B)
        prod = O.matmul(F[4], prod)
    else:
        assert F[4].shape[0] == 0
    D, kept = o.decode_matrix(K)
    assert list(kept) == list(range(k * a))
    assert np.array_equal(prod, D)


MBR_SPECIFIC = [
    ((3, 4, 6), [3, 4, 5]),
    ((4, 4, 6), [5, 1, 4, 2]),
    ((4, 6, 8), [0, 1, 2, 3]),
    ((8, 14, 16), list(range(8, 16))),
    ((8, 14, 16), [0, 1, 2, 6, 10, 12, 13, 15]),
    ((16, 30, 32), list(range(16, 32))),
]


@pytest.mark.parametrize("kdn,K", MBR_SPECIFIC, ids=lambda v: None)
def test_mbr_specific_factors_invert_the_received_rows(kdn, K):
    """The library's two PM-MBR factors: F1 F0 times the oracle's generator
    rows of the k d received blocks is the identity (they decode every
    object), and the nodes of K among the first k (rows [I_k, 0] of Psi)
    make their message symbols plain copies."""
    k, d, n = kdn
    c = pm.Code(k=k, d=d, n=n, kind=pm.PM_MBR)
    o = O.Code(O.MBR, k, d, n)
    F = [c.specific_factor(K, w) for w in range(5)]
    w = F[0].shape[0]
    assert F[0].shape == (w, k * d) and F[1].shape == (c.B, w)
    assert all(F[p].shape[0] == 0 for p in (2, 3, 4))
    assert k * (d - k) <= w <= k * d
    GK = np.concatenate([o.Gsys[i * d:(i + 1) * d] for i in K])
    assert np.array_equal(O.matmul(O.matmul(F[1], F[0]), GK), np.eye(c.B, dtype=np.uint8))
    # a message symbol held by a node l < k of K: one term, a copy of a copy
    sysK = [i for i in K if i < k]
    for a in sysK:
        for b in range(d):
            m = np.asarray(o.L).reshape(-1)[a * d + b]
            row = F[1][m]
            assert np.count_nonzero(row) == 1 and row.max() == 1
            src = F[0][np.flatnonzero(row)[0]]
            assert np.count_nonzero(src) == 1 and src.max() == 1
    if len(sysK) == k:
        assert (np.count_nonzero(F[0], axis=1) == 1).all() and (np.count_nonzero(F[1], axis=1) == 1).all()


def test_specific_decode_refusals():
    L = pm.lib()
    c = pm.Code(k=8, d=8, n=16, kind=pm.PM_RS)
    n = ctypes.c_size_t()
    assert L.pm_decode_specific_workspace(c.h, 4096, ctypes.byref(n)) == pm.PM_EUNSUPPORTED
    c = pm.Code(k=8, d=14, n=16, kind=pm.PM_MBR)
    assert L.pm_decode_specific_workspace(c.h, 4090, ctypes.byref(n)) == pm.PM_OK
    assert n.value == 8 * 14 * 4096
    bad = (ctypes.c_uint32 * 8)(0, 1, 2, 3, 4, 5, 6, 6)
    assert L.pm_decode_specific_factor(c.h, bad, 0, None, 0, None, None) == pm.PM_EINVAL
    c = pm.Code(k=4, d=6, n=8)
    bad = (ctypes.c_uint32 * 4)(0, 1, 1, 2)
    assert L.pm_decode_specific_factor(c.h, bad, 0, None, 0, None, None) == pm.PM_EINVAL
    good = (ctypes.c_uint32 * 4)(0, 1, 2, 3)
    assert L.pm_decode_specific_factor(c.h, good, 5, None, 0, None, None) == pm.PM_EINVAL
    n = ctypes.c_size_t()
    assert L.pm_decode_specific_workspace(c.h, 100, ctypes.byref(n)) == pm.PM_OK
    assert n.value == (c.k * (c.k - 1) + c.B + 2 * c.alpha ** 2 + c.B) * 112
    # workspace too small: refused before any GPU work
    st = L.pm_decode_specific(c.h, good, ctypes.c_void_p(1 << 20), 112, ctypes.c_void_p(1 << 22), 112, 100,
                              ctypes.c_void_p(1 << 24), n.value - 16, None)
    assert st == pm.PM_EINVAL


# ------------------------------------------------ GPU-side init: arguments --
def test_init_entry_points_refuse_bad_arguments_before_any_gpu_work():
    L = pm.lib()
    vp = ctypes.c_void_p
    c = pm.Code(k=8, d=14, n=16)
    B = c.B
    assert L.pm_decode_matrices(None, vp(1 << 20), 1, vp(1 << 21), B * B, None, vp(1 << 22), None) == pm.PM_EINVAL
    assert L.pm_decode_matrices(c.h, None, 1, vp(1 << 21), B * B, None, vp(1 << 22), None) == pm.PM_EINVAL
    assert L.pm_decode_matrices(c.h, vp(1 << 20), 1, None, B * B, None, vp(1 << 22), None) == pm.PM_EINVAL
    assert L.pm_decode_matrices(c.h, vp(1 << 20), 1, vp(1 << 21), B * B, None, None, None) == pm.PM_EINVAL
    assert L.pm_decode_matrices(c.h, vp(1 << 20), 1, vp(1 << 21), B * B - 1, None, vp(1 << 22), None) == pm.PM_EINVAL
    assert L.pm_decode_matrices(c.h, vp(1 << 20), 0, vp(1 << 21), B * B, None, vp(1 << 22), None) == pm.PM_OK
    inv = L.pm_gf_invert_batch
    assert inv(vp(1 << 20), 8, 64, 0, 1, vp(1 << 21), 8, 64, vp(1 << 22), None) == pm.PM_EINVAL    # m = 0
    assert inv(vp(1 << 20), 7, 64, 8, 1, vp(1 << 21), 8, 64, vp(1 << 22), None) == pm.PM_EINVAL    # a_ld < m
    assert inv(vp(1 << 20), 8, 64, 8, 1, vp(1 << 21), 7, 64, vp(1 << 22), None) == pm.PM_EINVAL    # inv_ld < m
    assert inv(vp(1 << 20), 8, 63, 8, 2, vp(1 << 21), 8, 64, vp(1 << 22), None) == pm.PM_EINVAL    # overlap
    assert inv(vp(1 << 20), 8, 64, 8, 2, vp(1 << 21), 8, 63, vp(1 << 22), None) == pm.PM_EINVAL
    assert inv(None, 8, 64, 8, 1, vp(1 << 21), 8, 64, vp(1 << 22), None) == pm.PM_EINVAL
    assert inv(vp(1 << 20), 8, 64, 8, 1, vp(1 << 21), 8, 64, None, None) == pm.PM_EINVAL
    assert inv(vp(1 << 20), 8, 64, 8, 0, vp(1 << 21), 8, 64, vp(1 << 22), None) == pm.PM_OK


@pytest.mark.parametrize("kw,ok,K", [
    (dict(k=8, d=14, n=16), (O.MSR, 8, 14, 16, O.SPARSE), [15, 3, 9, 0, 12, 6, 10, 1]),
    (dict(k=8, d=14, n=16, kind=pm.PM_MBR), (O.MBR, 8, 14, 16, O.SPARSE), [0, 1, 2, 6, 10, 12, 13, 15]),
    (dict(k=8, d=8, n=16, kind=pm.PM_RS), (O.RS, 8, 8, 16, O.SPARSE), list(range(8, 16))),
], ids=["msr8", "mbr8", "rs"])
def test_host_decode_matrix_matches_the_oracle(kw, ok, K):
    c = pm.Code(**kw)
    o = O.Code(*ok[:4], ok[4]) if ok[0] == O.MSR else O.Code(*ok[:4])
    D, kept = c.decode_matrix(K)
    Dw, kw_ = o.decode_matrix(K)
    assert np.array_equal(D, Dw) and kept == list(kw_)
    L = pm.lib()
    bad = (ctypes.c_uint32 * c.k)(*([0] * c.k))
    assert L.pm_decode_matrix(c.h, bad, None, 0, None) == pm.PM_EINVAL
    good = (ctypes.c_uint32 * c.k)(*K)
    assert L.pm_decode_matrix(c.h, good, ctypes.c_void_p(1), c.B * c.B - 1, None) == pm.PM_EINVAL

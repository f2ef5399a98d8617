"""Host side of the library's GF(2^16) codes (no GPU needed): its own
construction of the sparse PM-MSR code over GF(2^16) (Section 3.3) equals
the oracle's entry for entry, and calls it does not serve, or with bad
arguments, come back as statuses before any device work."""
import ctypes

import numpy as np
import pytest

from oracle import gf16 as F
from paper_1412_3022_amd import pm

CODES = [(3, 5, True), (4, 8, True), (4, 8, False), (8, 15, True), (8, 16, True), (8, 16, False),
         (40, 79, False)]


@pytest.mark.parametrize("k,n,sys_", CODES, ids=lambda v: str(v))
def test_construction_matches_oracle(k, n, sys_):
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_, check=k < 40)
    assert (c.alpha, c.B, c.enc_rows) == (o.alpha, o.B, o.enc.shape[0])
    assert np.array_equal(c.matrix(0), o.psi)
    assert np.array_equal(c.matrix(1).reshape(-1), o.lam)
    assert np.array_equal(c.matrix(2), o.G)
    assert np.array_equal(c.matrix(3), o.Gsys)
    assert np.array_equal(c.matrix(4), o.enc)
    nm = c.node_map()
    assert list(nm) == [t if src == "x" else o.B + t2 for t, (src, t2) in
                        ((t, o.node_map[t]) for t in range(n * o.alpha))]


def test_matrix_is_little_endian_two_bytes_per_entry():
    c = pm.Code(k=3, d=4, n=5, w=16)
    r, cl = ctypes.c_uint32(), ctypes.c_uint32()
    assert pm.lib().pm_code_matrix(c.h, 0, None, 0, ctypes.byref(r), ctypes.byref(cl)) == pm.PM_OK
    raw = np.zeros(2 * r.value * cl.value, np.uint8)
    assert pm.lib().pm_code_matrix(c.h, 0, raw.ctypes.data, raw.size - 1, None, None) == pm.PM_EINVAL
    assert pm.lib().pm_code_matrix(c.h, 0, raw.ctypes.data, raw.size, None, None) == pm.PM_OK
    psi = F.Code(3, 5).psi
    assert np.array_equal(raw[0::2].astype(np.uint16) | raw[1::2].astype(np.uint16) << 8, psi.reshape(-1))


def test_refusals_and_argument_errors_need_no_gpu():
    c = pm.Code(k=4, d=6, n=8, w=16)
    # GF(2^8)-only entry points
    assert pm.pm_set_variant(c.h, 0, 8, 4) == pm.PM_EUNSUPPORTED
    assert pm.lib().pm_decode_matrix(c.h, pm._u32arr([0, 1, 2, 3]), None, 0, None) == pm.PM_EUNSUPPORTED
    assert pm.pm_prepare(c.h, pm.OP_ENCODE, flags=pm.PM_PREPARE_BATCHED)[0] == pm.PM_EUNSUPPORTED
    # the specific decode: workspace of Z, the pairs, the phi^t S rows and Z
    n = ctypes.c_size_t()
    assert pm.lib().pm_decode_specific_workspace(c.h, 4096, ctypes.byref(n)) == pm.PM_OK
    assert n.value == (4 * 3 + 12 + 2 * 9 + 12) * 4096
    # the matrices are built and their bit-sliced kernels compiled (hipRTC
    # needs no device; with none here nothing is staged)
    assert pm.pm_prepare(c.h, 4, ids=[0, 1, 2, 3]) == (pm.PM_OK, 1)
    assert pm.pm_prepare(c.h, 4, ids=[0, 1, 2, 2])[0] == pm.PM_EINVAL
    assert pm.pm_prepare(c.h, pm.OP_ENCODE) == (pm.PM_OK, 1)
    assert pm.pm_prepare(c.h, pm.OP_HELPER, failed=2) == (pm.PM_OK, 1)
    assert pm.pm_prepare(c.h, pm.OP_NEWCOMER, failed=0, ids=[1, 2, 3, 4, 5, 6]) == (pm.PM_OK, 1)
    assert pm.pm_prepare(c.h, pm.OP_DECODE, ids=[7, 5, 3, 1]) == (pm.PM_OK, 1)
    # data calls: odd block sizes, bad regions and node lists
    assert pm.pm_encode(c.h, 4096, 64, 1 << 20, 64, 63) == pm.PM_EINVAL       # odd: not whole symbols
    assert pm.pm_encode(c.h, 4096, 64, 1 << 20, 64, 0) == pm.PM_EINVAL
    assert pm.pm_encode(c.h, 8, 64, 1 << 20, 64, 64) == pm.PM_EINVAL          # misaligned base
    assert pm.pm_encode(c.h, 4096, 64, 4096 + 64, 64, 64) == pm.PM_EINVAL     # overlap
    assert pm.pm_repair_helper(c.h, 99, 4096, 64, 1 << 20, 64) == pm.PM_EINVAL
    assert pm.pm_repair_newcomer(c.h, 0, [1, 2, 3, 4, 5, 5], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_repair_newcomer(c.h, 0, [0, 2, 3, 4, 5, 6], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_decode(c.h, [0, 1, 2, 2], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL
    assert pm.pm_decode(c.h, [0, 1, 2, 9], 4096, 64, 1 << 20, 64, 64) == pm.PM_EINVAL


@pytest.mark.parametrize("k,n,sys_,K", [(4, 8, True, [1, 4, 6, 7]), (4, 8, False, [7, 5, 3, 1]),
                                         (8, 16, True, [0, 3, 8, 9, 11, 12, 14, 15]),
                                         (16, 32, True, [0, 3, 9, 14, 15, 16, 17, 20, 22, 24, 25, 26, 28, 29, 30, 31])])
def test_specific_decode_factors_multiply_to_the_decode_matrix(k, n, sys_, K):
    """The library's five GF(2^16) factors of the specific decode (Section 4.1)
    multiply to the oracle's linearized decode matrix for the same nodes."""
    c = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
    o = F.Code(k, n, systematic_form=sys_)
    Fs = [c.specific_factor(K, w) for w in range(5)]
    prod = Fs[0]
    for f in Fs[1:]:
        if f.size:
            prod = F.matmul(f, prod)
    assert np.array_equal(prod, o.decode_matrix(K))
    assert (Fs[4].size > 0) == sys_


def test_split_kernels_compile_side_by_side_without_a_gpu():
    """The k = 8 decode from the 8 parity nodes (56 x 56 dense, past one
    bit-sliced kernel's size) is generated as two kernels whose hipRTC
    compiles run on two threads, joined before pm_prepare returns; with no
    device nothing is staged, and the call reports the operation
    specialized."""
    c = pm.Code(k=8, d=14, n=16, w=16)
    assert pm.pm_prepare(c.h, pm.OP_DECODE, ids=list(range(8, 16))) == (pm.PM_OK, 1)

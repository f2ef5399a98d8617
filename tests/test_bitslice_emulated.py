"""The generated bit-sliced kernels (single-set and multi-set), compiled for
the host and run thread by thread under AddressSanitizer, against the oracle:
encode, repair helper, repair newcomer and decode; ragged lengths (window tile
and byte tail); fewer and more work-group slots than row groups; and buffers
at addresses whose low 32 bits are >= 2^31.  Needs no GPU."""
import os
import shutil

import numpy as np
import pytest

import oracle as O
import bs_emulator as E
from paper_1412_3022_amd import pm, synth

pytestmark = pytest.mark.skipif(not os.path.exists(E.CLANG), reason="clang++ of the ROCm toolchain not found")

SIZES = [2048, 3000, 2049, 5000, 4096 + 17, 2063]
CASES = [
    # name, code, oracle code, failed node, helpers, decode nodes, slot counts
    ("msr4", dict(k=4, d=6, n=8), (O.MSR, 4, 6, 8, O.SPARSE), 5, [0, 1, 2, 3, 4, 6], [1, 4, 6, 7], (7, 3, 40)),
    ("mbr4", dict(k=4, d=5, n=7, kind=pm.PM_MBR), (O.MBR, 4, 5, 7, O.SPARSE), 2, [0, 1, 3, 4, 6], [0, 3, 5, 6],
     (9, 2)),
]


def _inputs(c, o, op, f, H, K, s, seed):
    X = synth.random_bytes(seed, c.B * s).reshape(c.B, s)
    P = o.encode(X, nthreads=4)
    nodes = {j: o.node_blocks(j, X, P) for j in range(c.n)}
    if op == pm.OP_ENCODE:
        return X, P
    if op == pm.OP_HELPER:
        return nodes[H[0]], O.apply(o.helper_row(f), nodes[H[0]])
    if op == pm.OP_NEWCOMER:
        return np.stack([O.apply(o.helper_row(f), nodes[h])[0] for h in H]), nodes[f]
    return np.concatenate([nodes[j] for j in K]), X


@pytest.mark.parametrize("name,kw,ok,f,H,K,slots", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("op", [pm.OP_ENCODE, pm.OP_HELPER, pm.OP_NEWCOMER, pm.OP_DECODE],
                         ids=["encode", "helper", "newcomer", "decode"])
def test_generated_kernels_match_oracle_on_host(tmp_path, name, kw, ok, f, H, K, slots, op):
    c, o = pm.Code(**kw), O.Code(*ok)
    src = E.generated_source(c, op, f, H if op == pm.OP_NEWCOMER else K, workdir=str(tmp_path))
    assert src is not None
    items = []
    for i, s in enumerate(SIZES):
        inp, want = _inputs(c, o, op, f, H, K, s, 700 + 31 * op + i)
        ld = (s + 15) // 16 * 16 + 16 * (i % 3)
        items.append(((inp, ld, want.shape[0], ld, s), want))
    for multi in (False, True):
        use = items if multi else items[:1]
        for sanitize, high in ((True, False), (False, True)):
            exe = E.build(src, multi, sanitize=sanitize)
            for P in slots:
                outs = E.run(exe, P, [u for u, _ in use], high=high)
                for got, (_, want) in zip(outs, use):
                    assert np.array_equal(got, want), (name, op, multi, P, high)


@pytest.mark.parametrize("kw,K", [(dict(k=5, d=8, n=10), list(range(5, 10))),
                                  (dict(k=6, d=10, n=12, systematic=False), [0, 2, 4, 6, 8, 10]),
                                  (dict(k=8, d=14, n=16, kind=pm.PM_MBR), [0, 1, 2, 6, 10, 12, 13, 15])],
                         ids=["msr5-sys", "msr6-nonsys", "mbr8-mixed"])
def test_specific_decode_factor_kernels_on_host(tmp_path, kw, K):
    """The generated kernels of the specific decode's factor matrices (MSR:
    node times phi products, pair solves, alpha x alpha solves, message
    symbols, systematic re-encoding; MBR: T beside copies, then the message
    symbols) against the oracle's product, on the host."""
    c = pm.Code(**kw)
    for w in range(5):
        F = c.specific_factor(K, w)
        if F.shape[0] == 0:
            continue
        src = E.generated_apply_source(F, workdir=str(tmp_path))
        assert src is not None, w
        s = 2048 + 77
        X = synth.random_bytes(900 + w, F.shape[1] * s).reshape(F.shape[1], s)
        want = O.apply(F, X, nthreads=4)
        ld = (s + 15) // 16 * 16 + 16
        for sanitize, high in ((True, False), (False, True)):
            exe = E.build(src, False, sanitize=sanitize)
            got, = E.run(exe, 5, [(X, ld, F.shape[0], ld, s)], high=high)
            assert np.array_equal(got, want), (w, high)

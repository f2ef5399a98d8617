"""GPU test of pm_decode_specific_noalloc, the specific decode for callers
that cannot allocate device memory: its intermediates live in the library's
fixed device scratch.  Its output must equal pm_decode_specific's (with a
caller workspace) byte for byte, on two calls in a row, the second with a
smaller block, and both must equal the object that was encoded."""
import numpy as np
import pytest
import torch

from gpu_util import PAD_OUT, device, out_regions, read, to_regions
from paper_1412_3022_amd import pm, synth

pytestmark = pytest.mark.gpu

CASES = [
    # (code, node set, first block size, second block size)
    (dict(k=8, d=14, n=16), [1, 3, 6, 8, 10, 11, 13, 15], 300_007, 4_099),
    (dict(k=8, d=14, n=16, kind=pm.PM_MBR), [0, 2, 5, 8, 9, 12, 14, 15], 500_000, 2_048),
    (dict(k=4, d=6, n=8), [4, 5, 6, 7], 65_549, 17),
]


def _node_blocks(code, X, P):
    """The k alpha blocks of every node after encode, from the node map."""
    nmap = code.node_map()
    full = np.concatenate([X, P])
    return full[nmap].reshape(code.n, code.alpha, -1)


@pytest.mark.parametrize("kw,nodes,s1,s2", CASES, ids=["msr-8-14-16", "mbr-8-14-16", "msr-4-6-8"])
def test_noalloc_specific_decode_equals_workspace_form(kw, nodes, s1, s2):
    dev = device()
    code = pm.Code(**kw)
    print("no-alloc specific decode", kw, nodes, s1, s2, flush=True)
    # before the node list is prepared the entry point refuses (host check)
    Y0 = torch.zeros((code.k * code.alpha, 16), dtype=torch.uint8, device=dev)
    X0 = torch.zeros((code.B, 16), dtype=torch.uint8, device=dev)
    st = pm.pm_decode_specific_noalloc(code.h, nodes, Y0.data_ptr(), 16, X0.data_ptr(), 16, 16)
    assert st == pm.PM_ENOTREADY
    code.prepare(pm.OP_DECODE_SPECIFIC, ids=nodes)
    for s in (s1, s2):
        X = synth.random_bytes(synth.CONFIG_SEED + 700 + s % 97, code.B * s).reshape(code.B, s)
        P = out_regions(code.enc_rows, s)
        code.encode(to_regions(X), P, s)
        Pn = read(P, s)
        held = _node_blocks(code, X, Pn)
        Y = to_regions(np.concatenate([held[i] for i in nodes]))
        X_ws = out_regions(code.B, s)
        code.decode_specific(nodes, Y, X_ws, s)
        X_na = out_regions(code.B, s)
        code.decode_specific_noalloc(nodes, Y, X_na, s)
        want = read(X_ws, s)
        got = read(X_na, s)
        assert np.array_equal(got, want), "no-alloc decode differs from the workspace form at s=%d" % s
        assert np.array_equal(got, X), "decode differs from the object at s=%d" % s


def test_noalloc_refuses_blocks_beyond_the_scratch():
    dev = device()
    code = pm.Code(k=8, d=14, n=16)
    nodes = list(range(8, 16))
    code.prepare(pm.OP_DECODE_SPECIFIC, ids=nodes)
    s = 8 << 20   # 266 workspace blocks of 8 MiB: far beyond 128 MiB
    assert pm.pm_decode_specific_workspace(code.h, s) > 128 << 20
    # full-size regions, so that the call is well formed apart from its size
    Y = torch.zeros((code.k * code.alpha, s), dtype=torch.uint8, device=dev)
    X = torch.full((code.B, s), PAD_OUT, dtype=torch.uint8, device=dev)
    st = pm.pm_decode_specific_noalloc(code.h, nodes, Y.data_ptr(), s, X.data_ptr(), s, s)
    assert st == pm.PM_ELIMIT
    assert "scratch" in pm.status_string(st)
    # nothing was launched: X still holds its fill
    torch.cuda.synchronize()
    assert bool((X == PAD_OUT).all())

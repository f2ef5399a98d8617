"""pm_repair: both repair steps in two launches (the d helper projections as
one multi-set launch, then the newcomer), checked against the oracle: the
workspace holds each helper's projection (the block it would send, Section
2) and the output the lost node's blocks, for every (f, H) of small codes and
for the configuration-1, configuration-3 and (16,30,32) shapes."""
from itertools import combinations

import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import device, out_regions, read, to_regions
from paper_1412_3022_amd import pm, synth

pytestmark = pytest.mark.gpu


def _oracle_for(kw):
    kind = {pm.PM_MSR: O.MSR, pm.PM_MBR: O.MBR, pm.PM_RS: O.RS}[kw.get("kind", pm.PM_MSR)]
    cons = O.VANILLA if kw.get("construction", pm.PM_SPARSE) == pm.PM_VANILLA else O.SPARSE
    x = np.array(kw["x"]) if kw.get("x") is not None else None
    return O.Code(kind, kw["k"], kw["d"], kw["n"], cons, kw.get("systematic", True), x=x)


def _check_repair(c, o, nodes, f, H, s):
    node_t = [to_regions(nodes[h]) for h in H]
    out = out_regions(c.alpha, s)
    ws = c.repair(f, list(H), node_t, out, s)
    assert np.array_equal(read(out, s), nodes[f]), (f, H, s)
    ld = (s + 15) // 16 * 16
    torch.cuda.synchronize()
    recv = ws[:len(H) * ld].view(len(H), ld)[:, :s].cpu().numpy()
    hrow = o.helper_row(f)
    for j, h in enumerate(H):
        assert np.array_equal(recv[j], O.apply(hrow, nodes[h])[0]), (f, h, s)


SMALL = [
    dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=list(range(1, 7))),
    dict(k=4, d=6, n=8, kind=pm.PM_MSR, construction=pm.PM_SPARSE),
    dict(k=4, d=6, n=7, kind=pm.PM_MSR, construction=pm.PM_SPARSE, systematic=False),
    dict(k=4, d=5, n=7, kind=pm.PM_MBR),
]


@pytest.mark.parametrize("kw", SMALL, ids=lambda kw: "%d-%d-%d-%d-%d" % (
    kw["kind"], kw.get("construction", 1), kw["k"], kw["d"], kw["n"]))
@pytest.mark.parametrize("s,prepared", [(64, False), (4099, False), (4099, True)])
def test_repair_every_failure_and_helper_set(kw, s, prepared):
    print("pm_repair %s s=%d prepared=%s" % (kw, s, prepared), flush=True)
    c, o = pm.Code(**kw), _oracle_for(kw)
    X = synth.random_bytes(301 + s + kw["n"], c.B * s).reshape(c.B, s)
    P = o.encode(X)
    nodes = {i: o.node_blocks(i, X, P) for i in range(c.n)}
    for f in range(c.n):
        if prepared:   # the helper vector's multi-set kernel: one projection launch
            assert c.prepare(pm.OP_HELPER, failed=f, batched=True)
        others = [i for i in range(c.n) if i != f]
        for H in combinations(others, c.d):
            _check_repair(c, o, nodes, f, H, s)


def test_repair_configuration_1():
    """Vanilla PM-MSR (3,4,6), x_i = i + 1, 1 MiB object: node 0 from
    helpers 1..4, after the init phase of both steps."""
    print("pm_repair config 1", flush=True)
    kw = dict(k=3, d=4, n=6, kind=pm.PM_MSR, construction=pm.PM_VANILLA, x=list(range(1, 7)))
    c, o = pm.Code(**kw), _oracle_for(kw)
    X, s = synth.split_object(1 << 20, c.B, synth.CONFIG_SEED + 1)
    P = o.encode(X)
    nodes = {i: o.node_blocks(i, X, P) for i in range(c.n)}
    c.prepare(pm.OP_REPAIR, failed=0, ids=[1, 2, 3, 4])
    _check_repair(c, o, nodes, 0, (1, 2, 3, 4), s)


@pytest.mark.parametrize("f", [0, 8])
def test_repair_configuration_3(f):
    """PM-MBR (8,14,16) on a 64 MiB object: node 0 (its helpers copy one
    block) and node 8 (full projections) from the first 14 survivors."""
    print("pm_repair config 3 f=%d" % f, flush=True)
    kw = dict(k=8, d=14, n=16, kind=pm.PM_MBR)
    c, o = pm.Code(**kw), _oracle_for(kw)
    X, s = synth.split_object(64 << 20, c.B, synth.CONFIG_SEED + 3)
    H = [i for i in range(c.n) if i != f][:c.d]
    c.prepare(pm.OP_REPAIR, failed=f, ids=H)
    P = o.encode(X, nthreads=16)
    nodes = {i: o.node_blocks(i, X, P) for i in H + [f]}
    _check_repair(c, o, nodes, f, tuple(H), s)


def test_repair_msr_16_30_32():
    print("pm_repair (16,30,32)", flush=True)
    kw = dict(k=16, d=30, n=32)
    c, o = pm.Code(**kw), _oracle_for(kw)
    s = 8192 + 48
    X = synth.random_bytes(0x16, c.B * s).reshape(c.B, s)
    P = o.encode(X, nthreads=16)
    f = 20
    H = [i for i in range(c.n) if i not in (f, 3)]
    c.prepare(pm.OP_REPAIR, failed=f, ids=H)
    nodes = {i: o.node_blocks(i, X, P) for i in H + [f]}
    _check_repair(c, o, nodes, f, tuple(H), s)


def test_repair_rejects_overlapping_workspace():
    c = pm.Code(k=4, d=6, n=8)
    s = 4096
    dev = device()
    node = torch.zeros((c.alpha, s), dtype=torch.uint8, device=dev)
    out = torch.zeros((c.alpha, s), dtype=torch.uint8, device=dev)
    need = pm.pm_repair_workspace(c.h, s)
    ws = torch.zeros(need, dtype=torch.uint8, device=dev)
    H = [0, 1, 2, 3, 4, 6]
    # the workspace may not be one of the helper inputs
    st = pm.pm_repair(c.h, 5, H, [ws.data_ptr()] + [node.data_ptr()] * 5, s, ws.data_ptr(), need,
                      out.data_ptr(), s, s)
    assert st == pm.PM_EINVAL
    st = pm.pm_repair(c.h, 5, H, [node.data_ptr()] * 6, s, ws.data_ptr(), need - 16, out.data_ptr(), s, s)
    assert st == pm.PM_EINVAL

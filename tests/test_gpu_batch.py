"""Batched work-list launches: every item equals the oracle and the same
operation run alone; graph replays give the same bytes every time."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_util import device
from paper_1412_3022_amd import pm, synth

pytestmark = pytest.mark.gpu

CODES = [
    ("msr4", dict(k=4, d=6, n=8), (O.MSR, 4, 6, 8, O.SPARSE)),
    ("msr8", dict(k=8, d=14, n=16), (O.MSR, 8, 14, 16, O.SPARSE)),
    ("msr16", dict(k=16, d=30, n=32), (O.MSR, 16, 30, 32, O.SPARSE)),
    ("mbr8", dict(k=8, d=14, n=16, kind=pm.PM_MBR), (O.MBR, 8, 14, 16, O.SPARSE)),
    ("rs", dict(k=8, d=8, n=16, kind=pm.PM_RS), (O.RS, 8, 8, 16, O.SPARSE)),
]


def _mixed_items(seed, count, max_bytes):
    """A seeded mix of encode / helper / newcomer / decode items over the
    codes above, with ragged block sizes; returns (items, expected)."""
    st = synth.Stream(seed)
    codes = {name: (pm.Code(**kw), O.Code(*ok)) for name, kw, ok in CODES}
    names = [c[0] for c in CODES]
    dev = device()
    items, expected = [], []
    for i in range(count):
        name = names[st.below(len(names))]
        c, o = codes[name]
        s = 1 + st.below(max_bytes)
        X = synth.random_bytes(seed * 7919 + i, c.B * s).reshape(c.B, s)
        P = o.encode(X, nthreads=8)
        nodes = {j: o.node_blocks(j, X, P) for j in range(c.n)}
        op = ["encode", "helper", "newcomer", "decode"][st.below(4)]
        ld = (s + 15) // 16 * 16 + 16 * st.below(3)
        if op == "encode":
            inp, want, extra = X, P, {}
        elif op == "helper":
            f = st.below(c.n)
            h = [j for j in range(c.n) if j != f][st.below(c.n - 1)]
            inp = nodes[h][:1] if c.kind == pm.PM_RS else nodes[h]
            want = O.apply(o.helper_row(f), inp)
            extra = {"failed": f}
        elif op == "newcomer":
            f = st.below(c.n)
            H = st.subset(c.n, c.d, exclude=[f])
            inp = np.stack([O.apply(o.helper_row(f), nodes[h])[0] for h in H])
            want = nodes[f]
            extra = {"failed": f, "ids": H}
        else:
            K = st.subset(c.n, c.k)
            inp = np.concatenate([nodes[j] for j in K])
            want = X
            extra = {"ids": K}
        tin = torch.zeros((inp.shape[0], ld), dtype=torch.uint8, device=dev)
        tin[:, :s] = torch.from_numpy(np.ascontiguousarray(inp)).to(dev)
        tout = torch.full((want.shape[0], ld), 0x5A, dtype=torch.uint8, device=dev)
        it = dict(code=c, op=op, inp=tin, out=tout, block_bytes=s, **extra)
        items.append(it)
        expected.append(want)
    return items, expected, codes


def _check(items, expected):
    torch.cuda.synchronize()
    for it, want in zip(items, expected):
        s = it["block_bytes"]
        got = it["out"].cpu().numpy()
        assert np.array_equal(got[:, :s], want), (it["op"], s)
        assert np.all(got[:, s:] == 0x5A)


@pytest.mark.parametrize("vec", [2, 4])
def test_mixed_batch_matches_oracle(vec):
    print("batch vec=%d" % vec, flush=True)
    items, expected, codes = _mixed_items(11, 60, 3000)
    b = pm.Batch(items, graph=False)
    b.set_variant(vec)
    units, classes = b.info()
    assert units > 0 and classes >= 2
    b.run()
    _check(items, expected)


def test_graph_replays_match_every_time():
    print("batch graph replays", flush=True)
    items, expected, codes = _mixed_items(12, 40, 5000)
    b = pm.Batch(items, graph=True)
    for rep in range(4):
        for it in items:
            it["out"].fill_(0x5A)          # eager work between replays
        torch.cuda.synchronize()
        b.run()
        _check(items, expected)


def test_batch_equals_single_calls_after_autotune():
    print("batch autotune", flush=True)
    items, expected, codes = _mixed_items(13, 30, 6000)
    b = pm.Batch(items, graph=True)
    vec = b.autotune(reps=2)
    assert vec in (2, 4)
    for it in items:
        it["out"].fill_(0x5A)
    b.run()
    _check(items, expected)
    # the same operations as single calls
    for it, want in zip(items, expected):
        c, s = it["code"], it["block_bytes"]
        out = torch.full_like(it["out"], 0x5A)
        if it["op"] == "encode":
            c.encode(it["inp"], out, s)
        elif it["op"] == "helper":
            c.repair_helper(it["failed"], it["inp"], out, s)
        elif it["op"] == "newcomer":
            c.repair_newcomer(it["failed"], it["ids"], it["inp"], out, s)
        else:
            c.decode(it["ids"], it["inp"], out, s)
        torch.cuda.synchronize()
        assert torch.equal(out, it["out"])


def test_config4_shape_scaled_down():
    """Configuration-4 shape at reduced total size: 256 objects, sizes
    log-uniform 4 KiB - 256 KiB, codes MSR (4,6), (8,14), (16,30) with n = 2k,
    all encoded in one batch; sampled outputs checked against the oracle."""
    print("config4 scaled", flush=True)
    st = synth.Stream(synth.CONFIG_SEED + 3)
    kinds = [(4, 6), (8, 14), (16, 30)]
    codes = {k: (pm.Code(k=k, d=d, n=2 * k), O.Code(O.MSR, k, d, 2 * k, O.SPARSE)) for k, d in kinds}
    dev = device()
    items, hosts = [], []
    for i in range(256):
        k, d = kinds[st.below(3)]
        c, o = codes[k]
        S = st.log_uniform(4 << 10, 256 << 10)
        X, s = synth.split_object(S, c.B, synth.CONFIG_SEED + 3 + 1000 * (i + 1))
        xin = torch.from_numpy(X).to(dev)
        out = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=dev)
        items.append(dict(code=c, op="encode", inp=xin, out=out, block_bytes=s))
        hosts.append((o, X, s))
    b = pm.Batch(items, graph=True)
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    for it, (o, X, s) in zip(items, hosts):
        pos = np.unique(np.concatenate([rng.integers(0, s, 64), [0, s - 1]]))
        got = it["out"].cpu().numpy()[:, pos]
        assert np.array_equal(got, O.apply(o.enc, X[:, pos]))


def _fixed_pattern_items(seed, count, max_bytes, fams):
    """Items over a few fixed matrices per code (encode, one repair pattern,
    one decode pattern), ragged sizes from 1 byte to max_bytes, so that a
    specialized plan compiles few kernels but runs many region sets."""
    st = synth.Stream(seed)
    dev = device()
    items, expected = [], []
    for i in range(count):
        c, o, f, H, K = fams[st.below(len(fams))]
        s = 1 + st.below(max_bytes) if st.below(4) else 2048 + st.below(16)
        X = synth.random_bytes(seed * 7919 + i, c.B * s).reshape(c.B, s)
        P = o.encode(X, nthreads=8)
        nodes = {j: o.node_blocks(j, X, P) for j in range(c.n)}
        op = ["encode", "helper", "newcomer", "decode"][st.below(4)]
        ld = (s + 15) // 16 * 16 + 16 * st.below(3)
        if op == "encode":
            inp, want, extra = X, P, {}
        elif op == "helper":
            inp = nodes[H[0]]
            want = O.apply(o.helper_row(f), inp)
            extra = {"failed": f}
        elif op == "newcomer":
            inp = np.stack([O.apply(o.helper_row(f), nodes[h])[0] for h in H])
            want = nodes[f]
            extra = {"failed": f, "ids": H}
        else:
            inp = np.concatenate([nodes[j] for j in K])
            want = X
            extra = {"ids": K}
        tin = torch.zeros((inp.shape[0], ld), dtype=torch.uint8, device=dev)
        tin[:, :s] = torch.from_numpy(np.ascontiguousarray(inp)).to(dev)
        tout = torch.full((want.shape[0], ld), 0x5A, dtype=torch.uint8, device=dev)
        items.append(dict(code=c, op=op, inp=tin, out=tout, block_bytes=s, **extra))
        expected.append(want)
    return items, expected


def _fams():
    fams = []
    for kw, ok, f, H, K in [
        (dict(k=4, d=6, n=8), (O.MSR, 4, 6, 8, O.SPARSE), 5, [0, 1, 2, 3, 4, 6], [1, 4, 6, 7]),
        (dict(k=8, d=14, n=16), (O.MSR, 8, 14, 16, O.SPARSE), 9, [0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 11, 12, 13, 14],
         [0, 3, 5, 8, 9, 11, 13, 15]),
    ]:
        fams.append((pm.Code(**kw), O.Code(*ok), f, H, K))
    return fams


def test_specialized_batch_matches_oracle():
    """PM_BATCH_SPECIALIZE: items of >= 2048 bytes run on the multi-set
    bit-sliced kernels (one launch per matrix), shorter ones on the table work
    lists; every item equals the oracle, run after run."""
    print("specialized batch, plain launches", flush=True)
    items, expected = _fixed_pattern_items(21, 48, 12000, _fams())
    assert any(it["block_bytes"] >= 2048 for it in items) and any(it["block_bytes"] < 2048 for it in items)
    plain = pm.Batch(items, graph=False)
    b = pm.Batch(items, graph=False, specialize=True)
    assert b.info()[1] > plain.info()[1]      # bit-sliced launches were added
    for rep in range(2):
        for it in items:
            it["out"].fill_(0x5A)
        torch.cuda.synchronize()
        b.run()
        _check(items, expected)


def test_specialized_batch_graph_replays():
    """The same specialized plan captured in a HIP graph: every replay gives
    the oracle's bytes."""
    print("specialized batch, graph replays", flush=True)
    items, expected = _fixed_pattern_items(22, 40, 12000, _fams())
    b = pm.Batch(items, graph=True, specialize=True)
    for rep in range(3):
        for it in items:
            it["out"].fill_(0x5A)
        torch.cuda.synchronize()
        b.run()
        _check(items, expected)


def test_specialized_batch_after_autotune():
    """The autotuner also times the bit-sliced multi-set launches at half,
    all and twice their resident work-group slots and keeps the fastest:
    after it, graph replays still give the oracle's bytes."""
    print("specialized batch, autotuned slots", flush=True)
    items, expected = _fixed_pattern_items(23, 40, 12000, _fams())
    b = pm.Batch(items, graph=True, specialize=True)
    assert b.autotune(reps=2) in (2, 4)
    for rep in range(2):
        for it in items:
            it["out"].fill_(0x5A)
        torch.cuda.synchronize()
        b.run()
        _check(items, expected)


def test_specialized_k16_encode_single_and_batched():
    """The k = 16 encode network (30 row groups of 8 x 30): its single-set
    kernel through pm_prepare and its multi-set kernel through a specialized
    batch, both against the oracle."""
    print("k16 specialized encode", flush=True)
    c = pm.Code(k=16, d=30, n=32)
    o = O.Code(O.MSR, 16, 30, 32, O.SPARSE)
    assert c.prepare(pm.OP_ENCODE) is True
    dev = device()
    items, expected = [], []
    for i, s in enumerate([2048, 2049, 5000, 3 * 2048 + 16, 20000]):
        X = synth.random_bytes(3100 + i, c.B * s).reshape(c.B, s)
        want = o.encode(X, nthreads=8)
        ld = (s + 15) // 16 * 16
        tin = torch.zeros((c.B, ld), dtype=torch.uint8, device=dev)
        tin[:, :s] = torch.from_numpy(X).to(dev)
        tout = torch.full((c.enc_rows, ld), 0x5A, dtype=torch.uint8, device=dev)
        items.append(dict(code=c, op="encode", inp=tin, out=tout, block_bytes=s))
        expected.append(want)
        single = torch.full_like(tout, 0x5A)
        c.encode(tin, single, s)
        torch.cuda.synchronize()
        got = single.cpu().numpy()
        assert np.array_equal(got[:, :s], want) and np.all(got[:, s:] == 0x5A)
    b = pm.Batch(items, graph=False, specialize=True)
    b.run()
    _check(items, expected)


@pytest.mark.timeout(400)
def test_config4_full_size_in_the_bench_launch_configuration():
    """Configuration 4 as bench.py times it: 4096 objects (log-uniform 64 KiB -
    16 MiB, sparse MSR (4,6), (8,14), (16,30), n = 2k, 12.3 GB of source),
    the encode kernels prepared in both forms, one graph-captured batch with
    autotuned tile width; every object equals its plain single call byte for
    byte, 256 seeded objects' whole 2 KiB tiles and tails equal the oracle,
    and a second replay gives the same bytes."""
    from paper_1412_3022_amd import workloads
    print("config4 full size", flush=True)
    objs, codes, inbuf, outbuf = workloads.batched_objects(4096, 64 << 10, 16 << 20, synth.CONFIG_SEED + 3, device())
    for c in codes.values():
        assert c.prepare(pm.OP_ENCODE) is True
        assert c.prepare(pm.OP_ENCODE, batched=True) is True
    oracles = {k: O.Code(O.MSR, k, c.d, c.n, O.SPARSE) for k, c in codes.items()}
    batch = pm.Batch([dict(code=o["code"], op="encode", inp=o["X"], out=o["P"], block_bytes=o["s"])
                      for o in objs], graph=True)
    batch.autotune(reps=1)
    units, launches = batch.info()
    assert launches == 5, launches      # three multi-set bit-sliced kernels + table kernels for short blocks
    outbuf.fill_(0x5A)
    batch.run()
    torch.cuda.synchronize()
    st = synth.Stream(0xC0F4)
    # every object, every byte, against its own plain single call
    for i, o in enumerate(objs):
        s, c = o["s"], o["code"]
        single = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=device())
        c.encode(o["X"], single, s)
        assert torch.equal(o["P"][:, :s], single), (i, c.k, s)
    # 256 objects against the oracle: whole 2 KiB tiles (first, a seeded
    # middle one, the last window) and the tail, plus scattered bytes
    sample = sorted(set(st.below(len(objs)) for _ in range(256)))
    snap = {}
    for i in sample:
        o = objs[i]
        s, c = o["s"], o["code"]
        s16 = s // 16 * 16
        pos = set(range(0, min(s, 2048))) | set(range(max(0, s - 64), s))
        if s16 >= 2048:
            mid = st.below(s16 // 2048) * 2048
            pos |= set(range(mid, mid + 2048)) | set(range(s16 - 2048, s16))
        pos |= {st.below(s) for _ in range(96)}
        pos = np.array(sorted(pos))
        assert pos.min() >= 0 and pos.max() < s
        X = o["X"][:, pos].cpu().numpy()
        got = o["P"][:, pos].cpu().numpy()
        assert np.array_equal(got, O.apply(oracles[c.k].enc, X, nthreads=16)), (i, c.k, s)
        snap[i] = (pos, got)
    outbuf.fill_(0x33)
    batch.run()
    torch.cuda.synchronize()
    for i in sample:
        pos, got = snap[i]
        assert np.array_equal(objs[i]["P"][:, pos].cpu().numpy(), got), i
    del batch

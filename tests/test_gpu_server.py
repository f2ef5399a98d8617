"""Served mode: every result is the same byte for byte whether the request
runs alone or inside the mix, micro-batches really overlap on the GPU, and
admission never holds more than the HBM budget."""
import time

import numpy as np
import pytest
import torch

from gpu_util import device
from paper_1412_3022_amd import pm, synth, workloads

pytestmark = pytest.mark.gpu


def _result(c, out_blocks, s):
    t = torch.empty((c["out_blocks"], c["out_ld"]), dtype=torch.uint8, device=device())
    pm.copy_device(t.data_ptr(), c["out"], t.numel())
    return t[:, :s]


def _alone(q):
    """The same request as plain single calls."""
    c, s = q["code"], q["block_bytes"]
    dev = device()
    if q["op"] == "encode":
        out = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=dev)
        c.encode(q["X"], out, s)
    elif q["op"] == "decode":
        out = torch.empty((c.B, s), dtype=torch.uint8, device=dev)
        c.decode(q["nodes"], q["Y"], out, s)
    else:
        recv = torch.empty((c.d, s), dtype=torch.uint8, device=dev)
        for j, node in enumerate(q["helper_nodes"]):
            c.repair_helper(q["failed"], node, recv[j:j + 1], s)
        out = torch.empty((c.alpha, s), dtype=torch.uint8, device=dev)
        c.repair_newcomer(q["failed"], q["helpers"], recv, out, s)
    torch.cuda.synchronize()
    return out


def _oracle_of(c):
    import oracle as O
    if c.kind == pm.PM_MBR:
        return O.Code(O.MBR, c.k, c.d, c.n)
    return O.Code(O.MSR, c.k, c.d, c.n, O.SPARSE)


def test_served_mix_equals_alone_and_overlaps():
    """Each served result equals the same request run alone; encodes also
    equal the oracle's encoding in full, repairs the lost node and decodes
    the object."""
    import oracle as O
    print("server mix", flush=True)
    wl = workloads.ServeWorkload(21, device(), 1 << 10, 256 << 10, resident_per_family=2)
    oracles = {c.h: _oracle_of(c) for c in wl.codes.values()}
    reqs, arrivals, nbytes = wl.requests(300, rate_per_s=2e5)
    budget = 32 << 20
    srv = pm.Server(budget, streams=3, max_batch=8)
    try:
        t0 = pm.table_bytes()
        comps = srv.replay(reqs, arrivals, keep=True)
        torch.cuda.synchronize()
        for q, c in zip(reqs, comps):
            assert c["status"] == pm.PM_OK, (q["op"], q["code"].k, q["code"].kind, q["block_bytes"], c["status"],
                                             t0, pm.table_bytes(), srv.stats())
            s = q["block_bytes"]
            got = _result(c, c["out_blocks"], s)
            want = _alone(q)
            assert torch.equal(got, want), (q["op"], s)
            if q["op"] == "repair":
                assert torch.equal(got, q["obj"]["nodes"][q["failed"]])
            elif q["op"] == "decode":
                assert torch.equal(got, q["obj"]["X"])
            else:
                X = q["X"][:, :s].cpu().numpy()
                assert np.array_equal(got.cpu().numpy(), O.apply(oracles[q["code"].h].enc, X, nthreads=8)), s
            srv.release(c["ticket"])
        st = srv.stats()
        assert st["completed"] == len(reqs)
        assert st["max_concurrent_batches"] >= 2, st
        assert st["arena_high_water"] <= budget
        assert st["arena_used"] == 0
        # latencies are ordered timestamps
        for c in comps:
            assert c["t_submit"] <= c["t_admit"] <= c["t_done"]
    finally:
        srv.close()


def test_budget_backpressure_completes_everything():
    print("server budget", flush=True)
    wl = workloads.ServeWorkload(22, device(), 64 << 10, 512 << 10, resident_per_family=1)
    reqs, arrivals, _ = wl.requests(60, rate_per_s=1e6)
    need = max(q["code"].enc_rows if q["op"] == "encode" else
               (q["code"].B if q["op"] == "decode" else q["code"].alpha + q["code"].d)
               for q in reqs) * max(q["block_bytes"] for q in reqs)
    budget = need + (1 << 16)          # arena for about one request at a time
    reserve = 32 << 20                 # plus the kernel tables' part of the budget
    srv = pm.Server(budget + reserve, streams=4, max_batch=4, table_reserve_bytes=reserve)
    try:
        comps = srv.replay(reqs, arrivals, keep=False)
        st = srv.stats()
        assert st["completed"] == len(reqs)
        assert all(c["status"] == pm.PM_OK for c in comps)
        assert st["arena_high_water"] <= budget
        assert st["arena_bytes"] + st["table_reserve_bytes"] <= budget + reserve
        assert st["table_bytes_high"] <= reserve
        assert st["arena_bytes"] + st["table_reserve_bytes"] <= budget + reserve
        assert st["table_bytes_high"] <= reserve
    finally:
        srv.close()


def test_queue_full_and_oversized_requests():
    print("server queue", flush=True)
    dev = device()
    c = pm.Code(k=4, d=6, n=8)
    s = 64 << 10
    X = torch.zeros((c.B, s), dtype=torch.uint8, device=dev)
    reserve = 16 << 20
    srv = pm.Server(c.enc_rows * s + 4096 + reserve, streams=2, max_batch=2, queue_cap=2,
                    table_reserve_bytes=reserve)
    try:
        t0 = srv.submit_encode(c, X, s)
        done = []
        deadline = time.time() + 30
        while not done and time.time() < deadline:
            done = srv.poll()
        assert done and done[0]["ticket"] == t0
        # the first result is held: the next two wait for memory, the third bounces
        assert srv.submit_encode(c, X, s) is not None
        assert srv.submit_encode(c, X, s) is not None
        assert srv.submit_encode(c, X, s) is None          # PM_EBUSY
        srv.release(t0)
        got = []
        deadline = time.time() + 30
        while len(got) < 2 and time.time() < deadline:
            for r in srv.poll():
                got.append(r)
                srv.release(r["ticket"])
        assert len(got) == 2
        big = torch.zeros((c.B, 4 * s), dtype=torch.uint8, device=dev)
        with pytest.raises(pm.PMError) as e:
            srv.submit_encode(c, big, 4 * s)
        assert e.value.status == pm.PM_ENOMEM
    finally:
        srv.close()


def test_served_mix_with_specialized_kernels():
    """With the encode, repair and decode matrices of two families prepared
    for batched use, their requests of >= 2048 bytes run on the multi-set
    bit-sliced kernels inside the micro-batches; every result still equals
    the same request run alone and the object it came from."""
    print("server mix specialized", flush=True)
    wl = workloads.ServeWorkload(33, device(), 1 << 10, 256 << 10, resident_per_family=2)
    for name in ("msr4", "msr8"):
        c = wl.codes[name]
        assert c.prepare(pm.OP_ENCODE, batched=True)
        for obj in wl.resident[name]:
            c.prepare(pm.OP_HELPER, failed=obj["failed"], batched=True)
            c.prepare(pm.OP_NEWCOMER, failed=obj["failed"], ids=obj["helpers"], batched=True)
            c.prepare(pm.OP_DECODE, ids=obj["K"], batched=True)
    reqs, arrivals, nbytes = wl.requests(200, rate_per_s=2e5)
    srv = pm.Server(64 << 20, streams=3, max_batch=8)
    try:
        comps = srv.replay(reqs, arrivals, keep=True)
        torch.cuda.synchronize()
        for q, c in zip(reqs, comps):
            assert c["status"] == pm.PM_OK
            s = q["block_bytes"]
            got = _result(c, c["out_blocks"], s)
            assert torch.equal(got, _alone(q)), (q["op"], s)
            if q["op"] == "repair":
                assert torch.equal(got, q["obj"]["nodes"][q["failed"]])
            elif q["op"] == "decode":
                assert torch.equal(got, q["obj"]["X"])
            srv.release(c["ticket"])
        assert srv.stats()["completed"] == len(reqs)
    finally:
        srv.close()


@pytest.mark.timeout(400)
def test_config5_full_size_in_the_bench_configuration():
    """Configuration 5 as bench.py serves it: the same mix (4 KiB - 64 MiB;
    MSR (4,6), (8,14), (16,30), MBR (8,14)), the same prepared kernels, a
    server of 8 streams x 128 requests; 1500 requests replayed as fast as
    they can be submitted.  Every repair equals the lost node's blocks and
    every decode the object (whole blocks); encodes are checked against the
    oracle on their first 2 KiB tile, their tail and scattered bytes."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    print("config5 full size", flush=True)
    wl = workloads.ServeWorkload(synth.CONFIG_SEED + 4, device(), 4 << 10, 64 << 20, resident_per_family=4)
    jobs = []
    for name, c in wl.codes.items():
        jobs.append((c, pm.OP_ENCODE, 0, None))
        for obj in wl.resident[name]:
            jobs.append((c, pm.OP_HELPER, obj["failed"], None))
            jobs.append((c, pm.OP_NEWCOMER, obj["failed"], obj["helpers"]))
            jobs.append((c, pm.OP_DECODE, 0, obj["K"]))
    with ThreadPoolExecutor(8) as ex:
        list(ex.map(lambda j: j[0].prepare(j[1], failed=j[2], ids=j[3], batched=True), jobs))
    oracles = {}
    for name, c in wl.codes.items():
        oracles[c.h] = O.Code(O.MBR, c.k, c.d, c.n) if c.kind == pm.PM_MBR else O.Code(O.MSR, c.k, c.d, c.n, O.SPARSE)
    reqs, _, _ = wl.requests(1500, rate_per_s=1.0)
    srv = pm.Server(64 * 10**9, streams=8, max_batch=128, queue_cap=1 << 16)
    st = synth.Stream(0xC0F5)
    try:
        comps = srv.replay(reqs, [0] * len(reqs), keep=True)
        torch.cuda.synchronize()
        assert srv.stats()["max_concurrent_batches"] > 1
        for q, c in zip(reqs, comps):
            assert c["status"] == pm.PM_OK
            s = q["block_bytes"]
            got = _result(c, c["out_blocks"], s)
            if q["op"] == "repair":
                assert torch.equal(got, q["obj"]["nodes"][q["failed"]]), s
            elif q["op"] == "decode":
                assert torch.equal(got, q["obj"]["X"]), s
            else:
                # the first 2 KiB wave tile whole, the tail, and scattered bytes
                pos = set(range(min(s, 2048))) | set(range(max(0, s - 64), s))
                pos = np.array(sorted(pos | {st.below(s) for _ in range(32)}))
                X = q["X"][:, pos].cpu().numpy()
                assert np.array_equal(got[:, pos].cpu().numpy(),
                                      O.apply(oracles[q["code"].h].enc, X, nthreads=16)), s
            srv.release(c["ticket"])
    finally:
        srv.close()


def test_failed_table_upload_fails_its_requests_only():
    """A kernel-table upload that fails (forced from the host) completes the
    requests of that micro-batch with PM_ENOMEM instead of reporting success
    for work that never ran; the server keeps serving, and the same request
    submitted again succeeds."""
    print("server upload failure", flush=True)
    dev = device()
    c = pm.Code(k=4, d=6, n=8)
    s = 4096
    X = torch.from_numpy(synth.random_bytes(synth.CONFIG_SEED + 51, c.B * s).reshape(c.B, s)).to(dev)
    P = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=dev)
    c.encode(X, P, s)
    torch.cuda.synchronize()
    nmap = torch.from_numpy(c.node_map().astype(np.int64)).to(dev)
    full = torch.cat([X, P])
    K = [1, 4, 6, 7]                         # a node set no call has decoded yet
    Y = torch.cat([full[nmap[i * c.alpha:(i + 1) * c.alpha]] for i in K]).contiguous()
    srv = pm.Server(256 << 20, streams=2, max_batch=1, table_reserve_bytes=64 << 20)
    try:
        pm.debug_fail_uploads(1)
        t0 = srv.submit_decode(c, K, Y, s)
        got = []
        deadline = time.time() + 30
        while not got and time.time() < deadline:
            got = srv.poll()
        assert got and got[0]["ticket"] == t0
        assert got[0]["status"] == pm.PM_ENOMEM
        srv.release(t0)
        t1 = srv.submit_decode(c, K, Y, s)
        got = []
        deadline = time.time() + 30
        while not got and time.time() < deadline:
            got = srv.poll()
        assert got and got[0]["ticket"] == t1 and got[0]["status"] == pm.PM_OK
        out = _result(got[0], c.B, s)
        assert torch.equal(out, X)
        st = srv.stats()
        assert st["failed"] == 1 and st["completed"] == 2
    finally:
        pm.debug_fail_uploads(0)
        srv.close()


def test_table_reserve_bounds_kernel_tables():
    """Decodes of many node sets of the (16,30,32) code each need their own
    dense 240 x 240 decode tables (over the bit-sliced size limit, so on the
    table kernels); with a reserve smaller than all of them, the server
    evicts least recently used patterns so the tables never exceed the
    reserve, and every decode still returns the object."""
    print("server table reserve", flush=True)
    dev = device()
    c = pm.Code(k=16, d=30, n=32)
    c.set_cache_limit(1024)
    s = 2048
    X = torch.from_numpy(synth.random_bytes(synth.CONFIG_SEED + 52, c.B * s).reshape(c.B, s)).to(dev)
    P = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=dev)
    c.encode(X, P, s)
    torch.cuda.synchronize()
    nmap = torch.from_numpy(c.node_map().astype(np.int64)).to(dev)
    full = torch.cat([X, P])
    rng = synth.Stream(0x7AB1E)
    sets = [sorted(rng.subset(c.n, c.k)) for _ in range(40)]
    Ys = [torch.cat([full[nmap[i * c.alpha:(i + 1) * c.alpha]] for i in K]).contiguous() for K in sets]
    pm.cache_release()
    base = pm.table_bytes()
    reserve = base + (12 << 20)             # room for about ten decode tables
    srv = pm.Server((256 << 20) + reserve, streams=2, max_batch=4, table_reserve_bytes=reserve)
    try:
        tickets = [srv.submit_decode(c, K, Y, s) for K, Y in zip(sets, Ys)]
        assert all(t is not None for t in tickets)
        done = {}
        deadline = time.time() + 120
        while len(done) < len(tickets) and time.time() < deadline:
            for r in srv.poll():
                done[r["ticket"]] = r
        assert len(done) == len(tickets)
        for t in tickets:
            r = done[t]
            assert r["status"] == pm.PM_OK
            assert torch.equal(_result(r, c.B, s), X)
            srv.release(t)
        st = srv.stats()
        assert st["table_bytes_high"] <= reserve, (st, reserve)
        assert st["arena_bytes"] + st["table_reserve_bytes"] <= (256 << 20) + reserve
    finally:
        srv.close()


def test_max_batch_bytes_closes_micro_batches():
    """With a byte limit below any request, every micro-batch takes exactly
    one request; with none, requests share micro-batches.  Results are the
    same either way."""
    print("server max_batch_bytes", flush=True)
    wl = workloads.ServeWorkload(23, device(), 4 << 10, 64 << 10, resident_per_family=1)
    reqs, arrivals, _ = wl.requests(40, rate_per_s=1e7)
    outs = {}
    for cap in (1, 0):
        srv = pm.Server(256 << 20, streams=2, max_batch=16, max_batch_bytes=cap)
        try:
            comps = srv.replay(reqs, [0] * len(reqs), keep=True)
            torch.cuda.synchronize()
            assert all(c["status"] == pm.PM_OK for c in comps)
            outs[cap] = [_result(c, c["out_blocks"], q["block_bytes"]).clone() for q, c in zip(reqs, comps)]
            for c in comps:
                srv.release(c["ticket"])
            st = srv.stats()
            if cap == 1:
                assert st["batches"] == len(reqs), st
            else:
                assert st["batches"] < len(reqs), st
        finally:
            srv.close()
    for a, b in zip(outs[1], outs[0]):
        assert torch.equal(a, b)

#!/usr/bin/env python3
"""Benchmark of the PM regenerating-code hot path on one MI355X.

Headline: GB/s of source bytes for the systematic sparse PM-MSR k=8, d=14,
n=16 encode of a 64 MiB object (56 sub-blocks of 1 198 400 B), one plain
launch per object, inputs resident in HBM.  A step encodes one object; K
steps rotate over 8 buffer sets (1 GiB) so the 256 MB Infinity Cache cannot
serve them.  The kernel's average launch time comes from HIP events on the
launch stream; the roofline figure divides the launch's algorithmic bytes
(read B sub-blocks, write the (n-k) alpha parity sub-blocks) by it.

Beside the headline the JSON line carries the other configuration-2 encodes
(vanilla non-systematic, vanilla systematic, Reed-Solomon), the MBR k=8
encode/repair/decode of configuration 3, and the CPU oracle timed on the host
cores over a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
NBUF = 8
PREWARM_S = 0.3   # untimed launches before the warmup steps of each encode case
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_msr_k8_sparse_encode_64MiB.txt")
CSRC = os.path.join(ROOT, "paper_1412_3022_amd", "csrc")
# the source a kernel's code comes from: the bit-sliced kernel is generated at
# run time by bitslice.cpp, the table kernels are compiled from kernels.hip
BITSLICE_SRC = os.path.join(CSRC, "bitslice.cpp")
TABLE_SRC = os.path.join(CSRC, "kernels.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the headline step is ~30 us: a long warmup brings the shader clock up
    # from idle before timing, and many steps give the sustained rate
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-extra", action="store_true", help="headline only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--sweep", action="store_true", help="print the headline kernel time of every variant")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched and served configurations")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--init-only", action="store_true",
                    help="only run the GPU-side init measurement (batched decode matrices)")
    ap.add_argument("--part", choices=("batched", "served", "served-only", "dense", "gf16", "repair-decode"),
                    help="only run configuration 4 (batched), 5 (served, or served-only without the "
                         "sequential baseline), the other configuration-2 encodes (dense), the GF(2^16) "
                         "codes (gf16) or the repairs and decodes (repair-decode) and print their fields")
    return ap.parse_args()


def calibrate_copy(torch, reps=10):
    """A plain device-to-device copy of known size: its FETCH_SIZE / WRITE_SIZE
    counters convert the engine's counters into HBM bytes."""
    n = 1 << 30
    src = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n, "reps": reps}), flush=True)


def kernel_name(variant):
    """Name of the kernel a (rows per group, dwords per lane) variant runs, as
    rocprofv3 reports it, and the source file its code comes from."""
    rg, vec = variant
    if vec == 32:
        return "pmbs", BITSLICE_SRC
    if vec > 20:
        return "pm_apply_pipe<%d, %d, 16>" % (rg, vec - 20), TABLE_SRC
    if vec > 10:
        return "pm_apply_lds<%d, %d>" % (rg, vec - 10), TABLE_SRC
    return "pm_apply_scalar<%d, %d>" % (rg, vec), TABLE_SRC


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, src):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on this kernel built from the current source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    vals = {}
    with open(PROFILE_TRAFFIC) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel") != kernel or vals.get("source_sha256_16") != source_hash(src):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


_T0 = time.perf_counter()


def progress(msg):
    """One line on stderr per finished stage (the JSON result is the only
    stdout line): a long run shows where it is."""
    print("bench: %s (%.0f s)" % (msg, time.perf_counter() - _T0), file=sys.stderr, flush=True)


class Timer:
    """Wall clock plus HIP events on the stream the kernels run on."""

    def __init__(self, torch):
        self.torch = torch

    def run(self, fn, steps, warmup, prewarm_s=0.0):
        """prewarm_s: before the warmup steps, run steps for at least this
        long (the shader clock ramps up from idle over some 100 ms, more
        than a short --warmup covers)."""
        torch = self.torch
        if prewarm_s > 0:
            t0 = time.perf_counter()
            i = 0
            while True:
                fn(i)
                i += 1
                if i % 64 == 0:
                    torch.cuda.synchronize()
                    if time.perf_counter() - t0 >= prewarm_s:
                        break
        for i in range(warmup):
            fn(i)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for i in range(steps):
            fn(i)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, e0.elapsed_time(e1) / 1e3


def encode_case(torch, pm, synth, kw, S, seed, steps, warmup, nbuf=NBUF, tune=True, sweep=False):
    dev = torch.device("cuda:0")
    code = pm.Code(**kw)
    X, s = synth.split_object(S, code.B, seed)
    xs = [torch.from_numpy(X).to(dev) for _ in range(nbuf)]
    outs = [torch.empty((code.enc_rows, s), dtype=torch.uint8, device=dev) for _ in range(nbuf)]
    stream = torch.cuda.current_stream().cuda_stream
    variant = None
    if sweep:
        for rg, vec in [(rg, vec) for rg in (4, 8, 16) for vec in (2, 4, 12, 14, 22, 24)] + [(8, 32)]:
                code.set_variant(pm.OP_ENCODE, rg, vec)
                def one(i):
                    j = i % nbuf
                    pm.pm_encode(code.h, xs[j].data_ptr(), s, outs[j].data_ptr(), s, s, stream)
                _, ev = Timer(torch).run(one, 40, 4)
                print(json.dumps({"variant": [rg, vec], "kernel_us": round(ev / 40 * 1e6, 2)}), file=sys.stderr,
                      flush=True)
        code.set_variant(pm.OP_ENCODE, 0, 0)
    if tune:
        st, rg, vec = pm.pm_autotune_encode(code.h, xs[0].data_ptr(), s, outs[0].data_ptr(), s, s, 20, stream)
        if st != pm.PM_OK:
            raise pm.PMError(st, "pm_autotune_encode")
        variant = [rg, vec]

    def step(i):
        j = i % nbuf
        st = pm.pm_encode(code.h, xs[j].data_ptr(), s, outs[j].data_ptr(), s, s, stream)
        if st != pm.PM_OK:
            raise pm.PMError(st, "pm_encode")

    wall, ev = Timer(torch).run(step, steps, warmup, prewarm_s=PREWARM_S)
    alg_bytes = (code.B + code.enc_rows) * s
    res = {"source_bytes": S, "block_bytes": s, "wall_s": wall, "event_s": ev,
           "gbps": S * steps / wall / 1e9, "kernel_us": ev / steps * 1e6,
           "alg_bytes_per_launch": alg_bytes, "hbm_gbps": alg_bytes * steps / ev / 1e9, "variant": variant}
    del xs, outs
    return code, res


def prepare_all(code, pm, f, H, K):
    """Init phase of the timed operations (matrices, inverses and their
    bit-sliced kernels), kept out of the data-phase timing as the paper's
    evaluation does; returns its wall time in seconds."""
    t0 = time.perf_counter()
    code.prepare(pm.OP_ENCODE)
    code.prepare(pm.OP_HELPER, failed=f)
    code.prepare(pm.OP_NEWCOMER, failed=f, ids=H)
    code.prepare(pm.OP_DECODE, ids=K)
    return time.perf_counter() - t0


def repair_case(torch, pm, code, node, f, H, reps, prefix, nsets=3):
    """Repair of node f from helpers H, after its init phase: pm_repair (the
    d projections as one multi-set launch, then the newcomer) against one
    pm_repair_helper call per helper and the newcomer, each timed with HIP
    events over `reps` repairs rotating over `nsets` copies of the helper
    blocks (about 160 MB each for the k=8 codes, so the 256 MB Infinity
    Cache cannot serve the next repair's inputs).  GB/s of repaired bytes
    (alpha blocks per repair)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    s = node(H[0]).shape[1]
    t0 = time.perf_counter()
    ready = code.prepare(pm.OP_REPAIR, failed=f, ids=H)
    init_s = time.perf_counter() - t0
    sets = [[node(h).clone() for h in H] for _ in range(nsets)]
    outs = [torch.empty((code.alpha, s), dtype=torch.uint8, device=dev) for _ in range(nsets)]
    ws_bytes = pm.pm_repair_workspace(code.h, s)
    wss = [torch.empty(ws_bytes, dtype=torch.uint8, device=dev) for _ in range(nsets)]
    ptrs = [[t.data_ptr() for t in st] for st in sets]

    def two(i):
        j = i % nsets
        st = pm.pm_repair(code.h, f, H, ptrs[j], s, wss[j].data_ptr(), ws_bytes, outs[j].data_ptr(), s, s, stream)
        if st != pm.PM_OK:
            raise pm.PMError(st, "pm_repair")

    _, ev = Timer(torch).run(two, reps, 4)
    res = {prefix + "_repair_gbps": code.alpha * s * reps / ev / 1e9,
           prefix + "_repair_us": ev / reps * 1e6,
           prefix + "_repair_init_s": init_s,
           prefix + "_repair_one_launch_projections": bool(ready)}
    torch.cuda.synchronize()
    want = node(f)
    res[prefix + "_repair_equal"] = all(bool(torch.equal(o, want)) for o in outs)
    recv = torch.empty((code.d, s), dtype=torch.uint8, device=dev)

    def per_helper(i):
        j = i % nsets
        for q in range(len(H)):
            pm.pm_repair_helper(code.h, f, ptrs[j][q], s, recv[q].data_ptr(), s, stream)
        pm.pm_repair_newcomer(code.h, f, H, recv.data_ptr(), s, outs[j].data_ptr(), s, s, stream)

    _, ev = Timer(torch).run(per_helper, reps, 4)
    res[prefix + "_repair_per_helper_gbps"] = code.alpha * s * reps / ev / 1e9
    del sets, outs, wss
    return res


def mbr_cases(torch, pm, synth, steps, warmup):
    """Configuration 3: PM-MBR (8,14,16), 64 MiB: encode, repair of node 8 from
    14 helpers (helper projections + newcomer solve), decode from a seeded
    random 8-subset, and the specific decode from it and from the parity
    nodes."""
    dev = torch.device("cuda:0")
    code = pm.Code(k=8, d=14, n=16, kind=pm.PM_MBR)
    S = 64 << 20
    X, s = synth.split_object(S, code.B, synth.CONFIG_SEED + 2)
    x = torch.from_numpy(X).to(dev)
    P = torch.empty((code.enc_rows, s), dtype=torch.uint8, device=dev)
    code.encode(x, P, s)
    nm = code.node_map()

    def node(i):
        return torch.stack([x[v] if v < code.B else P[v - code.B] for v in nm[i * code.alpha:(i + 1) * code.alpha]])

    out = {}
    stream = torch.cuda.current_stream().cuda_stream
    f = 8
    H = [i for i in range(code.n) if i != f][:code.d]
    K = synth.Stream(synth.CONFIG_SEED + 2).subset(code.n, code.k)
    out["mbr_init_s"] = prepare_all(code, pm, f, H, K)
    P2 = torch.empty_like(P)
    wall, ev = Timer(torch).run(lambda i: pm.pm_encode(code.h, x.data_ptr(), s, P2.data_ptr(), s, s, stream),
                                steps, warmup)
    out["mbr_encode_gbps"] = S * steps / wall / 1e9
    out.update(repair_case(torch, pm, code, node, f, H, max(20, steps // 20), "mbr"))
    n = max(20, steps // 20)
    Ys = [torch.cat([node(i) for i in K]) for _ in range(2)]
    xos = [torch.empty_like(x) for _ in range(2)]
    _, ev = Timer(torch).run(lambda i: pm.pm_decode(code.h, K, Ys[i % 2].data_ptr(), s, xos[i % 2].data_ptr(), s, s,
                                                    stream), n, 4)
    out["mbr_decode_gbps"] = S * n / ev / 1e9
    out["mbr_decode_nodes"] = K
    xo = xos[0]
    # the specific PM-MBR decode (pm_decode_specific: T, then S) from the same
    # nodes and, beside the linearized decode, from the 8 parity nodes (every
    # data block lost); its init (kernels of both passes) is reported apart
    Kp = list(range(code.k, code.n))
    t0 = time.perf_counter()
    code.prepare(pm.OP_DECODE, ids=Kp)
    ready = all(code.prepare(pm.OP_DECODE_SPECIFIC, ids=KK) for KK in (K, Kp))
    out["mbr_specific_init_s"] = time.perf_counter() - t0
    out["mbr_specific_all_passes_bitsliced"] = bool(ready)
    ws_bytes = pm.pm_decode_specific_workspace(code.h, s)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    equal = True
    for tag, KK in (("", K), ("_parity", Kp)):
        Y = torch.cat([node(i) for i in KK])
        if tag:
            _, ev = Timer(torch).run(
                lambda i: pm.pm_decode(code.h, KK, Y.data_ptr(), s, xo.data_ptr(), s, s, stream), n, 2)
            out["mbr_decode%s_linear_gbps" % tag] = S * n / ev / 1e9
            torch.cuda.synchronize()
            equal = equal and bool(torch.equal(xo, x))
        xo.zero_()
        _, ev = Timer(torch).run(
            lambda i: pm.pm_decode_specific(code.h, KK, Y.data_ptr(), s, xo.data_ptr(), s, s, ws.data_ptr(),
                                            ws_bytes, stream), n, 2)
        out["mbr_decode%s_specific_gbps" % tag] = S * n / ev / 1e9
        torch.cuda.synchronize()
        equal = equal and bool(torch.equal(xo, x))
    out["mbr_decode_results_equal"] = equal
    return out


def msr_repair_decode(torch, pm, synth, steps, warmup):
    """PM-MSR (8,14,16) sparse on the configuration-2 object: repair of node 8
    (full helpers) and decode from a seeded random 8-subset."""
    dev = torch.device("cuda:0")
    code = pm.Code(k=8, d=14, n=16)
    S = 64 << 20
    X, s = synth.split_object(S, code.B, synth.CONFIG_SEED + 1)
    x = torch.from_numpy(X).to(dev)
    P = torch.empty((code.enc_rows, s), dtype=torch.uint8, device=dev)
    code.encode(x, P, s)
    nm = code.node_map()

    def node(i):
        return torch.stack([x[v] if v < code.B else P[v - code.B] for v in nm[i * code.alpha:(i + 1) * code.alpha]])

    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    f = 8
    H = [i for i in range(code.n) if i != f][:code.d]
    K = synth.Stream(synth.CONFIG_SEED + 1).subset(code.n, code.k)
    out["msr_init_s"] = prepare_all(code, pm, f, H, K)
    out.update(repair_case(torch, pm, code, node, f, H, max(20, steps // 20), "msr"))
    n = max(20, steps // 20)
    Ys = [torch.cat([node(i) for i in K]) for _ in range(3)]
    xos = [torch.empty_like(x) for _ in range(3)]
    _, ev = Timer(torch).run(lambda i: pm.pm_decode(code.h, K, Ys[i % 3].data_ptr(), s, xos[i % 3].data_ptr(), s, s,
                                                    stream), n, 4)
    out["msr_decode_gbps"] = S * n / ev / 1e9
    out["msr_decode_nodes"] = K
    torch.cuda.synchronize()
    out["msr_decode_equal"] = all(bool(torch.equal(xo, x)) for xo in xos)
    return out


def msr16_decode_case(torch, pm, synth, steps, warmup):
    """PM-MSR (16,30,32) sparse, 64 MiB object, decoded from the 16 parity
    nodes (every data block lost): the linearized decode (dense 240 x 240
    inverse) against the specific decode (pm_decode_specific, after
    pm_prepare op 4 compiled its passes; that init time is reported apart);
    and the linearized decode from a mixed node set (9 systematic, 7 parity
    nodes: 135 blocks copied, 105 computed)."""
    dev = torch.device("cuda:0")
    code = pm.Code(k=16, d=30, n=32)
    S = 64 << 20
    X, s = synth.split_object(S, code.B, synth.CONFIG_SEED + 6)
    ld = (s + 15) // 16 * 16
    x = torch.zeros((code.B, ld), dtype=torch.uint8, device=dev)
    x[:, :s] = torch.from_numpy(X).to(dev)
    P = torch.empty((code.enc_rows, ld), dtype=torch.uint8, device=dev)
    code.encode(x, P, s)
    nm = code.node_map()
    K = list(range(16, 32))
    Y = torch.stack([x[v] if v < code.B else P[v - code.B] for i in K for v in nm[i * code.alpha:(i + 1) * code.alpha]])
    Y = Y.contiguous()
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    xl = torch.empty_like(x)
    n = max(20, steps // 20)
    _, ev = Timer(torch).run(lambda i: pm.pm_decode(code.h, K, Y.data_ptr(), ld, xl.data_ptr(), ld, s, stream),
                             n, 2)
    out["msr16_decode_linear_gbps"] = S * n / ev / 1e9
    t0 = time.perf_counter()
    ready = code.prepare(pm.OP_DECODE_SPECIFIC, ids=K)
    out["msr16_specific_init_s"] = time.perf_counter() - t0
    progress("(16,30,32) specific decode prepared")
    out["msr16_specific_all_passes_bitsliced"] = bool(ready)
    ws_bytes = pm.pm_decode_specific_workspace(code.h, s)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    xs = torch.empty_like(x)
    _, ev = Timer(torch).run(lambda i: pm.pm_decode_specific(code.h, K, Y.data_ptr(), ld, xs.data_ptr(), ld, s,
                                                             ws.data_ptr(), ws_bytes, stream), n, 2)
    out["msr16_decode_specific_gbps"] = S * n / ev / 1e9
    torch.cuda.synchronize()
    out["msr16_decode_results_equal"] = bool(torch.equal(xs[:, :s], xl[:, :s]) and torch.equal(xs[:, :s], x[:, :s]))
    # a mixed node set (9 systematic, 7 parity): the linearized decode copies
    # the 135 held blocks and computes the 105 lost ones on the matrix cores
    Km = [0, 6, 7, 9, 10, 11, 12, 13, 15, 16, 17, 20, 21, 23, 25, 29]
    Ym = torch.stack([x[v] if v < code.B else P[v - code.B] for i in Km for v in nm[i * code.alpha:(i + 1) * code.alpha]])
    Ym = Ym.contiguous()
    xm = torch.empty_like(x)
    _, ev = Timer(torch).run(lambda i: pm.pm_decode(code.h, Km, Ym.data_ptr(), ld, xm.data_ptr(), ld, s, stream),
                             n, 2)
    out["msr16_decode_mixed_linear_gbps"] = S * n / ev / 1e9
    torch.cuda.synchronize()
    out["msr16_decode_mixed_equal"] = bool(torch.equal(xm[:, :s], x[:, :s]))
    del x, P, Y, xl, xs, ws, Ym, xm
    return out


def dense_config2(torch, pm, synth, S, steps, warmup):
    """The other encodes of configuration 2 on the same 64 MiB object: the
    dense non-systematic vanilla form, the vanilla systematic form (dense
    G'') and RS(16,8); each autotuned, then timed like the headline."""
    codes = [
        ("msr_vanilla_nonsys", dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA,
                                    systematic=False)),
        ("msr_vanilla_sys", dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_VANILLA)),
        ("rs_16_8", dict(k=8, d=8, n=16, kind=pm.PM_RS)),
    ]
    out = {}
    for name, kw in codes:
        _, r = encode_case(torch, pm, synth, kw, S, synth.CONFIG_SEED + 1, max(20, steps // 4),
                           max(2, warmup // 4))
        out[name] = r
    return out


def gf16_cases(torch, pm, synth, steps, warmup):
    """Sparse PM-MSR over GF(2^16) (Section 3.3), 64 MiB objects: systematic
    encode at k = 8 (n = 16) and k = 16 (n = 32), non-systematic encode at
    k = 40 (n = 79, beyond the byte field's range) and k = 64 (n = 127, the
    top of the paper's range), and at k = 8 the repair of node 0 (helper and
    newcomer) and the decode from the last k nodes and from a half-systematic
    node set (its held blocks copied), and at k = 40 and 64 the specific
    decode (and at k = 40 the linearized one) from the last k nodes: on the
    generated bit-sliced kernels where the matrix is under their size limit
    (the *_bitsliced fields; past one kernel's size and within four, as
    several kernels compiled side by side: the k = 16 encode and the k = 8
    decode from the parity nodes), else the GF(2^16) table kernel.  GB/s of
    source bytes (node bytes for repair and decode); init times in seconds."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    S = 64 << 20
    out = {}

    def timed(fn, in_bytes, rows_in, rows_out, s, key):
        def step(i):
            st = fn(i)
            if st != pm.PM_OK:
                raise pm.PMError(st, key)
        wall, ev = Timer(torch).run(step, steps, warmup)
        out[key + "_gbps"] = in_bytes * steps / wall / 1e9
        out[key + "_kernel_us"] = ev / steps * 1e6
        out[key + "_hbm_gbps"] = (rows_in + rows_out) * s * steps / ev / 1e9

    for k, n, sys_ in ((8, 16, True), (16, 32, True), (40, 79, False), (64, 127, False)):
        code = pm.Code(k=k, d=2 * k - 2, n=n, systematic=sys_, w=16)
        s = synth.block_bytes_for(S, code.B)
        xs = [synth.random_bytes_torch(0x1600 + k + j, code.B * s, dev).view(code.B, s) for j in range(NBUF)]
        outs = [torch.empty((code.enc_rows, s), dtype=torch.uint8, device=dev) for _ in range(NBUF)]
        key = "gf16_k%d_%s_encode" % (k, "sys" if sys_ else "nonsys")
        t0 = time.time()
        out[key + "_bitsliced"] = code.prepare(pm.OP_ENCODE)
        out[key + "_init_s"] = time.time() - t0   # generation and hipRTC compile of the bit-sliced kernel
        progress("GF(2^16) k=%d encode prepared" % k)
        timed(lambda i: pm.pm_encode(code.h, xs[i % NBUF].data_ptr(), s, outs[i % NBUF].data_ptr(), s, s, stream),
              code.B * s, code.B, code.enc_rows, s, key)
        if k == 8:
            f, H, K = 0, list(range(1, 15)), list(range(8, 16))
            node = torch.empty((code.alpha, s), dtype=torch.uint8, device=dev)
            recv = torch.empty((code.d, s), dtype=torch.uint8, device=dev)
            rep_out = torch.empty((code.alpha, s), dtype=torch.uint8, device=dev)
            Y = torch.empty((code.B, s), dtype=torch.uint8, device=dev)
            code.prepare(pm.OP_HELPER, failed=f)
            out["gf16_k8_newcomer_bitsliced"] = code.prepare(pm.OP_NEWCOMER, failed=f, ids=H)
            out["gf16_k8_decode_bitsliced"] = code.prepare(pm.OP_DECODE, ids=K)
            progress("GF(2^16) k=8 repair and decodes prepared")
            timed(lambda i: pm.pm_repair_helper(code.h, f, node.data_ptr(), s, recv.data_ptr(), s, stream),
                  code.alpha * s, code.alpha, 1, s, "gf16_k8_helper")
            timed(lambda i: pm.pm_repair_newcomer(code.h, f, H, recv.data_ptr(), s, rep_out.data_ptr(), s, s,
                                                  stream), code.d * s, code.d, code.alpha, s, "gf16_k8_newcomer")
            timed(lambda i: pm.pm_decode(code.h, K, Y.data_ptr(), s, xs[i % NBUF].data_ptr(), s, s, stream),
                  code.B * s, code.B, code.B, s, "gf16_k8_decode")
            # half the nodes systematic: their blocks are copied, the lost half computed
            Km = [0, 1, 2, 3, 12, 13, 14, 15]
            out["gf16_k8_decode_mixed_bitsliced"] = code.prepare(pm.OP_DECODE, ids=Km)
            timed(lambda i: pm.pm_decode(code.h, Km, Y.data_ptr(), s, xs[i % NBUF].data_ptr(), s, s, stream),
                  code.B * s, code.B, code.B, s, "gf16_k8_decode_mixed")
        if k >= 40:
            # decode from the last k nodes: the specific decoder (Section 4.1;
            # factors need only alpha x alpha inverses) and, at k = 40, the
            # linearized one (a B x B inverse on the host, 2 s; 30 s at k = 64)
            K = list(range(n - k, n))
            Y = torch.empty((code.B, s), dtype=torch.uint8, device=dev)
            ws = torch.empty(pm.pm_decode_specific_workspace(code.h, s), dtype=torch.uint8, device=dev)
            t0 = time.time()
            code.prepare(pm.OP_DECODE_SPECIFIC, ids=K)
            out["gf16_k%d_specific_decode_init_s" % k] = time.time() - t0
            timed(lambda i: pm.pm_decode_specific(code.h, K, Y.data_ptr(), s, xs[i % NBUF].data_ptr(), s, s,
                                                  ws.data_ptr(), ws.numel(), stream),
                  code.B * s, code.B, code.B, s, "gf16_k%d_specific_decode" % k)
            if k == 40:
                t0 = time.time()
                code.prepare(pm.OP_DECODE, ids=K)
                out["gf16_k40_linear_decode_init_s"] = time.time() - t0
                timed(lambda i: pm.pm_decode(code.h, K, Y.data_ptr(), s, xs[i % NBUF].data_ptr(), s, s, stream),
                      code.B * s, code.B, code.B, s, "gf16_k40_linear_decode")
            del Y, ws
        del xs, outs
    return out


def gpu_init_case(torch, pm, synth):
    """GPU-side init (pm_decode_matrices, batched Gauss-Jordan): the decode
    matrices of every 8-subset of the 16 nodes of the (8,14,16) sparse MSR
    code in one launch, 1024 seeded node sets of the (16,30,32) code and
    2048 of the (8,14,16) MBR code; the library's host init of the same
    matrices (pm_decode_matrix, one thread) timed on a sample of the sets,
    and that sample compared with the GPU's matrices."""
    import itertools
    dev = torch.device("cuda:0")
    out = {}
    cases = [("msr8_all", dict(k=8, d=14, n=16), None, 200),
             ("msr16", dict(k=16, d=30, n=32), 1024, 8),
             ("mbr8", dict(k=8, d=14, n=16, kind=pm.PM_MBR), 2048, 100)]
    equal = True
    for name, kw, nsets, nsample in cases:
        code = pm.Code(**kw)
        if nsets is None:
            sets = [list(K) for K in itertools.combinations(range(code.n), code.k)]
        else:
            st = synth.Stream(synth.CONFIG_SEED + 7)
            sets = [st.subset(code.n, code.k) for _ in range(nsets)]
        S = torch.tensor(sets, dtype=torch.int32, device=dev)
        D, kept, status = code.decode_matrices(S)          # uploads the generator
        _, ev = Timer(torch).run(lambda i: code.decode_matrices(S), 5, 1)
        out["init_%s_sets" % name] = len(sets)
        out["init_%s_gpu_ms" % name] = ev / 5 * 1e3
        out["init_%s_gpu_sets_per_s" % name] = len(sets) * 5 / ev
        idx = synth.Stream(synth.CONFIG_SEED + 8).subset(len(sets), nsample)
        t0 = time.perf_counter()
        want = [code.decode_matrix(sets[i])[0] for i in idx]
        host = time.perf_counter() - t0
        out["init_%s_host_sets_per_s" % name] = nsample / host
        Dc, stc = D.cpu().numpy(), status.cpu().numpy()
        equal = equal and bool((stc == 0).all()) and all((Dc[i] == w).all() for i, w in zip(idx, want))
        del D, kept, status, S
    out["init_gpu_matches_host_sample"] = equal
    return out


def batched_case(torch, pm, synth, steps):
    """Configuration 4: 4096 objects, sizes log-uniform 64 KiB - 16 MiB,
    sparse PM-MSR (4,6), (8,14), (16,30), n = 2k, all encoded by one
    graph-captured batch (tile width and bit-sliced work-group slots autotuned;
    untuned_batched_gbps: the defaults), against one plain pm_encode
    launch per object on the same stream."""
    from paper_1412_3022_amd import workloads
    dev = torch.device("cuda:0")
    objs, codes, inbuf, outbuf = workloads.batched_objects(4096, 64 << 10, 16 << 20, synth.CONFIG_SEED + 3, dev)
    src = sum(o["S"] for o in objs)
    stream = torch.cuda.current_stream().cuda_stream
    # init phase, outside both timings: the bit-sliced encode kernels of the
    # three codes, single-set for the plain calls and multi-set for the batch
    t0 = time.perf_counter()
    for c in codes.values():
        c.prepare(pm.OP_ENCODE)
        c.prepare(pm.OP_ENCODE, batched=True)
    init_s = time.perf_counter() - t0
    # plain: one launch per object
    def plain(i):
        for o in objs:
            st = pm.pm_encode(o["code"].h, o["X"].data_ptr(), o["s"], o["P"].data_ptr(), o["s"], o["s"], stream)
            if st != pm.PM_OK:
                raise pm.PMError(st, "pm_encode")
    wall_plain, ev_plain = Timer(torch).run(plain, 2, 1)
    batch = pm.Batch([dict(code=o["code"], op="encode", inp=o["X"], out=o["P"], block_bytes=o["s"])
                      for o in objs], graph=True)   # uses the prepared multi-set kernels
    wall_u, _ = Timer(torch).run(lambda i: batch.run(), steps, 2)   # default tile widths and slots
    vec = batch.autotune(reps=2)
    units, classes = batch.info()
    wall_b, ev_b = Timer(torch).run(lambda i: batch.run(), steps, 2)
    res = {"objects": len(objs), "source_bytes": src, "plain_gbps": round(src * 2 / wall_plain / 1e9, 2),
           "batched_gbps": round(src * steps / wall_b / 1e9, 2),
           "untuned_batched_gbps": round(src * steps / wall_u / 1e9, 2),
           "batched_ms_per_run": round(wall_b / steps * 1e3, 3), "plain_ms_per_pass": round(wall_plain / 2 * 1e3, 3),
           "batch_units": units, "launches": classes, "tuned_dwords_per_lane": vec,
           "init_s": round(init_s, 2)}
    del batch, objs, inbuf, outbuf
    torch.cuda.synchronize()
    return res


def served_case(torch, pm, synth, nreq=20000, rho=0.8, sequential=True, streams=8, max_batch=128,
                max_batch_bytes=0):
    """Configuration 5: a Poisson stream of 20 000 requests (70% encode, 20%
    single-node repair, 10% k-subset decode; sizes log-uniform 4 KiB - 64 MiB;
    PM-MSR (4,6), (8,14), (16,30) and PM-MBR (8,14,16)) served under a 64 GB
    HBM budget.  The server's capacity on this mix is measured first with
    every request queued at once; the Poisson stream is then offered at rho
    times that capacity, and the same requests are also run one after another
    as plain single calls."""
    import numpy as np
    from paper_1412_3022_amd import workloads
    dev = torch.device("cuda:0")
    wl = workloads.ServeWorkload(synth.CONFIG_SEED + 4, dev, 4 << 10, 64 << 20, resident_per_family=4)
    # init phase: the bit-sliced encode kernels of every family (multi-set for
    # the server, single-set for the sequential plain calls) and the
    # multi-set repair (helper, newcomer) and decode kernels of every
    # resident object's failure pattern (dense k = 16 decodes are over the
    # size limit and stay on the table kernels, as do repairs and decodes in
    # the sequential plain calls).  hipRTC compiles on a thread pool.
    from concurrent.futures import ThreadPoolExecutor
    jobs = []
    for name, c in wl.codes.items():
        jobs.append((c, pm.OP_ENCODE, 0, None, False))
        jobs.append((c, pm.OP_ENCODE, 0, None, True))
        for obj in wl.resident[name]:
            jobs.append((c, pm.OP_HELPER, obj["failed"], None, True))
            jobs.append((c, pm.OP_NEWCOMER, obj["failed"], obj["helpers"], True))
            jobs.append((c, pm.OP_DECODE, 0, obj["K"], True))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(8) as ex:
        list(ex.map(lambda j: j[0].prepare(j[1], failed=j[2], ids=j[3], batched=j[4]), jobs))
    init_s = time.perf_counter() - t0
    progress("served: init done")
    budget = 64 * 10**9
    # 8 micro-batches in flight of up to 128 requests: on a 3 000-request
    # replay of this mix, 4 x 64 gave 0.54 TB/s, 8 x 64 0.72, 8 x 128 0.81,
    # 12 or 16 streams no more
    srv = pm.Server(budget, streams=streams, max_batch=max_batch, queue_cap=1 << 16, max_batch_bytes=max_batch_bytes)

    def span(comps, nbytes):
        t0 = min(c["t_submit"] for c in comps)
        t1 = max(c["t_done"] for c in comps)
        return float(sum(nbytes)) / ((t1 - t0) / 1e9) / 1e9

    sat, _, sat_bytes = wl.requests(nreq // 4, rate_per_s=1.0)
    # warm-up: one untimed pass over the same requests (device copies of
    # every program and table the mix touches are uploaded on first use)
    srv.replay(sat, [0] * len(sat))
    torch.cuda.synchronize()
    capacity = span(srv.replay(sat, [0] * len(sat)), sat_bytes)
    progress("served: capacity %.0f GB/s" % capacity)
    mean_bytes = float(np.mean(sat_bytes))
    rate = rho * capacity * 1e9 / mean_bytes
    reqs, arrivals, nbytes = wl.requests(nreq, rate_per_s=rate)
    srv.replay(reqs[:200], [0] * 200)
    torch.cuda.synchronize()
    comps = srv.replay(reqs, arrivals)
    stats = srv.stats()
    srv.close()
    lat = np.array([(c["t_done"] - c["t_submit"]) / 1e3 for c in comps])
    served = span(comps, nbytes)
    res = {"requests": nreq, "capacity_gbps": round(capacity, 2), "offered_rho": rho,
           "offered_rate_per_s": round(rate, 1), "mean_request_bytes": round(mean_bytes),
           "served_gbps": round(served, 2),
           "p50_us": round(float(np.percentile(lat, 50)), 1), "p99_us": round(float(np.percentile(lat, 99)), 1),
           "max_concurrent_batches": stats["max_concurrent_batches"], "batches": stats["batches"],
           "launch_host_us_per_batch": round(stats["launch_host_ns"] / max(stats["batches"], 1) / 1e3, 1),
           "failed": stats["failed"], "init_s": round(init_s, 2),
           "arena_high_water_bytes": stats["arena_high_water"], "hbm_budget_bytes": budget,
           "table_bytes_high": stats["table_bytes_high"], "table_reserve_bytes": stats["table_reserve_bytes"],
           "bytes_counted": "encode and decode: object bytes; repair: the alpha repaired blocks"}
    if not sequential:
        return res
    # the same requests as plain single calls, one after another
    stream = torch.cuda.current_stream().cuda_stream
    scratch = torch.empty(max(q["code"].d * q["block_bytes"] for q in reqs if q["op"] == "repair") + 256,
                          dtype=torch.uint8, device=dev)
    outb = torch.empty(max((q["code"].enc_rows if q["op"] == "encode" else q["code"].B) * q["block_bytes"]
                           for q in reqs) + 256, dtype=torch.uint8, device=dev)

    def seq(_):
        for q in reqs:
            c, s = q["code"], q["block_bytes"]
            if q["op"] == "encode":
                pm.pm_encode(c.h, q["X"].data_ptr(), s, outb.data_ptr(), s, s, stream)
            elif q["op"] == "decode":
                pm.pm_decode(c.h, q["nodes"], q["Y"].data_ptr(), s, outb.data_ptr(), s, s, stream)
            else:
                for j, node in enumerate(q["helper_nodes"]):
                    pm.pm_repair_helper(c.h, q["failed"], node.data_ptr(), node.stride(0),
                                        scratch.data_ptr() + j * s, s, stream)
                pm.pm_repair_newcomer(c.h, q["failed"], q["helpers"], scratch.data_ptr(), s, outb.data_ptr(), s,
                                      s, stream)
    wall_seq, _ = Timer(torch).run(seq, 1, 0)
    res["sequential_plain_gbps"] = round(float(sum(nbytes)) / wall_seq / 1e9, 2)
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(synth, budget_s=12.0):
    """The oracle (plain log/antilog C) on the host cores: the same encode on
    a bounded sample -- the first `w` bytes of every sub-block of the
    configuration-2 object -- with one thread (the paper measures one core)
    and with every host thread (at most 16), each repeated to about
    budget_s / 2 of CPU time."""
    import numpy as np
    import oracle as O
    code = O.Code(O.MSR, 8, 14, 16, O.SPARSE)
    X, s = synth.split_object(64 << 20, code.B, synth.CONFIG_SEED + 1)

    def run(threads, budget):
        w = 4096
        while True:
            sample = np.ascontiguousarray(X[:, :w])
            t0 = time.perf_counter()
            O.apply(code.enc, sample, nthreads=threads)
            dt = time.perf_counter() - t0
            if dt * threads > budget / 8 or w >= s:
                break
            w = min(s, w * 2)
        reps = 1
        while dt * threads < budget and reps < 64:
            reps *= 2
            t0 = time.perf_counter()
            for _ in range(reps):
                O.apply(code.enc, sample, nthreads=threads)
            dt = time.perf_counter() - t0
        return code.B * w * reps / dt / 1e9, w, reps, dt

    threads = min(os.cpu_count() or 1, 16)
    one, w1, r1, t1 = run(1, budget_s / 2)
    allc, w, reps, dt = run(threads, budget_s / 2)
    return {"value": allc, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "one_thread_value": one, "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "sample": "first %d B of each of the 56 sub-blocks of the 64 MiB object, encoded %d times "
                      "(%d source bytes), sparse systematic k=8 encode, %.2f s wall on %d threads; "
                      "one thread: first %d B x 56, %d times, %.2f s"
                      % (w, reps, code.B * w * reps, dt, threads, w1, r1, t1)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(objects and byte ranges split across GPUs with no exchange).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1412_3022_amd import pm, synth
    if not torch.cuda.is_available():
        print("no ROCm GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy(torch)
        return
    pm.lib()
    if args.init_only:
        print(json.dumps({k: (round(v, 3) if isinstance(v, float) else v)
                          for k, v in gpu_init_case(torch, pm, synth).items()}), flush=True)
        return
    if args.part == "batched":
        print(json.dumps({"batched": batched_case(torch, pm, synth, max(5, args.steps // 20))}), flush=True)
        return
    if args.part in ("served", "served-only"):
        # served-only: the server alone (no sequential plain-call baseline),
        # for profiles of the served kernels
        print(json.dumps({"served": served_case(torch, pm, synth, sequential=args.part == "served")}), flush=True)
        return
    if args.part == "gf16":
        print(json.dumps({k: (round(v, 2) if isinstance(v, float) else v)
                          for k, v in gf16_cases(torch, pm, synth, args.steps, args.warmup).items()}),
              flush=True)
        return
    if args.part == "repair-decode":
        out = {}
        for fn in (msr_repair_decode, mbr_cases, msr16_decode_case):
            out.update(fn(torch, pm, synth, args.steps, args.warmup))
        print(json.dumps({k: (round(v, 3) if isinstance(v, float) else v) for k, v in out.items()}), flush=True)
        return
    if args.part == "dense":
        res = dense_config2(torch, pm, synth, 64 << 20, args.steps, args.warmup)
        print(json.dumps({name: {"gbps": round(r["gbps"], 2), "kernel_us": round(r["kernel_us"], 3),
                                 "variant": r["variant"], "alg_bytes_per_launch": r["alg_bytes_per_launch"]}
                          for name, r in res.items()}), flush=True)
        return

    S = 64 << 20
    head_kw = dict(k=8, d=14, n=16, kind=pm.PM_MSR, construction=pm.PM_SPARSE)
    code, head = encode_case(torch, pm, synth, head_kw, S, synth.CONFIG_SEED + 1, args.steps, args.warmup,
                             sweep=args.sweep)
    extra = {"headline_kernel_us": round(head["kernel_us"], 3), "headline_variant": head["variant"],
             "headline_event_gbps": round(S / (head["kernel_us"] * 1e-6) / 1e9, 2)}
    progress("headline encode done")
    if not args.no_extra:
        for name, r in dense_config2(torch, pm, synth, S, args.steps, args.warmup).items():
            extra[name + "_encode_gbps"] = round(r["gbps"], 2)
            extra[name + "_variant"] = r["variant"]
        progress("dense encodes done")
        for fn, digits in ((msr_repair_decode, 2), (mbr_cases, 2), (msr16_decode_case, 2)):
            extra.update({k: (round(v, digits) if isinstance(v, float) else v)
                          for k, v in fn(torch, pm, synth, args.steps, args.warmup).items()})
            progress(fn.__name__ + " done")
        extra.update({k: (round(v, 3) if isinstance(v, float) else v)
                      for k, v in gpu_init_case(torch, pm, synth).items()})
        progress("GPU-side init done")
        extra.update({k: (round(v, 2) if isinstance(v, float) else v)
                      for k, v in gf16_cases(torch, pm, synth, args.steps, args.warmup).items()})
        progress("GF(2^16) cases done")
    batched = served = None
    if not args.no_batch:
        batched = batched_case(torch, pm, synth, max(5, args.steps // 20))
        progress("batched done")
        served = served_case(torch, pm, synth)
        progress("served done")
        # the same mix with micro-batches closed at 64 MiB of results: lower
        # latency, lower capacity (the server's per-micro-batch host work)
        served["latency_config"] = served_case(torch, pm, synth, sequential=False, max_batch_bytes=64 << 20)
        served["latency_config"]["max_batch_bytes"] = 64 << 20
        progress("served (64 MiB micro-batches) done")

    achieved = head["alg_bytes_per_launch"] / (head["kernel_us"] * 1e-6) / 1e9
    kname, ksrc = kernel_name(head["variant"])
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(kname, ksrc),
            "kernel": kname, "alg_bytes_per_launch": head["alg_bytes_per_launch"]}
    line = {
        "metric": "encode GB/s (source bytes) PM-MSR k=8 d=14 at 1 GPU; batched vs plain; serve p50/p99",
        "value": round(head["gbps"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["wall_s"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (splitmix64 uniform bytes, seed 0x5EED0001)",
        "config": {"workload": "PM-MSR sparse systematic encode k=8 d=14 n=16 GF(2^8), 64 MiB object "
                               "as 56 x 1198400 B sub-blocks, plain single launch per object",
                   "source_bytes_per_step": S, "buffer_sets": NBUF},
        "roofline": roof,
        "batched": batched,
        "served": served,
        "extra": extra,
        "paper_context": {"sparse_sys_k8_MBps": 790, "vanilla_sys_k8_MBps": 210, "rs_k8_MBps": 1640,
                          "cpu": "Xeon E5-2640 2.5 GHz, 1 core, 16 KB blocks"},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(synth)
        progress("CPU baseline done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

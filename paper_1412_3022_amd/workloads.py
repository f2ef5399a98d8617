"""Seeded synthetic workloads of the batched and served configurations.

Batched: many objects of log-uniform size, each drawn from the sparse
systematic PM-MSR codes (k, d) in {(4,6), (8,14), (16,30)} with n = 2k, all
encoded together.  Served: a Poisson stream of encode / single-node repair /
k-subset decode requests over PM-MSR (4,6), (8,14), (16,30) and PM-MBR
(8,14,16); repairs and decodes address objects kept resident on the device.

Object bytes come from the splitmix64 stream of ``synth`` (generated on the
device); every choice (code, size, failed node, helper set, node set,
arrival gap) is drawn from seeded splitmix64 streams.  Nothing here computes
any of the coding arithmetic: resident objects are encoded by the engine.
"""
from __future__ import annotations

import torch

from . import pm, synth

BATCH_CODES = [(4, 6), (8, 14), (16, 30)]
SERVE_FAMILIES = [
    ("msr4", dict(k=4, d=6, n=8)),
    ("msr8", dict(k=8, d=14, n=16)),
    ("msr16", dict(k=16, d=30, n=32)),
    ("mbr8", dict(k=8, d=14, n=16, kind=pm.PM_MBR)),
]


def batched_objects(count, lo, hi, seed, device, codes=None):
    """`count` objects with sizes log-uniform in [lo, hi] bytes.  Returns
    (objects, codes, in_buffer, out_buffer); each object is a dict with code,
    S (source bytes), s (block bytes), X (B x s view) and P (enc_rows x s view)."""
    st = synth.Stream(seed)
    codes = codes or {k: pm.Code(k=k, d=d, n=2 * k) for k, d in BATCH_CODES}
    specs = []
    for _ in range(count):
        k, _d = BATCH_CODES[st.below(len(BATCH_CODES))]
        S = st.log_uniform(lo, hi)
        c = codes[k]
        specs.append((c, S, synth.block_bytes_for(S, c.B)))
    in_total = sum(c.B * s for c, _, s in specs)
    out_total = sum(c.enc_rows * s for c, _, s in specs)
    inbuf = synth.random_bytes_torch(seed, in_total, device)
    outbuf = torch.empty(out_total, dtype=torch.uint8, device=device)
    objects, io, oo = [], 0, 0
    for c, S, s in specs:
        X = inbuf[io:io + c.B * s].view(c.B, s)
        X.view(-1)[S:].zero_()          # the object is zero padded to B s bytes
        P = outbuf[oo:oo + c.enc_rows * s].view(c.enc_rows, s)
        objects.append(dict(code=c, S=S, s=s, X=X, P=P))
        io += c.B * s
        oo += c.enc_rows * s
    return objects, codes, inbuf, outbuf


class ServeWorkload:
    """Resident objects and a seeded request stream for the served mode."""

    def __init__(self, seed, device, size_lo, size_hi, resident_per_family=4, pool_bytes=None):
        self.device = device
        self.st = synth.Stream(seed)
        self.size_lo, self.size_hi = size_lo, size_hi
        self.codes = {name: pm.Code(**kw) for name, kw in SERVE_FAMILIES}
        self.names = [n for n, _ in SERVE_FAMILIES]
        max_B = max(c.B for c in self.codes.values())
        pool = pool_bytes or (2 * size_hi + 64 * max_B + (1 << 20))
        self.pool = synth.random_bytes_torch(seed ^ 0x5EED, pool, device)
        self.resident = {n: [self._make_resident(n, seed * 131 + 17 * i + j)
                             for j in range(resident_per_family)]
                         for i, n in enumerate(self.names)}

    def _make_resident(self, name, seed):
        c = self.codes[name]
        S = self.st.log_uniform(self.size_lo, self.size_hi)
        s = synth.block_bytes_for(S, c.B)
        X = synth.random_bytes_torch(seed, c.B * s, self.device).view(c.B, s)
        X.view(-1)[S:].zero_()
        P = torch.empty((c.enc_rows, s), dtype=torch.uint8, device=self.device)
        c.encode(X, P, s)
        nm = c.node_map()
        nodes = [torch.stack([X[v] if v < c.B else P[v - c.B] for v in nm[i * c.alpha:(i + 1) * c.alpha]])
                 for i in range(c.n)]
        f = self.st.below(c.n)
        H = self.st.subset(c.n, c.d, exclude=[f])
        K = self.st.subset(c.n, c.k)
        Y = torch.cat([nodes[i] for i in K]).contiguous()
        return dict(code=c, name=name, S=S, s=s, X=X, nodes=nodes, failed=f, helpers=H, K=K, Y=Y)

    def _encode_input(self, c, S):
        s = synth.block_bytes_for(S, c.B)
        room = self.pool.numel() - c.B * s
        off = (self.st.below(max(1, room // 256)) * 256) if room > 0 else 0
        return self.pool[off:off + c.B * s].view(c.B, s), s

    def requests(self, count, rate_per_s, mix=(0.7, 0.2, 0.1)):
        """count requests; returns (requests, arrival_ns, source_bytes)."""
        reqs, arrivals, nbytes = [], [], []
        t = 0.0
        for _ in range(count):
            t += self.st.exponential(rate_per_s)
            arrivals.append(int(t * 1e9))
            u = self.st.uniform()
            name = self.names[self.st.below(len(self.names))]
            c = self.codes[name]
            if u < mix[0]:
                S = self.st.log_uniform(self.size_lo, self.size_hi)
                X, s = self._encode_input(c, S)
                reqs.append(dict(op="encode", code=c, X=X, block_bytes=s, S=S))
                nbytes.append(S)
            elif u < mix[0] + mix[1]:
                obj = self.resident[name][self.st.below(len(self.resident[name]))]
                reqs.append(dict(op="repair", code=c, failed=obj["failed"], helpers=obj["helpers"],
                                 helper_nodes=[obj["nodes"][h] for h in obj["helpers"]],
                                 block_bytes=obj["s"], obj=obj))
                nbytes.append(c.alpha * obj["s"])
            else:
                obj = self.resident[name][self.st.below(len(self.resident[name]))]
                reqs.append(dict(op="decode", code=c, nodes=obj["K"], Y=obj["Y"], block_bytes=obj["s"], obj=obj))
                nbytes.append(obj["S"])
        return reqs, arrivals, nbytes

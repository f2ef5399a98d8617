"""The batched GF(2^8) Gauss-Jordan kernel (csrc/gj.hip) run on the host.

Its own source, with host stand-ins (emu/gj_main.cpp: one OS thread per GPU
thread, barriers, an LDS block of exactly the kernel's size under
AddressSanitizer), computes decode matrices from the library's generator
rows for node sets, and inverses of caller matrices; every result is checked
against the oracle's decode matrices (Section 2: X = inverse(G~) Y~, the
first independent rows in order for MBR) and inverses."""
import os
import struct
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1412_3022_amd import pm, synth

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1412_3022_amd", "csrc")
SHARED = "extern __shared__ __align__(16) unsigned char sm[];"


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("gj")
    hdr = open(os.path.join(CSRC, "gj.hpp")).read().replace("#include <hip/hip_runtime.h>", "")
    src = open(os.path.join(CSRC, "gj.hip")).read()
    assert SHARED in src and '#include "gj.hpp"' in src
    src = src.replace('#include "gj.hpp"', hdr).replace(SHARED, "unsigned char *sm = g_sm;")
    with open(d / "gj_kernel.inc", "w") as f:
        f.write(src)
    out = str(d / "gj_main")
    subprocess.check_call(["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
                           "-pthread", "-I", str(d), os.path.join(HERE, "emu", "gj_main.cpp"), "-o", out])
    return out


def run(exe, tmp_path, src, B, nrows, src_ld, src_stride, count, sets=None, nsets=0, alpha=1, nnodes=0):
    d_ld, d_stride = B, B * B
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    src = np.ascontiguousarray(src, dtype=np.uint8).reshape(-1)
    with open(inp, "wb") as f:
        f.write(struct.pack("<12Q", count, B, nrows, nsets, alpha, nnodes, src_ld, src_stride, d_ld, d_stride,
                            1 if sets is not None else 0, src.size))
        f.write(src.tobytes())
        if sets is not None:
            f.write(np.ascontiguousarray(sets, dtype=np.uint32).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    subprocess.check_call([exe, str(inp), str(outp)], env=env, timeout=600)
    raw = open(outp, "rb").read()
    D = np.frombuffer(raw[:count * d_stride], np.uint8).reshape(count, B, B)
    kept = np.frombuffer(raw[count * d_stride:count * d_stride + 4 * count * B], np.uint32).reshape(count, B)
    st = np.frombuffer(raw[count * d_stride + 4 * count * B:], np.int32)
    return D, kept, st


CODES = [
    ("msr-cfg1", dict(k=3, d=4, n=6, construction=pm.PM_VANILLA, x=list(range(1, 7))),
     (O.MSR, 3, 4, 6, O.VANILLA)),
    ("msr8", dict(k=8, d=14, n=16), (O.MSR, 8, 14, 16, O.SPARSE)),
    ("msr4-nonsys", dict(k=4, d=6, n=8, systematic=False), (O.MSR, 4, 6, 8, O.SPARSE)),
    ("mbr4", dict(k=4, d=6, n=8, kind=pm.PM_MBR), (O.MBR, 4, 6, 8, None)),
    ("mbr8", dict(k=8, d=14, n=16, kind=pm.PM_MBR), (O.MBR, 8, 14, 16, None)),
    ("rs16-8", dict(k=8, d=8, n=16, kind=pm.PM_RS), (O.RS, 8, 8, 16, None)),
]


def oracle_code(ok, kw):
    kind, k, d, n, cons = ok
    if kind == O.MSR:
        x = np.array(kw["x"]) if "x" in kw else None
        return O.Code(kind, k, d, n, cons, kw.get("systematic", True), x=x)
    return O.Code(kind, k, d, n)


@pytest.mark.parametrize("name,kw,ok", CODES, ids=[c[0] for c in CODES])
def test_decode_matrices_on_host_match_the_oracle(exe, tmp_path, name, kw, ok):
    c = pm.Code(**kw)
    o = oracle_code(ok, kw)
    Gsys = c.matrix(3)
    rng = np.random.default_rng(len(name) * 7 + c.k)
    # (a block of 1024 host threads is slow: fewer sets when B > 64)
    sets = [list(range(c.n - c.k, c.n))] + ([list(range(c.k))] if c.B <= 64 else [])
    sets += [list(rng.permutation(c.n)[:c.k]) for _ in range(3 if c.B <= 64 else 1)]
    sets += [[0] * c.k, [c.n] + list(range(1, c.k))]       # repeated node, node id out of range
    D, kept, st = run(exe, tmp_path, Gsys, c.B, c.k * c.alpha, c.B, 0, len(sets), np.array(sets),
                      c.k, c.alpha, c.n)
    for i, K in enumerate(sets[:-2]):
        Dw, kw_ = o.decode_matrix(K)
        assert st[i] == 0, (K, st[i])
        assert np.array_equal(D[i], Dw), K
        assert list(kept[i]) == list(kw_), K
    assert list(st[-2:]) == [pm.PM_EINVAL, pm.PM_EINVAL]
    assert not D[-2:].any()


def test_inverses_on_host_match_the_oracle(exe, tmp_path):
    for m in (1, 5, 64, 65):
        count = 4 if m <= 64 else 2
        A = synth.random_bytes(70 + m, count * m * m).reshape(count, m, m).copy()
        A[1] = 0
        if m > 1:
            A[1, 0, m - 1] = 7
            A[1, 1:] = A[0, 1:]
            A[1, m - 1] = A[1, 0]              # two equal rows: singular
        if count > 2:
            A[2] = 0
            A[3] = np.eye(m, dtype=np.uint8)
        D, _, st = run(exe, tmp_path, A, m, m, m, m * m, count)
        for p in range(count):
            want = O.invert(A[p])
            if want is None:
                assert st[p] == pm.PM_ESINGULAR and not D[p].any(), (m, p)
            else:
                assert st[p] == 0 and np.array_equal(D[p], want), (m, p)

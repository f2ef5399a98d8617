"""The GF(2^16) region kernel (csrc/gf16.hip) run on the host.

Its own source, with host stand-ins for the two byte/bit builtins it uses
(emu/gf16_main.cpp, every lane of every wave in turn, buffers of exact size
under AddressSanitizer), multiplies regions of 16-bit symbols by matrices
packed here from the program and table layouts its header documents.  Every
result is compared with the oracle's GF(2^16) region product, and the bytes
past each block must stay untouched."""
import os
import struct
import subprocess

import numpy as np
import pytest

from oracle import gf16 as F

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1412_3022_amd", "csrc")
R = 8   # rows per group (kPm16Rows)


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("gf16")
    hdr = open(os.path.join(CSRC, "gf16k.hpp")).read().replace("#include <hip/hip_runtime.h>", "")
    src = open(os.path.join(CSRC, "gf16.hip")).read()
    assert '#include "gf16k.hpp"' in src and "constexpr uint32_t kPm16Rows = 8;" in hdr
    src = src.replace("#include <hip/hip_runtime.h>", "").replace('#include "gf16k.hpp"', hdr)
    with open(d / "gf16_kernel.inc", "w") as f:
        f.write(src)
    out = str(d / "gf16_main")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
                           "-I", str(d), os.path.join(HERE, "emu", "gf16_main.cpp"), "-o", out])
    return out


@pytest.fixture(scope="module")
def tables():
    """Byte h of c * (v x^(e_p)) for the six 3/3/2-bit pieces p of a symbol
    (e_p = 0, 3, 6, 8, 11, 14), per element c (the layout of gf16k.hpp), from
    the oracle's field."""
    ex = np.array([F.gpow(e) for e in range(65535)], np.int64)
    lg = np.full(65536, -1, np.int64)
    lg[ex] = np.arange(65535)
    c = np.arange(65536, dtype=np.int64)

    def mul(v):   # c * v for all c, v a constant
        if v == 0:
            return np.zeros(65536, np.int64)
        r = ex[(lg[c] + lg[v]) % 65535]
        r[0] = 0
        return r

    t = np.zeros((65536, 32), np.uint32)
    for p, (e, nv) in enumerate(zip((0, 3, 6, 8, 11, 14), (8, 8, 4, 8, 8, 4))):
        for h in range(2):
            for v in range(nv):
                b = ((mul(v << e) >> (8 * h)) & 0xFF).astype(np.uint32)
                t[:, 4 * p + 2 * h + v // 4] |= b << (8 * (v % 4))
    return t


def pack(A):
    """Program words of matrix A (gf16k.hpp): rows that are one input block
    times 1 in copy groups, the others in groups of R in row order."""
    rows, cols = A.shape
    unit = [r for r in range(rows) if (A[r] != 0).sum() == 1 and A[r].max() == 1]
    rest = [r for r in range(rows) if r not in unit]
    tgroups = [rest[i:i + R] for i in range(0, len(rest), R)]
    cgroups = [unit[i:i + R] for i in range(0, len(unit), R)]
    ng = len(tgroups) + len(cgroups)
    words = [ng] + [0] * (ng * (2 + R))
    for g, rs in enumerate(tgroups):
        rec, n = [], 0
        for c in range(cols):
            if not A[rs, c].any():
                continue
            rec.append(c)
            for i in range(0, R, 2):
                lo = int(A[rs[i], c]) if i < len(rs) else 0
                hi = int(A[rs[i + 1], c]) if i + 1 < len(rs) else 0
                rec.append(lo | hi << 16)
            n += 1
        gd = 1 + g * (2 + R)
        words[gd], words[gd + 1] = len(words), n
        for i in range(R):
            words[gd + 2 + i] = rs[i] if i < len(rs) else 0xFFFFFFFF
        words += rec
    for q, rs in enumerate(cgroups):
        gd = 1 + (len(tgroups) + q) * (2 + R)
        words[gd], words[gd + 1] = len(words), 0xFFFFFFFF
        for i in range(R):
            words[gd + 2 + i] = rs[i] if i < len(rs) else 0xFFFFFFFF
        words += [int(np.nonzero(A[r])[0][0]) for r in rs] + [0] * (R - len(rs))
    return np.array(words, np.uint32), ng


def run(exe, tmp_path, tables, A, X, in_ld, out_ld):
    A = np.ascontiguousarray(A, np.uint16)
    rows, cols = A.shape
    nsym = X.shape[1]
    s = 2 * nsym
    inb = np.zeros((cols, in_ld), np.uint8)
    inb[:, :s] = X.view(np.uint8).reshape(cols, s)
    words, ng = pack(A)
    p_in, p_out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(p_in, "wb") as f:
        f.write(struct.pack("<7Q", cols, rows, s, in_ld, out_ld, words.size, ng))
        f.write(inb.tobytes())
        f.write(words.tobytes())
        f.write(np.ascontiguousarray(tables).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    subprocess.check_call([exe, str(p_in), str(p_out)], env=env, timeout=600)
    out = np.frombuffer(open(p_out, "rb").read(), np.uint8).reshape(rows, out_ld)
    assert (out[:, s:] == 0x5A).all(), "bytes past the block were written"
    return np.ascontiguousarray(out[:, :s]).view(np.uint16)


CASES = [
    # (rows, cols, symbols, density): one symbol; a ragged unit; one tile
    # plus a ragged tail; several tiles and groups, a partial last group
    (3, 5, 1, 1.0),
    (5, 7, 3, 1.0),
    (9, 6, 1024 + 3, 0.6),
    (20, 12, 3 * 1024 + 5, 0.4),
    # dense: the first group reads every column with all 8 rows, the second
    # holds the zero row
    (16, 9, 1024 + 5, 1.0),
]


@pytest.mark.parametrize("rows,cols,nsym,dens", CASES)
def test_random_matrices(exe, tmp_path, tables, rows, cols, nsym, dens):
    rng = np.random.default_rng(rows * 1000 + nsym)
    A = rng.integers(1, 65536, (rows, cols), dtype=np.uint16)
    A[rng.random((rows, cols)) > dens] = 0
    A[rows // 2] = 0                       # a zero row is written as zeros
    A[0, 0] = 1
    X = rng.integers(0, 65536, (cols, nsym), dtype=np.uint16)
    X[:, 0] = 0xFFFF
    s = 2 * nsym
    ld = (s + 15) // 16 * 16 + 16
    got = run(exe, tmp_path, tables, A, X, ld, ld + 32)
    assert np.array_equal(got, F.apply(A, X))


def test_copy_groups(exe, tmp_path, tables):
    """Rows that are an input block as it is (a decode's blocks held by the
    nodes) go through copy groups; 11 of them fill one group and part of a
    second, beside computed rows, at a ragged size."""
    rng = np.random.default_rng(21)
    rows, cols, nsym = 19, 13, 1024 + 7
    A = rng.integers(1, 65536, (rows, cols), dtype=np.uint16)
    A[rng.random((rows, cols)) > 0.5] = 0
    for r, c in zip(range(0, rows, 2), rng.permutation(cols)):   # 10 unit rows
        A[r] = 0
        A[r, c] = 1
    A[1] = 0
    A[1, 3] = 1                                # 11th, the same block as another row may read
    X = rng.integers(0, 65536, (cols, nsym), dtype=np.uint16)
    ld = (2 * nsym + 15) // 16 * 16
    got = run(exe, tmp_path, tables, A, X, ld, ld + 16)
    assert np.array_equal(got, F.apply(A, X))


def test_systematic_encode_matrix(exe, tmp_path, tables):
    """The parity rows of the sparse PM-MSR (4, 6, 8) code over GF(2^16)."""
    c = F.Code(4, 8)
    rng = np.random.default_rng(7)
    nsym = 2 * 1024 + 7
    X = rng.integers(0, 65536, (c.B, nsym), dtype=np.uint16)
    ld = (2 * nsym + 15) // 16 * 16
    got = run(exe, tmp_path, tables, c.enc, X, ld, ld)
    assert np.array_equal(got, c.encode(X))

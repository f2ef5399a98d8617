"""The matrix-core kernel (csrc/mfma.hip) run on the host with its own
source and the library's operand packing (csrc/mfma.cpp): one OS thread per
GPU thread, the wave-wide matrix instruction emulated in the register layout
the library assumes, blocks placed right before an inaccessible page under
AddressSanitizer.  Outputs are compared with the oracle's region product
(out = A in over GF(2^8)) for dense and sparse matrices, ragged block sizes
(every tail case of the 128-byte position blocks) and non-identity input
maps.  The layout assumption itself is checked on the GPU by the parity
tests of the same kernel."""
import os
import struct
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1412_3022_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ of the ROCm toolchain not found")
    d = tmp_path_factory.mktemp("mfma")
    hdr = open(os.path.join(CSRC, "mfma.hpp")).read()
    assert "#include <hip/hip_runtime.h>" in hdr
    hdr = hdr.replace("#include <hip/hip_runtime.h>", "typedef int hipError_t;\ntypedef struct ihipStream_t *hipStream_t;")
    (d / "mfma.hpp").write_text(hdr)
    # the packing source next to the stand-in header, so its include finds it
    (d / "mfma.cpp").write_text(open(os.path.join(CSRC, "mfma.cpp")).read())
    src = open(os.path.join(CSRC, "mfma.hip")).read()
    src = src.replace("#include <hip/hip_runtime.h>", "").replace('#include "mfma.hpp"', "")
    decl = "extern __shared__ uint4 pm_mf_lds[];"
    assert decl in src
    src = src.replace(decl, "")   # the emulator's per-work-group buffer
    occ = "__attribute__((amdgpu_waves_per_eu(2, 2)))"
    assert occ in src
    src = src.replace(occ, "")    # a GPU register-allocation hint
    src = src[:src.index('extern "C" hipError_t pmk_mfma')]
    (d / "mfma_kernel.inc").write_text(src)
    out = str(d / "mfma_main")
    subprocess.check_call([CLANG, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
                           "-pthread", "-I", str(d), "-I", CSRC, os.path.join(HERE, "emu", "mfma_main.cpp"),
                           str(d / "mfma.cpp"), os.path.join(CSRC, "gf256.cpp"), "-o", out])
    return out


def _run(exe, tmp_path, A, in_map, X, ncu=None, subset=False):
    R, C = A.shape
    nin, s = X.shape
    ld = (s + 15) // 16 * 16
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(struct.pack("<5Q", R, C, nin, s, ld))
        f.write(np.ascontiguousarray(A, np.uint8).tobytes())
        f.write(np.asarray(in_map, np.uint32).tobytes())
        f.write(np.ascontiguousarray(X, np.uint8).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    if ncu:
        env["EMU_NCU"] = str(ncu)
    if subset:
        env["EMU_SUBSET"] = "1"
    r = subprocess.run([exe, str(inp), str(outp)], env=env, timeout=600, check=True, capture_output=True, text=True)
    plan = dict(zip(r.stdout.split()[0::2], map(int, r.stdout.split()[1::2])))
    return np.frombuffer(open(outp, "rb").read(), np.uint8).reshape(R, s), plan


CASES = [
    # rows, cols, inputs, block bytes, density, compute units planned for,
    # columns mapped to input blocks 0, 1, ... in order (else a permutation)
    (16, 8, 8, 128, 1.0, None, False),
    (16, 8, 8, 128, 1.0, None, True),
    (13, 9, 12, 300, 1.0, None, False),      # padded rows and columns, tail inside a position block
    (64, 64, 64, 129, 1.0, None, True),
    (100, 37, 40, 4, 0.7, None, False),      # one short position block
    (56, 56, 56, 1000, 0.25, None, False),
    (56, 56, 60, 1000, 0.25, None, True),
    (240, 240, 240, 257, 1.0, None, True),   # the (16,30,32) decode shape
    (24, 300, 300, 200, 1.0, None, False),   # 38 chunks
    (12, 24, 24, 5000, 1.0, 2, True),        # 2 position groups: several blocks per wave, the last group partial
    (9, 264, 270, 3000, 0.8, 5, False),      # 33 chunks, several blocks per wave
    (40, 512, 512, 130, 1.0, 3, True),       # 64 chunks (two tiles per work-group), more M blocks than CUs
    (40, 512, 512, 130, 1.0, 3, False),
]


@pytest.mark.parametrize("R,C,nin,s,dens,ncu,inord", CASES,
                         ids=["%dx%d-s%d%s%s" % (c[0], c[1], c[3], "-cu%d" % c[5] if c[5] else "",
                                                 "-inorder" if c[6] else "") for c in CASES])
def test_mfma_kernel_on_host_matches_the_oracle(exe, tmp_path, R, C, nin, s, dens, ncu, inord):
    rng = np.random.default_rng(R * 1000 + C + s)
    A = rng.integers(1, 256, (R, C), dtype=np.uint8)
    A[rng.random((R, C)) >= dens] = 0
    A[0, :] = 0
    A[0, C // 2] = 1          # a unit row
    in_map = np.arange(C) if inord else rng.permutation(nin)[:C]
    X = rng.integers(0, 256, (nin, s), dtype=np.uint8)
    got, plan = _run(exe, tmp_path, A, in_map, X, ncu)
    assert plan["T"] == (4 if (C + 7) // 8 <= 38 else 2)
    assert np.array_equal(got, O.apply(A, X[in_map], nthreads=4))


def test_only_the_computed_rows_on_the_matrix_cores(exe, tmp_path):
    """A decode-like matrix: rows that are one input block times 1 (blocks
    the node set holds) between dense rows.  With those rows left out of
    the program, the kernel writes exactly the other rows, each to its own
    output row, with the oracle's bytes; the unit rows' output stays as it
    was (zero here), for the library's copy launch."""
    rng = np.random.default_rng(91)
    R, C, s = 40, 48, 700
    A = rng.integers(1, 256, (R, C), dtype=np.uint8)
    A[rng.random((R, C)) >= 0.5] = 0
    unit = [0, 3, 4, 5, 17, 30, 39]
    for k, r in enumerate(unit):
        A[r, :] = 0
        A[r, (7 * k) % C] = 1
    in_map = rng.permutation(C)
    X = rng.integers(0, 256, (C, s), dtype=np.uint8)
    got, _ = _run(exe, tmp_path, A, in_map, X, subset=True)
    want = O.apply(A, X[in_map], nthreads=4)
    comp = [r for r in range(R) if r not in unit]
    assert np.array_equal(got[comp], want[comp])
    assert not got[unit].any()

"""Runs the library's generated bit-sliced kernels on the host.

The library writes each kernel source it generates to PMRC_BS_DUMP (and the
multi-set one to PMRC_BS_DUMP + ".multi") before handing it to hipRTC; a data
call on a machine without a GPU generates the source and then fails with
PM_EHIP.  Here that source gets the host stand-ins of emu/emu_prelude.h and
the driver emu/emu_main.inc, is compiled with clang++ (AddressSanitizer on),
and runs every thread of the launch in turn."""
import os
import subprocess
import tempfile

import numpy as np

from paper_1412_3022_amd import pm

HERE = os.path.dirname(os.path.abspath(__file__))
EMU = os.path.join(HERE, "emu")
CLANG = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")


def generated_source(code, op, failed=0, ids=None, workdir=None):
    """The single-set source path of `op`'s kernel (the multi-set one is the
    same path + ".multi"), or None if the matrix is not specialized."""
    path = os.path.join(workdir or tempfile.mkdtemp(), "op%d.hip" % op)
    os.environ["PMRC_BS_DUMP"] = path
    try:
        code.set_variant(op, 8, 32)
        s, base = 4096, 1 << 20
        big = base + 4096 * s
        L = pm.lib()
        arr = (lambda v: (pm.ctypes.c_uint32 * len(v))(*v))
        vp = pm.ctypes.c_void_p
        if op == pm.OP_ENCODE:
            st = L.pm_encode(code.h, vp(base), s, vp(big), s, s, None)
        elif op == pm.OP_HELPER:
            st = L.pm_repair_helper(code.h, failed, vp(base), s, vp(big), s, None)
        elif op == pm.OP_NEWCOMER:
            st = L.pm_repair_newcomer(code.h, failed, arr(ids), vp(base), s, vp(big), s, s, None)
        else:
            st = L.pm_decode(code.h, arr(ids), vp(base), s, vp(big), s, s, None)
    finally:
        del os.environ["PMRC_BS_DUMP"]
        code.set_variant(op, 0, 0)
    if not os.path.exists(path):
        return None
    assert st == pm.PM_EHIP, st   # generated, then no GPU to load it on
    return path


def generated_apply_source(A, workdir=None):
    """The single-set source of pm_apply's kernel for the matrix A (rows x
    cols, uint8), or None if the matrix is not specialized."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    path = os.path.join(workdir or tempfile.mkdtemp(), "apply.hip")
    os.environ["PMRC_BS_DUMP"] = path
    try:
        pm.pm_set_variant(None, pm.OP_APPLY, 8, 32)
        s, base = 4096, 1 << 20
        st = pm.pm_apply(A, base, s, base + (A.shape[1] + 1) * s * 2, s, s)
    finally:
        del os.environ["PMRC_BS_DUMP"]
        pm.pm_set_variant(None, pm.OP_APPLY, 0, 0)
    if not os.path.exists(path):
        return None
    assert st == pm.PM_EHIP, st
    return path


def build(source, multi, sanitize=True, tile=2048, kernel="pmbs"):
    """Compile one generated source for the host (tile: bytes of a block per
    wave tile, 4096 for the GF(2^16) kernels; kernel: the single-set
    kernel's name, pmbs16 for GF(2^16)); returns the executable."""
    src = source + (".multi" if multi else "")
    text = open(src).read()
    barrier = 'asm volatile("" : "+s"(ld), "+s"(old));'
    assert barrier in text
    text = text.replace(barrier, "")          # a compiler-only barrier, empty on the GPU too
    assert "asm" not in text
    cpp = src + ".emu.cpp"
    with open(cpp, "w") as f:
        f.write('#include "emu_prelude.h"\n' + text + '#include "emu_main.inc"\n')
    exe = src + (".asan" if sanitize else ".plain")
    cmd = [CLANG, "-O1", "-std=c++17", "-I" + EMU, "-DEMU_KIND=%d" % int(multi), "-DEMU_TILE=%d" % tile, "-DEMU_KERNEL=" + kernel, "-Wno-unused-value", cpp, "-o", exe]
    if sanitize:
        cmd[1:1] = ["-g", "-fsanitize=address"]
    subprocess.check_call(cmd)
    return exe


def run(exe, P, cases, high=False):
    """cases: (input rows x s uint8 array, in_ld, out_rows, out_ld, s) per
    item.  Returns each item's output rows (out_rows x s) and asserts that the
    row padding past s was not written."""
    work = tempfile.mkdtemp()
    args = [exe, str(P), str(len(cases))]
    outs = []
    for i, (inp, ld, out_rows, old, s) in enumerate(cases):
        rows = inp.shape[0]
        buf = np.full((rows, ld), 0xA5, np.uint8)
        buf[:, :s] = inp
        fin, fout = os.path.join(work, "in%d" % i), os.path.join(work, "out%d" % i)
        buf.reshape(-1)[:(rows - 1) * ld + s].tofile(fin)
        args += [fin, str(rows), str(ld), fout, str(out_rows), str(old), str(s)]
        outs.append((fout, out_rows, old, s))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    if high:
        env["EMU_HIGH"] = "1"
    r = subprocess.run(args, capture_output=True, text=True, env=env)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    res = []
    for fout, out_rows, old, s in outs:
        raw = np.fromfile(fout, np.uint8)
        full = np.full(out_rows * old, 0x5A, np.uint8)
        full[:raw.size] = raw
        o = full.reshape(out_rows, old)
        assert np.all(o[:, s:] == 0x5A), "write past the block end"
        res.append(o[:, :s].copy())
    return res

"""CPU oracle for the product-matrix regenerating-code data path.

TEST INFRASTRUCTURE ONLY.  The library (``paper_1412_3022_amd``) never imports
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` do.  The arithmetic lives in ``oracle.c`` (plain C,
log/antilog GF(2^8)); this module only marshals numpy arrays through ctypes
and composes the C steps in the order the paper describes them:

    Psi (Section 3.3 / Section 3.2) -> index matrix L (Section 3.1)
    -> linearized G (Section 3.1) -> systematic G' = G * inverse(G~)
    (Section 3.2) -> data phase Y = G X, repair, decode (Section 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from itertools import combinations

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "oracle16.c")]
_LIB = os.path.join(_HERE, "_liboracle.so")

MSR, MBR, RS = 0, 1, 2
VANILLA, SPARSE = 0, 1


def build(force: bool = False) -> str:
    """Compile oracle.c and oracle16.c with gcc into _liboracle.so (next to
    the sources)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(map(os.path.getmtime, _SRCS)):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", tmp] + _SRCS + ["-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        u8p = ctypes.POINTER(ctypes.c_uint8)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.or_init.restype = None
        for name in ("or_mul", "or_div"):
            getattr(L, name).argtypes = [ctypes.c_uint8, ctypes.c_uint8]
            getattr(L, name).restype = ctypes.c_uint8
        L.or_inv.argtypes = [ctypes.c_uint8]
        L.or_inv.restype = ctypes.c_uint8
        L.or_gpow.argtypes = [ctypes.c_long]
        L.or_gpow.restype = ctypes.c_uint8
        L.or_matmul.argtypes = [u8p, u8p, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_matmul.restype = None
        L.or_invert.argtypes = [u8p, u8p, ctypes.c_int]
        L.or_rank.argtypes = [u8p, ctypes.c_int, ctypes.c_int]
        L.or_dims.argtypes = [ctypes.c_int] * 4 + [ip, ip]
        L.or_msr_vanilla.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p, u8p]
        L.or_msr_sparse_printed.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
        L.or_msr_sparse.argtypes = [ctypes.c_int, ctypes.c_int, u8p, u8p]
        L.or_all_dsubsets_invertible.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_msr_valid.argtypes = [u8p, u8p, ctypes.c_int, ctypes.c_int]
        L.or_mbr_psi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p]
        L.or_index_msr.argtypes = [ctypes.c_int, ip]
        L.or_index_mbr.argtypes = [ctypes.c_int, ctypes.c_int, ip]
        L.or_linearize.argtypes = [u8p, ip] + [ctypes.c_int] * 4 + [u8p]
        L.or_linearize.restype = None
        L.or_specific_encode.argtypes = [u8p, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         pp, pp, ctypes.c_size_t]
        L.or_specific_encode.restype = None
        L.or_systematic.argtypes = [u8p, ctypes.c_int, ctypes.c_int, u8p]
        L.or_rs_generator.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
        L.or_apply.argtypes = [u8p, ctypes.c_int, ctypes.c_int, pp, pp, ctypes.c_size_t, ctypes.c_int]
        L.or_apply.restype = None
        L.or_helper_row.argtypes = [ctypes.c_int, u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p]
        L.or_helper_row.restype = None
        L.or_newcomer_matrix.argtypes = [ctypes.c_int, u8p, u8p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ip, u8p]
        L.or_decode_matrix.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, u8p, ip]
        L.or_msr_specific_decode.argtypes = [u8p, u8p, ip, ctypes.c_int, ctypes.c_int, ip, pp, ctypes.c_int,
                                             pp, ctypes.c_size_t]
        L.or_mbr_specific_decode.argtypes = [u8p, ip, ctypes.c_int, ctypes.c_int, ip, pp, pp, ctypes.c_size_t]
        L.or_init()
        _lib = L
    return _lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _ptrs(rows):
    arr = (ctypes.c_void_p * max(1, len(rows)))()
    for i, r in enumerate(rows):
        arr[i] = r.ctypes.data
    return arr


# ---------------------------------------------------------------- field --
def mul(a: int, b: int) -> int:
    return int(lib().or_mul(a, b))


def inv(a: int) -> int:
    return int(lib().or_inv(a))


def gpow(e: int) -> int:
    return int(lib().or_gpow(e))


# -------------------------------------------------------- linear algebra --
def matmul(A, B):
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.zeros((m, n), np.uint8)
    lib().or_matmul(_u8(A), _u8(B), _u8(C), m, k, n)
    return C


def invert(A):
    """Inverse of a square matrix, or None when singular."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    n = A.shape[0]
    Ai = np.zeros((n, n), np.uint8)
    return Ai if lib().or_invert(_u8(A), _u8(Ai), n) == 0 else None


def rank(A) -> int:
    A = np.ascontiguousarray(A, dtype=np.uint8)
    return int(lib().or_rank(_u8(A), A.shape[0], A.shape[1]))


# --------------------------------------------------------- constructions --
def dims(kind, k, d, n):
    a, b = ctypes.c_int(), ctypes.c_int()
    if lib().or_dims(kind, k, d, n, ctypes.byref(a), ctypes.byref(b)) != 0:
        raise ValueError("unsupported parameters kind=%d k=%d d=%d n=%d" % (kind, k, d, n))
    return a.value, b.value


def msr_vanilla(k, n, x=None):
    d = 2 * k - 2
    psi = np.zeros((n, d), np.uint8)
    lam = np.zeros(n, np.uint8)
    xs = None if x is None else np.ascontiguousarray(x, dtype=np.uint8)
    lib().or_msr_vanilla(k, n, None if xs is None else _u8(xs), _u8(psi), _u8(lam))
    return psi, lam


def msr_sparse_printed(k, n):
    d = 2 * k - 2
    psi = np.zeros((n, d), np.uint8)
    lam = np.zeros(n, np.uint8)
    if lib().or_msr_sparse_printed(k, n, _u8(psi), _u8(lam)) != 0:
        return None, None
    return psi, lam


def msr_sparse(k, n):
    d = 2 * k - 2
    psi = np.zeros((n, d), np.uint8)
    lam = np.zeros(n, np.uint8)
    if lib().or_msr_sparse(k, n, _u8(psi), _u8(lam)) != 0:
        return None, None
    return psi, lam


def all_dsubsets_invertible(psi, d, must=-1) -> bool:
    psi = np.ascontiguousarray(psi, dtype=np.uint8)
    return bool(lib().or_all_dsubsets_invertible(_u8(psi), psi.shape[0], d, must))


def msr_valid(psi, lam) -> bool:
    psi = np.ascontiguousarray(psi, dtype=np.uint8)
    lam = np.ascontiguousarray(lam, dtype=np.uint8)
    return bool(lib().or_msr_valid(_u8(psi), _u8(lam), psi.shape[0], psi.shape[1]))


def mbr_psi(k, d, n):
    psi = np.zeros((n, d), np.uint8)
    if lib().or_mbr_psi(k, d, n, _u8(psi)) != 0:
        raise ValueError("MBR base matrix singular")
    return psi


def index_msr(k):
    a = k - 1
    L = np.zeros((2 * a, a), np.int32)
    lib().or_index_msr(k, _i32(L))
    return L


def index_mbr(k, d):
    L = np.zeros((d, d), np.int32)
    lib().or_index_mbr(k, d, _i32(L))
    return L


def linearize(psi, L, alpha, B):
    psi = np.ascontiguousarray(psi, dtype=np.uint8)
    L = np.ascontiguousarray(L, dtype=np.int32)
    n, d = psi.shape
    G = np.zeros((n * alpha, B), np.uint8)
    lib().or_linearize(_u8(psi), _i32(L), n, d, alpha, B, _u8(G))
    return G


def specific_encode(psi, L, alpha, X):
    """C = Psi M byte by byte; returns the n*alpha node blocks (node-major)."""
    psi = np.ascontiguousarray(psi, dtype=np.uint8)
    L = np.ascontiguousarray(L, dtype=np.int32)
    X = np.ascontiguousarray(X, dtype=np.uint8)
    n, d = psi.shape
    s = X.shape[1]
    C = np.zeros((n * alpha, s), np.uint8)
    lib().or_specific_encode(_u8(psi), _i32(L), n, d, alpha, _ptrs(list(X)), _ptrs(list(C)), s)
    return C


def systematic(G, B):
    G = np.ascontiguousarray(G, dtype=np.uint8)
    Gp = np.zeros_like(G)
    if lib().or_systematic(_u8(G), G.shape[0], B, _u8(Gp)) != 0:
        return None
    return Gp


def rs_generator(k, n):
    G = np.zeros((n, k), np.uint8)
    if lib().or_rs_generator(k, n, _u8(G)) != 0:
        raise ValueError("RS Vandermonde top block singular")
    return G


# ------------------------------------------------------------ data phase --
def apply(A, X, nthreads=1):
    """out[r] = XOR_c A[r][c] * X[c] over byte regions (rows of X)."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    X = np.ascontiguousarray(X, dtype=np.uint8)
    rows, cols = A.shape
    assert X.shape[0] == cols
    s = X.shape[1]
    out = np.zeros((rows, s), np.uint8)
    if rows and s:
        lib().or_apply(_u8(A), rows, cols, _ptrs(list(X)), _ptrs(list(out)), s, int(nthreads))
    return out


def helper_row(kind, psi, alpha, f):
    psi = np.ascontiguousarray(psi, dtype=np.uint8)
    row = np.zeros(1 if kind == RS else alpha, np.uint8)
    lib().or_helper_row(kind, _u8(psi), psi.shape[1], alpha, f, _u8(row))
    return row.reshape(1, -1)


def newcomer_matrix(kind, psi_or_g, lam, d, alpha, f, H):
    psi_or_g = np.ascontiguousarray(psi_or_g, dtype=np.uint8)
    lam = np.ascontiguousarray(lam if lam is not None else np.zeros(psi_or_g.shape[0]), dtype=np.uint8)
    Ha = np.ascontiguousarray(H, dtype=np.int32)
    rows = 1 if kind == RS else alpha
    R = np.zeros((rows, d), np.uint8)
    if lib().or_newcomer_matrix(kind, _u8(psi_or_g), _u8(lam), d, alpha, f, _i32(Ha), _u8(R)) != 0:
        return None
    return R


def decode_matrix(Gsys, B, alpha, K):
    Gsys = np.ascontiguousarray(Gsys, dtype=np.uint8)
    Ka = np.ascontiguousarray(K, dtype=np.int32)
    D = np.zeros((B, B), np.uint8)
    kept = np.zeros(B, np.int32)
    if lib().or_decode_matrix(_u8(Gsys), B, alpha, _i32(Ka), len(K), _u8(D), _i32(kept)) != 0:
        return None, None
    return D, kept


# ------------------------------------------------------------ whole code --
class Code:
    """A PM-MSR / PM-MBR (or RS baseline) code assembled from the C steps.

    Attributes: psi (n x d), lam (MSR), L, G (n alpha x B, linearized),
    Gsys (generator the nodes are encoded with), enc (the rows encode writes),
    node_map (for each of the n alpha node blocks: ('x', i) or ('out', r)).
    """

    def __init__(self, kind, k, d, n, construction=SPARSE, systematic_form=True, x=None,
                 check=True):
        self.kind, self.k, self.n = kind, k, n
        self.d = k if kind == RS else d
        self.alpha, self.B = dims(kind, k, self.d, n)
        a, B = self.alpha, self.B
        self.lam = None
        if kind == MSR:
            if construction == VANILLA:
                self.psi, self.lam = msr_vanilla(k, n, x)
            else:
                self.psi, self.lam = msr_sparse(k, n)
                if self.psi is None:
                    raise ValueError("sparse construction unsupported for n=%d k=%d" % (n, k))
            if check and not msr_valid(self.psi, self.lam):
                raise ValueError("invalid MSR code (Lambda collision or singular d-subset)")
            self.L = index_msr(k)
            self.G = linearize(self.psi, self.L, a, B)
            if systematic_form:
                self.Gsys = systematic(self.G, B)
                if self.Gsys is None:
                    raise ValueError("first B rows of G are singular")
                self.enc = self.Gsys[B:]
                self.node_map = [("x", t) if t < B else ("out", t - B) for t in range(n * a)]
            else:
                self.Gsys = self.G
                self.enc = self.G
                self.node_map = [("out", t) for t in range(n * a)]
        elif kind == MBR:
            self.psi = mbr_psi(k, self.d, n)
            self.L = index_mbr(k, self.d)
            self.G = linearize(self.psi, self.L, a, B)
            self.Gsys = self.G
            kd = k * a
            self.enc = self.G[kd:]
            self.node_map = []
            for t in range(n * a):
                if t < kd:
                    nz = np.nonzero(self.G[t])[0]
                    assert len(nz) == 1 and self.G[t, nz[0]] == 1
                    self.node_map.append(("x", int(nz[0])))
                else:
                    self.node_map.append(("out", t - kd))
        elif kind == RS:
            self.G = rs_generator(k, n)
            self.Gsys = self.G
            self.psi = self.G
            self.enc = self.G[k:]
            self.node_map = [("x", t) if t < k else ("out", t - k) for t in range(n)]
        else:
            raise ValueError("kind")

    # data phase ---------------------------------------------------------
    def encode(self, X, nthreads=1):
        return apply(self.enc, X, nthreads)

    def node_blocks(self, i, X, out):
        rows = []
        for t in range(i * self.alpha, (i + 1) * self.alpha):
            src, idx = self.node_map[t]
            rows.append(X[idx] if src == "x" else out[idx])
        return np.stack(rows)

    def helper_row(self, f):
        return helper_row(self.kind, self.psi, self.alpha, f)

    def newcomer_matrix(self, f, H):
        return newcomer_matrix(self.kind, self.psi, self.lam, self.d, self.alpha, f, list(H))

    def repair(self, f, H, nodes):
        """nodes: dict node -> (alpha x s) blocks.  Returns node f's blocks."""
        hrow = self.helper_row(f)
        recv = np.stack([apply(hrow, nodes[h])[0] for h in H])
        R = self.newcomer_matrix(f, H)
        if R is None:
            raise np.linalg.LinAlgError("singular helper set")
        return apply(R, recv)

    def decode_matrix(self, K):
        return decode_matrix(self.Gsys, self.B, self.alpha, list(K))

    def decode_specific(self, K, Y):
        """The same decode by the specific PM-MSR or PM-MBR algorithm."""
        if self.kind == MSR:
            return msr_specific_decode(self.psi, self.lam, self.L, self.k, K, Y, self.Gsys is not self.G)
        if self.kind == MBR:
            return mbr_specific_decode(self.psi, self.L, self.k, self.d, K, Y)
        raise ValueError("specific decoding is defined here for PM-MSR and PM-MBR")

    def decode(self, K, Y):
        """Y: (k alpha x s) blocks of the nodes in K, node-major."""
        D, kept = self.decode_matrix(K)
        if D is None:
            raise np.linalg.LinAlgError("undecodable node set")
        return apply(D, Y[kept])


def msr_specific_decode(psi, lam, L, k, K, Y, systematic_form=True):
    """Specific PM-MSR decoding from the k nodes K (their k alpha blocks Y,
    node-major); returns the B data blocks, or None if singular."""
    Y = np.ascontiguousarray(Y, dtype=np.uint8)
    s = Y.shape[1]
    alpha = k - 1
    B = alpha * (alpha + 1)
    X = np.zeros((B, s), np.uint8)
    rc = lib().or_msr_specific_decode(_u8(psi), _u8(lam), _i32(np.ascontiguousarray(L, dtype=np.int32)), k,
                                      psi.shape[0], _i32(np.array(K, dtype=np.int32)), _ptrs(list(Y)),
                                      1 if systematic_form else 0, _ptrs(list(X)), s)
    if rc == -2:
        raise ValueError("Psi is not of the form [Phi, Lambda Phi]")
    return None if rc != 0 else X


def mbr_specific_decode(psi, L, k, d, K, Y):
    """Specific PM-MBR decoding from the k nodes K (their k d blocks Y,
    node-major); returns the B data blocks, or None if singular."""
    K = list(K)
    if len(K) != k:
        raise ValueError("K must list k nodes")
    Y = np.ascontiguousarray(Y, dtype=np.uint8)
    if Y.shape[0] != k * d:
        raise ValueError("Y must hold k d blocks")
    s = Y.shape[1]
    B = k * d - k * (k - 1) // 2
    X = np.zeros((B, s), np.uint8)
    rc = lib().or_mbr_specific_decode(_u8(np.ascontiguousarray(psi, dtype=np.uint8)),
                                      _i32(np.ascontiguousarray(L, dtype=np.int32)), k, d,
                                      _i32(np.array(K, dtype=np.int32)), _ptrs(list(Y)), _ptrs(list(X)), s)
    return None if rc != 0 else X


def subsets(n, m):
    return combinations(range(n), m)

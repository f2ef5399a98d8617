"""GF(2^16) part of the CPU oracle (TEST INFRASTRUCTURE ONLY, like the rest
of this package).

Section 3.3 extends the sparse PM-MSR construction from k <= 39 in GF(2^8)
to k <= 64 in GF(2^16).  This module marshals numpy arrays through ctypes to
``oracle16.c`` and assembles those codes in the paper's order: Psi and Lambda
(Section 3.3) -> index matrix L (Section 3.1) -> linearized G (Section 3.1)
-> systematic G' (Section 3.2) -> encode, repair, decode (Section 2).

Regions are numpy uint16 arrays of shape (blocks, symbols); their bytes
(``.view(np.uint8)`` on a little-endian host) are the library's layout: symbol
p in bytes 2p (low) and 2p + 1 (high).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _i32, _ptrs, index_msr, lib as _lib8

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = _lib8()
        u16p = ctypes.POINTER(ctypes.c_uint16)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.or16_init.restype = None
        for name in ("or16_mul", "or16_div"):
            getattr(L, name).argtypes = [ctypes.c_uint16, ctypes.c_uint16]
            getattr(L, name).restype = ctypes.c_uint16
        L.or16_inv.argtypes = [ctypes.c_uint16]
        L.or16_inv.restype = ctypes.c_uint16
        L.or16_gpow.argtypes = [ctypes.c_long]
        L.or16_gpow.restype = ctypes.c_uint16
        L.or16_matmul.argtypes = [u16p, u16p, u16p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or16_matmul.restype = None
        L.or16_invert.argtypes = [u16p, u16p, ctypes.c_int]
        L.or16_rank.argtypes = [u16p, ctypes.c_int, ctypes.c_int]
        for name in ("or16_msr_sparse_printed", "or16_msr_sparse"):
            getattr(L, name).argtypes = [ctypes.c_int, ctypes.c_int, u16p, u16p]
        L.or16_all_dsubsets_invertible.argtypes = [u16p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or16_msr_valid.argtypes = [u16p, u16p, ctypes.c_int, ctypes.c_int]
        L.or16_linearize.argtypes = [u16p, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, u16p]
        L.or16_linearize.restype = None
        L.or16_specific_encode.argtypes = [u16p, ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, pp, pp,
                                           ctypes.c_size_t]
        L.or16_specific_encode.restype = None
        L.or16_systematic.argtypes = [u16p, ctypes.c_int, ctypes.c_int, u16p]
        L.or16_apply.argtypes = [u16p, ctypes.c_int, ctypes.c_int, pp, pp, ctypes.c_size_t]
        L.or16_apply.restype = None
        L.or16_newcomer_matrix.argtypes = [u16p, u16p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, u16p]
        L.or16_decode_matrix.argtypes = [u16p, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, u16p]
        L.or16_msr_specific_decode.argtypes = [u16p, u16p, ip, ctypes.c_int, ip, pp, ctypes.c_int, pp,
                                               ctypes.c_size_t]
        L.or16_init()
        _lib = L
    return _lib


def _u16(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16))


def _c16(a):
    return np.ascontiguousarray(a, dtype=np.uint16)


# ---------------------------------------------------------------- field --
def mul(a: int, b: int) -> int:
    return int(lib().or16_mul(a, b))


def inv(a: int) -> int:
    return int(lib().or16_inv(a))


def gpow(e: int) -> int:
    return int(lib().or16_gpow(e))


# -------------------------------------------------------- linear algebra --
def matmul(A, B):
    A, B = _c16(A), _c16(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.zeros((m, n), np.uint16)
    lib().or16_matmul(_u16(A), _u16(B), _u16(C), m, k, n)
    return C


def invert(A):
    """Inverse of a square matrix, or None when singular."""
    A = _c16(A)
    n = A.shape[0]
    Ai = np.zeros((n, n), np.uint16)
    return Ai if lib().or16_invert(_u16(A), _u16(Ai), n) == 0 else None


def rank(A) -> int:
    A = _c16(A)
    return int(lib().or16_rank(_u16(A), A.shape[0], A.shape[1]))


# --------------------------------------------------------- construction --
def msr_sparse_printed(k, n):
    d = 2 * k - 2
    psi = np.zeros((n, d), np.uint16)
    lam = np.zeros(n, np.uint16)
    if lib().or16_msr_sparse_printed(k, n, _u16(psi), _u16(lam)) != 0:
        return None, None
    return psi, lam


def msr_sparse(k, n):
    d = 2 * k - 2
    psi = np.zeros((n, d), np.uint16)
    lam = np.zeros(n, np.uint16)
    if lib().or16_msr_sparse(k, n, _u16(psi), _u16(lam)) != 0:
        return None, None
    return psi, lam


def all_dsubsets_invertible(psi, d, must=-1) -> bool:
    psi = _c16(psi)
    return bool(lib().or16_all_dsubsets_invertible(_u16(psi), psi.shape[0], d, must))


def msr_valid(psi, lam) -> bool:
    psi, lam = _c16(psi), _c16(lam)
    return bool(lib().or16_msr_valid(_u16(psi), _u16(lam), psi.shape[0], psi.shape[1]))


def linearize(psi, L, alpha, B):
    psi = _c16(psi)
    L = np.ascontiguousarray(L, dtype=np.int32)
    n, d = psi.shape
    G = np.zeros((n * alpha, B), np.uint16)
    lib().or16_linearize(_u16(psi), _i32(L), n, d, alpha, B, _u16(G))
    return G


def specific_encode(psi, L, alpha, X):
    """C = Psi M symbol by symbol; the n alpha node blocks, node-major."""
    psi = _c16(psi)
    L = np.ascontiguousarray(L, dtype=np.int32)
    X = _c16(X)
    n, d = psi.shape
    C = np.zeros((n * alpha, X.shape[1]), np.uint16)
    lib().or16_specific_encode(_u16(psi), _i32(L), n, d, alpha, _ptrs(list(X)), _ptrs(list(C)), X.shape[1])
    return C


def systematic(G, B):
    G = _c16(G)
    Gp = np.zeros_like(G)
    return Gp if lib().or16_systematic(_u16(G), G.shape[0], B, _u16(Gp)) == 0 else None


# ------------------------------------------------------------ data phase --
def apply(A, X):
    """out[r] = sum_c A[r][c] * X[c] over regions of 16-bit symbols."""
    A, X = _c16(A), _c16(X)
    rows, cols = A.shape
    assert X.shape[0] == cols
    out = np.zeros((rows, X.shape[1]), np.uint16)
    if rows and X.shape[1]:
        lib().or16_apply(_u16(A), rows, cols, _ptrs(list(X)), _ptrs(list(out)), X.shape[1])
    return out


def newcomer_matrix(psi, lam, alpha, f, H):
    psi, lam = _c16(psi), _c16(lam)
    d = psi.shape[1]
    if len(H) != d:
        raise ValueError("a repair takes d = %d helpers" % d)
    R = np.zeros((alpha, d), np.uint16)
    Ha = np.ascontiguousarray(H, dtype=np.int32)
    if lib().or16_newcomer_matrix(_u16(psi), _u16(lam), d, alpha, f, _i32(Ha), _u16(R)) != 0:
        return None
    return R


def decode_matrix(Gsys, B, alpha, K):
    Gsys = _c16(Gsys)
    D = np.zeros((B, B), np.uint16)
    Ka = np.ascontiguousarray(K, dtype=np.int32)
    if len(K) * alpha != B:
        raise ValueError("a decode takes k = %d nodes" % (B // alpha))
    if lib().or16_decode_matrix(_u16(Gsys), B, alpha, _i32(Ka), len(K), _u16(D)) != 0:
        return None
    return D


def msr_specific_decode(psi, lam, L, k, K, Y, systematic_form=True):
    """Specific PM-MSR decoding from the k nodes K (their k alpha blocks Y,
    node-major, uint16 symbols); the B data blocks, or None if singular."""
    K = list(K)
    if len(K) != k:
        raise ValueError("K must list k nodes")
    Y = _c16(Y)
    alpha = k - 1
    if Y.shape[0] != k * alpha:
        raise ValueError("Y must hold k alpha blocks")
    B = alpha * (alpha + 1)
    X = np.zeros((B, Y.shape[1]), np.uint16)
    rc = lib().or16_msr_specific_decode(_u16(_c16(psi)), _u16(_c16(lam)), _i32(np.ascontiguousarray(L, np.int32)), k,
                                        _i32(np.array(K, np.int32)), _ptrs(list(Y)), 1 if systematic_form else 0,
                                        _ptrs(list(X)), Y.shape[1])
    if rc == -2:
        raise ValueError("Psi is not of the form [Phi, Lambda Phi]")
    return None if rc != 0 else X


class Code:
    """Sparse PM-MSR over GF(2^16) (Section 3.3), systematic (Section 3.2) or
    not.  Attributes as the GF(2^8) oracle's Code: psi, lam, L, G, Gsys, enc,
    node_map."""

    def __init__(self, k, n, systematic_form=True, check=True):
        self.k, self.n = k, n
        self.d = d = 2 * k - 2
        self.alpha = a = k - 1
        self.B = B = k * a
        self.psi, self.lam = msr_sparse(k, n)
        if self.psi is None:
            raise ValueError("construction failed for k=%d n=%d" % (k, n))
        if check and not msr_valid(self.psi, self.lam):
            raise ValueError("invalid encoding matrix")
        self.L = index_msr(k)
        self.G = linearize(self.psi, self.L, a, B)
        if systematic_form:
            self.Gsys = systematic(self.G, B)
            self.enc = self.Gsys[B:]
            self.node_map = [("x", t) if t < B else ("out", t - B) for t in range(n * a)]
        else:
            self.Gsys = self.G
            self.enc = self.G
            self.node_map = [("out", t) for t in range(n * a)]
        self.enc_rows = self.enc.shape[0]

    def encode(self, X):
        return apply(self.enc, X)

    def node_blocks(self, i, X, out):
        rows = []
        for t in range(i * self.alpha, (i + 1) * self.alpha):
            src, idx = self.node_map[t]
            rows.append(X[idx] if src == "x" else out[idx])
        return np.stack(rows)

    def helper_row(self, f):
        return self.psi[f, :self.alpha].reshape(1, -1).copy()

    def newcomer_matrix(self, f, H):
        return newcomer_matrix(self.psi, self.lam, self.alpha, f, list(H))

    def repair(self, f, H, nodes):
        hrow = self.helper_row(f)
        recv = np.stack([apply(hrow, nodes[h])[0] for h in H])
        R = self.newcomer_matrix(f, H)
        if R is None:
            raise np.linalg.LinAlgError("singular helper set")
        return apply(R, recv)

    def decode_matrix(self, K):
        return decode_matrix(self.Gsys, self.B, self.alpha, list(K))

    def decode_specific(self, K, Y):
        return msr_specific_decode(self.psi, self.lam, self.L, self.k, K, Y, self.Gsys is not self.G)

    def decode(self, K, Y):
        D = self.decode_matrix(K)
        if D is None:
            raise np.linalg.LinAlgError("undecodable node set")
        return apply(D, Y)

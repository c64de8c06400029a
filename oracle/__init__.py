"""CPU oracle for C = A^t A, packed lower triangle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never does, and this package imports nothing
from it.

Functions
  classical(A)              plain definition, k ascending (Section 3, block
                            equations; output n(n+1)/2 entries)
  classical_mt(A, ...)      the same definition, threaded; bitwise equal
  ata(A, cutoff, ...)       Algorithm 1 with HASA off-diagonal products,
                            returns (C, counts)
  hasa(X, Y, cutoff, ...)   the rectangular Strassen/Winograd routine alone
  ata_mult_count(m, n, c)   multiplication count of Algorithm 1 (no data)
  potrf(Cp, n)              Cholesky factor of packed C (row by row), with
                            LAPACK's info (first non-positive pivot + 1)
  potrs(L, n, B)            L L^t X = B by forward and back substitution
  atb(A, B)                 A^t B, the normal equations' right-hand side
                            (these three follow Section 1's least-squares use
                            of A^t A and their textbook definitions)
  project(A, B)             A (A^t A)^-1 A^t B, the projection onto the
                            column space (Section 1's projection matrix):
                            the steps above, then a matrix product
  bf16_round, bf16_split, e4m3_round, pow2_column_scales
                            number-format conversions used by the reduced
                            precision forms, written from the format
                            definitions (IEEE-754 binary32 -> bfloat16 with
                            round-to-nearest-even; OCP 8-bit e4m3)
  gram_bf16x3(A32), gram_fp8(A32)
                            classical products of the converted operands
                            (hi^t hi + hi^t lo + lo^t hi; de-scaled e4m3),
                            in FP64
  ata_lowp(A32, fmt, cutoff, levels)
                            Algorithm 1 with HASA levels whose operand sums
                            are formed in FP32 and converted before each
                            product (the reduced-precision Strassen form)
  unpack, pack              packed lower <-> full symmetric matrix
  rel_fro, scaled_err, freivalds_residual
                            checkers: relative Frobenius error of packed
                            results (off-diagonal entries counted twice),
                            largest |dC_ij| / sqrt(C_ii C_jj), and the
                            Freivalds residual |C x - A^t (A x)| / (|A|_F^2 |x|)

Every function is pinned by tests that do not reuse it (hand values, closed
forms, brute force, library routines, planted mistakes).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import build, lib_path

__all__ = [
    "classical", "classical_mt", "ata", "hasa", "ata_mult_count", "unpack", "pack",
    "tri", "rel_fro", "scaled_err", "freivalds_residual", "bf16_round", "bf16_split",
    "e4m3_round", "pow2_column_scales", "gram_bf16x3", "gram_fp8", "STRASSEN", "WINOGRAD", "load",
    "potrf", "potrs", "atb", "project", "ata_lowp",
]

STRASSEN = 0
WINOGRAD = 1
_VARIANTS = {"strassen": STRASSEN, "winograd": WINOGRAD, STRASSEN: STRASSEN, WINOGRAD: WINOGRAD}

_lib = None


class Counts(ctypes.Structure):
    _fields_ = [
        ("mults", ctypes.c_int64),
        ("adds", ctypes.c_int64),
        ("ata_leaves", ctypes.c_int64),
        ("hasa_leaves", ctypes.c_int64),
        ("hasa_calls", ctypes.c_int64),
        ("max_hasa_depth", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def load():
    """Load the compiled oracle, compiling it first if no build exists."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.ora_classical.argtypes = [dp, i64, i64, i64, dp]
    lib.ora_classical.restype = None
    lib.ora_classical_mt.argtypes = [dp, i64, i64, i64, i64, i64, dp, ctypes.c_int]
    lib.ora_classical_mt.restype = ctypes.c_int
    lib.ora_ata.argtypes = [dp, i64, i64, i64, dp, i64, ctypes.c_int, ctypes.c_int,
                            ctypes.POINTER(Counts)]
    lib.ora_ata.restype = None
    lib.ora_hasa.argtypes = [dp, i64, dp, i64, i64, i64, i64, dp, i64, i64, ctypes.c_int,
                             ctypes.c_int, ctypes.POINTER(Counts)]
    lib.ora_hasa.restype = None
    lib.ora_ata_mult_count.argtypes = [i64, i64, i64, ctypes.c_int]
    lib.ora_ata_mult_count.restype = i64
    lib.ora_potrf.argtypes = [dp, i64]
    lib.ora_potrf.restype = i64
    lib.ora_potrs.argtypes = [dp, i64, dp, i64, i64]
    lib.ora_potrs.restype = None
    lib.ora_atb.argtypes = [dp, i64, i64, i64, dp, i64, i64, dp, i64]
    lib.ora_atb.restype = None
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_rows(A: np.ndarray):
    """Return (buffer, m, n, lda) for a row-major float64 matrix view."""
    A = np.asarray(A)
    if A.dtype != np.float64:
        raise TypeError("the oracle works in float64")
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    m, n = A.shape
    if A.strides[1] != 8 or (m > 1 and A.strides[0] % 8) or (m > 1 and A.strides[0] < 8 * n):
        A = np.ascontiguousarray(A)
    lda = A.strides[0] // 8 if m > 1 else max(n, 1)
    return A, m, n, lda


def tri(n: int) -> int:
    return n * (n + 1) // 2


def classical(A: np.ndarray) -> np.ndarray:
    """Packed lower triangle of A^t A by the plain definition (k ascending)."""
    A, m, n, lda = _as_rows(A)
    C = np.zeros(tri(n), dtype=np.float64)
    if n:
        load().ora_classical(_dptr(A), m, n, lda, _dptr(C))
    return C


def classical_mt(A: np.ndarray, rows=None, threads: int | None = None) -> np.ndarray:
    """Packed rows [i0, i1) of the lower triangle (all rows by default), by the
    plain definition, tiled and threaded; bitwise equal to classical()."""
    A, m, n, lda = _as_rows(A)
    i0, i1 = (0, n) if rows is None else rows
    if threads is None:
        threads = os.cpu_count() or 1
    C = np.zeros(tri(i1) - tri(i0), dtype=np.float64)
    if i1 > i0:
        rc = load().ora_classical_mt(_dptr(A), m, n, lda, i0, i1, _dptr(C), int(threads))
        if rc < 0:
            raise ValueError("bad row range")
    return C


def ata(A: np.ndarray, cutoff: int = 32, variant="strassen", max_depth: int = -1):
    """Algorithm 1 (ATA) with HASA off-diagonal products.

    cutoff: base case when m <= cutoff or n <= cutoff; HASA stops at
    min(M, K, N) <= cutoff.  max_depth >= 0 additionally caps the number of
    Strassen levels inside each HASA call.  Returns (packed C, counts dict).
    """
    if cutoff < 1:
        raise ValueError("cutoff must be >= 1")
    A, m, n, lda = _as_rows(A)
    C = np.zeros(tri(n), dtype=np.float64)
    cnt = Counts()
    if n:
        load().ora_ata(_dptr(A), m, n, lda, _dptr(C), int(cutoff), _VARIANTS[variant],
                       int(max_depth), ctypes.byref(cnt))
    return C, cnt.as_dict()


def hasa(X: np.ndarray, Y: np.ndarray, cutoff: int = 32, variant="strassen", max_depth: int = -1):
    """D = X Y by the rectangular Strassen recursion.  Returns (D, counts)."""
    if cutoff < 1:
        raise ValueError("cutoff must be >= 1")
    X, M, K, ldx = _as_rows(X)
    Y, K2, N, ldy = _as_rows(Y)
    if K != K2:
        raise ValueError("inner dimensions differ")
    D = np.zeros((M, N), dtype=np.float64)
    cnt = Counts()
    if M and N:
        load().ora_hasa(_dptr(X), ldx, _dptr(Y), ldy, M, K, N, _dptr(D), max(N, 1), int(cutoff),
                        _VARIANTS[variant], int(max_depth), ctypes.byref(cnt))
    return D, cnt.as_dict()


def ata_mult_count(m: int, n: int, cutoff: int, max_depth: int = -1) -> int:
    """Scalar multiplications of Algorithm 1 for an m x n input."""
    return int(load().ora_ata_mult_count(int(m), int(n), int(cutoff), int(max_depth)))


def potrf(Cp: np.ndarray, n: int):
    """Cholesky factor of the packed lower SPD matrix Cp (a copy is factored).
    Returns (packed L, info): info 0, or p + 1 for the first row p whose pivot
    is not positive (rows from p on are then unspecified)."""
    L = np.array(Cp, dtype=np.float64, copy=True)
    if L.shape != (tri(n),):
        raise ValueError("packed length must be n(n+1)/2")
    info = int(load().ora_potrf(_dptr(L), n)) if n else 0
    return L, info


def potrs(L: np.ndarray, n: int, B: np.ndarray) -> np.ndarray:
    """X with L L^t X = B for packed lower L; B is n x nrhs (or length n)."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    X = np.array(B, dtype=np.float64, copy=True, order="C")
    vec = X.ndim == 1
    X2 = X.reshape(n, 1) if vec else X
    if n and X2.shape[1]:
        load().ora_potrs(_dptr(L), n, _dptr(X2), X2.shape[1], X2.shape[1])
    return X2.reshape(-1) if vec else X2


def atb(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A^t B for A m x n and B m x nrhs (or length m), i ascending."""
    A, m, n, lda = _as_rows(A)
    Bv = np.ascontiguousarray(B, dtype=np.float64)
    vec = Bv.ndim == 1
    B2 = Bv.reshape(m, 1) if vec else Bv
    r = B2.shape[1]
    out = np.zeros((n, r))
    if n and r:
        load().ora_atb(_dptr(A), m, n, lda, _dptr(B2), r, r, _dptr(out), r)
    return out.reshape(-1) if vec else out


def project(A: np.ndarray, B: np.ndarray, info_out: list | None = None) -> np.ndarray:
    """P B for the projection P = A (A^t A)^-1 A^t onto the columns of A
    (Section 1): the normal equations solved through the plain product, its
    Cholesky factor and the two substitutions, then A X."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    L, info = potrf(classical(A), n)
    if info_out is not None:
        info_out.append(info)
    X = potrs(L, n, atb(A, B))
    return A @ X


# -------------------------------------------------------------------------
# Layout helpers and checks
# -------------------------------------------------------------------------

def unpack(Cp: np.ndarray, n: int) -> np.ndarray:
    """Full symmetric n x n matrix from the row-major packed lower triangle
    (entry (i, j), j <= i, at i(i+1)/2 + j)."""
    full = np.zeros((n, n), dtype=np.asarray(Cp).dtype)
    il = np.tril_indices(n)
    full[il] = Cp  # row-major order of tril_indices matches the packing
    full.T[il] = Cp
    return full


def pack(full: np.ndarray) -> np.ndarray:
    n = full.shape[0]
    return np.ascontiguousarray(full[np.tril_indices(n)])


def rel_fro(C: np.ndarray, ref: np.ndarray, n: int) -> float:
    """Relative Frobenius error of packed C against packed ref, measured on
    the full symmetric matrices (off-diagonal entries counted twice)."""
    C = np.asarray(C, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = C - ref
    diag = np.array([tri(i + 1) - 1 for i in range(n)], dtype=np.int64)
    w = np.full(d.shape, 2.0)
    w[diag] = 1.0
    num = float(np.sqrt(np.sum(w * d * d)))
    den = float(np.sqrt(np.sum(w * ref * ref)))
    return num / den if den > 0 else num


def scaled_err(C: np.ndarray, ref: np.ndarray, n: int) -> float:
    """max |C_ij - ref_ij| / sqrt(ref_ii ref_jj) over the lower triangle."""
    C = np.asarray(C, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    diag = np.array([ref[tri(i + 1) - 1] for i in range(n)])
    ii, jj = np.tril_indices(n)
    den = np.sqrt(np.abs(diag[ii] * diag[jj]))
    den[den == 0] = 1.0
    return float(np.max(np.abs(C - ref) / den)) if n else 0.0


def freivalds_residual(Cp: np.ndarray, A: np.ndarray, x: np.ndarray) -> float:
    """|| C x - A^t (A x) || / (||A||_F^2 ||x||): a probabilistic check of C = A^t A
    in O(mn + n^2) work."""
    n = A.shape[1]
    C = unpack(np.asarray(Cp, dtype=np.float64), n)
    A = np.asarray(A, dtype=np.float64)
    lhs = C @ x
    rhs = A.T @ (A @ x)
    scale = float(np.sum(A * A)) * float(np.linalg.norm(x))
    return float(np.linalg.norm(lhs - rhs)) / scale if scale > 0 else float(np.linalg.norm(lhs - rhs))


# -------------------------------------------------------------------------
# Number formats for the reduced-precision forms
# -------------------------------------------------------------------------

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round binary32 values to bfloat16 (round to nearest, ties to even),
    returned as binary32.  bfloat16 keeps the top 16 bits of binary32; NaN
    stays NaN."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


def bf16_split(x: np.ndarray):
    """hi = bf16(x), lo = bf16(x - hi) with x - hi formed exactly in binary32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round((x - hi).astype(np.float32))
    return hi, lo


E4M3_MAX = 448.0


def e4m3_round(x: np.ndarray) -> np.ndarray:
    """Round binary32 values to OCP e4m3 (1 sign, 4 exponent bits with bias 7,
    3 mantissa bits, no infinities, max finite 448), ties to even, saturating
    to +-448; returned as float64 values."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    # normal binade [2^e, 2^(e+1)), e in [-6, 8], step 2^(e-3); subnormals step 2^-9
    _, ex = np.frexp(np.where(a > 0, a, 1.0))  # a = f 2^ex with f in [0.5, 1)
    e = np.clip(ex.astype(np.float64) - 1.0, -6, 8)
    step = np.exp2(e - 3)
    q = a / step
    r = np.round(q)  # numpy rounds half to even
    out = r * step
    out = np.minimum(out, E4M3_MAX)
    out[a == 0] = 0.0
    return np.copysign(out, x)


def gram_bf16x3(A32: np.ndarray) -> np.ndarray:
    """What the bfloat16 split form computes, in exact-as-possible FP64:
    packed lower of hi^t hi + hi^t lo + lo^t hi with hi, lo = bf16_split(A)
    (the lo^t lo term is dropped by the method)."""
    hi, lo = bf16_split(np.asarray(A32, dtype=np.float32))
    hi = hi.astype(np.float64)
    lo = lo.astype(np.float64)
    full = hi.T @ hi + hi.T @ lo + lo.T @ hi
    return pack(full)


def gram_fp8(A32: np.ndarray) -> np.ndarray:
    """What the e4m3 form computes, in FP64: with power-of-two column scales
    s, Q = e4m3(A diag(s)) and C = diag(s)^-1 Q^t Q diag(s)^-1 (packed lower)."""
    A32 = np.asarray(A32, dtype=np.float32)
    s = pow2_column_scales(A32.astype(np.float64))
    Q = e4m3_round(A32.astype(np.float64) * s[None, :])
    full = (Q.T @ Q) / s[:, None] / s[None, :]
    return pack(full)


def _lowp_leaf(X: np.ndarray, Y: np.ndarray, fmt: str, xs=None, ys=None) -> np.ndarray:
    """X (M x K) Y (K x N) of binary32 operands in a reduced-precision form,
    exactly in FP64: 'bf16x3' splits each operand (hi = bf16(x),
    lo = bf16(x - hi)) and keeps hi hi + hi lo + lo hi; 'fp8' rounds
    diag(xs) X and Y diag(ys) to e4m3 and scales back, with xs, ys the
    power-of-two scales of X's rows and Y's columns (computed from the
    operands when not given)."""
    X = np.asarray(X, dtype=np.float32)
    Y = np.asarray(Y, dtype=np.float32)
    if fmt == "bf16x3":
        xh, xl = bf16_split(X)
        yh, yl = bf16_split(Y)
        xh, xl, yh, yl = (v.astype(np.float64) for v in (xh, xl, yh, yl))
        return xh @ yh + xh @ yl + xl @ yh
    if fmt == "fp8":
        if xs is None:
            xs = pow2_column_scales(X.T.astype(np.float64))
        if ys is None:
            ys = pow2_column_scales(Y.astype(np.float64))
        qx = e4m3_round(X.astype(np.float64) * xs[:, None])
        qy = e4m3_round(Y.astype(np.float64) * ys[None, :])
        return (qx @ qy) / xs[:, None] / ys[None, :]
    raise ValueError("format must be 'bf16x3' or 'fp8'")


# Strassen (1969) and Winograd (1971) products as (left terms, right terms):
# each term (sign, row half, column half) of X or Y; result quadrants below.
_LP_STRASSEN = [
    ([(1, 0, 0), (1, 1, 1)], [(1, 0, 0), (1, 1, 1)]),  # M1 = (X11 + X22)(Y11 + Y22)
    ([(1, 1, 0), (1, 1, 1)], [(1, 0, 0)]),             # M2 = (X21 + X22) Y11
    ([(1, 0, 0)], [(1, 0, 1), (-1, 1, 1)]),            # M3 = X11 (Y12 - Y22)
    ([(1, 1, 1)], [(1, 1, 0), (-1, 0, 0)]),            # M4 = X22 (Y21 - Y11)
    ([(1, 0, 0), (1, 0, 1)], [(1, 1, 1)]),             # M5 = (X11 + X12) Y22
    ([(1, 1, 0), (-1, 0, 0)], [(1, 0, 0), (1, 0, 1)]), # M6 = (X21 - X11)(Y11 + Y12)
    ([(1, 0, 1), (-1, 1, 1)], [(1, 1, 0), (1, 1, 1)]), # M7 = (X12 - X22)(Y21 + Y22)
]
_LP_STRASSEN_D = [  # D_ac = sum of sign * M_p, in product order
    [(1, 0), (1, 3), (-1, 4), (1, 6)], [(1, 2), (1, 4)], [(1, 1), (1, 3)], [(1, 0), (-1, 1), (1, 2), (1, 5)]]


def _lowp_hasa(X, Y, fmt, cutoff, levels):
    """HASA (Strassen levels down to min(M, K, N) <= cutoff or `levels`
    levels) with every operand sum formed in binary32 and every leaf product
    taken in the reduced-precision form; combinations in FP64."""
    M, K = X.shape
    N = Y.shape[1]
    if levels == 0 or min(M, K, N) <= cutoff:
        return _lowp_leaf(X, Y, fmt)
    M1, K1, N1 = (M + 1) // 2, (K + 1) // 2, (N + 1) // 2

    def quad(Z, a, b, R, C):
        q = np.zeros((R, C), dtype=np.float32)
        blk = Z[a * R:(a + 1) * R, b * C:(b + 1) * C]
        q[:blk.shape[0], :blk.shape[1]] = blk
        return q

    Xq = {(a, b): quad(X, a, b, M1, K1) for a in (0, 1) for b in (0, 1)}
    Yq = {(a, b): quad(Y, a, b, K1, N1) for a in (0, 1) for b in (0, 1)}

    def opsum(q, terms):
        acc = None
        for sg, a, b in terms:
            v = q[(a, b)] if sg > 0 else -q[(a, b)]
            acc = v if acc is None else (acc + v).astype(np.float32)  # binary32 sum
        return acc

    P = [_lowp_hasa(opsum(Xq, xt), opsum(Yq, yt), fmt, cutoff, levels - 1) for xt, yt in _LP_STRASSEN]
    D = np.zeros((2 * M1, 2 * N1))
    for q, terms in enumerate(_LP_STRASSEN_D):
        acc = np.zeros((M1, N1))
        for sg, p in terms:
            acc = acc + sg * P[p]
        a, c = q >> 1, q & 1
        D[a * M1:(a + 1) * M1, c * N1:(c + 1) * N1] = acc
    return D[:M, :N]


def ata_lowp(A32: np.ndarray, fmt: str, cutoff: int, levels: int) -> np.ndarray:
    """Algorithm 1 in a reduced-precision form (packed lower C in FP64): the
    base-case blocks are products of the converted input (e4m3 with the
    power-of-two scale of each whole column of A, as one converted copy of A
    would hold it); each off-diagonal HASA product runs at most `levels`
    Strassen levels with binary32 operand sums and converted leaf operands
    (_lowp_hasa); the sums of the recursion are in FP64.  Strassen variant
    only.  For small inputs (a reference for tests)."""
    A32 = np.asarray(A32, dtype=np.float32)
    m, n = A32.shape
    cs = pow2_column_scales(A32.astype(np.float64)) if fmt == "fp8" else None
    C = np.zeros((n, n))

    def leaf(rows, c0, c1, d0, d1):
        X = A32[rows[0]:rows[1], c0:c1].T
        Y = A32[rows[0]:rows[1], d0:d1]
        if fmt == "fp8":
            return _lowp_leaf(X, Y, fmt, cs[c0:c1], cs[d0:d1])
        return _lowp_leaf(X, Y, fmt)

    def rec(r0, r1, c0, c1):
        mm, nn = r1 - r0, c1 - c0
        if mm <= 0 or nn <= 0:
            return
        if mm <= cutoff or nn <= cutoff:
            C[c0:c1, c0:c1] += leaf((r0, r1), c0, c1, c0, c1)
            return
        m1, n1 = (mm + 1) // 2, (nn + 1) // 2
        rec(r0, r0 + m1, c0, c0 + n1)
        rec(r0 + m1, r1, c0, c0 + n1)
        rec(r0, r0 + m1, c0 + n1, c1)
        rec(r0 + m1, r1, c0 + n1, c1)
        for (a0, a1) in ((r0, r0 + m1), (r0 + m1, r1)):
            if a1 > a0:
                X = A32[a0:a1, c0 + n1:c1].T
                Y = A32[a0:a1, c0:c0 + n1]
                C[c0 + n1:c1, c0:c0 + n1] += _lowp_hasa(X, Y, fmt, cutoff, levels)

    rec(0, m, 0, n)
    return pack(np.tril(C) + np.tril(C, -1).T)


def pow2_column_scales(A: np.ndarray, target: float = E4M3_MAX) -> np.ndarray:
    """Per-column power-of-two scales s_j = 2^floor(log2(target / max_k |A_kj|));
    a zero column gets scale 1."""
    amax = np.max(np.abs(np.asarray(A, dtype=np.float64)), axis=0) if A.shape[0] else np.zeros(A.shape[1])
    s = np.ones_like(amax)
    nz = amax > 0
    s[nz] = np.exp2(np.floor(np.log2(target / amax[nz])))
    return s

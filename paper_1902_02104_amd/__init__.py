"""MI355X-native A^t A (Arrigoni & Massini, ATA with Strassen off-diagonal
products): thin ctypes binding of libata.so.

Every step of the product runs in the library's HIP kernels; PyTorch only
provides device memory and streams.  The binding fails loudly when the
library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

__all__ = [
    "F64", "F32", "F32_BF16X3", "F32_FP8", "OUT_F64", "STRASSEN", "WINOGRAD",
    "load", "gram", "plan_info", "workspace_bytes", "default_cutoff", "status_string",
    "AtaError", "lib_path", "tri",
]

F64 = 0
F32 = 1
F32_BF16X3 = 2
F32_FP8 = 3
OUT_F64 = 0x100
STRASSEN = 0
WINOGRAD = 1
DEFAULT_MAX_DEPTH = 1
OPT_PRODUCT_TILES = 0x1
OPT_EQUILIBRATE = 0x2
OPT_OPERAND_SUMS = 0x4
OPT_ADAPTIVE = 0x8
OPT_EQUILIBRATE_AUTO = 0x10

_PKG = os.path.dirname(os.path.abspath(__file__))
_lib = None


def lib_path() -> str:
    return os.path.join(_PKG, "libata.so")


class AtaError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        extra = ""
        if status == 2 and _lib is not None:
            extra = " (hip error %d)" % _lib.ata_last_hip_error()
        super().__init__("%s: status %d (%s)%s" % (what or "ata", status, msg, extra))


class Opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("max_depth", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PlanStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "mults", "classical_mults", "syrk_tasks", "gemm_tasks", "strassen_tasks", "combine_tasks",
        "work_items", "phases", "ata_depth", "max_hasa_depth", "workspace_bytes", "cutoff",
        "strassen_mults", "gemm_mults", "syrk_mults", "combine_elems", "lp_staging")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def load():
    """Load the in-tree libata.so.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError("libata.so not built: run paper_1902_02104_amd/build.py (or "
                           "__graft_entry__.build()) first; there is no fallback path")
    lib = ctypes.CDLL(path)
    i64, vp, ci = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
    lib.ata.argtypes = [vp, i64, i64, i64, vp, ci, ci, vp]
    lib.ata.restype = ci
    lib.ata_ex.argtypes = [vp, i64, i64, i64, vp, ci, ci, vp, ctypes.POINTER(Opts), vp, ctypes.c_size_t]
    lib.ata_ex.restype = ci
    lib.ata_ex_noalloc.argtypes = [vp, i64, i64, i64, vp, ci, ci, vp, ctypes.POINTER(Opts),
                                   ctypes.POINTER(ctypes.c_size_t)]
    lib.ata_ex_noalloc.restype = ci
    lib.ata_workspace_bytes.argtypes = [i64, i64, ci, ci, ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_size_t)]
    lib.ata_workspace_bytes.restype = ci
    lib.ata_plan_info.argtypes = [i64, i64, ci, ci, ctypes.POINTER(Opts), ctypes.POINTER(PlanStats)]
    lib.ata_plan_info.restype = ci
    lib.ata_default_cutoff.argtypes = [i64, i64, ci]
    lib.ata_default_cutoff.restype = ci
    lib.ata_status_string.argtypes = [ci]
    lib.ata_status_string.restype = ctypes.c_char_p
    lib.ata_last_hip_error.argtypes = []
    lib.ata_last_hip_error.restype = ci
    lib.ata_version.argtypes = []
    lib.ata_version.restype = ctypes.c_char_p
    lib.ata_release_caches.argtypes = []
    lib.ata_release_caches.restype = None
    lib.ata_precision_convert.argtypes = [ci, vp, i64, vp, vp, vp]
    lib.ata_precision_convert.restype = ci
    lib.ata_profile_enable.argtypes = [ci]
    lib.ata_profile_enable.restype = ci
    lib.ata_profile_collect.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), ci]
    lib.ata_profile_collect.restype = ci
    lib.ata_aat.argtypes = [vp, i64, i64, i64, vp, ci, ci, vp]
    lib.ata_aat.restype = ci
    lib.ata_potrf.argtypes = [vp, i64, ci, vp, vp]
    lib.ata_potrf.restype = ci
    lib.ata_potrs.argtypes = [vp, i64, vp, i64, i64, ci, vp]
    lib.ata_potrs.restype = ci
    lib.ata_atb.argtypes = [vp, i64, i64, i64, vp, i64, i64, vp, i64, ci, vp]
    lib.ata_atb.restype = ci
    lib.ata_normal_solve.argtypes = [vp, i64, i64, i64, vp, i64, i64, vp, i64, ci, ci, vp, vp]
    lib.ata_normal_solve.restype = ci
    lib.ata_project.argtypes = [vp, i64, i64, i64, vp, i64, i64, vp, i64, ci, ci, vp, vp]
    lib.ata_project.restype = ci
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().ata_status_string(int(status)).decode()


def tri(n: int) -> int:
    return n * (n + 1) // 2


def _opts(variant, max_depth, dtype=F64, intile=None, equilibrate=None, operand_sums=False, adaptive=None):
    """The options struct for a call, or None for the library's defaults
    (ATA_DEFAULT_MAX_DEPTH levels, adaptive depth, equilibration with
    Strassen levels, product tiles for FP64) when nothing is chosen."""
    if (max_depth is None and intile is None and equilibrate is None and not operand_sums and adaptive is None
            and variant in ("strassen", STRASSEN)):
        return None
    o = Opts()
    o.variant = {"strassen": STRASSEN, "winograd": WINOGRAD}.get(variant, variant)
    if max_depth is None:
        # reduced-precision leaves are classical; the other forms take the default level count
        max_depth = 0 if (dtype & 0xff) in (F32_BF16X3, F32_FP8) else DEFAULT_MAX_DEPTH
    o.max_depth = int(max_depth)
    intile = True if intile is None else intile
    o.flags = ((0 if intile else OPT_PRODUCT_TILES) | (OPT_EQUILIBRATE if equilibrate else 0)
               | (OPT_OPERAND_SUMS if operand_sums else 0) | (OPT_ADAPTIVE if adaptive else 0))
    return o


def _optp(o):
    return ctypes.byref(o) if o is not None else None


def plan_info(m: int, n: int, cutoff: int = 0, dtype: int = F64, variant="strassen", max_depth=None,
              intile=None, equilibrate=None, operand_sums=False, adaptive=None) -> dict:
    """Host-only description of the device plan (no GPU needed)."""
    st = PlanStats()
    o = _opts(variant, max_depth, dtype, intile, equilibrate, operand_sums, adaptive)
    rc = load().ata_plan_info(int(m), int(n), int(dtype), int(cutoff), _optp(o), ctypes.byref(st))
    if rc:
        raise AtaError(rc, "ata_plan_info")
    return st.as_dict()


def workspace_bytes(m: int, n: int, cutoff: int = 0, dtype: int = F64, variant="strassen", max_depth=None,
                    intile=None, equilibrate=None, operand_sums=False, adaptive=None) -> int:
    out = ctypes.c_size_t(0)
    o = _opts(variant, max_depth, dtype, intile, equilibrate, operand_sums, adaptive)
    rc = load().ata_workspace_bytes(int(m), int(n), int(dtype), int(cutoff), _optp(o), ctypes.byref(out))
    if rc:
        raise AtaError(rc, "ata_workspace_bytes")
    return int(out.value)


def precision_convert(x, dtype: int, stream=None):
    """Element conversions of the reduced-precision forms, run on the device:
    F32_BF16X3 -> (hi, lo) int16 tensors of bfloat16 bits; F32_FP8 -> uint8
    tensor of OCP e4m3 bytes."""
    import torch
    lib = load()
    x = x.contiguous()
    if x.dtype != torch.float32 or not x.is_cuda:
        raise ValueError("x must be a float32 device tensor")
    if (dtype & 0xff) == F32_BF16X3:
        o0 = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
        o1 = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
        p1 = ctypes.c_void_p(o1.data_ptr())
    elif (dtype & 0xff) == F32_FP8:
        o0 = torch.empty(x.numel(), dtype=torch.uint8, device=x.device)
        o1, p1 = None, None
    else:
        raise ValueError("dtype must be F32_BF16X3 or F32_FP8")
    with torch.cuda.device(x.device):
        rc = lib.ata_precision_convert(int(dtype), ctypes.c_void_p(x.data_ptr()), x.numel(),
                                       ctypes.c_void_p(o0.data_ptr()), p1, _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_precision_convert")
    return (o0, o1) if o1 is not None else o0


KERNEL_KINDS = ("strassen", "gemm", "syrk", "combine", "other", "factor_panel", "factor_update", "solve", "tiles")


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events on its stream."""
    load().ata_profile_enable(1 if on else 0)


def profile_collect() -> dict:
    """Wait for recorded launches; return {kind: (total_ms, launches)} and clear."""
    k = len(KERNEL_KINDS)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    rc = load().ata_profile_collect(ms, cnt, k)
    if rc < 0 or rc > k:
        raise AtaError(rc, "ata_profile_collect")
    return {name: (ms[i], int(cnt[i])) for i, name in enumerate(KERNEL_KINDS)}


def release_caches() -> None:
    """Free cached plans, their device tables and helper streams (waits for
    the devices that hold them to go idle)."""
    load().ata_release_caches()


def default_cutoff(m: int, n: int, dtype: int = F64) -> int:
    return int(load().ata_default_cutoff(int(m), int(n), int(dtype)))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def gram(A, cutoff: int = 0, dtype: int | None = None, variant="strassen", max_depth=None, out=None,
         workspace=None, stream=None, intile=None, equilibrate=None, operand_sums=False, adaptive=None):
    """Packed lower triangle of A^t A for a 2-D CUDA tensor A (row-major rows,
    unit column stride, row stride >= n).  Asynchronous on `stream` (default:
    torch's current stream).  Returns the packed output tensor.  intile: run
    the last Strassen level inside each workgroup tile (default), else as
    product tiles summed by a combination pass (OPT_PRODUCT_TILES);
    equilibrate: power-of-two column scaling around the product
    (OPT_EQUILIBRATE); operand_sums: product tiles on operand sums formed in
    a memory pass (OPT_OPERAND_SUMS)."""
    import torch
    lib = load()
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    m, n = A.shape
    if n > 0 and m > 0 and A.stride(1) != 1:
        raise ValueError("A needs unit column stride")
    lda = A.stride(0) if m > 1 else max(n, 1)
    if dtype is None:
        dtype = F64 if A.dtype == torch.float64 else F32
    want_in = torch.float64 if (dtype & 0xff) == F64 else torch.float32
    if A.dtype != want_in:
        raise TypeError("A must be %s for dtype %#x" % (want_in, dtype))
    out_t = torch.float64 if ((dtype & 0xff) == F64 or dtype & OUT_F64) else torch.float32
    if out is None:
        out = torch.empty(tri(n), dtype=out_t, device=A.device)
    elif out.dtype != out_t or out.numel() < tri(n) or not out.is_contiguous():
        raise ValueError("bad output tensor")
    o = _opts(variant, max_depth, dtype, intile, equilibrate, operand_sums, adaptive)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    with torch.cuda.device(A.device):
        rc = lib.ata_ex(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(out.data_ptr()), int(dtype),
                        int(cutoff), _stream_handle(stream), _optp(o),
                        ctypes.c_void_p(ws_ptr) if ws_ptr else None, ws_bytes)
    if rc:
        raise AtaError(rc, "ata_ex")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # ATA_NOALLOC_SCRATCH_BYTES


def gram_noalloc(A, out, cutoff: int = 0, dtype: int | None = None, variant="strassen", max_depth=None,
                 stream=None, intile=None, equilibrate=None, operand_sums=False, adaptive=None):
    """gram() through ata_ex_noalloc: no device allocation by the library (the
    plan tables and workspace live in its fixed per-GPU scratch array), so
    the output tensor `out` must be given.  Returns (out, scratch bytes the
    call used).  Calls that overlap on one GPU race on the shared array."""
    import torch
    lib = load()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    m, n = A.shape
    if n > 0 and m > 0 and A.stride(1) != 1:
        raise ValueError("A needs unit column stride")
    lda = A.stride(0) if m > 1 else max(n, 1)
    if dtype is None:
        dtype = F64 if A.dtype == torch.float64 else F32
    want_in = torch.float64 if (dtype & 0xff) == F64 else torch.float32
    if A.dtype != want_in:
        raise TypeError("A must be %s for dtype %#x" % (want_in, dtype))
    out_t = torch.float64 if ((dtype & 0xff) == F64 or dtype & OUT_F64) else torch.float32
    if out.dtype != out_t or out.numel() < tri(n) or not out.is_contiguous() or not out.is_cuda:
        raise ValueError("bad output tensor")
    o = _opts(variant, max_depth, dtype, intile, equilibrate, operand_sums, adaptive)
    used = ctypes.c_size_t(0)
    with torch.cuda.device(A.device):
        rc = lib.ata_ex_noalloc(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(out.data_ptr()), int(dtype),
                                int(cutoff), _stream_handle(stream), _optp(o), ctypes.byref(used))
    if rc:
        raise AtaError(rc, "ata_ex_noalloc")
    return out, int(used.value)


def gram_rows(A, cutoff: int = 0, dtype: int | None = None, out=None, stream=None):
    """Packed lower triangle of the companion product A A^t (m x m) for a 2-D
    device tensor A, through the product of A^t with itself (ata_aat)."""
    import torch
    lib = load()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    m, n = A.shape
    if n > 0 and m > 0 and A.stride(1) != 1:
        raise ValueError("A needs unit column stride")
    lda = A.stride(0) if m > 1 else max(n, 1)
    if dtype is None:
        dtype = F64 if A.dtype == torch.float64 else F32
    want_in = torch.float64 if (dtype & 0xff) == F64 else torch.float32
    if A.dtype != want_in:
        raise TypeError("A must be %s for dtype %#x" % (want_in, dtype))
    out_t = torch.float64 if ((dtype & 0xff) == F64 or dtype & OUT_F64) else torch.float32
    if out is None:
        out = torch.empty(tri(m), dtype=out_t, device=A.device)
    elif out.dtype != out_t or out.numel() < tri(m) or not out.is_contiguous():
        raise ValueError("bad output tensor")
    with torch.cuda.device(A.device):
        rc = lib.ata_aat(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(out.data_ptr()), int(dtype),
                         int(cutoff), _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_aat")
    return out


# -------------------------------------------------------------------------
# Normal equations: Cholesky factor, triangular solves, A^t B
# -------------------------------------------------------------------------

def _solve_dtype(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("float64 or float32 tensors only")


def _rows2d(B, n, dtype, what):
    """(tensor, rows, nrhs, row stride) of a length-n vector or n x r matrix
    with unit column stride on the device."""
    if not B.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if _solve_dtype(B) != dtype:
        raise TypeError("%s must have the factor's dtype" % what)
    if B.dim() == 1:
        if B.shape[0] != n or (n > 1 and B.stride(0) != 1):
            raise ValueError("%s must be a contiguous vector of length %d" % (what, n))
        return B, n, 1, 1
    if B.dim() != 2 or B.shape[0] != n:
        raise ValueError("%s must have %d rows" % (what, n))
    r = B.shape[1]
    if n > 0 and r > 0 and B.stride(1) != 1:
        raise ValueError("%s needs unit column stride" % what)
    return B, n, r, (B.stride(0) if n > 1 else max(r, 1))


def _order(packed, n):
    if n is None:
        n = int((math.isqrt(8 * packed.numel() + 1) - 1) // 2)
    if packed.dim() != 1 or packed.numel() < tri(n) or not packed.is_contiguous():
        raise ValueError("packed triangle must be a contiguous vector of n(n+1)/2 entries")
    return n


def cholesky(C, n: int | None = None, info=None, stream=None):
    """Cholesky factor of the packed lower SPD matrix C (device tensor), in
    place: C then holds L with L L^t = C.  info: optional int32 device tensor
    of one element that receives 0, or p + 1 for the first column p whose
    pivot is not positive.  Returns C."""
    import torch
    lib = load()
    if not C.is_cuda:
        raise ValueError("C must be a device tensor")
    n = _order(C, n)
    if info is not None and (info.dtype != torch.int32 or not info.is_cuda or info.numel() < 1):
        raise ValueError("info must be an int32 device tensor")
    with torch.cuda.device(C.device):
        rc = lib.ata_potrf(ctypes.c_void_p(C.data_ptr()), n, _solve_dtype(C),
                           ctypes.c_void_p(info.data_ptr()) if info is not None else None, _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_potrf")
    return C


def cholesky_solve(L, B, n: int | None = None, stream=None):
    """Solve L L^t X = B in place (B: length-n vector or n x r matrix on the
    device, unit column stride) for the packed factor L.  Returns B."""
    import torch
    lib = load()
    n = _order(L, n)
    dt = _solve_dtype(L)
    B, _, r, ldb = _rows2d(B, n, dt, "B")
    with torch.cuda.device(L.device):
        rc = lib.ata_potrs(ctypes.c_void_p(L.data_ptr()), n, ctypes.c_void_p(B.data_ptr()), r, ldb, dt,
                           _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_potrs")
    return B


def atb(A, B, out=None, stream=None):
    """A^t B for device tensors A (m x n) and B (length m or m x r)."""
    import torch
    lib = load()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    m, n = A.shape
    if m > 0 and n > 0 and A.stride(1) != 1:
        raise ValueError("A needs unit column stride")
    lda = A.stride(0) if m > 1 else max(n, 1)
    dt = _solve_dtype(A)
    B, _, r, ldb = _rows2d(B, m, dt, "B")
    shape = (n,) if B.dim() == 1 else (n, r)
    if out is None:
        out = torch.empty(shape, dtype=A.dtype, device=A.device)
    out, _, _, ldo = _rows2d(out, n, dt, "out")
    with torch.cuda.device(A.device):
        rc = lib.ata_atb(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(B.data_ptr()), r, ldb,
                         ctypes.c_void_p(out.data_ptr()), ldo, dt, _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_atb")
    return out


def normal_solve(A, B, cutoff: int = 0, X=None, info=None, stream=None):
    """Least-squares solution X = (A^t A)^-1 A^t B through the normal
    equations: the packed product, its Cholesky factor, A^t B and the two
    triangular solves, all on the device.  info as for cholesky().  Returns X."""
    import torch
    lib = load()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    m, n = A.shape
    if m > 0 and n > 0 and A.stride(1) != 1:
        raise ValueError("A needs unit column stride")
    lda = A.stride(0) if m > 1 else max(n, 1)
    dt = _solve_dtype(A)
    B, _, r, ldb = _rows2d(B, m, dt, "B")
    if X is None:
        X = torch.empty((n,) if B.dim() == 1 else (n, r), dtype=A.dtype, device=A.device)
    X, _, _, ldx = _rows2d(X, n, dt, "X")
    if info is not None and (info.dtype != torch.int32 or not info.is_cuda or info.numel() < 1):
        raise ValueError("info must be an int32 device tensor")
    with torch.cuda.device(A.device):
        rc = lib.ata_normal_solve(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(B.data_ptr()), r, ldb,
                                  ctypes.c_void_p(X.data_ptr()), ldx, dt, int(cutoff),
                                  ctypes.c_void_p(info.data_ptr()) if info is not None else None,
                                  _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_normal_solve")
    return X


def project(A, B, cutoff: int = 0, out=None, info=None, stream=None):
    """P B for the projection P = A (A^t A)^-1 A^t onto the columns of A
    (device tensors; B of length m or m x r): the normal equations on the
    device, then A X.  info as for cholesky().  Returns out."""
    import torch
    lib = load()
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    m, n = A.shape
    if m > 0 and n > 0 and A.stride(1) != 1:
        raise ValueError("A needs unit column stride")
    lda = A.stride(0) if m > 1 else max(n, 1)
    dt = _solve_dtype(A)
    B, _, r, ldb = _rows2d(B, m, dt, "B")
    if out is None:
        out = torch.empty((m,) if B.dim() == 1 else (m, r), dtype=A.dtype, device=A.device)
    out, _, _, ldo = _rows2d(out, m, dt, "out")
    if info is not None and (info.dtype != torch.int32 or not info.is_cuda or info.numel() < 1):
        raise ValueError("info must be an int32 device tensor")
    with torch.cuda.device(A.device):
        rc = lib.ata_project(ctypes.c_void_p(A.data_ptr()), m, n, lda, ctypes.c_void_p(B.data_ptr()), r, ldb,
                             ctypes.c_void_p(out.data_ptr()), ldo, dt, int(cutoff),
                             ctypes.c_void_p(info.data_ptr()) if info is not None else None,
                             _stream_handle(stream))
    if rc:
        raise AtaError(rc, "ata_project")
    return out

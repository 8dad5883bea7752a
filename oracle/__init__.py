"""CPU oracle for split-BF16 GEMM, LU and iterative refinement.

TEST INFRASTRUCTURE ONLY: the slow, plain statement of what the GPU library
computes, written from the paper (Henry, Tang & Heinecke 2019).  Only the test
suite, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.

Pins: every function here is checked against the paper's invariants, closed
forms, library routines or exact arithmetic in ``tests/test_oracle_*.py``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_int = ctypes.c_int


def lib():
    """Load (building on first use if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_bf16_rne.argtypes = [ctypes.c_float]
        L.orc_bf16_rne.restype = ctypes.c_uint16
        L.orc_split.argtypes = [_f32p, _i64, _u16p, _u16p, ctypes.c_void_p]
        L.orc_split.restype = None
        L.orc_gemm_ex.argtypes = [_int, _int, _i64, _i64, _i64, ctypes.c_float,
                                  _f32p, _i64, _f32p, _i64, ctypes.c_float,
                                  _f32p, _i64]
        L.orc_gemm_ex.restype = _int
        L.orc_dot_partials.argtypes = [_i64, _f32p, _i64, _f32p, _i64, _f32p]
        L.orc_dot_partials.restype = _int
        L.orc_gemm_entries.argtypes = [_int, _i64, _f32p, _i64, _f32p, _i64,
                                       _i64, _i64p, _i64p, _f32p]
        L.orc_gemm_entries.restype = _int
        L.orc_sgemm.argtypes = [_i64, _i64, _i64, ctypes.c_float, _f32p, _i64,
                                _f32p, _i64, ctypes.c_float, _f32p, _i64]
        L.orc_sgemm.restype = _int
        L.orc_sgemm_entries.argtypes = [_i64, _f32p, _i64, _f32p, _i64, _i64,
                                        _i64p, _i64p, _f32p]
        L.orc_sgemm_entries.restype = _int
        L.orc_lu.argtypes = [_int, _i64, _f32p, _i64, _i32p, _i64]
        L.orc_lu.restype = _int
        L.orc_lu_solve.argtypes = [_i64, _f32p, _i64, _i32p, _f32p]
        L.orc_lu_solve.restype = _int
        L.orc_ir.argtypes = [_i64, _f32p, _i64, _f32p, _i64, _i32p, _f64p,
                             _f64p, ctypes.c_double, _int,
                             ctypes.POINTER(_int), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(_int), _f64p]
        L.orc_ir.restype = _int
        L.orc_gmres_ir.argtypes = [_i64, _f32p, _i64, _f32p, _i64, _i32p, _f64p, _f64p,
                                   ctypes.c_double, _int, _int, ctypes.c_double,
                                   ctypes.POINTER(_int), ctypes.POINTER(_int),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_int), _f64p]
        L.orc_gmres_ir.restype = _int
        L.orc_residual.argtypes = [_i64, _f32p, _i64, _f64p, _f64p, _f64p]
        L.orc_residual.restype = None
        L.orc_inf_norm_mat.argtypes = [_i64, _f32p, _i64]
        L.orc_inf_norm_mat.restype = ctypes.c_double
        L.orc_lu_fmt.argtypes = [_int, _i64, _f32p, _i64, _i32p]
        L.orc_lu_fmt.restype = _int
        L.orc_round_fmt.argtypes = [ctypes.c_double, _int]
        L.orc_round_fmt.restype = ctypes.c_double
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = _int
        _lib = L
    return _lib


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def num_threads() -> int:
    return lib().orc_num_threads()


def bf16_rne(x: float) -> int:
    """FP32 -> BF16 bit pattern, round to nearest even, saturating (Sec. II-A)."""
    return int(lib().orc_bf16_rne(float(np.float32(x))))


def split(a, nterms: int = 3):
    """Sec. II-A split of every element; returns uint16 planes (b0, b1[, b2])."""
    a = _c32(a)
    flat = a.reshape(-1)
    b0 = np.empty(flat.shape, np.uint16)
    b1 = np.empty(flat.shape, np.uint16)
    b2 = np.empty(flat.shape, np.uint16) if nterms == 3 else None
    lib().orc_split(flat, flat.size, b0, b1,
                    b2.ctypes.data_as(ctypes.c_void_p) if b2 is not None else None)
    planes = [b0.reshape(a.shape), b1.reshape(a.shape)]
    if b2 is not None:
        planes.append(b2.reshape(a.shape))
    return tuple(planes)


def bf16_bits_to_f32(h):
    """Widen BF16 bit patterns to the FP32 values they denote (exact)."""
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def gemm(variant: int, A, B, C=None, alpha: float = 1.0, beta: float = 0.0,
         fp64_sum: bool = False):
    """Split GEMM C = alpha*(A x B) + beta*C with `variant` products (Sec. II-D, IV-A)."""
    A = _c32(A)
    B = _c32(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    if C is None:
        C = np.zeros((M, N), np.float32)
    C = _c32(C).copy()
    rc = lib().orc_gemm_ex(variant, int(fp64_sum), M, N, K, alpha, A,
                           max(K, 1), B, max(N, 1), beta, C, max(N, 1))
    if rc != 0:
        raise ValueError(f"orc_gemm_ex returned {rc}")
    return C


def dot_partials(x, y):
    """The nine FP32 partial inner products Z^(i,j) (Sec. II-D) of x . y."""
    x = _c32(x)
    y = _c32(y)
    Z = np.zeros(9, np.float32)
    rc = lib().orc_dot_partials(x.size, x, 1, y, 1, Z)
    if rc:
        raise ValueError(rc)
    return Z.reshape(3, 3)


def gemm_entries(variant: int, A, B, rows, cols):
    """Entries C[rows[t], cols[t]] of the split product A x B (alpha=1, beta=0)."""
    A = _c32(A)
    B = _c32(B)
    rows = np.ascontiguousarray(rows, np.int64)
    cols = np.ascontiguousarray(cols, np.int64)
    out = np.zeros(rows.size, np.float32)
    rc = lib().orc_gemm_entries(variant, A.shape[1], A, A.shape[1], B, B.shape[1],
                                rows.size, rows, cols, out)
    if rc:
        raise ValueError(rc)
    return out


def sgemm(A, B, C=None, alpha: float = 1.0, beta: float = 0.0):
    """Plain FP32 GEMM, one FMA per term in index order (Sec. II-C)."""
    A = _c32(A)
    B = _c32(B)
    M, K = A.shape
    _, N = B.shape
    if C is None:
        C = np.zeros((M, N), np.float32)
    C = _c32(C).copy()
    rc = lib().orc_sgemm(M, N, K, alpha, A, max(K, 1), B, max(N, 1), beta, C,
                         max(N, 1))
    if rc:
        raise ValueError(rc)
    return C


def sgemm_entries(A, B, rows, cols):
    A = _c32(A)
    B = _c32(B)
    rows = np.ascontiguousarray(rows, np.int64)
    cols = np.ascontiguousarray(cols, np.int64)
    out = np.zeros(rows.size, np.float32)
    rc = lib().orc_sgemm_entries(A.shape[1], A, A.shape[1], B, B.shape[1],
                                 rows.size, rows, cols, out)
    if rc:
        raise ValueError(rc)
    return out


def lu(A, update_variant: int = 6, nb: int = 64):
    """Blocked right-looking LU with partial pivoting; returns (LU, ipiv, info)."""
    A = _c32(A).copy()
    n = A.shape[0]
    ipiv = np.zeros(n, np.int32)
    info = lib().orc_lu(update_variant, n, A, max(n, 1), ipiv, nb)
    if info < 0:
        raise ValueError(f"orc_lu argument error {info}")
    return A, ipiv, info


FMT_BF16, FMT_FP16 = 1, 2


def lu_fmt(A, fmt: int):
    """Single-format LU with partial pivoting (the BF16 / FP16 rows of the
    Sec. IV-B tables): A rounded to the format, every multiplier and update
    rounded to it once.  Returns (LU, ipiv, info); the factors are FP32 arrays
    whose values lie in the format."""
    A = _c32(A).copy()
    n = A.shape[0]
    ipiv = np.zeros(n, np.int32)
    info = lib().orc_lu_fmt(fmt, n, A, max(n, 1), ipiv)
    if info < 0:
        raise ValueError(f"orc_lu_fmt argument error {info}")
    return A, ipiv, info


def round_fmt(x: float, fmt: int) -> float:
    """x rounded once to the format (1: BF16, 2: FP16), nearest even."""
    return lib().orc_round_fmt(float(x), fmt)


def lu_solve(LU, ipiv, b):
    LU = _c32(LU)
    b = _c32(b).copy()
    lib().orc_lu_solve(LU.shape[0], LU, max(LU.shape[0], 1),
                       np.ascontiguousarray(ipiv, np.int32), b)
    return b


def residual(A, b, x):
    A = _c32(A)
    b = np.ascontiguousarray(b, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    r = np.zeros_like(b)
    lib().orc_residual(A.shape[0], A, max(A.shape[0], 1), b, x, r)
    return r


def ir(A, LU, ipiv, b, tol: float = 1e-14, max_iter: int = 30):
    """Residual-form iterative refinement (Sec. III).

    Returns dict(x, iters, eta, status, eta_hist)."""
    A = _c32(A)
    LU = _c32(LU)
    n = A.shape[0]
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(n, np.float64)
    it = ctypes.c_int(0)
    eta = ctypes.c_double(0.0)
    st = ctypes.c_int(0)
    hist = np.full(max_iter + 1, np.nan)
    rc = lib().orc_ir(n, A, max(n, 1), LU, max(n, 1),
                      np.ascontiguousarray(ipiv, np.int32), b, x, tol, max_iter,
                      ctypes.byref(it), ctypes.byref(eta), ctypes.byref(st), hist)
    if rc:
        raise ValueError(rc)
    return dict(x=x, iters=it.value, eta=eta.value, status=st.value,
                eta_hist=hist[: it.value + 1])


def gmres_ir(A, LU, ipiv, b, tol: float = 1e-14, max_iter: int = 30, restart: int = 50,
             inner_tol: float = 1e-8):
    """Refinement with LU-preconditioned FP64 GMRES as the correction solver
    (Sec. III, Sec. IV-B).  Returns dict(x, iters, inner, eta, status, eta_hist)."""
    A = _c32(A)
    LU = _c32(LU)
    n = A.shape[0]
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(n, np.float64)
    it = ctypes.c_int(0)
    inner = ctypes.c_int(0)
    eta = ctypes.c_double(0.0)
    st = ctypes.c_int(0)
    hist = np.full(max_iter + 1, np.nan)
    rc = lib().orc_gmres_ir(n, A, max(n, 1), LU, max(n, 1), np.ascontiguousarray(ipiv, np.int32),
                            b, x, tol, max_iter, restart, inner_tol, ctypes.byref(it),
                            ctypes.byref(inner), ctypes.byref(eta), ctypes.byref(st), hist)
    if rc:
        raise ValueError(rc)
    return dict(x=x, iters=it.value, inner=inner.value, eta=eta.value, status=st.value,
                eta_hist=hist[: it.value + 1])

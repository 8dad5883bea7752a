"""ctypes declarations for libbfx.so (the C ABI in include/bfx.h).

The library must have been built (``python -m paper_1904_06376_amd.build`` or
``__graft_entry__.build()``).  There is no fallback: if libbfx.so is missing the
import fails with an error that says so.
"""
import ctypes
import os

# torch first: its HIP runtime is then the one libbfx.so binds to, so that
# device memory allocated by torch and by the library share one runtime.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

lib = ctypes.CDLL(LIB_PATH)

c_i64 = ctypes.c_int64
c_int = ctypes.c_int
c_f32 = ctypes.c_float
c_f64 = ctypes.c_double
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t


class GemmDesc(ctypes.Structure):
    _fields_ = [("M", c_i64), ("N", c_i64), ("K", c_i64),
                ("A", c_vp), ("lda", c_i64),
                ("B", c_vp), ("ldb", c_i64),
                ("C", c_vp), ("ldc", c_i64),
                ("alpha", c_f32), ("beta", c_f32)]


class SolveDesc(ctypes.Structure):
    _fields_ = [("n", c_i64), ("A", c_vp), ("lda", c_i64), ("b", c_vp), ("x", c_vp)]


class IrOpts(ctypes.Structure):
    _fields_ = [("tol", c_f64), ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("tol", c_f64), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("inner_tol", c_f64)]


class BatchedSolveOpts(ctypes.Structure):
    _fields_ = [("tol", c_f64), ("max_iter", ctypes.c_int32), ("gmres_max_iter", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("inner_tol", c_f64), ("lu_format", ctypes.c_int32),
                ("mode", ctypes.c_int32)]


class GmresResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("inner", ctypes.c_int32), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("eta", c_f64)]


class IrResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("eta", c_f64)]


SIGNATURES = {
    "bfx_version": ([], c_int),
    "bfx_last_error_string": ([], ctypes.c_char_p),
    "bfx_split_f32": ([c_vp, c_i64, c_int, c_vp, c_vp, c_vp, c_vp], c_int),
    "bfx_gemm": ([c_int, c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64,
                  c_f32, c_vp, c_i64, c_vp, c_size, c_vp], c_int),
    "bfx_gemm_ex": ([c_int, c_int, c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64,
                     c_f32, c_vp, c_i64, c_vp, c_size, c_vp], c_int),
    "bfx_gemm_ws_size": ([c_int, c_i64, c_i64, c_i64], c_size),
    "bfx_gemm_noalloc": ([c_int, c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64,
                          c_f32, c_vp, c_i64, c_vp], c_int),
    "bfx_gemm_noalloc_scratch_bytes": ([], c_size),
    "bfx_split_blocks_size": ([c_int, c_i64, c_i64], c_size),
    "bfx_split_blocks": ([c_int, c_int, c_i64, c_i64, c_vp, c_i64, c_vp, c_size, c_vp], c_int),
    "bfx_gemm_blocks": ([c_int, c_i64, c_i64, c_i64, c_f32, c_vp, c_vp, c_f32, c_vp, c_i64, c_vp],
                        c_int),
    "bfx_sgemm_fp32": ([c_i64, c_i64, c_i64, c_f32, c_vp, c_i64, c_vp, c_i64,
                        c_f32, c_vp, c_i64, c_vp, c_size, c_vp], c_int),
    "bfx_sgemm_ws_size": ([c_i64, c_i64, c_i64], c_size),
    "bfx_gemm_batched_plan_create": ([c_int, c_i64, ctypes.POINTER(GemmDesc),
                                      ctypes.c_char_p, ctypes.POINTER(c_vp)], c_int),
    "bfx_plan_launch": ([c_vp, c_vp], c_int),
    "bfx_plan_launch_per_problem": ([c_vp, c_vp], c_int),
    "bfx_plan_info": ([c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)], c_int),
    "bfx_plan_destroy": ([c_vp], c_int),
    "bfx_lu_factor": ([c_int, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_size, c_vp], c_int),
    "bfx_lu_ws_size": ([c_i64], c_size),
    "bfx_ir_solve": ([c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp,
                      ctypes.POINTER(IrOpts), ctypes.POINTER(IrResult), c_vp, c_size,
                      c_vp], c_int),
    "bfx_ir_ws_size": ([c_i64], c_size),
    "bfx_gmres_ir_solve": ([c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp,
                            ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresResult), c_vp,
                            c_size, c_vp], c_int),
    "bfx_gmres_ir_ws_size": ([c_i64, c_int], c_size),
    "bfx_lu_solve_f32": ([c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_size, c_vp], c_int),
    "bfx_lu_ir_batched_plan_create": ([c_int, c_i64, ctypes.POINTER(SolveDesc),
                                       ctypes.POINTER(BatchedSolveOpts), ctypes.POINTER(c_vp)], c_int),
    "bfx_solve_plan_launch": ([c_vp, c_vp], c_int),
    "bfx_solve_plan_launch_per_problem": ([c_vp, c_vp], c_int),
    "bfx_solve_plan_results": ([c_vp, ctypes.POINTER(GmresResult), ctypes.POINTER(ctypes.c_int32)], c_int),
    "bfx_solve_plan_factors": ([c_vp, c_i64, c_vp, c_vp], c_int),
    "bfx_solve_plan_destroy": ([c_vp], c_int),
}

EXPORTED = []
for _name, (_args, _res) in SIGNATURES.items():
    _fn = getattr(lib, _name, None)
    if _fn is None:
        continue
    _fn.argtypes = _args
    _fn.restype = _res
    EXPORTED.append(_name)


class BfxError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != 0:
        msg = lib.bfx_last_error_string().decode()
        raise BfxError(f"{what} returned {rc}" + (f": {msg}" if rc <= -1000 else ""))

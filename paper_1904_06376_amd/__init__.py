"""bfx: FP32-accurate GEMM, LU and iterative refinement from BF16 pieces on MI355X.

Python binding of libbfx.so (C ABI declared in include/bfx.h).  Method:
Henry, Tang & Heinecke, "Leveraging the bfloat16 Artificial Intelligence
Datatype For Higher-Precision Computations" (2019).
"""
from ._lib import EXPORTED, BfxError, lib  # noqa: F401  (fails loudly if unbuilt)
from .api import (BatchedGemmPlan, BatchedSolvePlan, gemm, gemm_blocks,  # noqa: F401
                  gemm_ws_size, gmres_ir_solve, ir_solve, lu_factor, lu_solve_f32,
                  sgemm_fp32, split, split_blocks)

__all__ = ["split", "gemm", "gemm_ws_size", "split_blocks", "gemm_blocks", "sgemm_fp32", "BatchedGemmPlan", "BatchedSolvePlan",
           "lu_factor", "lu_solve_f32", "ir_solve", "gmres_ir_solve", "BfxError", "EXPORTED"]

"""Torch-facing wrappers over the libbfx C ABI: argument checks and marshalling
only.  Every computation runs in the HIP kernels of libbfx.so; tensors supply
device memory and the current HIP stream."""
from __future__ import annotations

import ctypes
import os

import torch

from ._lib import (BatchedSolveOpts, GemmDesc, GmresOpts, GmresResult, IrOpts, IrResult, SolveDesc,
                   check, lib)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


def _rows(t: torch.Tensor, name: str):
    """Row-major 2-D view with unit column stride; returns the leading dimension."""
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    M, N = t.shape
    if M == 0 or N == 0 or M == 1:
        return max(N, 1)
    if N > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t.stride(0)


def _ws(nbytes: int, device):
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def split(a: torch.Tensor, nterms: int = 3):
    """Sec. II-A split; returns nterms int16 tensors holding BF16 bit patterns."""
    _dev(a, torch.float32, "a")
    a = a.contiguous()
    outs = [torch.empty(a.shape, dtype=torch.int16, device=a.device) for _ in range(nterms)]
    b2 = outs[2].data_ptr() if nterms == 3 else None
    check(lib.bfx_split_f32(a.data_ptr(), a.numel(), nterms, outs[0].data_ptr(),
                            outs[1].data_ptr(), b2, _stream()), "bfx_split_f32")
    return tuple(outs)


def gemm_ws_size(variant: int, M: int, N: int, K: int) -> int:
    return lib.bfx_gemm_ws_size(variant, M, N, K)


FP64_SUM = 1   # bfx_gemm_ex flag: the "d" option (final sum and epilogue in FP64)


def gemm(variant: int, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None,
         alpha: float = 1.0, beta: float = 0.0, ws: torch.Tensor | None = None,
         fp64_sum: bool = False):
    """Split-BF16 GEMM C = alpha*(A x B) + beta*C with `variant` in {1,3,6,7,8,9}
    or a per-operand split count 10*pa + pb in {12,13,21,23,31,32}; fp64_sum
    selects the "d" option.

    `ws`: optional uint8 device tensor of at least gemm_ws_size(...) bytes,
    allocated here when missing or too small; it holds split-K partial sums,
    or, for large products, both operands' BF16 planes (split once per call)."""
    _dev(A, torch.float32, "A")
    _dev(B, torch.float32, "B")
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
        beta = 0.0
    _dev(C, torch.float32, "C")
    need = gemm_ws_size(variant, M, N, K)
    if ws is None or ws.numel() < need:
        ws = _ws(need, A.device)
    check(lib.bfx_gemm_ex(variant, FP64_SUM if fp64_sum else 0, M, N, K, alpha, A.data_ptr(),
                          _rows(A, "A"), B.data_ptr(), _rows(B, "B"), beta, C.data_ptr(),
                          _rows(C, "C"), ws.data_ptr() if ws is not None else None, need,
                          _stream()),
          "bfx_gemm_ex")
    return C


def split_blocks(X: torch.Tensor, nterms: int, trans: bool = False) -> torch.Tensor:
    """One operand into `nterms` BF16 planes of the pre-split block layout
    (Sec. II-A): trans=False for A (M x K), trans=True for B (K x N).  Returns
    the planes as an int16 tensor of bfx_split_blocks_size / 2 elements."""
    _dev(X, torch.float32, "X")
    if trans:
        K, R = X.shape
    else:
        R, K = X.shape
    nbytes = lib.bfx_split_blocks_size(nterms, R, K)
    out = torch.empty(max(nbytes // 2, 8), dtype=torch.int16, device=X.device)
    check(lib.bfx_split_blocks(nterms, int(trans), R, K, X.data_ptr(), _rows(X, "X"),
                               out.data_ptr(), out.numel() * 2, _stream()), "bfx_split_blocks")
    return out


def planes(variant: int) -> int:
    """BF16 terms of each operand that `variant` reads (bfx_split_blocks' nterms)."""
    if variant >= 10:
        return max(divmod(variant, 10))
    return {1: 1, 3: 2}.get(variant, 3)


def gemm_blocks(variant: int, M: int, N: int, K: int, Ab: torch.Tensor, Bb: torch.Tensor,
                C: torch.Tensor | None = None, alpha: float = 1.0, beta: float = 0.0,
                device=None):
    """C = alpha*(A x B) + beta*C from operands pre-split by split_blocks (with
    planes(variant) terms each: the kernel reads that many planes of both)."""
    P = planes(variant)
    if (Ab.numel() * Ab.element_size() < lib.bfx_split_blocks_size(P, M, K)
            or Bb.numel() * Bb.element_size() < lib.bfx_split_blocks_size(P, N, K)):
        raise ValueError(f"variant {variant} reads {P} planes of each operand: split them with nterms={P}")
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=device or Ab.device)
        beta = 0.0
    _dev(C, torch.float32, "C")
    check(lib.bfx_gemm_blocks(variant, M, N, K, alpha, Ab.data_ptr(), Bb.data_ptr(), beta,
                              C.data_ptr(), _rows(C, "C"), _stream()), "bfx_gemm_blocks")
    return C


def sgemm_fp32(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None,
               alpha: float = 1.0, beta: float = 0.0):
    """Plain FP32 vector-ALU GEMM (the comparator)."""
    _dev(A, torch.float32, "A")
    _dev(B, torch.float32, "B")
    M, K = A.shape
    _, N = B.shape
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
        beta = 0.0
    need = lib.bfx_sgemm_ws_size(M, N, K)
    ws = _ws(need, A.device)
    check(lib.bfx_sgemm_fp32(M, N, K, alpha, A.data_ptr(), _rows(A, "A"), B.data_ptr(),
                             _rows(B, "B"), beta, C.data_ptr(), _rows(C, "C"),
                             ws.data_ptr() if ws is not None else None, need, _stream()),
          "bfx_sgemm_fp32")
    return C


def default_tune_table(variant: int) -> str | None:
    """The autotuner's table shipped with the package for `variant`, if any."""
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune", f"gfx950_x{variant}.json")
    return p if os.path.exists(p) else None


class BatchedGemmPlan:
    """One persistent, graph-captured launch over many independent GEMMs.

    tune_table: path of an autotuner table; None uses the packaged table of the
    variant when there is one, "" the built-in defaults."""

    def __init__(self, variant: int, problems, tune_table: str | None = None):
        if tune_table is None:
            tune_table = default_tune_table(variant)
        self._keep = problems
        descs = (GemmDesc * len(problems))()
        for i, (A, B, C, alpha, beta) in enumerate(problems):
            M, K = A.shape
            N = B.shape[1]
            descs[i] = GemmDesc(M, N, K, A.data_ptr(), _rows(A, "A"), B.data_ptr(),
                                _rows(B, "B"), C.data_ptr(), _rows(C, "C"), alpha, beta)
        h = ctypes.c_void_p()
        tt = tune_table.encode() if tune_table else None
        check(lib.bfx_gemm_batched_plan_create(variant, len(problems), descs, tt,
                                                ctypes.byref(h)), "plan_create")
        self._h = h

    def launch(self):
        check(lib.bfx_plan_launch(self._h, _stream()), "bfx_plan_launch")

    def launch_per_problem(self):
        check(lib.bfx_plan_launch_per_problem(self._h, _stream()), "launch_per_problem")

    def info(self):
        t = ctypes.c_int64()
        p = ctypes.c_int64()
        check(lib.bfx_plan_info(self._h, ctypes.byref(t), ctypes.byref(p)), "plan_info")
        return t.value, p.value

    def close(self):
        if getattr(self, "_h", None):
            lib.bfx_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lu_factor(A: torch.Tensor, variant: int = 6):
    """In-place LU with partial pivoting; returns (A, ipiv int32, info int32 tensor)."""
    _dev(A, torch.float32, "A")
    n = A.shape[0]
    if A.shape[1] != n:
        raise ValueError("A must be square")
    ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    need = lib.bfx_lu_ws_size(n)
    ws = _ws(need, A.device)
    check(lib.bfx_lu_factor(variant, n, A.data_ptr(), _rows(A, "A"), ipiv.data_ptr(),
                            info.data_ptr(), ws.data_ptr() if ws is not None else None,
                            need, _stream()), "bfx_lu_factor")
    return A, ipiv[:n], info


def lu_solve_f32(LU: torch.Tensor, ipiv: torch.Tensor, rhs: torch.Tensor):
    n = LU.shape[0]
    _dev(rhs, torch.float32, "rhs")
    need = lib.bfx_ir_ws_size(n)
    ws = _ws(need, LU.device)
    check(lib.bfx_lu_solve_f32(n, LU.data_ptr(), _rows(LU, "LU"), ipiv.data_ptr(),
                               rhs.data_ptr(), ws.data_ptr() if ws is not None else None,
                               need, _stream()), "bfx_lu_solve_f32")
    return rhs


class DeviceResult:
    """A bfx_ir_result / bfx_gmres_result that the library writes in device
    memory.  Reading a field copies it to the host (which waits for the
    solve); ``device`` is the raw byte tensor for callers that stay on the
    device."""

    def __init__(self, ctype, device):
        self._ctype = ctype
        self.device = torch.zeros(ctypes.sizeof(ctype), dtype=torch.uint8, device=device)
        self._host = None

    def ptr(self):
        return ctypes.cast(ctypes.c_void_p(self.device.data_ptr()), ctypes.POINTER(self._ctype))

    def to_dict(self):
        if self._host is None:
            raw = bytes(self.device.cpu().numpy().tobytes())
            r = self._ctype.from_buffer_copy(raw)
            self._host = {name: getattr(r, name) for name, _ in self._ctype._fields_ if name != "reserved"}
        return self._host

    def __getitem__(self, key):
        return self.to_dict()[key]

    def __repr__(self):
        return repr(self.to_dict())


def ir_solve(A: torch.Tensor, LU: torch.Tensor, ipiv: torch.Tensor, b: torch.Tensor,
             tol: float = 1e-14, max_iter: int = 30, x: torch.Tensor | None = None):
    """Residual-form iterative refinement, queued on the current stream
    without waiting; returns (x, result) where result is a DeviceResult
    (fields iters, status, eta, read on first access)."""
    n = A.shape[0]
    _dev(b, torch.float64, "b")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    need = lib.bfx_ir_ws_size(n)
    ws = _ws(need, A.device)
    opts = IrOpts(tol, max_iter, 0)
    res = DeviceResult(IrResult, A.device)
    check(lib.bfx_ir_solve(n, A.data_ptr(), _rows(A, "A"), LU.data_ptr(), _rows(LU, "LU"),
                           ipiv.data_ptr(), b.data_ptr(), x.data_ptr(), ctypes.byref(opts),
                           res.ptr(), ws.data_ptr() if ws is not None else None,
                           need, _stream()), "bfx_ir_solve")
    res._keep = ws
    return x, res


def gmres_ir_solve(A: torch.Tensor, LU: torch.Tensor, ipiv: torch.Tensor, b: torch.Tensor,
                   tol: float = 1e-14, max_iter: int = 10, restart: int = 50,
                   inner_tol: float = 1e-8, x: torch.Tensor | None = None):
    """Refinement with LU-preconditioned FP64 GMRES as the correction solver,
    queued without waiting; returns (x, DeviceResult with iters, inner,
    status, eta)."""
    n = A.shape[0]
    _dev(b, torch.float64, "b")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    need = lib.bfx_gmres_ir_ws_size(n, restart)
    ws = _ws(need, A.device)
    opts = GmresOpts(tol, max_iter, restart, inner_tol)
    res = DeviceResult(GmresResult, A.device)
    check(lib.bfx_gmres_ir_solve(n, A.data_ptr(), _rows(A, "A"), LU.data_ptr(), _rows(LU, "LU"),
                                 ipiv.data_ptr(), b.data_ptr(), x.data_ptr(), ctypes.byref(opts),
                                 res.ptr(), ws.data_ptr() if ws is not None else None,
                                 need, _stream()), "bfx_gmres_ir_solve")
    res._keep = ws
    return x, res


class BatchedSolvePlan:
    """Many LU + refinement solves in one persistent, graph-captured launch;
    problems that LU-IR leaves unconverged continue with GMRES-IR when
    gmres_max_iter > 0 (restart 0 = a full Krylov space).  lu_format 1 / 2:
    single-format BF16 / FP16 LU; mode 1: GMRES-IR from the start.

    problems: list of (A float32 n x n, b float64 n, x float64 n) GPU tensors."""

    def __init__(self, variant: int, problems, tol: float = 1e-14, max_iter: int = 30,
                 gmres_max_iter: int = 10, restart: int = 0, inner_tol: float = 1e-8,
                 lu_format: int = 0, mode: int = 0):
        self._keep = problems
        descs = (SolveDesc * len(problems))()
        for i, (A, b, x) in enumerate(problems):
            _dev(A, torch.float32, "A")
            _dev(b, torch.float64, "b")
            _dev(x, torch.float64, "x")
            descs[i] = SolveDesc(A.shape[0], A.data_ptr(), _rows(A, "A"), b.data_ptr(), x.data_ptr())
        opts = BatchedSolveOpts(tol, max_iter, gmres_max_iter, restart, inner_tol, lu_format, mode)
        h = ctypes.c_void_p()
        check(lib.bfx_lu_ir_batched_plan_create(variant, len(problems), descs, ctypes.byref(opts),
                                                 ctypes.byref(h)), "solve_plan_create")
        self._h = h
        self.count = len(problems)

    def launch(self):
        check(lib.bfx_solve_plan_launch(self._h, _stream()), "bfx_solve_plan_launch")

    def launch_per_problem(self):
        check(lib.bfx_solve_plan_launch_per_problem(self._h, _stream()), "solve_per_problem")

    def results(self):
        res = (GmresResult * max(self.count, 1))()
        info = (ctypes.c_int32 * max(self.count, 1))()
        check(lib.bfx_solve_plan_results(self._h, res, info), "bfx_solve_plan_results")
        return [dict(iters=r.iters, inner=r.inner, status=r.status, eta=r.eta, info=int(i))
                for r, i in zip(list(res)[: self.count], list(info)[: self.count])]

    def factors(self, index: int):
        """(LU, ipiv) of problem `index` as host arrays (after a launch)."""
        import numpy as np
        n = self._keep[index][0].shape[0]
        lu = np.zeros((n, n), np.float32)
        piv = np.zeros(n, np.int32)
        check(lib.bfx_solve_plan_factors(self._h, index, lu.ctypes.data, piv.ctypes.data),
              "bfx_solve_plan_factors")
        return lu, piv

    def close(self):
        if getattr(self, "_h", None):
            lib.bfx_solve_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

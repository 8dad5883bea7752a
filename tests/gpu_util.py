"""Helpers for GPU parity tests: host<->device movement and bound checks."""
import numpy as np
import torch

U = 2.0 ** -24


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bits16(t):
    return host(t).view(np.uint16)


def gemm_bound(variant, K):
    """Componentwise error bound relative to |A||B|: the FP32 accumulation's
    2K 2^-24 plus the dropped split terms' 3 2^-16 (x3) or 3 2^-8 (x1) (Sec.
    II-D, II-G); for K < 8 the dropped-term allowance (513/512) 2^-23 is added."""
    k = 2 * K + (8 if K < 8 else 0)
    if variant >= 10:
        # per-operand split counts 10 pa + pb: the weaker operand's count decides
        variant = 1 if min(divmod(variant, 10)) == 1 else 3
    if variant >= 6:
        return k * U
    if variant == 3:
        return 3 * 2.0 ** -16 + k * U
    return 3 * 2.0 ** -8 + k * U


def ref64(A, B):
    return A.astype(np.float64) @ B.astype(np.float64)


def absref(A, B):
    return np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))

"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds none of the split-BF16 arithmetic: it only draws random
numbers (NumPy PCG64 from an explicit seed, generated in FP64 and rounded once
to FP32) in the shapes and value distributions of the paper's experiments
(Sec. IV-A: uniform [-1,1] as with drand48; a wide exponent range; a Gaussian
exponent range; Sec. IV-B: conditioned dense systems).

Recipes (each is stated again in the design doc):
  uniform      iid U[-1, 1]
  normal       iid N(0, 1)
  wide         +-2^u, u ~ U[-20, 20] continuous, random sign
  gauss_exp    +-m * 2^e, m ~ U[1, 2), e = round(N(0, 8)) clipped to [-100, 100]
  max_exp      +-m * 2^e, m ~ U[1, 2), e uniform over the integers of [-E, E],
               E = floor((126 - log2 K) / 2) - 1 (finite K-term sums)
  cancellation B[:, j] = -A[j, :]^T + 1e-4 * N(0, 1)  (B's j-th column is the
               negated j-th row of A plus noise)
  batched      shapes M, N, K iid uniform over {32, 48, ..., 512}; entries N(0,1)
  conditioned  A = U diag(s) V^T, U and V orthogonal from the Householder QR
               of a Gaussian matrix with the signs of diag(R) folded in
               (Haar distributed), s_i = kappa^(-(i-1)/(n-1)); A rounded to
               FP32; x_true ~ N(0,1); b = A32 x_true in FP64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "uniform", "normal", "wide", "gauss_exp", "max_exp", "cancellation",
    "batched_shapes", "batched_problems", "haar", "conditioned_system",
    "batch_sizes",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=shape).astype(np.float32)


def normal(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(size=shape).astype(np.float32)


def wide(shape, seed: int, umax: float = 20.0) -> np.ndarray:
    g = rng(seed)
    u = g.uniform(-umax, umax, size=shape)
    s = np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
    return (s * np.exp2(u)).astype(np.float32)


def gauss_exp(shape, seed: int, sigma: float = 8.0, emax: int = 100) -> np.ndarray:
    g = rng(seed)
    m = g.uniform(1.0, 2.0, size=shape)
    e = np.clip(np.rint(g.normal(0.0, sigma, size=shape)), -emax, emax)
    s = np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
    return (s * m * np.exp2(e)).astype(np.float32)


def max_exp(shape, seed: int, K: int = 256) -> np.ndarray:
    """The "maximal exponent" inputs of Sec. IV-A (Fig. 3): random sign,
    mantissa uniform in [1, 2), exponent uniform over the integers of
    [-E, E] with E = floor((126 - log2 K) / 2) - 1, the widest symmetric range
    whose products and K-term sums stay finite in FP32 (E = 58 for K = 256).
    Products then reach down to 2^-116, below the 2^-110 limit of an exact
    split (Sec. II-F)."""
    E = int((126 - np.log2(max(K, 1))) // 2) - 1
    g = rng(seed)
    m = g.uniform(1.0, 2.0, size=shape)
    e = g.integers(-E, E + 1, size=shape)
    s = np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
    return (s * m * np.exp2(e.astype(np.float64))).astype(np.float32)


def cancellation(M: int, K: int, seed: int, noise: float = 1e-4):
    """A (M x K) uniform; B (K x M) with column j = -(row j of A) + noise."""
    g = rng(seed)
    A64 = g.uniform(-1.0, 1.0, size=(M, K))
    A = A64.astype(np.float32)
    B = (-A.astype(np.float64).T + noise * g.standard_normal(size=(K, M))).astype(np.float32)
    return A, np.ascontiguousarray(B)


def batched_shapes(count: int, seed: int, lo: int = 32, hi: int = 512, step: int = 16):
    g = rng(seed)
    vals = np.arange(lo, hi + 1, step)
    return g.choice(vals, size=(count, 3)).astype(np.int64)


def batched_problems(count: int, seed: int, lo: int = 32, hi: int = 512, step: int = 16):
    """List of (A, B) FP32 pairs with uniformly drawn multiple-of-16 shapes."""
    shapes = batched_shapes(count, seed, lo, hi, step)
    g = rng(seed + 1)
    out = []
    for (M, N, K) in shapes:
        A = g.standard_normal(size=(M, K)).astype(np.float32)
        B = g.standard_normal(size=(K, N)).astype(np.float32)
        out.append((A, B))
    return shapes, out


def haar(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: Householder QR of a Gaussian."""
    Z = g.standard_normal(size=(n, n))
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def conditioned_system(n: int, kappa: float, seed: int):
    """(A32, b64, x_true) with A = U diag(s) V^T, s geometric from 1 to 1/kappa."""
    g = rng(seed)
    U = haar(n, g)
    V = haar(n, g)
    if n > 1:
        s = kappa ** (-np.arange(n) / (n - 1))
    else:
        s = np.ones(1)
    A = ((U * s[None, :]) @ V.T).astype(np.float32)
    x_true = g.standard_normal(size=n)
    b = A.astype(np.float64) @ x_true
    return A, b, x_true


def batch_sizes(count: int, seed: int, lo: int = 64, hi: int = 1024) -> np.ndarray:
    return rng(seed).integers(lo, hi + 1, size=count).astype(np.int64)


def conditioned_system_torch(n: int, kappa: float, seed: int, device):
    """Large-n version of `conditioned_system` generated on the GPU: Gaussian
    matrices from torch's seeded device generator, Householder QR (sign of
    diag(R) folded in), A = U diag(s) V^T in FP64 rounded to FP32,
    x_true ~ N(0,1), b = A32 x_true in FP64.  Returns (A32, b64) on `device`."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def haar_t():
        Z = torch.randn(n, n, dtype=torch.float64, device=device, generator=g)
        Q, R = torch.linalg.qr(Z)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        del Z, R
        return Q * d[None, :]

    U = haar_t()
    V = haar_t()
    s = kappa ** (-torch.arange(n, dtype=torch.float64, device=device) / max(n - 1, 1))
    A = ((U * s[None, :]) @ V.T.contiguous()).to(torch.float32)
    del U, V
    x_true = torch.randn(n, dtype=torch.float64, device=device, generator=g)
    b = A.to(torch.float64) @ x_true
    return A.contiguous(), b


def batch_systems_torch(count: int, kappa: float, seed: int, device, lo: int = 64, hi: int = 1024):
    """`count` conditioned systems with n ~ U{lo..hi} (same recipe as
    `conditioned_system_torch`, one seed per problem).  Returns a list of
    (A32, b64) device tensors and the sizes."""
    sizes = batch_sizes(count, seed, lo, hi)
    out = [conditioned_system_torch(int(n), kappa, seed * 100003 + i, device)
           for i, n in enumerate(sizes)]
    return out, sizes

"""GPU split GEMM (bfx_gemm) and FP32 comparator (bfx_sgemm_fp32) vs the oracle.

Bar: every entry within the paper's componentwise bound of the exact product
(FP64 of FP32 inputs) and within twice that bound of the oracle; exactly equal
where the result is exact in any order (integers, identity operands); the
FP32 comparator bit-identical to the oracle's FMA chain."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import absref, bits16, dev, gemm_bound, host, ref64

pytestmark = pytest.mark.gpu

# K % 4 == 0 and N % 4 == 0 with 16-byte aligned rows take the
# wave-specialised engine (partial tiles masked); the other shapes the general
# engine.
SHAPES = [(256, 256, 256), (200, 130, 77), (129, 257, 33), (17, 300, 5), (1, 1, 1),
          (64, 64, 1000), (300, 40, 600), (3, 5, 4096), (130, 132, 128),
          (200, 132, 96), (129, 256, 36), (1, 4, 4), (65, 64, 44), (127, 128, 1028),
          (200, 130, 96), (65, 63, 44)]


def _check_bound(variant, A, B, C, Corc=None, alpha=1.0):
    K = A.shape[1]
    z = alpha * ref64(A, B)
    zh = abs(alpha) * absref(A, B)
    bnd = gemm_bound(variant, K) * zh + 1e-38
    err = np.abs(C.astype(np.float64) - z)
    worst = float(np.max(err / bnd)) if err.size else 0.0
    assert np.all(err <= bnd), f"variant {variant}: max err/bound {worst}"
    if Corc is not None:
        d = np.abs(C.astype(np.float64) - Corc.astype(np.float64))
        assert np.all(d <= 2 * bnd)
    return worst


@pytest.mark.parametrize("variant", [1, 3, 6, 9])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_parity_uniform(bfx, orc, variant, shape):
    M, N, K = shape
    A = workloads.uniform((M, K), M * 7 + K)
    B = workloads.uniform((K, N), N * 11 + K)
    C = host(bfx.gemm(variant, dev(A), dev(B)))
    Co = orc.gemm(variant, A, B)
    if variant == 1:
        # one BF16 term: same products as the oracle, only the order differs
        d = np.abs(C.astype(np.float64) - Co)
        assert np.all(d <= 2 * K * 2.0 ** -24 * absref(A, B) + 1e-38)
    else:
        _check_bound(variant, A, B, C, Co)


@pytest.mark.parametrize("gen", ["normal", "wide", "gauss_exp"])
@pytest.mark.parametrize("variant", [3, 6, 7, 8, 9])
def test_gemm_parity_distributions(bfx, orc, gen, variant):
    f = getattr(workloads, gen)
    A = f((160, 300), 21)
    B = f((300, 144), 22)
    C = host(bfx.gemm(variant, dev(A), dev(B)))
    _check_bound(variant, A, B, C, orc.gemm(variant, A, B))


@pytest.mark.parametrize("variant", [1, 3, 6, 9])
def test_gemm_integers_exact(bfx, orc, variant):
    g = np.random.default_rng(5)
    A = g.integers(-8, 9, (150, 70)).astype(np.float32)
    B = g.integers(-8, 9, (70, 190)).astype(np.float32)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    np.testing.assert_array_equal(host(bfx.gemm(variant, dev(A), dev(B))), exact)


@pytest.mark.parametrize("variant", [6, 9])
def test_gemm_identity_exact(bfx, variant):
    """a0 + (a1 + a2) rebuilds a exactly in any summation order: A x I == A."""
    A = workloads.normal((190, 160), 6)
    I = np.eye(160, dtype=np.float32)
    np.testing.assert_array_equal(host(bfx.gemm(variant, dev(A), dev(I))), A)
    I2 = np.eye(190, dtype=np.float32)
    np.testing.assert_array_equal(host(bfx.gemm(variant, dev(I2), dev(A))), A)


def test_gemm_alpha_beta(bfx, orc):
    A = workloads.uniform((140, 90), 7)
    B = workloads.uniform((90, 150), 8)
    C0 = workloads.uniform((140, 150), 9)
    got = host(bfx.gemm(6, dev(A), dev(B), dev(C0), alpha=-1.0, beta=1.0))
    exact = C0.astype(np.float64) - ref64(A, B)
    bnd = gemm_bound(6, 90) * absref(A, B) + 2.0 ** -24 * np.abs(exact) + 1e-38
    assert np.all(np.abs(got - exact) <= bnd)
    Cn = np.full((140, 150), np.nan, np.float32)
    got = host(bfx.gemm(6, dev(A), dev(B), dev(Cn), alpha=2.0, beta=0.0))
    assert np.all(np.isfinite(got))
    _check_bound(6, A, B, got, alpha=2.0)


def test_gemm_strided_and_unaligned(bfx, orc):
    A = workloads.normal((100, 131), 10)
    B = workloads.normal((131, 97), 11)
    tA = dev(np.pad(A, ((0, 0), (0, 5))))[:, :131]      # lda = 136
    tB = dev(np.pad(B, ((0, 0), (0, 3))))[:, :97]       # ldb = 100
    C = host(bfx.gemm(6, tA, tB))
    _check_bound(6, A, B, C, orc.gemm(6, A, B))
    tA2 = dev(np.pad(A, ((0, 0), (0, 2))))[:, :131]     # lda = 133: scalar loads
    C2 = host(bfx.gemm(6, tA2, dev(B)))
    _check_bound(6, A, B, C2)


def test_gemm_nonfinite_pattern(bfx, orc):
    A = workloads.uniform((70, 64), 12)
    B = workloads.uniform((64, 66), 13)
    A[3, 10] = np.inf
    B[20, 5] = np.nan
    A[50, 7] = 3e38        # saturating split, finite
    for v in (3, 6, 9):
        C = host(bfx.gemm(v, dev(A), dev(B)))
        Co = orc.gemm(v, A, B)
        np.testing.assert_array_equal(np.isfinite(C), np.isfinite(Co))
        np.testing.assert_array_equal(np.isnan(C), np.isnan(Co))


@pytest.mark.parametrize("variant", [1, 3, 6, 9])
@pytest.mark.parametrize("shape", [(256, 128, 256), (200, 132, 72)])
def test_gemm_fast_path_nonfinite_and_saturating(bfx, orc, variant, shape):
    """Shapes the wave-specialised engine takes (full and partial tiles):
    values whose first BF16 term would be Inf/NaN are re-split exactly out
    of band."""
    M, K, N = shape
    A = workloads.uniform((M, K), 14)
    B = workloads.uniform((K, N), 15)
    A[5, 3] = np.inf
    A[M - 56, K - 28] = -np.inf
    B[64, N - 3] = np.nan
    A[130, 31] = 3.3e38      # rounds past the largest BF16: saturating split
    B[K - 1, N - 1] = -3.39e38
    C = host(bfx.gemm(variant, dev(A), dev(B)))
    Co = orc.gemm(variant, A, B)
    np.testing.assert_array_equal(np.isfinite(C), np.isfinite(Co))
    np.testing.assert_array_equal(np.isnan(C), np.isnan(Co))
    fin = np.isfinite(Co)
    A2 = np.where(np.isfinite(A), A, 0).astype(np.float32)
    B2 = np.where(np.isfinite(B), B, 0).astype(np.float32)
    zh = absref(A2, B2)
    bnd = gemm_bound(variant, K) * zh + 1e-30
    assert np.all(np.abs(C[fin] - Co[fin]) <= 2 * bnd[fin])


@pytest.mark.parametrize("variant", [3, 6, 9])
def test_gemm_fast_vs_general_engine(bfx, orc, variant):
    """The same aligned product through the fast path and (with lda not a
    multiple of 4) through the general engine: both within the bound."""
    A = workloads.normal((384, 256), 16)
    B = workloads.normal((256, 512), 17)
    Cf = host(bfx.gemm(variant, dev(A), dev(B)))
    tA = dev(np.pad(A, ((0, 0), (0, 1))))[:, :256]
    Cg = host(bfx.gemm(variant, tA, dev(B)))
    bnd = gemm_bound(variant, 256) * absref(A, B)
    z = ref64(A, B)
    assert np.all(np.abs(Cf - z) <= bnd) and np.all(np.abs(Cg - z) <= bnd)
    assert np.all(np.abs(Cf - Cg) <= 2 * bnd)


@pytest.mark.parametrize("variant", [3, 6, 9])
def test_gemm_partial_tiles_fast_vs_general(bfx, orc, variant):
    """Partial tiles through the wave-specialised engine (masked loads and
    epilogue) and through the general engine: both within the bound."""
    A = workloads.normal((200, 132), 18)
    B = workloads.normal((132, 72), 19)
    Cf = host(bfx.gemm(variant, dev(A), dev(B)))
    tA = dev(np.pad(A, ((0, 0), (0, 1))))[:, :132]
    Cg = host(bfx.gemm(variant, tA, dev(B)))
    bnd = gemm_bound(variant, 132) * absref(A, B)
    z = ref64(A, B)
    assert np.all(np.abs(Cf - z) <= bnd) and np.all(np.abs(Cg - z) <= bnd)
    assert np.all(np.abs(Cf - Cg) <= 2 * bnd)
    # the masked region of C is untouched: write into a larger buffer
    big = torch.full((210, 80), 7.0, dtype=torch.float32, device="cuda")
    bfx.gemm(variant, dev(A), dev(B), big[:200, :72])
    hb = host(big)
    assert np.all(hb[200:] == 7.0) and np.all(hb[:, 72:] == 7.0)
    np.testing.assert_array_equal(hb[:200, :72], Cf)


def test_gemm_K0(bfx):
    A = np.zeros((5, 0), np.float32)
    B = np.zeros((0, 7), np.float32)
    C = host(bfx.gemm(6, dev(A), dev(B)))
    assert np.all(C == 0)


@pytest.mark.parametrize("shape", [(256, 256, 256), (200, 130, 77), (1, 1, 1), (129, 257, 33),
                                   (64, 64, 500)])
def test_sgemm_bitwise_equals_oracle(bfx, orc, shape):
    """Without split-K every output is the oracle's FMA chain: bit-identical."""
    M, N, K = shape
    A = workloads.normal((M, K), 40 + M)
    B = workloads.normal((K, N), 41 + N)
    np.testing.assert_array_equal(host(bfx.sgemm_fp32(dev(A), dev(B))), orc.sgemm(A, B))
    C0 = workloads.normal((M, N), 42)
    np.testing.assert_array_equal(host(bfx.sgemm_fp32(dev(A), dev(B), dev(C0), 0.5, -2.0)),
                                  orc.sgemm(A, B, C0, 0.5, -2.0))


def test_sgemm_splitk_long_k(bfx, orc):
    """Few tiles and a long K: the comparator splits K (fixed-order sum of the
    chains of each range); within the FP32 bound of the exact product."""
    A = workloads.uniform((64, 1 << 16), 50)
    B = workloads.uniform((1 << 16, 64), 51)
    assert bfx.lib.bfx_sgemm_ws_size(64, 64, 1 << 16) > 0
    C = host(bfx.sgemm_fp32(dev(A), dev(B)))
    K = A.shape[1]
    assert np.all(np.abs(C - ref64(A, B)) <= K * 2.0 ** -24 * absref(A, B))


# ---- full-size workloads: sampled entries checked against the oracle ----------

def _sampled(bfx, orc, A, B, variant, nsample, seed):
    C = host(bfx.gemm(variant, dev(A), dev(B)))
    g = np.random.default_rng(seed)
    r = g.integers(0, A.shape[0], nsample)
    c = g.integers(0, B.shape[1], nsample)
    orc_vals = orc.gemm_entries(variant, A, B, r, c)
    z = np.einsum("ij,ji->i", A[r].astype(np.float64), B[:, c].astype(np.float64))
    zh = np.einsum("ij,ji->i", np.abs(A[r].astype(np.float64)), np.abs(B[:, c].astype(np.float64)))
    bnd = gemm_bound(variant, A.shape[1]) * zh + 1e-38
    got = C[r, c].astype(np.float64)
    assert np.all(np.abs(got - z) <= bnd), float(np.max(np.abs(got - z) / bnd))
    assert np.all(np.abs(orc_vals - z) <= bnd)
    assert np.all(np.abs(got - orc_vals) <= 2 * bnd)
    assert np.all(np.isfinite(C))
    return C


@pytest.mark.parametrize("gen", ["normal", "wide"])
def test_gemm_8192_sampled(bfx, orc, gen):
    f = getattr(workloads, gen)
    A = f((8192, 8192), 100)
    B = f((8192, 8192), 101)
    for v in (3, 6, 9):
        _sampled(bfx, orc, A, B, v, 256, 7 + v)


@pytest.mark.parametrize("cancel", [False, True])
def test_gemm_long_k_splitk(bfx, orc, cancel):
    """64 x 64 x 2^20 (split-K path): all 4096 entries against the FP64 product,
    a sample against the oracle."""
    K = 1 << 20
    if cancel:
        A, B = workloads.cancellation(64, K, 200)
    else:
        A = workloads.uniform((64, K), 201)
        B = workloads.uniform((K, 64), 202)
    z = ref64(A, B)
    zh = absref(A, B)
    for v in (3, 6, 9):
        assert bfx.gemm_ws_size(v, 64, 64, K) > 0
        C = host(bfx.gemm(v, dev(A), dev(B)))
        bnd = gemm_bound(v, K) * zh
        assert np.all(np.abs(C - z) <= bnd)
    g = np.random.default_rng(3)
    r = g.integers(0, 64, 24)
    c = g.integers(0, 64, 24)
    o = orc.gemm_entries(6, A, B, r, c)
    C6 = host(bfx.gemm(6, dev(A), dev(B)))
    assert np.all(np.abs(C6[r, c] - o) <= 2 * gemm_bound(6, K) * zh[r, c])


@pytest.mark.parametrize("variant", [3, 6, 9])
@pytest.mark.parametrize("K", [96, 160])
def test_gemm_persistent_equals_one_tile_launch(bfx, variant, K):
    """Problems made of full 128 x 128 tiles take the persistent launch (64 x
    64 tiles for K <= 128, 128 x 128 above); with 2176 x 2176 outputs some
    workgroups compute several tiles back to back.  Four more columns make
    the tiling partial, which takes the one-tile-per-workgroup launch: every
    output element is accumulated in the same order, so the common columns
    must be bitwise equal, for beta = 0 and beta != 0, and the persistent
    result must meet the bound of the exact product."""
    M = 2176
    A = workloads.normal((M, K), 61)
    B = workloads.normal((K, M + 4), 62)
    C0 = workloads.normal((M, M + 4), 63)
    tA, tB = dev(A), dev(B)
    for alpha, beta in ((1.0, 0.0), (-1.0, 1.0)):
        Cp = dev(C0[:, :M])
        bfx.gemm(variant, tA, tB[:, :M], Cp, alpha=alpha, beta=beta)
        Cr = dev(C0)
        bfx.gemm(variant, tA, tB, Cr, alpha=alpha, beta=beta)
        np.testing.assert_array_equal(host(Cp), host(Cr)[:, :M])
    rows = np.arange(0, M, 97)
    Cp = host(bfx.gemm(variant, tA, tB[:, :M]))
    z = ref64(A[rows], B[:, :M])
    bnd = gemm_bound(variant, K) * absref(A[rows], B[:, :M])
    assert np.all(np.abs(Cp[rows] - z) <= bnd)


def _gemm_fused(bfx, variant, A, B, C, alpha, beta):
    """bfx_gemm without a workspace: the in-kernel split (no pre-split planes)."""
    from paper_1904_06376_amd.api import _stream
    M, K = A.shape
    N = B.shape[1]
    rc = bfx.lib.bfx_gemm(variant, M, N, K, alpha, A.data_ptr(), K, B.data_ptr(), N, beta,
                          C.data_ptr(), N, None, 0, _stream())
    assert rc == 0


@pytest.mark.parametrize("variant", [1, 3, 6, 7, 8, 9])
@pytest.mark.parametrize("shape", [(2048, 2048, 512), (2085, 2148, 1000), (2176, 2048, 1536)])
def test_gemm_presplit_equals_fused(bfx, variant, shape):
    """With a workspace of bfx_gemm_ws_size bytes, problems of >= 256 output
    tiles and K >= 512 split each operand once into BF16 planes (zero-padded
    128 x 32 blocks) and run the products on them; without one, the split
    happens inside the GEMM kernel.  Both split exactly (Sec. II-A) and
    accumulate every output in the same order, so the results must be
    bitwise equal, for beta = 0 and beta != 0, ragged M, N and K included,
    and with zeros, subnormals, values near FLT_MAX, infinities and NaNs in
    the operands."""
    M, N, K = shape
    A = workloads.normal((M, K), 71)
    B = workloads.normal((K, N), 72)
    A[3, :7] = [0.0, -0.0, 1e-39, -3e-41, 3.3e38, np.inf, 1e-30]
    A[M - 1, K - 5:] = [np.nan, 2.0 ** -126, -2.0 ** -140, 1e38, 5.0]
    B[:9, N - 1] = [np.inf, -np.inf, 0.0, 1e-40, 3.4e38, -3.4e38, 2.0 ** -130, 7.0, np.nan]
    C0 = workloads.normal((M, N), 73)
    assert bfx.gemm_ws_size(variant, M, N, K) > 0
    tA, tB = dev(A), dev(B)
    for alpha, beta in ((1.0, 0.0), (-0.75, 1.25)):
        Cp = dev(C0)
        bfx.gemm(variant, tA, tB, Cp, alpha=alpha, beta=beta)
        Cf = dev(C0)
        _gemm_fused(bfx, variant, tA, tB, Cf, alpha, beta)
        np.testing.assert_array_equal(host(Cp).view(np.uint32), host(Cf).view(np.uint32))


def _unblock(blocks, nterms, R, K):
    """Host-side reading of the pre-split block layout (include/bfx.h): plane
    t, block (r, s) at element (t * RB * KS + r * KS + s) * 4096; row n in
    64-byte row n ^ ((n >> 2) & 1), chunk c at position c ^ ((n >> 1) & 3)."""
    RB, KS = -(-R // 128), -(-K // 32)
    b = blocks.reshape(nterms, RB, KS, 128, 4, 8)          # plane, r, s, phys row, chunk pos, k%8
    n = np.arange(128)
    phys = n ^ ((n >> 2) & 1)
    out = np.empty((nterms, RB, 128, KS, 4, 8), np.uint16)
    for c in range(4):
        pos = c ^ ((n >> 1) & 3)
        out[:, :, :, :, c, :] = b[:, :, :, phys, pos, :].transpose(0, 1, 3, 2, 4)
    full = out.reshape(nterms, RB * 128, KS * 32)
    return full[:, :R, :K], full


@pytest.mark.parametrize("shape", [(200, 77), (128, 32), (1, 1), (257, 1000), (130, 4)])
@pytest.mark.parametrize("nterms", [1, 2, 3])
def test_split_blocks_layout_vs_oracle(bfx, orc, shape, nterms):
    """bfx_split_blocks of A (R x K) and of B (K x R, trans) hold the oracle's
    Sec. II-A terms of every element at the documented positions, zeros in the
    padding; special values included."""
    R, K = shape
    X = workloads.normal((R, K), 81) * np.float32(3.0)
    X.ravel()[:6] = [np.inf, -np.nan, 1e-40, 3.4e38, -0.0, 2.0 ** -133][:X.size]
    ref = orc.split(X, 3)
    for trans in (False, True):
        src = X.T.copy() if trans else X
        got = bits16(bfx.split_blocks(dev(src), nterms, trans=trans))
        inner, full = _unblock(got, nterms, R, K)
        for t in range(nterms):
            np.testing.assert_array_equal(inner[t], ref[t])
        pad = full.copy()
        pad[:, :R, :K] = 0
        assert not pad.any()


@pytest.mark.parametrize("variant", [1, 3, 6, 9])
@pytest.mark.parametrize("shape", [(200, 132, 96), (129, 256, 36), (1, 4, 4), (65, 64, 44),
                                   (256, 256, 256), (300, 44, 200), (127, 128, 480)])
def test_gemm_blocks_small_shapes(bfx, orc, variant, shape):
    """bfx_gemm_blocks on small and ragged shapes: within the bound of the
    exact product, within twice the bound of the oracle, and bitwise equal to
    bfx_gemm's in-kernel split (these shapes take its wave-specialised engine
    without split-K, which accumulates in the same order)."""
    M, N, K = shape
    P = {1: 1, 3: 2, 6: 3, 9: 3}[variant]
    A = workloads.normal((M, K), 91)
    B = workloads.normal((K, N), 92)
    C0 = workloads.normal((M, N), 93)
    tA, tB = dev(A), dev(B)
    Ab = bfx.split_blocks(tA, P)
    Bb = bfx.split_blocks(tB, P, trans=True)
    for alpha, beta in ((1.0, 0.0), (0.5, -2.0)):
        Cb = dev(C0)
        bfx.gemm_blocks(variant, M, N, K, Ab, Bb, Cb, alpha=alpha, beta=beta)
        Cf = dev(C0)
        _gemm_fused(bfx, variant, tA, tB, Cf, alpha, beta)
        np.testing.assert_array_equal(host(Cb).view(np.uint32), host(Cf).view(np.uint32))
    Cb = host(bfx.gemm_blocks(variant, M, N, K, Ab, Bb))
    _check_bound(variant, A, B, Cb, orc.gemm(variant, A, B))


def test_gemm_blocks_K0_scales_C(bfx):
    """K = 0: no products, C = beta C (beta = 0: C = 0), the operands unread."""
    C0 = workloads.normal((70, 40), 95)
    e = torch.empty(8, dtype=torch.int16, device="cuda")
    C = dev(C0)
    bfx.gemm_blocks(6, 70, 40, 0, e, e, C, alpha=2.0, beta=-0.5)
    np.testing.assert_array_equal(host(C), np.float32(-0.5) * C0)
    C = dev(C0)
    bfx.gemm_blocks(6, 70, 40, 0, e, e, C, alpha=2.0, beta=0.0)
    assert not host(C).any()


@pytest.mark.parametrize("variant", [3, 6])
@pytest.mark.parametrize("offset", [0, 1])
def test_gemm_presplit_strided_views(bfx, variant, offset):
    """The pre-split path on row-major views with leading dimensions larger
    than the row length (lda = K + 12, ldb = N + 8, ldc = N + 4) and, with
    offset 1, operands that start one element past a 16-byte boundary (the
    splits then take their scalar loads): bitwise equal to the in-kernel
    split on contiguous copies, columns outside the view untouched."""
    M, N, K = 2048, 2100, 640
    A = workloads.normal((M, K + 12 + offset), 101)
    B = workloads.normal((K, N + 8 + offset), 102)
    Cw = workloads.normal((M, N + 4), 103)
    tAw, tBw = dev(A), dev(B)
    tA = tAw[:, offset:offset + K]
    tB = tBw[:, offset:offset + N]
    tCw = dev(Cw)
    tC = tCw[:, :N]
    assert bfx.gemm_ws_size(variant, M, N, K) > 0
    bfx.gemm(variant, tA, tB, tC, alpha=1.5, beta=0.25)
    Cf = dev(np.ascontiguousarray(Cw[:, :N]))
    _gemm_fused(bfx, variant, dev(np.ascontiguousarray(A[:, offset:offset + K])),
                dev(np.ascontiguousarray(B[:, offset:offset + N])), Cf, 1.5, 0.25)
    got = host(tCw)
    np.testing.assert_array_equal(got[:, :N].view(np.uint32), host(Cf).view(np.uint32))
    np.testing.assert_array_equal(got[:, N:], Cw[:, N:])


@pytest.mark.parametrize("variant", [7, 8])
@pytest.mark.parametrize("shape", [(256, 256, 256), (200, 132, 96), (129, 257, 33), (65, 63, 44),
                                   (64, 64, 1000)])
def test_gemm_x7_x8_vs_oracle(bfx, orc, variant, shape):
    """Variants 7 (x6 plus A1 B2) and 8 (bins 0-3) of Sec. II-D / IV-A:
    within the bound of the exact product and twice of it from the oracle's
    bin-by-bin sum, on the wave-specialised, general and split-K engines
    (the shapes select them)."""
    M, N, K = shape
    A = workloads.wide((M, K), 111)
    B = workloads.wide((K, N), 112)
    C = host(bfx.gemm(variant, dev(A), dev(B)))
    _check_bound(variant, A, B, C, orc.gemm(variant, A, B))


def test_gemm_x7_x8_errors_between_x3_and_x9(bfx):
    """On wide-range operands (2^u, u ~ U[-20, 20]) the summed absolute
    errors against FP64 of x6, x7, x8 and x9 agree within 25% (the FP32
    accumulation dominates once bins 0-2 are in, Sec. II-D, II-G) and all are
    far below x3's (which drops bin 2, about 2^-16 of the product)."""
    A = workloads.wide((256, 512), 121)
    B = workloads.wide((512, 256), 122)
    z = ref64(A, B)
    err = {}
    for v in (3, 6, 7, 8, 9):
        err[v] = float(np.sum(np.abs(host(bfx.gemm(v, dev(A), dev(B))).astype(np.float64) - z)))
    hi = max(err[v] for v in (6, 7, 8, 9))
    lo = min(err[v] for v in (6, 7, 8, 9))
    assert hi <= 1.25 * lo, err
    assert err[3] > 8 * hi, err


PER_OPERAND = (12, 13, 21, 23, 31, 32)


@pytest.mark.parametrize("variant", PER_OPERAND)
@pytest.mark.parametrize("shape", [(200, 130, 77), (129, 257, 33), (256, 256, 256), (65, 64, 44),
                                   (3, 5, 4096)])
def test_gemm_per_operand_vs_oracle(bfx, orc, variant, shape):
    """Per-operand split counts (Sec. II-G): every entry within the bound of the
    weaker operand's count and within twice it of the oracle."""
    M, N, K = shape
    A = workloads.gauss_exp((M, K), 900 + M, sigma=2)
    B = workloads.gauss_exp((K, N), 901 + N, sigma=2)
    C = host(bfx.gemm(variant, dev(A), dev(B)))
    _check_bound(variant, A, B, C, orc.gemm(variant, A, B))


def _terms(orc, X, nterms):
    planes = [orc.bf16_bits_to_f32(h).reshape(X.shape).astype(np.float64) for h in orc.split(X.ravel())]
    return sum(planes[:nterms]).astype(np.float32)


@pytest.mark.parametrize("variant", PER_OPERAND)
def test_gemm_per_operand_equals_full_when_dropped_terms_vanish(bfx, orc, variant):
    """With A holding no terms beyond its pa-th and B none beyond its pb-th, the
    dropped products are exact zeros: the GPU result has the bits of the full
    variant (x6, or x3 when both counts are at most 2) on the same engine."""
    pa, pb = divmod(variant, 10)
    full = 3 if max(pa, pb) <= 2 else 6
    A = _terms(orc, workloads.normal((200, 77), 910), pa)
    B = _terms(orc, workloads.normal((77, 130), 911), pb)
    tA, tB = dev(A), dev(B)
    np.testing.assert_array_equal(host(bfx.gemm(variant, tA, tB)).view(np.uint32),
                                  host(bfx.gemm(full, tA, tB)).view(np.uint32))


@pytest.mark.parametrize("variant", [23, 32, 13])
def test_gemm_per_operand_presplit(bfx, orc, variant):
    """2048 x 2048 x 512 with the workspace: the pre-split products kernel
    (bfx_split_blocks planes) against the general engine (small workspace) and
    the oracle on sampled entries."""
    n, K = 2048, 512
    A = workloads.normal((n, K), 920)
    B = workloads.normal((K, n), 921)
    tA, tB = dev(A), dev(B)
    C1 = host(bfx.gemm(variant, tA, tB))                                  # planes path
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    C2 = torch.empty((n, n), dtype=torch.float32, device="cuda")
    from paper_1904_06376_amd._lib import check, lib
    check(lib.bfx_gemm(variant, n, n, K, 1.0, tA.data_ptr(), K, tB.data_ptr(), n, 0.0,
                       C2.data_ptr(), n, ws.data_ptr(), 16, torch.cuda.current_stream().cuda_stream),
          "bfx_gemm")
    C2 = host(C2)
    g = np.random.default_rng(3)
    rows, cols = g.integers(0, n, 200), g.integers(0, n, 200)
    z = np.einsum("ij,ji->i", A[rows].astype(np.float64), B[:, cols].astype(np.float64))
    zh = np.einsum("ij,ji->i", np.abs(A[rows]).astype(np.float64), np.abs(B[:, cols]).astype(np.float64))
    bnd = gemm_bound(variant, K) * zh
    eo = orc.gemm_entries(variant, A, B, rows, cols)
    for C in (C1, C2):
        got = C[rows, cols].astype(np.float64)
        assert np.all(np.abs(got - z) <= bnd)
        assert np.all(np.abs(got - eo) <= 2 * bnd)
    assert np.all(np.abs(C1.astype(np.float64) - C2) <= 2 * gemm_bound(variant, K) * absref(A, B))


@pytest.mark.parametrize("shape", [(200, 130, 77), (256, 256, 256), (64, 64, 1 << 16)])
def test_gemm_fp64_sum(bfx, orc, shape):
    """The "d" option (Sec. IV-A): with alpha = 1, beta = 0 the FP64 sum of the
    two FP32 accumulators rounds to the bits of the FP32 sum; with alpha, beta
    the FP64 epilogue stays within the bound of the exact result and within
    twice it of the oracle's "d" (split-K shape included)."""
    M, N, K = shape
    A = workloads.uniform((M, K), 930 + K)
    B = workloads.uniform((K, N), 931 + K)
    C0 = workloads.uniform((M, N), 932)
    tA, tB = dev(A), dev(B)
    np.testing.assert_array_equal(host(bfx.gemm(6, tA, tB, fp64_sum=True)).view(np.uint32),
                                  host(bfx.gemm(6, tA, tB)).view(np.uint32))
    alpha, beta = 2.5, -0.75
    for v in (3, 6, 9):
        C = host(bfx.gemm(v, tA, tB, dev(C0), alpha=alpha, beta=beta, fp64_sum=True))
        Co = orc.gemm(v, A, B, C0, alpha=alpha, beta=beta, fp64_sum=True)
        z = alpha * ref64(A, B) + beta * C0.astype(np.float64)
        bnd = gemm_bound(v, K) * abs(alpha) * absref(A, B) + 2 * 2.0 ** -24 * (
            np.abs(alpha * ref64(A, B)) + np.abs(beta * C0.astype(np.float64))) + 1e-38
        assert np.all(np.abs(C - z) <= bnd), v
        assert np.all(np.abs(C.astype(np.float64) - Co) <= 2 * bnd), v

"""Pins for the oracle's blocked LU (SGETRF semantics with split-GEMM trailing
updates, Sec. I, IV-A) and residual-form iterative refinement (Sec. III, IV-B).
Checked against LAPACK (scipy getrf/solve), backward-error bounds, pivot
structure on diagonally dominant input, the singular-pivot convention, and the
paper's IR table (FP32-level LU at n=50 converges in a few iterations)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import workloads


def perm_from_ipiv(ipiv, n):
    p = np.arange(n)
    for i, q in enumerate(ipiv):
        p[[i, q]] = p[[q, i]]
    return p


def unpack(LU):
    n = LU.shape[0]
    L = np.tril(LU.astype(np.float64), -1) + np.eye(n)
    Uf = np.triu(LU.astype(np.float64))
    return L, Uf


@pytest.mark.parametrize("n,nb", [(1, 8), (7, 3), (64, 16), (130, 32), (200, 64)])
@pytest.mark.parametrize("variant", [0, 6, 9])
def test_lu_backward_error(orc, n, nb, variant):
    A = workloads.normal((n, n), 40 + n)
    LU, ipiv, info = orc.lu(A, variant, nb)
    assert info == 0
    assert np.all(ipiv >= np.arange(n)) and np.all(ipiv < n)
    p = perm_from_ipiv(ipiv, n)
    L, Uf = unpack(LU)
    R = A.astype(np.float64)[p] - L @ Uf
    scale = np.abs(L) @ np.abs(Uf)
    # componentwise backward error of Gaussian elimination: |PA - LU| <= gamma_n |L||U|
    assert np.all(np.abs(R) <= 2 * n * 2.0 ** -24 * scale + 1e-30)


@pytest.mark.parametrize("n", [16, 50, 97])
def test_lu_pivots_match_lapack(orc, n):
    """Partial pivoting on generic data picks the same rows as LAPACK dgetrf."""
    A = workloads.uniform((n, n), 60 + n)
    LU, ipiv, info = orc.lu(A, 6, 16)
    lu64, piv64 = sla.lu_factor(A.astype(np.float64))
    np.testing.assert_array_equal(ipiv, piv64)
    np.testing.assert_allclose(LU, lu64, rtol=0, atol=2e-4 * np.abs(lu64).max())


def test_lu_unblocked_equals_sgetrf_like_scipy_single(orc):
    """nb >= n is unblocked right-looking elimination in FP32: same pivots as
    LAPACK sgetrf and factors within a few FP32 ulps of it."""
    n = 40
    A = workloads.uniform((n, n), 70)
    LU, ipiv, _ = orc.lu(A, 0, n)
    lu32, piv32, info = sla.lapack.sgetrf(A)
    np.testing.assert_array_equal(ipiv, piv32)
    np.testing.assert_allclose(LU, lu32, rtol=0, atol=1e-5 * np.abs(lu32).max())


def test_diagonally_dominant_no_pivoting(orc):
    n = 96
    A = workloads.uniform((n, n), 71)
    A += np.diag(np.abs(A).sum(axis=0) + 1).astype(np.float32)   # column dominance
    _, ipiv, info = orc.lu(A, 6, 32)
    assert info == 0
    np.testing.assert_array_equal(ipiv, np.arange(n))


def test_singular_info(orc):
    """An exactly zero pivot sets info = column + 1 and the factorisation completes."""
    n = 20
    A = workloads.uniform((n, n), 72)
    A[:, 6] = 0
    LU, ipiv, info = orc.lu(A, 6, 8)
    assert info == 7
    assert np.all(np.isfinite(LU[:, :6]))
    lu32, piv32, info32 = sla.lapack.sgetrf(A)
    assert info32 == 7


def test_fig5_split_lu_more_accurate_than_fp32_lu(orc):
    """Sec. IV-A, Fig. 5: the x6 LU is more accurate element-wise than the FP32
    LU, both measured against the FP64 LU (same pivots), on [-1,1] and [-1e10,1e10]."""
    n = 128
    for scale in (1.0, 1e10):
        ratios = []
        for s in range(3):
            A = (workloads.uniform((n, n), 80 + s) * np.float32(scale)).astype(np.float32)
            lu64, piv64 = sla.lu_factor(A.astype(np.float64))
            l6, p6, _ = orc.lu(A, 6, 32)
            l0, p0, _ = orc.lu(A, 0, 32)
            if not (np.array_equal(p6, piv64) and np.array_equal(p0, piv64)):
                continue
            e6 = np.mean(np.abs(l6 - lu64))
            e0 = np.mean(np.abs(l0 - lu64))
            ratios.append(e6 / e0)
        assert ratios and max(ratios) < 1.0, ratios


def test_lu_solve_matches_lapack(orc):
    n = 60
    A = workloads.normal((n, n), 90)
    b = workloads.normal((n,), 91)
    LU, ipiv, _ = orc.lu(A, 6, 16)
    x = orc.lu_solve(LU, ipiv, b)
    xr = np.linalg.solve(A.astype(np.float64), b.astype(np.float64))
    assert np.max(np.abs(x - xr)) / np.max(np.abs(xr)) < 1e-4


@pytest.mark.parametrize("kappa", [1e1, 1e2, 1e3, 1e4])
def test_ir_table_fp32_rows(orc, kappa):
    """Sec. IV-B IR table: with an FP32-accurate LU, dense unsymmetric n=50 systems
    with kappa up to 1e4 all converge in a few iterations (the paper's FP32 rows:
    100% converged, 2.39-3.47 mean iterations to its own tolerance)."""
    its = []
    for s in range(10):
        A, b, xt = workloads.conditioned_system(50, kappa, 1000 + s)
        LU, ipiv, _ = orc.lu(A, 6, 16)
        res = orc.ir(A, LU, ipiv, b, tol=1e-14, max_iter=30)
        assert res["status"] == 0 and res["eta"] <= 1e-14, res
        its.append(res["iters"])
        # eta recomputed independently with numpy
        r = b - A.astype(np.float64) @ res["x"]
        eta = np.abs(r).max() / (np.abs(A.astype(np.float64)).sum(1).max() * np.abs(res["x"]).max() + np.abs(b).max())
        assert eta <= 1e-14 * 1.01
        # forward error consistent with a backward-stable FP64 solve
        xr = np.linalg.solve(A.astype(np.float64), b)
        assert np.max(np.abs(res["x"] - xr)) / np.max(np.abs(xr)) <= 50 * kappa * 2.0 ** -52
    assert 1 <= np.mean(its) <= 5


def test_ir_residual_matches_numpy(orc):
    A, b, _ = workloads.conditioned_system(30, 10.0, 7)
    x = np.random.default_rng(1).normal(size=30)
    r = orc.residual(A, b, x)
    np.testing.assert_allclose(r, b - A.astype(np.float64) @ x, rtol=0, atol=1e-13)


def test_ir_status_codes(orc):
    A, b, _ = workloads.conditioned_system(40, 1e4, 3)
    LU, ipiv, _ = orc.lu(A, 6, 16)
    res = orc.ir(A, LU, ipiv, b, tol=1e-14, max_iter=0)
    assert res["status"] == 1 and res["iters"] == 0 and res["eta"] > 1e-14
    # an LU with an exactly zero pivot produces a non-finite solve
    As = A.copy()
    As[:, 3] = 0
    LUs, ps, info = orc.lu(As, 6, 16)
    assert info > 0
    res = orc.ir(As, LUs, ps, b, tol=1e-14, max_iter=5)
    assert res["status"] == 3


def test_ir_high_kappa_lu_ir_does_not_reach_fp64(orc):
    """Sec. III: IR breaks down when kappa is large against the LU's precision.
    With kappa(A32) far above 1/2^-24, LU-IR does not reach 1e-14 (reported, the
    GMRES variant is the remedy)."""
    A, b, _ = workloads.conditioned_system(60, 1e12, 5)
    LU, ipiv, _ = orc.lu(A, 6, 16)
    res = orc.ir(A, LU, ipiv, b, tol=1e-14, max_iter=30)
    assert res["status"] in (1, 2) and res["eta"] > 1e-14


@pytest.mark.parametrize("n", [10, 50, 100])
def test_gmres_table_diagonally_dominant(orc, n):
    """Sec. IV-B GMRES table: row- and column-diagonally dominant unsymmetric
    matrices with an FP32-level LU as preconditioner all converge (FP32 rows:
    100% converged, 2.0 iterations on average)."""
    its = []
    for s in range(10):
        g = np.random.default_rng(2000 + 17 * n + s)
        A = g.uniform(-1, 1, (n, n))
        d = np.maximum(np.abs(A).sum(0), np.abs(A).sum(1)) + 1.0
        A = (A + np.diag(d * np.sign(g.uniform(-1, 1, n)))).astype(np.float32)
        b = A.astype(np.float64) @ g.normal(size=n)
        LU, ipiv, _ = orc.lu(A, 6, 16)
        np.testing.assert_array_equal(ipiv, np.arange(n))   # dominance: no pivoting
        res = orc.gmres_ir(A, LU, ipiv, b)
        assert res["status"] == 0 and res["eta"] <= 1e-14
        its.append(res["iters"])
    assert np.mean(its) <= 2.0


@pytest.mark.parametrize("kappa", [1e8, 1e10])
def test_gmres_ir_beyond_lu_ir(orc, kappa):
    """Sec. III: GMRES with the low-precision LU as preconditioner reaches an
    FP64-level backward error in one or two refinement steps where plain LU-IR
    needs many or fails; the solution agrees with LAPACK's FP64 solve to
    within the conditioning."""
    n = 150
    A, b, _ = workloads.conditioned_system(n, kappa, 77)
    LU, ipiv, _ = orc.lu(A, 6, 32)
    g = orc.gmres_ir(A, LU, ipiv, b, restart=n)
    assert g["status"] == 0 and g["eta"] <= 1e-14 and g["iters"] <= 3, g
    r = b - A.astype(np.float64) @ g["x"]
    eta = np.abs(r).max() / (np.abs(A.astype(np.float64)).sum(1).max() * np.abs(g["x"]).max() + np.abs(b).max())
    assert eta <= 1.01e-14
    xr = np.linalg.solve(A.astype(np.float64), b)
    sv = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    k32 = sv[0] / sv[-1]
    assert np.max(np.abs(g["x"] - xr)) <= 10 * k32 * 2.0 ** -52 * np.sqrt(n) * np.max(np.abs(xr))
    ir = orc.ir(A, LU, ipiv, b)
    assert ir["status"] != 0 or ir["iters"] > g["iters"]


def test_gmres_full_krylov_space_is_exact(orc):
    """With restart >= n the Krylov space of the preconditioned operator spans
    R^n, so one GMRES cycle solves the correction equation to rounding level
    even for a singular-value spread far beyond 1/2^-24."""
    n = 40
    A, b, _ = workloads.conditioned_system(n, 1e12, 78)
    LU, ipiv, _ = orc.lu(A, 6, 8)
    g = orc.gmres_ir(A, LU, ipiv, b, restart=n, inner_tol=0.0)
    assert g["status"] == 0 and g["eta"] <= 1e-14 and g["iters"] <= 2
    assert g["inner"] <= 2 * n


# ---------------------------------------------------------------------------
# Single-format LU (the BF16 and FP16 rows of the Sec. IV-B tables)
# ---------------------------------------------------------------------------
FMT_BITS = {1: (8, -126, 127), 2: (11, -14, 15)}


def test_round_fmt_matches_library_casts_and_rationals(orc):
    """The format rounding equals torch's FP32 -> BF16 cast and numpy's FP32 ->
    FP16 cast (nearest even, gradual underflow, overflow to Inf) on FP32 inputs
    across the exponent range, ties included, and an exact-rational rounding on
    FP64 inputs."""
    import torch
    from tests.exact import _round_to_grid
    g = np.random.default_rng(77)
    e = g.integers(-150, 128, 4000)
    x = (g.uniform(1, 2, 4000) * np.exp2(e.astype(np.float64)) * np.where(g.random(4000) < 0.5, -1, 1))
    x32 = x.astype(np.float32)
    ties = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 65520.0, 65519.0, 1.5 * 2 ** -24, 2.5 * 2 ** -133,
                     3.3895e38, 3.4e38], np.float32)
    x32 = np.concatenate([x32, ties, -ties])
    bf = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy()
    hf = x32.astype(np.float16).astype(np.float64)
    for v, b, h in zip(x32, bf, hf):
        assert orc.round_fmt(float(v), 1) == float(b), (v, b)
        assert orc.round_fmt(float(v), 2) == h or (np.isnan(h) and False), (v, h)
    for v in x[:1000]:
        for fmt, (p, emin, emax) in FMT_BITS.items():
            assert orc.round_fmt(float(v), fmt) == _round_to_grid(Fraction(float(v)), p, emin, emax)


def _lu_fmt_emulated(A, fmt):
    """Exact-rational statement of the single-format elimination: every value a
    rational, rounded to the format by integer arithmetic (tests/exact.py)."""
    from tests.exact import _round_to_grid
    p, emin, emax = FMT_BITS[fmt]

    def R(q):
        return Fraction(_round_to_grid(q, p, emin, emax))

    n = A.shape[0]
    M = [[R(Fraction(float(A[i, j]))) for j in range(n)] for i in range(n)]
    piv = []
    for c in range(n):
        best, pr = abs(M[c][c]), c
        for r in range(c + 1, n):
            if abs(M[r][c]) > best:
                best, pr = abs(M[r][c]), r
        piv.append(pr)
        M[c], M[pr] = M[pr], M[c]
        if M[c][c] == 0:
            continue
        for r in range(c + 1, n):
            l = R(M[r][c] / M[c][c])
            M[r][c] = l
            for q in range(c + 1, n):
                M[r][q] = R(M[r][q] - l * M[c][q])
    return np.array([[float(v) for v in row] for row in M], np.float64), np.array(piv, np.int32)


@pytest.mark.parametrize("fmt", [1, 2])
def test_lu_fmt_equals_exact_rational_emulation(orc, fmt):
    """Bit for bit on small matrices of several exponent ranges: every multiplier
    and update rounded once to the format (a missing or extra rounding, or an
    FP32 intermediate, changes some entries)."""
    for seed in range(6):
        n = 3 + seed
        A = workloads.gauss_exp((n, n), 1500 + seed, sigma=2) if seed % 2 else \
            workloads.uniform((n, n), 1500 + seed)
        LU, ipiv, info = orc.lu_fmt(A, fmt)
        LUe, pe = _lu_fmt_emulated(A, fmt)
        np.testing.assert_array_equal(ipiv, pe)
        np.testing.assert_array_equal(LU.astype(np.float64), LUe)


@pytest.mark.parametrize("fmt,n", [(1, 50), (2, 50), (1, 100), (2, 100)])
def test_lu_fmt_backward_error(orc, fmt, n):
    """Gaussian elimination with unit roundoff u of the format: the factors
    reproduce the rounded matrix to gamma_n |L||U| componentwise, and the
    error is of the format's size, not of FP32's."""
    u = 2.0 ** -FMT_BITS[fmt][0]
    A = workloads.normal((n, n), 1600 + n + fmt)
    LU, ipiv, info = orc.lu_fmt(A, fmt)
    assert info == 0
    Af = np.vectorize(lambda v: orc.round_fmt(float(v), fmt))(A.astype(np.float64))
    p = np.arange(n)
    for i, q in enumerate(ipiv):
        p[[i, q]] = p[[q, i]]
    L = np.tril(LU.astype(np.float64), -1) + np.eye(n)
    U = np.triu(LU.astype(np.float64))
    R = np.abs(Af[p] - L @ U)
    gam = n * u / (1 - n * u)
    assert np.all(R <= gam * (np.abs(L) @ np.abs(U)) + 1e-300)
    assert R.max() / np.abs(Af).max() > 2.0 ** -24


def test_ir_and_gmres_tables_single_format_ordering(orc):
    """IR table (n = 50) and GMRES table (diagonally dominant) of Sec. IV-B,
    qualitatively: LU-IR from the FP32-accurate split LU converges in fewer
    steps than from an FP16 LU, and that in fewer than from a BF16 LU; with
    GMRES-IR all three converge, BF16 needing the most GMRES steps."""
    its = {1: [], 2: [], 0: []}
    for s in range(10):
        A, b, _ = workloads.conditioned_system(50, 100.0, 1700 + s)
        for fmt in (0, 1, 2):
            LU, ipiv, _ = orc.lu(A, 6, 64) if fmt == 0 else orc.lu_fmt(A, fmt)
            r = orc.ir(A, LU, ipiv, b, max_iter=100)
            assert r["status"] == 0, (fmt, r)
            its[fmt].append(r["iters"])
    assert np.mean(its[0]) < np.mean(its[2]) < np.mean(its[1])
    inner = {1: [], 2: [], 0: []}
    for s in range(10):
        g = np.random.default_rng(1800 + s)
        n = 50
        A = g.uniform(-1, 1, (n, n))
        d = np.maximum(np.abs(A).sum(0), np.abs(A).sum(1)) + 1.0
        A = (A + np.diag(d * np.sign(g.uniform(-1, 1, n)))).astype(np.float32)
        b = A.astype(np.float64) @ g.normal(size=n)
        for fmt in (0, 1, 2):
            LU, ipiv, _ = orc.lu(A, 6, 64) if fmt == 0 else orc.lu_fmt(A, fmt)
            r = orc.gmres_ir(A, LU, ipiv, b, restart=n)
            assert r["status"] == 0, (fmt, r)
            inner[fmt].append(r["inner"])
    assert np.mean(inner[0]) < np.mean(inner[2]) < np.mean(inner[1])

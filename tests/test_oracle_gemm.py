"""Pins for the oracle's split GEMM (Sec. II-C..II-G, IV-A) and its plain FP32
comparator.  Checked against: exact integer products, identity and permutation
invariants, the paper's componentwise error bounds against an FP64 product,
the exact-Z0 special case, exact-rational emulation on tiny inputs, the worked
example's stated ordering and the Fig. 2 accuracy ordering."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import workloads
from tests.exact import add32, fl32, fma32, frac

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -24
VARIANTS = (1, 3, 6, 7, 8, 9)


def ref64(A, B):
    """FP64 product of FP32 inputs: every scalar product exact, sum error ~K 2^-53."""
    return A.astype(np.float64) @ B.astype(np.float64)


def absref(A, B):
    return np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))


def bound(variant, K):
    """Componentwise bounds relative to |A||B|: 2k 2^-24 for six or more products,
    3*2^-16 + 2k 2^-24 for three; below K=8 the dropped terms alone can reach
    (513/512) 2^-23 (Sec. II-G), so 8*2^-24 is added."""
    k = 2 * K + (8 if K < 8 else 0)
    if variant >= 6:
        return k * U
    if variant == 3:
        return 3 * 2.0 ** -16 + k * U
    return 3 * 2.0 ** -8 + k * U


@pytest.mark.parametrize("variant", VARIANTS)
def test_integer_inputs_exact(orc, variant):
    """Small integers are BF16 numbers and all sums are exact: every variant must
    equal the exact integer product (catches transposed or misindexed operands)."""
    g = np.random.default_rng(11)
    A = g.integers(-8, 9, size=(13, 29)).astype(np.float32)
    B = g.integers(-8, 9, size=(29, 7)).astype(np.float32)
    exact = A.astype(np.int64) @ B.astype(np.int64)
    np.testing.assert_array_equal(orc.gemm(variant, A, B), exact.astype(np.float32))
    np.testing.assert_array_equal(orc.sgemm(A, B), exact.astype(np.float32))


@pytest.mark.parametrize("variant", (6, 7, 8, 9))
def test_identity_reproduces_operand(orc, variant):
    """With six or more products A x I == A and I x B == B bit for bit, because
    a0 + (a1 + a2) rebuilds a exactly (Sec. II-A); the paper's x3 keeps a0 + a1."""
    A = workloads.normal((17, 23), 12)
    I = np.eye(23, dtype=np.float32)
    np.testing.assert_array_equal(orc.gemm(variant, A, I), A)
    np.testing.assert_array_equal(orc.gemm(variant, np.eye(17, dtype=np.float32), A), A)


def test_identity_x3_drops_third_term(orc):
    A = workloads.uniform((16, 16), 13)
    b0, b1, _ = orc.split(A)
    two = orc.bf16_bits_to_f32(b0) + orc.bf16_bits_to_f32(b1)
    got = orc.gemm(3, A, np.eye(16, dtype=np.float32))
    np.testing.assert_array_equal(got, two)
    assert np.any(got != A)


@pytest.mark.parametrize("variant", (3, 6, 9))
def test_row_col_permutation_equivariance(orc, variant):
    g = np.random.default_rng(14)
    A = workloads.uniform((12, 40), 15)
    B = workloads.uniform((40, 9), 16)
    pr = g.permutation(12)
    pc = g.permutation(9)
    C = orc.gemm(variant, A, B)
    np.testing.assert_array_equal(orc.gemm(variant, A[pr], B[:, pc]), C[pr][:, pc])


@pytest.mark.parametrize("gen", ["uniform", "normal", "wide", "gauss_exp"])
@pytest.mark.parametrize("K", [1, 5, 32, 100, 257])
def test_componentwise_bounds(orc, gen, K):
    """Spec bounds: x6/x9 within 2k 2^-24 |A||B| and x3 within
    (3*2^-16 + 2k 2^-24)|A||B| of the exact product; FP32 within gamma_k."""
    f = getattr(workloads, gen)
    A = f((23, K), 100 + K)
    B = f((K, 19), 200 + K)
    z = ref64(A, B)
    zh = absref(A, B)
    for v in (3, 6, 7, 8, 9):
        err = np.abs(orc.gemm(v, A, B).astype(np.float64) - z)
        assert np.all(err <= bound(v, K) * zh), (v, float(np.max(err / zh)))
    err = np.abs(orc.sgemm(A, B).astype(np.float64) - z)
    gam = K * U / (1 - K * U)
    assert np.all(err <= gam * zh * (1 + 1e-12) + 1e-300)


def test_x3_is_not_x6(orc):
    """The two-term variant must actually lose the 2^-16 bin (guards a variant mix-up)."""
    A = workloads.uniform((32, 64), 17)
    B = workloads.uniform((64, 32), 18)
    z = ref64(A, B)
    zh = absref(A, B)
    e3 = np.max(np.abs(orc.gemm(3, A, B) - z) / zh)
    e6 = np.max(np.abs(orc.gemm(6, A, B) - z) / zh)
    assert e3 > 2.0 ** -20 and e6 < 2.0 ** -20 and e3 > 8 * e6


def test_exact_Z0_special_case(orc):
    """Sec. II-E special case: inputs in [1,2), K <= 64: every a0*b0 is a multiple
    of 2^-14 below 4, so the FP32 chain Z^(0,0) is exact and
    |Z_2 - z| <= 1.01 (gamma_3 + 2 gamma_k 2^-8) zhat (the paper's 1.01 gamma_3
    plus the lower bins' own accumulation error)."""
    g = np.random.default_rng(19)
    K = 64
    x = g.uniform(1, 2, K).astype(np.float32)
    y = g.uniform(1, 2, K).astype(np.float32)
    Z = orc.dot_partials(x, y)
    a0 = orc.bf16_bits_to_f32(orc.split(x)[0]).astype(np.float64)
    c0 = orc.bf16_bits_to_f32(orc.split(y)[0]).astype(np.float64)
    assert Z[0, 0] == np.sum(a0 * c0)
    A = x[None, :]
    B = y[:, None]
    z = float(sum(frac(p) * frac(q) for p, q in zip(x, y)))
    zh = abs(z)
    got = float(orc.gemm(6, A, B)[0, 0])
    g3 = 3 * U / (1 - 3 * U)
    gk = K * U / (1 - K * U)
    assert abs(got - z) <= 1.01 * (g3 + 2 * gk * 2.0 ** -8) * zh


def test_partial_magnitudes(orc):
    """Sec. II-E: |Z^(i,j)| <= (1 + gamma_n) eps_b^(i+j) zhat (with the (1+2^-8)^2
    slack of |x^(0)| <= (1+2^-8)|x|)."""
    g = np.random.default_rng(20)
    for n in (8, 64, 500):
        x = g.uniform(-1, 1, n).astype(np.float32)
        y = g.normal(size=n).astype(np.float32)
        Z = orc.dot_partials(x, y)
        zh = float(np.sum(np.abs(x.astype(np.float64) * y)))
        gam = n * U / (1 - n * U)
        for i in range(3):
            for j in range(3):
                assert abs(Z[i, j]) <= (1 + gam) * (1 + 2.0 ** -8) ** 2 * 2.0 ** (-8 * (i + j)) * zh


def _emulate(variant, x, y):
    """Exact-rational emulation of the Sec. II-D algorithm for one entry: split by
    nearest-even rounding of rationals, FP32 FMA chains, FP32 bin sums."""
    from tests.exact import bf16_nearest

    def split(v):
        t0 = bf16_nearest(frac(v))
        r1 = frac(v) - Fraction(t0)
        t1 = bf16_nearest(r1)
        r2 = r1 - Fraction(t1)
        t2 = bf16_nearest(r2)
        return [t0, t1, t2]

    xs = [split(v) for v in x]
    ys = [split(v) for v in y]
    need = {1: lambda i, j: i + j == 0, 3: lambda i, j: i + j <= 1,
            6: lambda i, j: i + j <= 2, 9: lambda i, j: True}[variant]
    Z = [[np.float32(0)] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            if not need(i, j):
                continue
            acc = np.float32(0)
            for a, b in zip(xs, ys):
                acc = fma32(a[i], b[j], acc)
            Z[i][j] = acc
    Z0 = Z[0][0]
    if variant == 1:
        return Z0
    Z1 = add32(Z[0][1], Z[1][0])
    if variant == 3:
        return add32(Z0, Z1)
    Z2 = add32(Z[0][2], add32(Z[1][1], Z[2][0]))
    if variant == 6:
        return add32(Z0, add32(Z1, Z2))
    Z3 = add32(Z[1][2], Z[2][1])
    return add32(Z0, add32(Z1, add32(Z2, add32(Z3, Z[2][2]))))


@pytest.mark.parametrize("variant", (1, 3, 6, 9))
def test_exact_rational_emulation_tiny(orc, variant):
    """Brute force on tiny inputs: the C oracle equals an exact-rational emulation
    of the algorithm bit for bit (checks FMA, ordering and the bin brackets)."""
    for seed in range(4):
        A = workloads.gauss_exp((3, 5), 300 + seed, sigma=3)
        B = workloads.gauss_exp((5, 2), 400 + seed, sigma=3)
        C = orc.gemm(variant, A, B)
        for i in range(3):
            for j in range(2):
                e = _emulate(variant, A[i], B[:, j])
                assert C[i, j] == e, (variant, seed, i, j, C[i, j], e)


def test_worked_example_ordering(orc):
    """Sec. II-G: for x = 0.5789..., y = -7447.66... six products are less accurate
    than FP32, while adding a1*b2 (seven products) is at least as accurate."""
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    x = np.float32(ex["x"])
    y = np.float32(ex["y"])
    exact = frac(x) * frac(y)

    def err(v):
        return abs(Fraction(float(v)) - exact)

    fp32 = fl32(exact)
    assert orc.sgemm(np.array([[x]]), np.array([[y]]))[0, 0] == fp32
    r = {v: orc.gemm(v, np.array([[x]]), np.array([[y]]))[0, 0] for v in (3, 6, 7, 9)}
    assert err(r[6]) > err(fp32)
    assert err(r[7]) <= err(fp32)
    assert err(r[9]) <= err(fp32)
    assert err(r[3]) > err(r[6])


def test_sgemm_K1_is_correctly_rounded_product(orc):
    g = np.random.default_rng(21)
    A = workloads.wide((40, 1), 22)
    B = workloads.wide((1, 30), 23)
    expect = (A.astype(np.float64) @ B.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(orc.sgemm(A, B), expect)


def test_epilogue_alpha_beta(orc):
    """C = fma(alpha, X, beta*C); beta = 0 means C is not read (BLAS)."""
    A = workloads.uniform((6, 11), 24)
    B = workloads.uniform((11, 5), 25)
    X = orc.gemm(6, A, B)
    C0 = workloads.uniform((6, 5), 26)
    alpha, beta = np.float32(-1.5), np.float32(0.75)
    got = orc.gemm(6, A, B, C0, alpha, beta)
    for i in range(6):
        for j in range(5):
            bc = fl32(frac(beta) * frac(C0[i, j]))
            assert got[i, j] == fma32(alpha, X[i, j], bc)
    Cnan = np.full((6, 5), np.nan, np.float32)
    np.testing.assert_array_equal(orc.gemm(6, A, B, Cnan, alpha, 0.0), (alpha * X).astype(np.float32))
    np.testing.assert_array_equal(orc.sgemm(A, B, Cnan, 2.0, 0.0), 2 * orc.sgemm(A, B))


def test_entries_match_full(orc):
    A = workloads.normal((20, 70), 27)
    B = workloads.normal((70, 15), 28)
    g = np.random.default_rng(29)
    r = g.integers(0, 20, 50)
    c = g.integers(0, 15, 50)
    for v in (3, 6, 9):
        full = orc.gemm(v, A, B)
        np.testing.assert_array_equal(orc.gemm_entries(v, A, B, r, c), full[r, c])
    np.testing.assert_array_equal(orc.sgemm_entries(A, B, r, c), orc.sgemm(A, B)[r, c])


def test_fig2_accuracy_ordering(orc):
    """Sec. IV-A, Fig. 2: on [-1,1] data the mean relative Frobenius error vs an
    FP64 product orders x3 > FP32 > x6 >= x6 with an FP64 final sum."""
    errs = {k: [] for k in ("x3", "fp32", "x6", "x6d")}
    for s in range(8):
        A = workloads.uniform((64, 256), 500 + s)
        B = workloads.uniform((256, 64), 600 + s)
        z = ref64(A, B)
        nz = np.linalg.norm(z)
        errs["x3"].append(np.linalg.norm(orc.gemm(3, A, B) - z) / nz)
        errs["fp32"].append(np.linalg.norm(orc.sgemm(A, B) - z) / nz)
        errs["x6"].append(np.linalg.norm(orc.gemm(6, A, B) - z) / nz)
        errs["x6d"].append(np.linalg.norm(orc.gemm(6, A, B, fp64_sum=True) - z) / nz)
    m = {k: float(np.mean(v)) for k, v in errs.items()}
    assert m["x3"] > m["fp32"] > m["x6"] >= m["x6d"], m


def test_nonfinite_propagation(orc):
    """Inf/NaN inputs give non-finite outputs exactly in their row/column."""
    A = workloads.uniform((8, 16), 30)
    B = workloads.uniform((16, 6), 31)
    A[2, 5] = np.inf
    B[7, 4] = np.nan
    for v in (3, 6, 9):
        C = orc.gemm(v, A, B)
        bad = ~np.isfinite(C)
        expect = np.zeros_like(bad)
        expect[2, :] = True
        expect[:, 4] = True
        np.testing.assert_array_equal(bad, expect)


def test_argument_errors(orc):
    A = np.zeros((2, 2), np.float32)
    with pytest.raises(ValueError):
        orc.gemm(5, A, A)
    with pytest.raises(ValueError):
        orc.gemm(2, A, A)

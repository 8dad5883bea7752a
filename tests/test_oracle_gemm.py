"""Pins for the oracle's split GEMM (Sec. II-C..II-G, IV-A) and its plain FP32
comparator.  Checked against: exact integer products, identity and permutation
invariants, the paper's componentwise error bounds against an FP64 product,
the exact-Z0 special case, exact-rational emulation on tiny inputs (FP32 and
FP64 bin sums), product-membership probes for every variant, the worked
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
# per-operand split counts (Sec. II-G): 10 * (terms of A) + (terms of B)
PER_OPERAND = (12, 13, 21, 23, 31, 32)


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


def _emulate(variant, x, y, fp64_sum=False):
    """Exact-rational emulation of the Sec. II-D algorithm for one entry: split by
    nearest-even rounding of rationals, FP32 FMA chains, bin sums in the printed
    brackets (FP32, or FP64 for the "d" option of Sec. IV-A, whose FP64 result is
    then rounded once to FP32).  Bins: Z0 = Z00, Z1 = Z01 + Z10,
    Z2 = Z02 + (Z11 + Z20), Z3 = Z12 + Z21, Z4 = Z22; x7 adds Z12 alone as the
    bin after Z2."""
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
    if variant in PER_OPERAND:
        pa, pb = divmod(variant, 10)
        need = lambda i, j: i < pa and j < pb and i + j <= 2  # noqa: E731
        # bins and brackets of x3 (both counts <= 2) or x6, absent products as +0 chains
        variant = 3 if max(pa, pb) <= 2 else 6
    else:
        need = {1: lambda i, j: i + j == 0, 3: lambda i, j: i + j <= 1,
                6: lambda i, j: i + j <= 2, 7: lambda i, j: i + j <= 2 or (i, j) == (1, 2),
                8: lambda i, j: i + j <= 3, 9: lambda i, j: True}[variant]
    Z = [[np.float32(0)] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            if not need(i, j):
                continue
            acc = np.float32(0)
            for a, b in zip(xs, ys):
                acc = fma32(a[i], b[j], acc)
            Z[i][j] = acc
    if fp64_sum:
        # FP64 additions of exact FP32 values: float(Fraction) rounds to nearest
        def add(a, b):
            return float(frac(a) + frac(b))
    else:
        add = add32
    Z0 = Z[0][0]
    if variant == 1:
        r = Z0
    else:
        Z1 = add(Z[0][1], Z[1][0])
        if variant == 3:
            r = add(Z0, Z1)
        else:
            Z2 = add(Z[0][2], add(Z[1][1], Z[2][0]))
            if variant == 6:
                r = add(Z0, add(Z1, Z2))
            elif variant == 7:
                r = add(Z0, add(Z1, add(Z2, Z[1][2])))
            else:
                Z3 = add(Z[1][2], Z[2][1])
                if variant == 8:
                    r = add(Z0, add(Z1, add(Z2, Z3)))
                else:
                    r = add(Z0, add(Z1, add(Z2, add(Z3, Z[2][2]))))
    return fl32(frac(r)) if fp64_sum else r


@pytest.mark.parametrize("variant", VARIANTS + PER_OPERAND)
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


def _cancelling_pairs(rows, cols, seed):
    """Operands whose products cancel in their leading terms: row i of A is
    (a, a(1 + d)) with |d| <= 1e-3 and column j of B is (b, -b), so the bin-0
    chain nearly cancels and the lower bins decide the low bits of the result,
    where an FP32 and an FP64 bin sum round differently."""
    g = np.random.default_rng(seed)
    A = g.uniform(-1, 1, (rows, 2)).astype(np.float32)
    A[:, 1] = A[:, 0] * (1 + g.uniform(-1e-3, 1e-3, rows)).astype(np.float32)
    B = g.uniform(-1, 1, (2, cols)).astype(np.float32)
    B[1, :] = -B[0, :]
    return A, B


@pytest.mark.parametrize("variant", (3, 6, 7, 8, 9))
def test_exact_rational_emulation_fp64_sum(orc, variant):
    """The "d" option of Sec. IV-A (bins and final sum in FP64, one rounding to
    FP32 at the end) equals its exact-rational emulation bit for bit, on data
    where it differs from the FP32 bin sum (an FP32 sum in its place fails; x3
    has a single addition, which rounds once either way)."""
    differ = 0
    for seed in range(6):
        A, B = _cancelling_pairs(6, 6, 330 + seed)
        C = orc.gemm(variant, A, B, fp64_sum=True)
        differ += int(np.sum(C != orc.gemm(variant, A, B)))
        for i in range(6):
            for j in range(6):
                e = _emulate(variant, A[i], B[:, j], fp64_sum=True)
                assert C[i, j] == e, (variant, seed, i, j, C[i, j], e)
    if variant >= 6:
        assert differ > 0, "inputs do not separate the FP64 from the FP32 bin sum"
    else:
        assert differ == 0


def test_each_product_is_in_exactly_its_variants(orc):
    """Which products each variant includes (Sec. II-D: x3 = bins 0-1, x6 = bins
    0-2, x8 = bins 0-3, x9 = all; x7 = x6 + Z^(1,2), the worked example of
    Sec. II-G), isolated with K = 2 operands built from a = 1 + 2^-9 + 2^-18,
    a' = 1 + 2^-9 + 2^-19, c = 1 + 2^-9 and c' = 1 + 2^-10, which split as
    (1, 2^-9, 2^-18), (1, 2^-9, 2^-19), (1, 2^-9, 0) and (1, 2^-10, 0):
      x = (a, a),  y = (a, -a'):  only Z^(i,2) = a_i 2^-19 survive;
      x = (a, -a'), y = (a, a):   only Z^(2,j) = 2^-19 a_j survive;
      x = (a, a),  y = (c, -c'):  only Z^(i,1) = a_i 2^-10 survive;
      x = (c, -c'), y = (a, a):   only Z^(1,j) = 2^-10 a_j survive.
    Every chain and bin sum is exact, so the result is the exact sum of the
    included products; a product dropped from or added to any variant (x8 without
    Z^(2,1), x7 with Z^(2,1), ...) changes one of the two results."""
    a = np.float32(1.0 + 2.0 ** -9 + 2.0 ** -18)
    a2 = np.float32(1.0 + 2.0 ** -9 + 2.0 ** -19)
    ta = [float(orc.bf16_bits_to_f32(h)[0]) for h in orc.split(np.array([a]))]
    ta2 = [float(orc.bf16_bits_to_f32(h)[0]) for h in orc.split(np.array([a2]))]
    c = np.float32(1.0 + 2.0 ** -9)
    c2 = np.float32(1.0 + 2.0 ** -10)
    tc = [float(orc.bf16_bits_to_f32(h)[0]) for h in orc.split(np.array([c]))]
    tc2 = [float(orc.bf16_bits_to_f32(h)[0]) for h in orc.split(np.array([c2]))]
    assert ta == [1.0, 2.0 ** -9, 2.0 ** -18] and ta2 == [1.0, 2.0 ** -9, 2.0 ** -19]
    assert tc == [1.0, 2.0 ** -9, 0.0] and tc2 == [1.0, 2.0 ** -10, 0.0]
    included = {
        1: {(0, 0)},
        3: {(0, 0), (0, 1), (1, 0)},
        6: {(i, j) for i in range(3) for j in range(3) if i + j <= 2},
        7: {(i, j) for i in range(3) for j in range(3) if i + j <= 2} | {(1, 2)},
        8: {(i, j) for i in range(3) for j in range(3) if i + j <= 3},
        9: {(i, j) for i in range(3) for j in range(3)},
    }
    for v in PER_OPERAND:
        pa, pb = divmod(v, 10)
        included[v] = {(i, j) for i in range(pa) for j in range(pb) if i + j <= 2}
    F = Fraction
    probes = {
        "column": (np.array([[a, a]], np.float32), np.array([[a], [-a2]], np.float32),
                   lambda i, j: F(ta[i]) * (F(ta[j]) - F(ta2[j]))),
        "row": (np.array([[a, -a2]], np.float32), np.array([[a], [a]], np.float32),
                lambda i, j: (F(ta[i]) - F(ta2[i])) * F(ta[j])),
        "column1": (np.array([[a, a]], np.float32), np.array([[c], [-c2]], np.float32),
                    lambda i, j: F(ta[i]) * (F(tc[j]) - F(tc2[j]))),
        "row1": (np.array([[c, -c2]], np.float32), np.array([[a], [a]], np.float32),
                 lambda i, j: (F(tc[i]) - F(tc2[i])) * F(ta[j])),
    }
    seen = {}
    for name, (X, Y, Zij) in probes.items():
        for v, inc in included.items():
            exact = sum((Zij(i, j) for (i, j) in inc), F(0))
            assert fl32(exact) == exact  # representable: the result must be exact
            seen[(name, v)] = exact
            for d in (False, True):
                got = orc.gemm(v, X, Y, fp64_sum=d)[0, 0]
                assert F(float(got)) == exact, (name, v, d, float(got), float(exact))
    # the probes separate every pair of variants
    for v in included:
        for w in included:
            if v < w:
                assert any(seen[(p, v)] != seen[(p, w)] for p in probes), (v, w)


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


def _terms(X, nterms):
    """X rounded to its first `nterms` BF16 terms (values with no further terms)."""
    planes = orc_split_planes(X)
    out = np.zeros(X.shape, np.float64)
    for p in planes[:nterms]:
        out += p
    return out.astype(np.float32)


def orc_split_planes(X):
    import oracle
    return [oracle.bf16_bits_to_f32(h).reshape(X.shape).astype(np.float64) for h in oracle.split(X.ravel())]


@pytest.mark.parametrize("variant", PER_OPERAND)
def test_per_operand_equals_full_when_dropped_terms_vanish(orc, variant):
    """Sec. II-G, different split counts per operand: when A has no terms beyond
    its pa-th and B none beyond its pb-th, the products the variant drops are
    exactly zero and it returns the bits of the variant with all terms (x6, or
    x3 when both counts are at most 2); on general data it does not (the
    dropped products matter), and its error is within the bound of the weaker
    operand's count."""
    pa, pb = divmod(variant, 10)
    full = 3 if max(pa, pb) <= 2 else 6
    for seed in range(3):
        A = workloads.gauss_exp((17, 33), 700 + seed, sigma=2)
        B = workloads.gauss_exp((33, 9), 800 + seed, sigma=2)
        At, Bt = _terms(A, pa), _terms(B, pb)
        np.testing.assert_array_equal(orc.gemm(variant, At, Bt).view(np.uint32),
                                      orc.gemm(full, At, Bt).view(np.uint32))
        assert np.any(orc.gemm(variant, A, B) != orc.gemm(full, A, B))
        K = A.shape[1]
        z = A.astype(np.float64) @ B.astype(np.float64)
        zh = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
        bnd = (3 * 2.0 ** -8 if min(pa, pb) == 1 else 3 * 2.0 ** -16) + 2 * K * U
        assert np.all(np.abs(orc.gemm(variant, A, B) - z) <= bnd * zh)

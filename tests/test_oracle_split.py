"""Pins for the oracle's FP32 -> BF16 conversion and three-way split (Sec. II-A,
II-F, II-G).  Each test checks the oracle against something other than itself:
torch's CPU bfloat16 cast, exact rational rounding, the exactness domain and
residual bounds the paper states, and its statistical claims."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from tests.exact import bf16_nearest, frac

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bits(x):
    return np.asarray(x, np.float32).view(np.uint32)


def _f(h):
    return (np.asarray(h, np.uint16).astype(np.uint32) << 16).view(np.float32)


def _stratified_finite(seed, per_exp=400):
    """Random finite FP32 patterns covering every biased exponent 0..254."""
    g = np.random.default_rng(seed)
    exps = np.repeat(np.arange(0, 255, dtype=np.uint32), per_exp)
    mant = g.integers(0, 1 << 23, size=exps.size, dtype=np.uint32)
    sign = g.integers(0, 2, size=exps.size, dtype=np.uint32) << 31
    return (sign | (exps << 23) | mant).view(np.float32)


def test_b0_matches_torch_bf16_cast(orc):
    """b0 = (B16)a must equal torch's CPU RNE cast wherever that does not overflow."""
    a = _stratified_finite(1)
    extra = np.array([0x3F808000, 0x3F818000, 0x3F80_8001, 0x3F80_7FFF,
                      0x0000_8000, 0x0001_8000, 0x0000_0001, 0x807F_FFFF,
                      0x7F7F_7FFF], np.uint32).view(np.float32)
    a = np.concatenate([a, extra])
    b0, _, _ = orc.split(a)
    t = torch.from_numpy(a.copy()).to(torch.bfloat16).view(torch.int16).numpy()
    t = t.view(np.uint16)
    ok = np.isfinite(_f(t))           # torch overflows to Inf; the oracle saturates
    assert ok.mean() > 0.99
    np.testing.assert_array_equal(b0[ok], t[ok])


def test_b0_matches_exact_rational_rounding(orc):
    """Brute force: nearest BF16 by exact rational distance, ties to even."""
    g = np.random.default_rng(2)
    a = _stratified_finite(3, per_exp=6)
    # force exact ties and near-ties
    ties = (g.integers(0, 1 << 31, size=200, dtype=np.uint32) & 0x7FFF0000) | 0x8000
    a = np.concatenate([a, ties.view(np.float32)])
    a = a[np.abs(a) < np.float32(3.38e38)]
    b0 = orc.split(a)[0]
    for v, h in zip(a, b0):
        expect = bf16_nearest(frac(v))
        assert _f(h) == np.float32(expect), (hex(int(_bits(v))), hex(int(h)))


def test_special_values(orc):
    inf = np.float32(np.inf)
    a = np.array([0.0, -0.0, inf, -inf, np.nan], np.float32)
    a[4] = np.array([0x7FA00001], np.uint32).view(np.float32)[0]   # signalling NaN
    b0, b1, b2 = orc.split(a)
    assert list(b0) == [0x0000, 0x8000, 0x7F80, 0xFF80, 0x7FC0]
    assert list(b1) == [0, 0, 0, 0, 0]
    assert list(b2) == [0, 0, 0, 0, 0]
    neg_nan = np.array([0xFFC12345], np.uint32).view(np.float32)
    assert orc.split(neg_nan)[0][0] == 0xFFC0


def test_saturation_keeps_split_exact_at_top_of_range(orc):
    """Values that would round to Inf saturate to the largest BF16 (reading R-sat);
    the split then stays exact up to FLT_MAX, as the usable range [-110,127] needs."""
    pats = np.arange(0x7F7F8000, 0x7F800000, 7, dtype=np.uint32)
    a = np.concatenate([pats, pats | 0x80000000]).view(np.float32)
    b0, b1, b2 = orc.split(a)
    assert np.all((b0 & 0x7FFF) == 0x7F7F)
    s = _f(b0).astype(np.float64) + _f(b1) + _f(b2)
    np.testing.assert_array_equal(s, a.astype(np.float64))


def test_split_exact_in_paper_range(orc):
    """Sec. II-F: for exponents >= -110 the three terms represent a exactly."""
    a = _stratified_finite(4, per_exp=800)
    mag = np.abs(a.astype(np.float64))
    a = a[(mag >= 2.0 ** -110) | (mag == 0)]
    b0, b1, b2 = orc.split(a)
    s = _f(b0).astype(np.float64) + _f(b1).astype(np.float64) + _f(b2).astype(np.float64)
    np.testing.assert_array_equal(s, a.astype(np.float64))


def test_split_below_range_error_bound(orc):
    """Below 2^-110 the low terms fall under the BF16 subnormal grid (2^-133):
    the lost part is at most half a grid step."""
    a = _stratified_finite(5, per_exp=400)
    a = a[(np.abs(a.astype(np.float64)) < 2.0 ** -110) & (a != 0)]
    b0, b1, b2 = orc.split(a)
    s = _f(b0).astype(np.float64) + _f(b1) + _f(b2)
    err = np.abs(a.astype(np.float64) - s)
    assert err.max() <= 2.0 ** -134
    # and it is genuinely lossy there (the paper's worst case)
    assert (err > 0).mean() > 0.4


def test_paper_bad_number_loses_bits(orc):
    """Sec. II-F: exponent field 1, bit 16 set, bits 0-15 all ones (~1.1939e-38):
    b1 = b2 = 0 and only the top bits survive."""
    a = np.array([(1 << 23) | (1 << 16) | 0xFFFF], np.uint32).view(np.float32)
    assert abs(float(a[0]) - 1.1939e-38) < 1e-41
    b0, b1, b2 = orc.split(a)
    assert _f(b1)[0] == 0 and _f(b2)[0] == 0
    assert _f(b0)[0] != a[0]


def test_residual_bounds(orc):
    """Sec. II-G: |b1| <= 2^-8 |b0| and |b2| <= 2^-8 |b1| (round to nearest)."""
    a = _stratified_finite(6, per_exp=400)
    a = a[np.abs(a.astype(np.float64)) >= 2.0 ** -100]
    b0, b1, b2 = (_f(b).astype(np.float64) for b in orc.split(a))
    assert np.all(np.abs(b1) <= 2.0 ** -8 * np.abs(b0))
    assert np.all(np.abs(b2) <= 2.0 ** -8 * np.abs(b1))


def test_mean_term_ratios_768(orc):
    """Sec. II-G: for uniformly distributed data |a1| ~ |a0|/768, |a2| ~ |a0|/768^2."""
    a = np.random.default_rng(7).uniform(-1, 1, 200_000).astype(np.float32)
    b0, b1, b2 = (_f(b).astype(np.float64) for b in orc.split(a))
    m1 = np.mean(np.abs(b1) / np.abs(b0))
    m2 = np.mean(np.abs(b2) / np.abs(b0))
    assert abs(m1 * 768 - 1) < 0.10, m1
    assert abs(m2 * 768 ** 2 - 1) < 0.10, m2


def test_dropped_terms_E_bound_and_mean(orc):
    """Sec. II-G: E = a1 b2 + a2 b1 + a2 b2 satisfies |E| <= (513/512) 2^-23 |a0 b0|;
    on average it is a few 1e-9 of |a0 b0| (the paper quotes ~4.412e-9)."""
    g = np.random.default_rng(8)
    x = g.uniform(-1, 1, 100_000).astype(np.float32)
    y = g.uniform(-1, 1, 100_000).astype(np.float32)
    a0, a1, a2 = (_f(b).astype(np.float64) for b in orc.split(x))
    c0, c1, c2 = (_f(b).astype(np.float64) for b in orc.split(y))
    E = a1 * c2 + a2 * c1 + a2 * c2
    p = np.abs(a0 * c0)
    assert np.all(np.abs(E) <= (513 / 512) * 2.0 ** -23 * p)
    mean = np.mean(np.abs(E) / p)
    assert 1e-9 < mean < 1e-8, mean


def test_worked_example_split_terms(orc):
    """Sec. II-G worked example: the split terms of x and y are exact
    decompositions with the magnitude ordering of the bins."""
    ex = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    x = np.float32(ex["x"])
    y = np.float32(ex["y"])
    for v in (x, y):
        h = orc.split(np.array([v]))
        terms = [Fraction(float(_f(t)[0])) for t in h]
        assert sum(terms) == Fraction(float(v))
        assert abs(terms[1]) <= abs(terms[0]) / 256
        assert abs(terms[2]) <= abs(terms[1]) / 256

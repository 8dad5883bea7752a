"""GPU split (bfx_split_f32) vs the oracle: bit-exact on the 256^3 workload's
131072 inputs, on every FP32 exponent, on special values, and exhaustively over
all 2^32 bit patterns."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import bits16, dev

pytestmark = pytest.mark.gpu


def _check(bfx, orc, a, nterms=3):
    got = bfx.split(dev(a), nterms)
    exp = orc.split(a, nterms)
    for p in range(nterms):
        np.testing.assert_array_equal(bits16(got[p]), exp[p], err_msg=f"plane {p}")


def test_split_gemm256_inputs(bfx, orc):
    A = workloads.uniform((256, 256), 0)
    B = workloads.uniform((256, 256), 1)
    _check(bfx, orc, np.concatenate([A.ravel(), B.ravel()]))


def test_split_all_exponents_and_specials(bfx, orc):
    g = np.random.default_rng(3)
    exps = np.repeat(np.arange(256, dtype=np.uint32), 512)
    pats = (g.integers(0, 2, exps.size, dtype=np.uint32) << 31) | (exps << 23) | \
        g.integers(0, 1 << 23, exps.size, dtype=np.uint32)
    extra = np.array([0, 0x80000000, 0x7F800000, 0xFF800000, 0x7FC00000, 0x7FA00001,
                      0xFFC12345, 0x7F7F8000, 0x7F7FFFFF, 0xFF7F8000, 0x00000001,
                      0x00008000, 0x00018000, 0x3F808000, 0x3F818000], np.uint32)
    a = np.concatenate([pats, extra, np.arange(0x7F7F8000, 0x7F800000, dtype=np.uint32)])
    _check(bfx, orc, a.view(np.float32))
    _check(bfx, orc, a.view(np.float32), nterms=2)


@pytest.mark.parametrize("n", [0, 1, 3, 5, 1023, 4097])
def test_split_ragged_lengths(bfx, orc, n):
    a = workloads.normal((n,), 10 + n)
    _check(bfx, orc, a)


def test_split_unaligned_view(bfx, orc):
    a = workloads.normal((1001,), 5)
    t = dev(a)[1:]
    got = bfx.split(t.contiguous()[0:999])   # contiguous offset copy
    exp = orc.split(a[1:1000])
    for p in range(3):
        np.testing.assert_array_equal(bits16(got[p]), exp[p])


@pytest.mark.timeout(600)
def test_split_exhaustive_2pow32(bfx, orc):
    """Every one of the 2^32 FP32 bit patterns splits exactly as the oracle does."""
    chunk = 1 << 26
    mism = 0
    for c in range(1 << 32 >> 26):
        lo = c * chunk
        a = np.arange(lo, lo + chunk, dtype=np.uint64).astype(np.uint32).view(np.float32)
        got = bfx.split(dev(a))
        exp = orc.split(a)
        for p in range(3):
            mism += int(np.count_nonzero(bits16(got[p]) != exp[p]))
        del got
    assert mism == 0

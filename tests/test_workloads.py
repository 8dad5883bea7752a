"""The seeded generators are deterministic and have the stated distributions."""
import numpy as np

import workloads


def test_deterministic_and_dtypes():
    for f in (workloads.uniform, workloads.normal, workloads.wide, workloads.gauss_exp):
        a = f((31, 17), 5)
        assert a.dtype == np.float32 and a.shape == (31, 17)
        np.testing.assert_array_equal(a, f((31, 17), 5))
        assert not np.array_equal(a, f((31, 17), 6))


def test_wide_range_exponents():
    a = workloads.wide((200_000,), 1)
    e = np.log2(np.abs(a.astype(np.float64)))
    assert e.min() >= -20.001 and e.max() <= 20.001
    assert abs(np.mean(e)) < 0.2 and abs((a < 0).mean() - 0.5) < 0.01


def test_cancellation_structure():
    A, B = workloads.cancellation(8, 4096, 3)
    assert A.shape == (8, 4096) and B.shape == (4096, 8)
    d = B + A.T
    assert np.abs(d).max() < 1e-3 and np.abs(d).std() > 5e-5


def test_batched_shapes():
    s = workloads.batched_shapes(4096, 0)
    assert s.shape == (4096, 3)
    assert set(np.unique(s)) <= set(range(32, 513, 16))
    assert len(np.unique(s)) == 31


def test_conditioned_system_kappa():
    A, b, xt = workloads.conditioned_system(64, 1e4, 2)
    sv = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    assert abs(sv[0] / sv[-1] / 1e4 - 1) < 1e-3
    np.testing.assert_allclose(b, A.astype(np.float64) @ xt)


def test_max_exp_range_and_finite_products():
    a = workloads.max_exp((256, 256), 3, K=256)
    e = np.floor(np.log2(np.abs(a.astype(np.float64))))
    assert e.min() == -58 and e.max() == 58
    assert abs((a < 0).mean() - 0.5) < 0.01
    np.testing.assert_array_equal(a, workloads.max_exp((256, 256), 3, K=256))
    p = np.abs(a.astype(np.float64)) @ np.abs(a.astype(np.float64))
    assert np.all(p < np.finfo(np.float32).max)

"""Persistent, graph-captured batched split GEMM (bfx_gemm_batched_plan_*):
every problem within the componentwise bound of its exact product and of the
oracle; identical to the one-launch-per-problem path; unchanged across graph
replays with eager work in between."""
import json
import os

import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import absref, dev, gemm_bound, host, ref64

pytestmark = pytest.mark.gpu


def _problems(count, seed, lo=32, hi=512):
    shapes, probs = workloads.batched_problems(count, seed, lo, hi)
    return shapes, probs


def _build(bfx, probs, beta=0.0):
    tens = []
    for (A, B) in probs:
        tA, tB = dev(A), dev(B)
        tC = torch.full((A.shape[0], B.shape[1]), 7.0, dtype=torch.float32, device="cuda")
        tens.append((tA, tB, tC, 1.0, beta))
    return tens


@pytest.mark.parametrize("variant", [3, 6, 9])
def test_batched_parity(bfx, orc, variant):
    shapes, probs = _problems(24, 11 + variant)
    tens = _build(bfx, probs)
    plan = bfx.BatchedGemmPlan(variant, tens)
    ntiles, nprob = plan.info()
    assert nprob == 24 and ntiles >= 24
    plan.launch()
    for (A, B), (_, _, tC, _, _) in zip(probs, tens):
        C = host(tC)
        bnd = gemm_bound(variant, A.shape[1]) * absref(A, B)
        assert np.all(np.abs(C - ref64(A, B)) <= bnd)
        Co = orc.gemm(variant, A, B)
        assert np.all(np.abs(C - Co) <= 2 * bnd)
    plan.close()


def test_batched_matches_per_problem_and_replays(bfx):
    """The per-problem path may split K (different summation order), so the two
    agree within twice the bound; graph replays are bit-identical."""
    shapes, probs = _problems(40, 5)
    tens = _build(bfx, probs)
    plan = bfx.BatchedGemmPlan(6, tens)
    plan.launch_per_problem()
    per = [host(t[2]).copy() for t in tens]
    plan.launch()
    ref = [host(t[2]).copy() for t in tens]
    for (A, B), a, b in zip(probs, per, ref):
        bnd = gemm_bound(6, A.shape[1]) * absref(A, B)
        assert np.all(np.abs(a - b) <= 2 * bnd)
        assert np.all(np.abs(b - ref64(A, B)) <= bnd)
    for rep in range(4):
        for t in tens:
            t[2].fill_(float("nan"))
        # eager work and a sync between replays
        _ = torch.randn(1000, device="cuda").sum().item()
        plan.launch()
        torch.cuda.synchronize()
        for r, t in zip(ref, tens):
            np.testing.assert_array_equal(host(t[2]), r)
    plan.close()


def test_batched_beta_and_ragged(bfx, orc):
    """beta = 1 accumulation, shapes not multiples of 16, empty problems; the
    plan mixes both engines (K % 4 == 0 goes to the wave-specialised one)."""
    g = np.random.default_rng(9)
    probs = []
    for (M, N, K) in [(33, 47, 19), (1, 1, 1), (130, 70, 257), (0, 5, 5), (64, 64, 0), (200, 300, 31),
                      (33, 47, 20), (130, 70, 256), (200, 300, 36), (1, 1, 4), (300, 270, 516)]:
        probs.append((workloads.normal((M, K), M + N), workloads.normal((K, N), K + 3)))
    tens = []
    C0s = []
    for (A, B) in probs:
        C0 = g.normal(size=(A.shape[0], B.shape[1])).astype(np.float32)
        C0s.append(C0)
        tens.append((dev(A), dev(B), dev(C0), -1.0, 1.0))
    plan = bfx.BatchedGemmPlan(6, tens)
    plan.launch()
    for (A, B), C0, t in zip(probs, C0s, tens):
        C = host(t[2])
        exact = C0.astype(np.float64) - ref64(A, B)
        bnd = gemm_bound(6, max(A.shape[1], 1)) * absref(A, B) + 2.0 ** -24 * np.abs(exact) + 1e-38
        assert np.all(np.abs(C - exact) <= bnd)
    plan.close()


def test_batched_tune_table(bfx, tmp_path):
    """A tuning table forcing each tile shape: the four general-engine shapes
    give identical results (same summation order inside a K-step), so do the
    two wave-specialised shapes; across engines the product order differs and
    the results agree within twice the bound."""
    shapes, probs = _problems(12, 21, 32, 300)
    outs = []
    for tile in range(6):
        table = {"arch": "gfx950", "variant": 6,
                 "entries": [{"m": m, "n": n, "tile": tile} for m in (64, 128, 256, 512)
                             for n in (64, 128, 256, 512)]}
        path = tmp_path / f"t{tile}.json"
        path.write_text(json.dumps(table))
        tens = _build(bfx, probs)
        plan = bfx.BatchedGemmPlan(6, tens, str(path))
        plan.launch()
        outs.append([host(t[2]).copy() for t in tens])
        plan.close()
    for k in (1, 2, 3):
        for a, b in zip(outs[0], outs[k]):
            np.testing.assert_array_equal(a, b)
    for a, b in zip(outs[4], outs[5]):
        np.testing.assert_array_equal(a, b)
    for (A, B), a, b in zip(probs, outs[0], outs[4]):
        bnd = gemm_bound(6, A.shape[1]) * absref(A, B)
        assert np.all(np.abs(b - ref64(A, B)) <= bnd)
        assert np.all(np.abs(a - b) <= 2 * bnd)


def test_batched_4096_workload_sampled(bfx, orc):
    """The 4096-problem workload: every output finite, a sample of problems
    checked entirely against the FP64 product and the oracle."""
    shapes, probs = _problems(4096, 0)
    tens = _build(bfx, probs)
    plan = bfx.BatchedGemmPlan(6, tens)
    plan.launch()
    torch.cuda.synchronize()
    idx = np.random.default_rng(1).choice(4096, 12, replace=False)
    for i in idx:
        A, B = probs[i]
        C = host(tens[i][2])
        bnd = gemm_bound(6, A.shape[1]) * absref(A, B)
        assert np.all(np.abs(C - ref64(A, B)) <= bnd)
    for t in tens:
        assert torch.isfinite(t[2]).all().item()
    plan.close()

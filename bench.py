#!/usr/bin/env python3
"""Benchmark of the split-BF16 GEMM / LU / IR library on one MI355X.

Timed step: one bf16x6 split GEMM C = A x B with M = N = K = 8192, FP32 in and
out, A and B iid N(0,1) already resident in HBM.  Every step splits both
operands into BF16 terms (one pass per operand) and runs the products; `value`
is FP32-equivalent throughput 2MNK / t in TFLOP/s over the whole step.  The
roofline object covers the dominant kernel (the products on the split
operands), timed on its own with HIP events.  The same run also reports, as extra fields:
the x3 and x9 variants, the plain FP32 vector-ALU GEMM comparator and torch's
FP32 matmul (library context), errors against an FP64 product on sampled
entries, the 64 x 64 x 2^20 split-K shape (GB/s), the 4096-problem batched
launch against one launch per problem, and LU + iterative refinement solves.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_TFLOPS = 2500.0     # MI355X dense BF16 MFMA
HBM_PEAK_GBS = 8000.0
PMC_RECORD = os.path.join(ROOT, "profiles", "gemm_planes_x6_8192_hbm_bytes.json")


def gemm_source_sha1():
    import hashlib
    d = os.path.join(ROOT, "paper_1904_06376_amd", "csrc")
    src = b"".join(open(os.path.join(d, n), "rb").read()
                   for n in ("common.hpp", "gemm_tile.hpp", "gemm.hip"))
    return hashlib.sha1(src).hexdigest()


def measured_traffic():
    """Per-launch HBM bytes of the x6 kernel from the committed counter record
    (FETCH_SIZE and WRITE_SIZE runs, scaled by a 1 GiB copy), or None when the
    GEMM sources changed since the counters were taken."""
    try:
        rec = json.load(open(PMC_RECORD))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha1") != gemm_source_sha1():
        return None
    return rec.get("traffic_bytes")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--skip-extras", action="store_true",
                    help="only the timed step, roofline and CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU oracle sample")
    ap.add_argument("--full-krylov", action="store_true",
                    help="also run GMRES-IR at n = 16384, kappa = 1e12 (a Krylov space of ~n, minutes)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for counter runs: one 1 GiB device-to-device copy (calibration "
                         "of the HBM byte counters) followed by one x6 GEMM, no timing")
    return ap.parse_args()


def time_launches(torch, fn, reps, stream):
    """Average duration of fn() over reps launches, with HIP events on `stream`."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for s, e in ev:
        s.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    ts = [s.elapsed_time(e) for s, e in ev]
    return float(np.mean(ts)), float(np.median(ts))


def sampled_errors(A, B, C, variant, nsample=256, seed=0):
    g = np.random.default_rng(seed)
    r = g.integers(0, A.shape[0], nsample)
    c = g.integers(0, B.shape[1], nsample)
    Ar = A[r].astype(np.float64)
    Bc = B[:, c].astype(np.float64)
    z = np.einsum("ij,ji->i", Ar, Bc)
    zh = np.einsum("ij,ji->i", np.abs(Ar), np.abs(Bc))
    K = A.shape[1]
    if variant >= 6:            # x6, x7, x8, x9: 2K 2^-24 |A||B|
        bnd = 2 * K * 2.0 ** -24
    elif variant == 3:
        bnd = 3 * 2.0 ** -16 + 2 * K * 2.0 ** -24
    else:                       # FP32 comparators (variant 0): gamma_K
        bnd = K * 2.0 ** -24
    got = C[r, c].astype(np.float64)
    ratio = np.abs(got - z) / (bnd * zh)
    rel = np.linalg.norm(got - z) / np.linalg.norm(z)
    return dict(max_err_over_bound=float(ratio.max()), rel_err_sample=float(rel),
                max_componentwise=float(np.max(np.abs(got - z) / zh)))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        sys.exit(2)

    import torch
    import paper_1904_06376_amd as bfx
    import workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    n = args.size
    if args.pmc_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)          # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del src, dst
        tA = torch.from_numpy(workloads.normal((n, n), 100)).to(dev)
        tB = torch.from_numpy(workloads.normal((n, n), 101)).to(dev)
        tC = torch.empty((n, n), dtype=torch.float32, device=dev)
        bfx.gemm(6, tA, tB, tC)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": "done", "copy_bytes": 1 << 30, "gemm": [n, n, n]}))
        return
    log(f"[bench] generating {n}x{n} N(0,1) operands")
    A = workloads.normal((n, n), 100)
    B = workloads.normal((n, n), 101)
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    tC = torch.empty((n, n), dtype=torch.float32, device=dev)
    flop = 2.0 * n * n * n

    ws_gemm = torch.empty(bfx.gemm_ws_size(9, n, n, n), dtype=torch.uint8, device=dev)

    def step(v=6):
        bfx.gemm(v, tA, tB, tC, ws=ws_gemm)

    # ---------------- timed region: K steps of the x6 GEMM ----------------
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = flop / (ms_per_step * 1e-3) / 1e12
    log(f"[bench] x6 {n}^3: {ms_per_step:.3f} ms/step, {value:.1f} TFLOP/s FP32-equivalent")

    # whole-call duration (split passes + products) with HIP events
    avg_ms, med_ms = time_launches(torch, step, max(args.steps, 5), stream)
    # dominant kernel alone (roofline): the products on operands split once
    Ab = bfx.split_blocks(tA, 3)
    Bb = bfx.split_blocks(tB, 3, trans=True)
    tG = torch.empty_like(tC)

    def products():
        bfx.gemm_blocks(6, n, n, n, Ab, Bb, tG)

    for _ in range(2):
        products()
    k_ms, _ = time_launches(torch, products, max(args.steps, 5), stream)
    torch.cuda.synchronize()
    assert torch.equal(tG, tC), "products on pre-split operands differ from the full call"
    sp_ms, _ = time_launches(torch, lambda: (bfx.split_blocks(tA, 3), bfx.split_blocks(tB, 3, trans=True)),
                             5, stream)
    del tG
    bf16_flop = 6 * flop
    achieved = bf16_flop / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(), "kernel": "gemm_planes_kernel<6>",
                "algorithmic_flop_per_launch": bf16_flop, "avg_launch_ms": round(k_ms, 4),
                "step_ms": round(avg_ms, 4), "step_minus_products_ms": round(avg_ms - k_ms, 4),
                "bfx_split_blocks_A_and_B_ms": round(sp_ms, 4)}

    C6 = tC.cpu().numpy()
    errors = {"x6": sampled_errors(A, B, C6, 6)}

    extras = {}
    if not args.skip_extras:
        # 256^3, U[-1,1]: split of all 131072 inputs against the oracle, and the
        # mean relative Frobenius error over 100 seeds per variant (Fig. 2 style)
        small = {}
        Ssplit = np.concatenate([workloads.uniform((256, 256), 0).ravel(),
                                 workloads.uniform((256, 256), 1).ravel()])
        planes = [x.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
                  for x in bfx.split(torch.from_numpy(Ssplit).to(dev), 3)]
        total = sum(pl.view(np.float32).astype(np.float64) for pl in planes)
        small["split_131072_sum_exact"] = bool(np.array_equal(total, Ssplit.astype(np.float64)))
        # (the mean relative Frobenius errors over 1000 seeds are in paper_figures)
        tS1 = torch.empty((256, 256), dtype=torch.float32, device=dev)
        tA1 = torch.from_numpy(workloads.uniform((256, 256), 0)).to(dev)
        tB1 = torch.from_numpy(workloads.uniform((256, 256), 1)).to(dev)
        us = {}
        for v in (3, 6, 9):
            ms, _ = time_launches(torch, lambda: bfx.gemm(v, tA1, tB1, tS1), 20, stream)
            us[f"x{v}"] = round(ms * 1e3, 1)
        small["launch_us"] = us
        extras["gemm_256"] = small
        log(f"[bench] 256^3 {small}")

        variants = {}
        for v in (3, 7, 8, 9):
            for _ in range(2):
                step(v)
            ms, _ = time_launches(torch, lambda: step(v), 5, stream)
            variants[f"x{v}"] = {"ms": round(ms, 3), "tflops_fp32eq": round(flop / ms / 1e9, 2),
                                 "tflops_bf16": round(v * flop / ms / 1e9, 2)}
            errors[f"x{v}"] = sampled_errors(A, B, tC.cpu().numpy(), v)
        variants["x6"] = {"ms": round(avg_ms, 3), "tflops_fp32eq": round(flop / avg_ms / 1e9, 2),
                          "tflops_bf16": round(6 * flop / avg_ms / 1e9, 2),
                          "products_kernel_ms": round(k_ms, 3)}
        # FP32 comparators
        tS = torch.empty_like(tC)
        bfx.sgemm_fp32(tA, tB, tS)
        ms_s, _ = time_launches(torch, lambda: bfx.sgemm_fp32(tA, tB, tS), 3, stream)
        errors["fp32_vector"] = sampled_errors(A, B, tS.cpu().numpy(), 0)
        torch.backends.cuda.matmul.allow_tf32 = False
        torch.matmul(tA, tB, out=tS)
        ms_t, _ = time_launches(torch, lambda: torch.matmul(tA, tB, out=tS), 5, stream)
        errors["torch_fp32"] = sampled_errors(A, B, tS.cpu().numpy(), 0)
        extras["variants"] = variants
        extras["fp32_vector_gemm"] = {"ms": round(ms_s, 3), "tflops": round(flop / ms_s / 1e9, 2)}
        extras["torch_fp32_matmul"] = {"ms": round(ms_t, 3), "tflops": round(flop / ms_t / 1e9, 2)}
        extras["speedup_x6_vs_fp32_vector"] = round(ms_s / avg_ms, 3)
        extras["speedup_x6_vs_torch_fp32"] = round(ms_t / avg_ms, 3)
        del tS
        log(f"[bench] variants {variants} fp32-vector {ms_s:.2f} ms torch-fp32 {ms_t:.2f} ms")

        # wide-range input set (2^u, u ~ U[-20,20])
        W1 = workloads.wide((n, n), 102)
        W2 = workloads.wide((n, n), 103)
        tW1 = torch.from_numpy(W1).to(dev)
        tW2 = torch.from_numpy(W2).to(dev)
        wide_err = {}
        for v in (3, 6, 9):
            bfx.gemm(v, tW1, tW2, tC)
            wide_err[f"x{v}"] = sampled_errors(W1, W2, tC.cpu().numpy(), v)
        torch.matmul(tW1, tW2, out=tC)
        wide_err["torch_fp32"] = sampled_errors(W1, W2, tC.cpu().numpy(), 0)
        extras["errors_wide"] = wide_err
        del tW1, tW2, W1, W2

        # split-K, 64 x 64 x 2^20
        K3 = 1 << 20
        X = torch.from_numpy(workloads.uniform((64, K3), 201)).to(dev)
        Y = torch.from_numpy(workloads.uniform((K3, 64), 202)).to(dev)
        Z = torch.empty((64, 64), dtype=torch.float32, device=dev)
        ws = torch.empty(max(bfx.gemm_ws_size(6, 64, 64, K3), 1), dtype=torch.uint8, device=dev)
        sk = {}
        for v in (3, 6, 9):
            bfx.gemm(v, X, Y, Z, ws=ws)
            ms, _ = time_launches(torch, lambda: bfx.gemm(v, X, Y, Z, ws=ws), 10, stream)
            sk[f"x{v}"] = {"us": round(ms * 1e3, 1),
                           "GBps": round(2 * 64 * K3 * 4 / (ms * 1e-3) / 1e9, 1)}
        bfx.sgemm_fp32(X, Y, Z)
        ms_s, _ = time_launches(torch, lambda: bfx.sgemm_fp32(X, Y, Z), 5, stream)
        sk["fp32_vector"] = {"us": round(ms_s * 1e3, 1),
                             "GBps": round(2 * 64 * K3 * 4 / (ms_s * 1e-3) / 1e9, 1)}
        # cancellation variant: errors against FP64, diagonal and off-diagonal apart
        Xc, Yc = workloads.cancellation(64, K3, 203)
        X.copy_(torch.from_numpy(Xc))
        Y.copy_(torch.from_numpy(Yc))
        z = Xc.astype(np.float64) @ Yc.astype(np.float64)
        zh = np.abs(Xc).astype(np.float64) @ np.abs(Yc).astype(np.float64)
        diag = np.eye(64, dtype=bool)
        canc = {}
        for v in (3, 6, 9, 0):
            if v:
                bfx.gemm(v, X, Y, Z, ws=ws)
            else:
                bfx.sgemm_fp32(X, Y, Z)
            got = Z.cpu().numpy().astype(np.float64)
            bnd = {3: 3 * 2.0 ** -16 + 2 * K3 * 2.0 ** -24, 6: 2 * K3 * 2.0 ** -24,
                   9: 2 * K3 * 2.0 ** -24, 0: K3 * 2.0 ** -24}[v]
            ratio = np.abs(got - z) / (bnd * zh)
            rel = np.abs(got - z) / np.abs(z)
            canc["fp32_vector" if v == 0 else f"x{v}"] = {
                "max_err_over_bound": float(ratio.max()),
                "max_rel_diag": float(rel[diag].max()),
                "median_rel_offdiag": float(np.median(rel[~diag])),
                "median_cancellation_offdiag": float(np.median(np.abs(z[~diag]) / zh[~diag]))}
        sk["cancellation"] = canc
        extras["splitk_64x64x1M"] = sk
        del X, Y, Z, ws, Xc, Yc
        log(f"[bench] split-K {sk}")

        # batched: 4096 uneven problems
        shapes, probs = workloads.batched_problems(4096, 0)
        tens = []
        for (a, b) in probs:
            tens.append((torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev),
                         torch.empty((a.shape[0], b.shape[1]), dtype=torch.float32, device=dev),
                         1.0, 0.0))
        tune = os.path.join(ROOT, "paper_1904_06376_amd", "tune", "gfx950_x6.json")
        plan = bfx.BatchedGemmPlan(6, tens, tune if os.path.exists(tune) else None)
        plan.launch()
        plan.launch_per_problem()
        torch.cuda.synchronize()
        ms_p, _ = time_launches(torch, plan.launch, 10, stream)
        ms_pp, _ = time_launches(torch, plan.launch_per_problem, 3, stream)
        bflop = float(sum(2.0 * M * N * K for M, N, K in shapes))
        extras["batched_4096"] = {"persistent_ms": round(ms_p, 3), "per_problem_ms": round(ms_pp, 3),
                                  "speedup": round(ms_pp / ms_p, 2),
                                  "tflops_fp32eq": round(bflop / ms_p / 1e9, 2),
                                  "tiles": plan.info()[0]}
        plan.close()
        del tens, probs
        log(f"[bench] batched {extras['batched_4096']}")

        # LU + IR solves
        try:
            extras["solves"] = bench_solves(torch, bfx, workloads, dev, stream, full_krylov=args.full_krylov)
        except Exception as e:  # report, do not hide
            extras["solves"] = {"error": repr(e)}
        log(f"[bench] solves {extras['solves']}")
        try:
            extras["batched_solves_512"] = bench_batched_solves(torch, bfx, workloads, dev, stream)
        except Exception as e:
            extras["batched_solves_512"] = {"error": repr(e)}
        log(f"[bench] batched solves {extras['batched_solves_512']}")
        try:
            extras["paper_figures"] = bench_paper_figures(torch, bfx, workloads, dev)
        except Exception as e:
            extras["paper_figures"] = {"error": repr(e)}
        log(f"[bench] paper figures {extras['paper_figures']}")
        try:
            extras["paper_tables"] = bench_paper_tables(torch, bfx, workloads, dev)
        except Exception as e:
            extras["paper_tables"] = {"error": repr(e)}
        log(f"[bench] paper tables {extras['paper_tables']}")

    # ---------------- CPU baseline: the oracle on a row sample ----------------
    import oracle as orc
    cores = orc.num_threads()
    # Each oracle call has a fixed part (splitting all of B) and a part
    # proportional to the rows of C: after a warm-up call, calibrate on 8 and
    # 40 rows and size the sample so that the timed call takes about
    # --cpu-seconds.
    def timed(r):
        t = time.perf_counter()
        orc.gemm(6, A[:r], B)
        return time.perf_counter() - t
    timed(2)
    ta, tb = timed(8), timed(40)
    per_row = max((tb - ta) / 32.0, 1e-3)
    fixed = max(ta - 8 * per_row, 0.0)
    rows2 = int(min(2048, max(8, (args.cpu_seconds - fixed) / per_row)))
    t0 = time.perf_counter()
    orc.gemm(6, A[:rows2], B)
    dt2 = time.perf_counter() - t0
    cpu_val = 2.0 * rows2 * n * n / dt2 / 1e12
    cpu = {"value": cpu_val, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
           "sample": f"bf16x6 oracle on {rows2} rows of C ({rows2}x{n}x{n}, full K), {dt2:.1f} s"}
    log(f"[bench] cpu oracle {cpu}")

    out = {
        "metric": "bf16x6 split-BF16 GEMM throughput (FP32-equivalent) at the paper's error bound",
        "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"split-BF16 GEMM {n}x{n}x{n}, FP32 operands N(0,1), "
                               "bf16x6 on MFMA with FP32 accumulation",
                   "variant": "bf16x6", "M": n, "N": n, "K": n, "parallelism": "single-gpu"},
        "roofline": roofline, "cpu_baseline": cpu, "errors": errors,
        "paper_projection": "up to 5.2x over FP32 for a 32x-density BF16 unit (projection, not a target)",
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def eta_check(torch, A, b, x):
    """Normwise backward error of x recomputed in FP64 from A (FP32, promoted
    exactly), b and x: |b - A x|_inf / (|A|_inf |x|_inf + |b|_inf)."""
    A64 = A.to(torch.float64)
    r = b - A64 @ x
    den = A64.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()
    return float((r.abs().max() / den).item())


def bench_solves(torch, bfx, workloads, dev, stream, n=16384, full_krylov=False):
    """One n x n system per kappa: LU (bf16x6 trailing updates) + LU-IR, and
    for kappa >= 1e8 GMRES-IR with a Krylov space large enough to converge
    (kappa = 1e12 needs about n GMRES steps: run at n = 16384 only with
    full_krylov, else at n = 4096).  eta is recomputed in FP64 from x."""
    res = {}
    # one warm-up factorisation: the first in a process also creates the
    # LU's streams and events and makes the first launches of its kernels
    W = torch.from_numpy(workloads.normal((2048, 2048), 6)).to(dev)
    bfx.lu_factor(W, 6)
    torch.cuda.synchronize()
    del W
    for kappa in (1e1, 1e4, 1e8, 1e12):
        t0 = time.perf_counter()
        A, b = workloads.conditioned_system_torch(n, kappa, 7, dev)
        log(f"[bench] generated n={n} kappa={kappa:g} system in {time.perf_counter() - t0:.1f}s")
        LU = A.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ipiv, info = bfx.lu_factor(LU, 6)
        torch.cuda.synchronize()
        t_lu = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, r = bfx.ir_solve(A, LU, ipiv, b)
        torch.cuda.synchronize()
        t_ir = time.perf_counter() - t0
        row = {"lu_ms": round(t_lu * 1e3, 2), "lu_tflops_fp32eq": round(2 / 3 * n ** 3 / t_lu / 1e12, 2),
               "info": int(info.item()),
               "lu_ir": {"ms": round(t_ir * 1e3, 2), "iters": r["iters"], "status": r["status"],
                         "eta": r["eta"], "eta_recomputed": eta_check(torch, A, b, x),
                         "solves_per_s": round(1.0 / (t_lu + t_ir), 3)}}
        del x
        if kappa >= 1e8 and (kappa < 1e12 or full_krylov):
            budget = dict(max_iter=3, restart=n if kappa >= 1e12 else 4096)
            log(f"[bench] n={n} kappa={kappa:g}: GMRES-IR {budget}")
            t0 = time.perf_counter()
            xg, g = bfx.gmres_ir_solve(A, LU, ipiv, b, **budget)
            torch.cuda.synchronize()
            t_g = time.perf_counter() - t0
            row["gmres_ir"] = {"ms": round(t_g * 1e3, 2), "iters": g["iters"], "inner": g["inner"],
                               "status": g["status"], "eta": g["eta"],
                               "eta_recomputed": eta_check(torch, A, b, xg), "budget": budget,
                               "ms_per_gmres_step": round(t_g * 1e3 / max(g["inner"], 1), 3),
                               "solves_per_s": round(1.0 / (t_lu + t_g), 4)}
            del xg
        res[f"n{n}_kappa{kappa:g}"] = row
        log(f"[bench] n={n} kappa={kappa:g}: {row}")
        del A, b, LU
        torch.cuda.empty_cache()
    if not full_krylov:
        # kappa = 1e12: GMRES-IR with a full Krylov space at n = 4096
        m = 4096
        A, b = workloads.conditioned_system_torch(m, 1e12, 7, dev)
        LU = A.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ipiv, info = bfx.lu_factor(LU, 6)
        torch.cuda.synchronize()
        t_lu = time.perf_counter() - t0
        budget = dict(max_iter=3, restart=m)
        t0 = time.perf_counter()
        xg, g = bfx.gmres_ir_solve(A, LU, ipiv, b, **budget)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t0
        res[f"n{m}_kappa1e+12"] = {
            "lu_ms": round(t_lu * 1e3, 2), "info": int(info.item()),
            "gmres_ir": {"ms": round(t_g * 1e3, 2), "iters": g["iters"], "inner": g["inner"],
                         "status": g["status"], "eta": g["eta"],
                         "eta_recomputed": eta_check(torch, A, b, xg), "budget": budget,
                         "ms_per_gmres_step": round(t_g * 1e3 / max(g["inner"], 1), 3),
                         "solves_per_s": round(1.0 / (t_lu + t_g), 4)}}
        log(f"[bench] n={m} kappa=1e12: {res[f'n{m}_kappa1e+12']}")
        del A, b, LU, xg
        torch.cuda.empty_cache()
    return res


def bench_batched_solves(torch, bfx, workloads, dev, stream, count=512):
    """512 systems, n uniform in [64, 1024], one persistent launch of LU + IR
    per kappa (GMRES-IR with a full Krylov space for the systems LU-IR leaves
    unconverged); one launch per problem timed on a 64-system subset at 1e4.
    eta is recomputed in FP64 from every x."""
    out = {}
    for kappa in (1e1, 1e4, 1e8, 1e12):
        t0 = time.perf_counter()
        systems, sizes = workloads.batch_systems_torch(count, kappa, 11, dev)
        log(f"[bench] generated {count} systems (n in [64,1024], kappa {kappa:g}) in "
            f"{time.perf_counter() - t0:.1f}s")
        probs = [(A, b, torch.empty(b.shape[0], dtype=torch.float64, device=dev)) for (A, b) in systems]
        plan = bfx.BatchedSolvePlan(6, probs)
        plan.launch()
        res = plan.results()
        ms, _ = time_launches(torch, plan.launch, 1 if kappa >= 1e12 else 3, stream)
        conv = sum(1 for r in res if r["status"] == 0)
        etas = [eta_check(torch, A, b, x) for (A, b, x) in probs]
        row = {"ms": round(ms, 3), "solves_per_s": round(count / (ms * 1e-3), 1),
               "converged": conv, "count": count,
               "max_eta": max(r["eta"] for r in res), "max_eta_recomputed": max(etas),
               "converged_recomputed": sum(1 for e in etas if e <= 1e-14),
               "mean_iters": round(float(np.mean([r["iters"] for r in res])), 2),
               "gmres_used": sum(1 for r in res if r["inner"] > 0),
               "mean_gmres_steps_when_used": round(float(np.mean([r["inner"] for r in res if r["inner"] > 0]
                                                                 or [0])), 1),
               "lu_flop_fp32eq": float(sum(2.0 / 3.0 * int(n) ** 3 for n in sizes))}
        plan.close()
        if kappa == 1e4:
            sub = probs[:64]
            plan2 = bfx.BatchedSolvePlan(6, sub)
            plan2.launch_per_problem()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan2.launch_per_problem()
            torch.cuda.synchronize()
            per = (time.perf_counter() - t0) / len(sub)
            plan2.close()
            row["per_problem_ms_each"] = round(per * 1e3, 3)
            row["per_problem_extrapolated_ms"] = round(per * 1e3 * count, 1)
            row["speedup_vs_per_problem"] = round(per * 1e3 * count / ms, 1)
        out[f"kappa{kappa:g}"] = row
        log(f"[bench] batched solves kappa={kappa:g}: {row}")
        del probs, systems
    return out


def bench_paper_figures(torch, bfx, workloads, dev, n=256, seeds=1000, lu_n=256, lu_runs=100):
    """The GEMM and LU accuracy experiments of Sec. IV-A on the GPU.
    Figs. 2-4: mean relative Frobenius error ||C - AB|| / ||AB|| against the
    FP64 product over `seeds` pairs of n x n operands (Fig. 2 uniform [-1,1],
    Fig. 3 maximal exponent range, Fig. 4 Gaussian exponents), for x3, x6, x6
    with the FP64 final sum ("d"), x9, the FP32 vector-ALU GEMM and torch's
    FP32 matmul.  Fig. 5: mean element error of the LU factors against the
    FP64 elimination with the same pivots, FP32-GEMM LU over x6 LU (> 1: x6
    more accurate), on [-1, 1] and [-1e10, 1e10]."""
    out = {}
    keys = ("x3", "x6", "x6d", "x9", "fp32_vector", "torch_fp32")
    tC = torch.empty((n, n), dtype=torch.float32, device=dev)
    torch.backends.cuda.matmul.allow_tf32 = False
    gens = (("fig2_uniform", lambda shape, sd: workloads.uniform(shape, sd)),
            ("fig3_max_exponent", lambda shape, sd: workloads.max_exp(shape, sd, K=n)),
            ("fig4_gauss_exponent", lambda shape, sd: workloads.gauss_exp(shape, sd)))
    for name, gen in gens:
        t0 = time.perf_counter()
        errs = torch.zeros((len(keys), seeds), dtype=torch.float64, device=dev)
        for sd in range(seeds):
            tA = torch.from_numpy(gen((n, n), 50000 + 2 * sd)).to(dev)
            tB = torch.from_numpy(gen((n, n), 50001 + 2 * sd)).to(dev)
            Z = tA.double() @ tB.double()
            zn = torch.linalg.norm(Z)
            for k, key in enumerate(keys):
                if key == "fp32_vector":
                    bfx.sgemm_fp32(tA, tB, tC)
                elif key == "torch_fp32":
                    torch.matmul(tA, tB, out=tC)
                else:
                    bfx.gemm(int(key[1]), tA, tB, tC, fp64_sum=key.endswith("d"))
                errs[k, sd] = torch.linalg.norm(tC.double() - Z) / zn
        m = errs.mean(dim=1).cpu().numpy()
        out[name] = {key: float(v) for key, v in zip(keys, m)}
        out[name]["seeds"] = seeds
        log(f"[bench] {name}: {out[name]} ({time.perf_counter() - t0:.1f}s)")

    def lu64_same_pivots(A, piv):
        p = np.arange(lu_n)
        for i, q in enumerate(piv):
            p[[i, q]] = p[[q, i]]
        M = A.double()[torch.from_numpy(p).to(dev)]
        for c in range(lu_n - 1):
            M[c + 1:, c] /= M[c, c]
            M[c + 1:, c + 1:] -= torch.outer(M[c + 1:, c], M[c, c + 1:])
        return M

    fig5 = {}
    for scale in (1.0, 1e10):
        ratios = []
        for r in range(lu_runs):
            A = torch.from_numpy(workloads.uniform((lu_n, lu_n), 60000 + r) * np.float32(scale)).to(dev)
            errs = []
            for v in (6, 0):
                LU = A.clone()
                _, ipiv, _ = bfx.lu_factor(LU, v)
                ref = lu64_same_pivots(A, ipiv.cpu().numpy())
                errs.append(float((LU.double() - ref).abs().mean().item()))
            ratios.append(errs[1] / errs[0])
        fig5[f"range_{scale:g}"] = {"mean_improvement": float(np.mean(ratios)),
                                    "min_improvement": float(np.min(ratios)), "runs": lu_runs, "n": lu_n}
    out["fig5_lu_fp32gemm_over_x6"] = fig5
    return out


def bench_paper_tables(torch, bfx, workloads, dev, count=100):
    """The Sec. IV-B tables on the GPU, `count` systems per row, with the
    split-BF16 LU (the FP32-accurate row) and single-format BF16 and FP16 LUs.
    IR table: n = 50, kappa 10 .. 1e4, LU-IR (max 100 steps).  GMRES table:
    diagonally dominant n = 10, 50, 100, GMRES-IR.  % converged to eta <=
    1e-14 and mean refinement steps (and GMRES steps) of the converged."""
    fmts = {"fp32_split": 0, "bf16": 1, "fp16": 2}
    ir = {}
    for kappa in (1e1, 1e2, 1e3, 1e4):
        systems = [workloads.conditioned_system(50, kappa, 70000 + s) for s in range(count)]
        row = {}
        for fname, f in fmts.items():
            probs = [(torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev),
                      torch.empty(50, dtype=torch.float64, device=dev)) for (A, b, _) in systems]
            plan = bfx.BatchedSolvePlan(6, probs, lu_format=f, max_iter=100, gmres_max_iter=0)
            plan.launch()
            res = plan.results()
            plan.close()
            conv = [r for r in res if r["status"] == 0]
            row[fname] = {"converged_pct": 100.0 * len(conv) / count,
                          "mean_iters": round(float(np.mean([r["iters"] for r in conv])), 2) if conv else None}
        ir[f"kappa{kappa:g}"] = row
    gm = {}
    for n in (10, 50, 100):
        systems = []
        for s in range(count):
            g = np.random.default_rng(80000 + 17 * n + s)
            A = g.uniform(-1, 1, (n, n))
            d = np.maximum(np.abs(A).sum(0), np.abs(A).sum(1)) + 1.0
            A = (A + np.diag(d * np.sign(g.uniform(-1, 1, n)))).astype(np.float32)
            systems.append((A, A.astype(np.float64) @ g.normal(size=n)))
        row = {}
        for fname, f in fmts.items():
            probs = [(torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev),
                      torch.empty(n, dtype=torch.float64, device=dev)) for (A, b) in systems]
            plan = bfx.BatchedSolvePlan(6, probs, lu_format=f, mode=1)
            plan.launch()
            res = plan.results()
            plan.close()
            conv = [r for r in res if r["status"] == 0]
            row[fname] = {"converged_pct": 100.0 * len(conv) / count,
                          "mean_iters": round(float(np.mean([r["iters"] for r in conv])), 2) if conv else None,
                          "mean_gmres_steps": round(float(np.mean([r["inner"] for r in conv])), 2) if conv else None}
        gm[f"n{n}"] = row
    return {"ir_table_n50": ir, "gmres_table_diag_dominant": gm}


if __name__ == "__main__":
    main()

"""Run one library workload a few times (for profilers such as rocprofv3).

    python paper_1904_06376_amd/run_workload.py gemm   --n 8192 --variant 6 --reps 5
    python paper_1904_06376_amd/run_workload.py splitk --variant 6 --reps 10
    python paper_1904_06376_amd/run_workload.py lu     --n 16384 --kappa 1e4
    python paper_1904_06376_amd/run_workload.py lu     --n 16384 --plain --reps 3
    python paper_1904_06376_amd/run_workload.py batched-gemm --count 4096 --reps 3
    python paper_1904_06376_amd/run_workload.py batched-solve --count 512 --reps 2
    python paper_1904_06376_amd/run_workload.py lu-update --n 16384 --reps 5
    python paper_1904_06376_amd/run_workload.py save-system --n 16384 --kappa 1e8 --out /tmp/s16k
    python paper_1904_06376_amd/run_workload.py refine --src /tmp/s16k --solver gmres --restart 200 --max-iter 1

save-system generates a conditioned system, factors it and writes A, the
factors, the pivots and b to <out>_A.npy, <out>_LU.npy, <out>_ipiv.npy and
<out>_b.npy; refine loads them and runs only the refinement (LU-IR or
GMRES-IR), so that a profiler sees the refinement kernels alone.

Inputs are the seeded synthetic workloads of the benchmark; nothing is timed
here except a one-line summary printed at the end.
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["gemm", "splitk", "lu", "batched-gemm", "batched-solve",
                                            "lu-update", "save-system", "refine"])
    ap.add_argument("--out", default="/tmp/bfx_system")
    ap.add_argument("--src", default="/tmp/bfx_system")
    ap.add_argument("--solver", choices=["ir", "gmres"], default="gmres")
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--max-iter", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--variant", type=int, default=6)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--kappa", type=float, default=1e4)
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--plain", action="store_true", help="lu: factor a seeded normal matrix, no refinement")
    a = ap.parse_args()

    import torch
    import paper_1904_06376_amd as bfx
    import workloads

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    if a.workload == "gemm":
        A = torch.from_numpy(workloads.normal((a.n, a.n), 100)).to(dev)
        B = torch.from_numpy(workloads.normal((a.n, a.n), 101)).to(dev)
        C = torch.empty_like(A)
        for _ in range(a.reps):
            bfx.gemm(a.variant, A, B, C)
    elif a.workload == "splitk":
        K = 1 << 20
        X = torch.from_numpy(workloads.uniform((64, K), 201)).to(dev)
        Y = torch.from_numpy(workloads.uniform((K, 64), 202)).to(dev)
        Z = torch.empty((64, 64), dtype=torch.float32, device=dev)
        for _ in range(a.reps):
            bfx.gemm(a.variant, X, Y, Z)
    elif a.workload == "lu" and a.plain:
        # factorisation only, of a seeded normal matrix (no QR-built system)
        A = torch.from_numpy(workloads.normal((a.n, a.n), 7)).to(dev)
        for _ in range(a.reps):
            LU = A.clone()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, ipiv, info = bfx.lu_factor(LU, a.variant)
            torch.cuda.synchronize()
            print(f"lu {1e3 * (time.perf_counter() - t1):.1f} ms, info {int(info.item())}", flush=True)
    elif a.workload == "lu":
        A, b = workloads.conditioned_system_torch(a.n, a.kappa, 7, dev)
        for _ in range(a.reps):
            LU = A.clone()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, ipiv, info = bfx.lu_factor(LU, a.variant)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            x, res = bfx.ir_solve(A, LU, ipiv, b)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            print(f"lu {1e3 * (t2 - t1):.1f} ms, ir {1e3 * (t3 - t2):.1f} ms, {res}", flush=True)
    elif a.workload == "save-system":
        import numpy as np
        A, b = workloads.conditioned_system_torch(a.n, a.kappa, 7, dev)
        LU = A.clone()
        _, ipiv, info = bfx.lu_factor(LU, a.variant)
        torch.cuda.synchronize()
        for name, t in (("A", A), ("LU", LU), ("ipiv", ipiv), ("b", b)):
            np.save(f"{a.out}_{name}.npy", t.cpu().numpy())
        print(f"saved n={a.n} kappa={a.kappa:g} info={int(info.item())} to {a.out}_*.npy", flush=True)
    elif a.workload == "refine":
        import numpy as np
        A, LU, ipiv, b = (torch.from_numpy(np.load(f"{a.src}_{name}.npy")).to(dev)
                          for name in ("A", "LU", "ipiv", "b"))
        for _ in range(a.reps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if a.solver == "ir":
                x, res = bfx.ir_solve(A, LU, ipiv, b, max_iter=a.max_iter)
            else:
                x, res = bfx.gmres_ir_solve(A, LU, ipiv, b, restart=a.restart, max_iter=a.max_iter)
            torch.cuda.synchronize()
            print(f"{a.solver} {1e3 * (time.perf_counter() - t1):.1f} ms, {res}", flush=True)
    elif a.workload == "lu-update":
        # the first trailing update of an n x n LU: A22 -= L21 x U12, K = 128,
        # all three operands strided views of one n x n matrix
        M = torch.from_numpy(workloads.normal((a.n, a.n), 102)).to(dev)
        L21, U12, A22 = M[128:, :128], M[:128, 128:], M[128:, 128:]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * a.reps)]
        for r in range(a.reps):
            ev[2 * r].record()
            bfx.gemm(a.variant, L21, U12, A22, alpha=-1.0, beta=1.0)
            ev[2 * r + 1].record()
        torch.cuda.synchronize()
        ms = [ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(a.reps)]
        m = a.n - 128
        print(f"lu-update {m}x{m}x128: " + " ".join(f"{x:.3f}" for x in ms) + " ms; "
              f"{a.variant * 2.0 * m * m * 128 / (min(ms) * 1e-3) / 1e12:.0f} TFLOP/s BF16, "
              f"{8.0 * m * m / (min(ms) * 1e-3) / 1e9:.0f} GB/s of C", flush=True)
    elif a.workload == "batched-gemm":
        shapes, probs = workloads.batched_problems(a.count, 0)
        tens = [(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev),
                 torch.empty((x.shape[0], y.shape[1]), dtype=torch.float32, device=dev), 1.0, 0.0)
                for (x, y) in probs]
        plan = bfx.BatchedGemmPlan(a.variant, tens)
        for _ in range(a.reps):
            plan.launch()
        plan.close()
    else:
        systems, sizes = workloads.batch_systems_torch(a.count, a.kappa, 11, dev)
        probs = [(A, b, torch.empty(b.shape[0], dtype=torch.float64, device=dev))
                 for (A, b) in systems]
        plan = bfx.BatchedSolvePlan(a.variant, probs)
        for _ in range(a.reps):
            plan.launch()
        plan.results()
        plan.close()
    torch.cuda.synchronize()
    print(f"{a.workload}: done in {time.perf_counter() - t0:.2f} s", flush=True)


if __name__ == "__main__":
    main()

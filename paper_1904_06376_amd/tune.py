"""Autotuner for the batched split-GEMM tile shapes.

For every (M, N) bucket (upper bounds 64, 128, 256, 512) it builds a batch of
problems whose M and N are drawn from that bucket (K from the whole range),
runs the persistent plan once per candidate tile shape (forced through a
one-shape tuning table), times the graph launches with HIP events, and writes
the fastest shape per bucket to a JSON table that
`bfx_gemm_batched_plan_create` reads:

    {"arch": "gfx950", "variant": 6,
     "entries": [{"m": 64, "n": 128, "tile": 2, "ms": {...}}, ...]}

Usage: python -m paper_1904_06376_amd.tune --variant 6 --out <path>
"""
import argparse
import json
import os
import sys
import tempfile

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

# 0-3: general engine (256 threads); 4-5: wave-specialised engine (512 threads)
TILES = {0: "64x64", 1: "128x128", 2: "128x64", 3: "64x128", 4: "ws64x64", 5: "ws128x128"}
EDGES = [(32, 64), (80, 128), (144, 256), (272, 512)]


def _time(fn, reps=10):
    fn()
    torch.cuda.synchronize()
    s = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    e = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
    for i in range(reps):
        s[i].record()
        fn()
        e[i].record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in zip(s, e)]))


def tune(variant=6, count=256, seed=0, out=None, log=print):
    import paper_1904_06376_amd as bfx
    g = np.random.default_rng(seed)
    entries = []
    with tempfile.TemporaryDirectory() as td:
        for bm, (mlo, mhi) in enumerate(EDGES):
            for bn, (nlo, nhi) in enumerate(EDGES):
                Ms = g.choice(np.arange(mlo, mhi + 1, 16), count)
                Ns = g.choice(np.arange(nlo, nhi + 1, 16), count)
                Ks = g.choice(np.arange(32, 513, 16), count)
                probs = []
                for M, N, K in zip(Ms, Ns, Ks):
                    A = torch.randn(int(M), int(K), device="cuda")
                    B = torch.randn(int(K), int(N), device="cuda")
                    C = torch.empty(int(M), int(N), device="cuda")
                    probs.append((A, B, C, 1.0, 0.0))
                times = {}
                for tile in TILES:
                    path = os.path.join(td, f"t{tile}.json")
                    with open(path, "w") as f:
                        json.dump({"arch": "gfx950", "variant": variant,
                                   "entries": [{"m": EDGES[bm][1], "n": EDGES[bn][1],
                                                "tile": tile}]}, f)
                    plan = bfx.BatchedGemmPlan(variant, probs, path)
                    times[TILES[tile]] = _time(plan.launch)
                    plan.close()
                best = min(TILES, key=lambda t: times[TILES[t]])
                entries.append({"m": EDGES[bm][1], "n": EDGES[bn][1], "tile": best,
                                "ms": {k: round(v, 4) for k, v in times.items()}})
                log(f"bucket m<={EDGES[bm][1]} n<={EDGES[bn][1]}: best {TILES[best]} {times}")
    table = {"arch": "gfx950", "variant": variant, "count_per_bucket": count,
             "tiles": TILES, "entries": entries}
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        with open(out, "w") as f:
            json.dump(table, f, indent=1)
    return table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--variant", type=int, default=6)
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--out", default=os.path.join(HERE, "tune", "gfx950_x6.json"))
    a = ap.parse_args()
    tune(a.variant, a.count, out=a.out)

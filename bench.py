"""Benchmark: walk steps/s of the MLMC solve of x = exp(tA) v on one MI355X.

Workload (one "step" of this benchmark = one complete MLMC solve, Algorithm 1 to a
target RMSE, through the C-ABI): the 2D 5-point Dirichlet Laplacian on a 256 x 256 grid
(n = 65536), t = h^2/2 so that ||tA||_1 = 4, v ~ N(0, 1) (seeded), full vector, FP32
path weights with compensated FP32 row sums and an FP64 level combine, levels from
l0 = 2 (six levels at the default target). Inputs are resident in HBM before timing.

Prints one JSON line with the metric, a roofline entry for the walk kernel and the
oracle's CPU throughput on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU work of the walk kernel, in lane-instructions of a minimal gfx950
# implementation: a step consumes one 32-bit Philox word (a Philox4x32-10 block is 10
# rounds of 2 32x32->64 multiplies and 2 three-input xors, so 10 instructions per word)
# plus its threshold compare; a jump draws one block for slot, coin and holding time
# (40), evaluates two FP64 logarithms (about 40 each, division included), gathers and
# selects the alias entry and updates the weights (about 30); a walk evaluates exp and
# expm1 of its weights and adds to the compensated sums (about 50).
OPS_PER_STEP = 11
OPS_PER_JUMP = 150
OPS_PER_WALK = 50
# MI355X vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# bytes the jumps must gather: one 16-byte alias slot and one 32-byte row record
BYTES_PER_JUMP = 48


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--pilot", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(A, t, v, l0, walks, target_s):
    """The oracle (plain FP64 C, OpenMP over rows) on a bounded sample of the same
    workload: a random subset of rows with the solve's sample sizes scaled down so that
    the run takes about target_s seconds. Returns walk steps per second."""
    import numpy as np

    from oracle import mlmc as orc

    tables = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    threads = orc.max_threads()
    rng = np.random.default_rng(5)
    # calibration on a small slice
    rows = rng.choice(A.n, size=256, replace=False)
    t0 = time.perf_counter()
    orc.level_sums(tables, t, l0, l0, 1, v, rows, 0, 256)
    cal = time.perf_counter() - t0
    speed = 256 * 256 * (1 << l0) / max(cal, 1e-6)
    steps_full = sum(w * (1 << (l0 + q)) for q, w in enumerate(walks)) * A.n
    frac = min(1.0, target_s * speed / steps_full)
    n_rows = max(64, min(A.n, int(A.n * math.sqrt(frac))))
    scale = min(1.0, frac * A.n / n_rows)
    rows = np.sort(rng.choice(A.n, size=n_rows, replace=False))
    Ms = [max(1, int(round(w * scale))) for w in walks]
    steps = 0
    t0 = time.perf_counter()
    for q, M in enumerate(Ms):
        orc.level_sums(tables, t, l0 + q, l0, 1, v, rows, 0, M)
        steps += n_rows * M * (1 << (l0 + q))
    el = time.perf_counter() - t0
    return {"value": steps / el, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_rows} of {A.n} rows, walks per level {Ms} (the solve's sample "
                      f"sizes x {scale:.2e}), levels {l0}..{l0 + len(Ms) - 1}, FP64, "
                      f"{steps:.3e} steps in {el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the walk kernel is "
                                   "measured at one GPU's share of the work (--gpus 1)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1904_12754_amd import api, exact, inputs

    dev = torch.device("cuda:0")
    A, t, v = inputs.workload_laplace2d(args.grid)
    x_exact = exact.expv_laplace2d(v, t)
    u = torch.as_tensor(v.astype(np.float32), device=dev)
    plan = api.Plan(A, t, precision="fp32")
    stream = torch.cuda.current_stream()

    def solve(seed):
        return plan.run(u, eps=args.eps, seed=seed, pilot_walks=args.pilot, max_levels=12)

    for w in range(args.warmup):
        solve(10_000 + w)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, st = solve(20_000 + k)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stream.synchronize()

    steps = sum(s["steps"] for s in stats)
    jumps = sum(s["total_jumps"] for s in stats)
    walks_total = sum(sum(s["walks"]) * plan.n_rows for s in stats)
    wk_ms = sum(s["walk_kernel_ms"] for s in stats)
    launches = sum(s["walk_launches"] for s in stats)
    last = stats[-1]
    xg = x.cpu().numpy()[:, 0]
    true_rmse = float(np.sqrt(np.mean((xg - x_exact) ** 2)))

    ops = OPS_PER_STEP * steps + OPS_PER_JUMP * jumps + OPS_PER_WALK * walks_total
    achieved = ops / (wk_ms * 1e-3)
    roofline = {
        "bound": "alu",
        "kernel": "level_walks_r1<float,float>",
        "achieved": achieved / 1e12,
        "peak": VALU_PEAK_LANE_OPS / 1e12,
        "unit": "T lane-ops/s",
        "frac": achieved / VALU_PEAK_LANE_OPS,
        "traffic": None,
        "per_unit": {"ops_per_step": OPS_PER_STEP, "ops_per_jump": OPS_PER_JUMP,
                     "ops_per_walk": OPS_PER_WALK},
        "launch_avg_ms": wk_ms / max(launches, 1),
        "launches": launches,
        "gathered_GBps": BYTES_PER_JUMP * jumps / (wk_ms * 1e-3) / 1e9,
    }
    line = {
        "metric": "walk steps/s",
        "value": steps / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"2D 5-point Dirichlet Laplacian {args.grid}x{args.grid} (n={A.n}), "
                        f"t=h^2/2 (||tA||_1=4), v~N(0,1); adaptive MLMC (Algorithm 1) to "
                        f"RMSE {args.eps:g}; FP32 weights, Kahan FP32 row sums, FP64 combine",
            "n": A.n, "eps": args.eps, "l0": last["l0"], "levels": last["num_levels"],
            "walks_per_row_per_level": last["walks"],
            "time_to_rmse_s": elapsed / args.steps,
            "true_rmse_vs_exact": true_rmse,
            "est_rmse": math.sqrt(last["est_variance"] + last["est_bias"] ** 2),
            "jumps_per_s": jumps / elapsed,
            "walk_kernel_share": wk_ms * 1e-3 / elapsed,
            "path_decisions": "fp64 + u32 (bit-identical to the FP64 oracle)",
        },
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A, t, v, last["l0"], last["walks"], args.cpu_seconds)
    print(json.dumps(line), flush=True)
    plan.close()


if __name__ == "__main__":
    main()

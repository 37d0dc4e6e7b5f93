"""Benchmark: walk steps/s and time-to-RMSE of the MLMC solve of x = exp(tA) v on one MI355X.

Headline workload (one "step" of this benchmark = one complete MLMC solve, Algorithm 1 to a
target RMSE, through the C-ABI): the 2D 5-point Dirichlet Laplacian on a 256 x 256 grid
(n = 65536), t = h^2/2 so that ||tA||_1 = 4, v ~ N(0, 1) (seeded), full vector, FP32
path weights with compensated FP32 row sums and an FP64 level combine, levels from
l0 = 2. Inputs are resident in HBM before timing.

The same run also measures the other four workloads (outside the timed region): the FP64
1D Laplacian against the dense exponential, the Barabasi-Albert graph with 64 right-hand
sides, the batch of 512 uneven instances, and the learned proposal against the plain jump
law on the 3D convection-diffusion operator; every result states its true error against
an FP64 reference (bench_reference.py). Machine probes (random 16-byte gathers at several
table sizes, integer VALU issue) calibrate the rooflines.

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

# Minimal VALU work of the walks, in lane-instructions of a gfx950 sequence: a step consumes
# a quarter of a Philox4x32-10 block (10 rounds of two v_mad_u64_u32 and two v_bitop3_b32
# three-input xors: 40 per block, 10 per step) and one compare; a jump consumes one block
# (40), the alias selection and gather addressing (~8), the holding-time bracket (~8) and the
# run update of the weights (~9); a walk end scales and exponentiates its exponent and
# applies the sign (3), gathers u and multiplies (2), adds to the two compensated sums (9)
# and to the counters (3), plus an expm1 (~23) above the base level; with several
# right-hand sides a walk that moved adds one product and two compensated sums per
# right-hand side (10). The random draws are part of the method's cost (the per-step term
# of the cost model of section 4), so the generator counts as work.
OPS_PER_STEP = 11
OPS_PER_JUMP = 65
OPS_PER_WALK_BASE = 17
OPS_PER_WALK_ABOVE = 40
OPS_PER_RHS_SAMPLE = 10
# MI355X integer VALU: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz (a wave64
# instruction issues over four cycles; the FP32 vector figure of 157.3 TFLOP/s counts two
# flops per FMA and dual-issue, which 32-bit integer instructions do not have)
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# MI355X HBM3E peak bandwidth
HBM_PEAK_BPS = 8.0e12
# Algorithmic bytes: a jump gathers its 16-byte alias slot and the 24-byte record of the row
# it lands on (the layout here pads that record to 32 bytes); a walk end reads R values of
# u (4 bytes each; a walk that never jumped ends at its start row, whose u row is read once
# per row and level); each (row, level, right-hand side) writes two FP64 sums.
BYTES_PER_JUMP = 40
# HBM traffic of the walk kernel from the FETCH_SIZE / WRITE_SIZE counters (calibrated on a
# plain copy), recorded with the hash of the kernel source it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_kernel_traffic.json")
# the walk kernel's sources and the build script that holds its compiler flags
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1904_12754_amd", "csrc", f)
                  for f in ("kernels.hip", "walk_engine.h", "common.h", "kernels.h")] + [
                      os.path.join(ROOT, "paper_1904_12754_amd", "build.py")]


def kernel_sources_sha256() -> str:
    """Hash of the sources the walk kernel is compiled from and of its build flags."""
    import hashlib

    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_traffic(launches_walks):
    """Calibrated HBM bytes per walk-kernel launch, or None when the counters were taken on
    another version of the kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        sha = kernel_sources_sha256()
    except OSError:
        return None
    if rec.get("kernel_sha256") != sha:
        return None
    return rec["bytes_per_walk"] * launches_walks


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--pilot", type=int, default=0,
                    help="Algorithm 1's M0 (0: the library's rule, 2^18 samples per level)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--cd-grid", type=int, default=128)
    ap.add_argument("--cd-pilot", type=int, default=0)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-loose", action="store_true",
                    help="skip the solves to RMSE 1e-2 after the timed region")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the 1D Laplacian, Barabasi-Albert and batch workloads")
    ap.add_argument("--mode", choices=["bench", "kernel", "copy", "batch", "tc", "learned",
                                       "classical", "config1", "probe"],
                    default="bench",
                    help="kernel: only the dominant walk-kernel launch (level l0 + --level, "
                         "--walks per row), for counter runs; copy: a plain device copy of "
                         "--bytes, the calibration for the traffic counters; probe: the "
                         "machine probes alone")
    ap.add_argument("--profile-run", action="store_true",
                    help="batch, tc and learned modes under a counter profiler: only the "
                         "workload itself (no one-run-per-instance comparison, no small-"
                         "instance batch, no machine probes, no CPU reference)")
    ap.add_argument("--level", type=int, default=0)
    ap.add_argument("--walks", type=int, default=65536)
    ap.add_argument("--bytes", type=int, default=1 << 30)
    return ap.parse_args()


# ---- machine probes and rooflines -------------------------------------------------------
PROBE_LOG2 = (18, 19, 21, 23, 25, 28)      # 4 MB .. 4 GB tables of 16-byte records
LDS_PROBE_LOG2 = 11                         # 32 KB: four workgroups' copies fit in a CU's LDS


def machine_probes():
    """Integer VALU issue rate and uniformly random 16-byte gather rates by table size."""
    import torch

    from paper_1904_12754_amd import api

    n, s = api.probe_valu(32, 8192)
    out = {"valu_lane_ops_per_s": n / s, "gather_per_s": {}}
    table = torch.zeros((16 << max(PROBE_LOG2)) // 4, dtype=torch.int32, device="cuda")
    for lg in PROBE_LOG2:
        g, s = api.probe_gather(table, lg, 32, 64 if lg <= 21 else 32)
        out["gather_per_s"][str(16 << lg)] = g / s
    # what staging rows' tables in LDS could gain per gather: a 32 KB table gathered from
    # LDS and from device memory (where the caches hold it), as rates (8 streams per lane)
    # and as the latency of serial gathers (one dependent stream per lane; 16 waves per CU
    # keep 16 x 64 gathers in flight per CU)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    lds = {"table_bytes": 16 << LDS_PROBE_LOG2, "waves_per_cu": 16}
    for where in ("global", "lds"):
        g, s = api.probe_gather(table, LDS_PROBE_LOG2, 16, 256, lds=where == "lds")
        lds[f"{where}_gathers_per_s"] = g / s
        g, s = api.probe_gather(table, LDS_PROBE_LOG2, 16, 256, lds=where == "lds", dependent=True)
        lds[f"{where}_latency_ns"] = 16 * 64 * cus / (g / s) * 1e9
    out["lds_vs_global"] = lds
    del table
    torch.cuda.empty_cache()
    return out


def probe_rate_for(probes, ws_bytes):
    """The probe's gather rate at the smallest measured table holding ws_bytes."""
    sizes = sorted(int(k) for k in probes["gather_per_s"])
    size = next((z for z in sizes if z >= ws_bytes), sizes[-1])
    return size, probes["gather_per_s"][str(size)]


def walk_roofline(kernel, seconds, launches, steps, jumps, walks_base, walks_above, rows_levels,
                  nrhs, ws_bytes, probes, traffic=None):
    """Rooflines of one walk kernel over `seconds` of its launches (summed event-pair
    durations): VALU issue (the binding one for these workloads), and the algorithmic bytes
    and gathers against the HBM peak and the probe's gather rate at the working-set size."""
    walks = walks_base + walks_above
    moved = min(walks, jumps) if nrhs > 1 else walks
    ops = (OPS_PER_STEP * steps + OPS_PER_JUMP * jumps + OPS_PER_WALK_BASE * walks_base +
           OPS_PER_WALK_ABOVE * walks_above + (OPS_PER_RHS_SAMPLE * nrhs * moved if nrhs > 1 else 0))
    nbytes = BYTES_PER_JUMP * jumps + 4 * nrhs * moved + (4 + 16) * nrhs * rows_levels
    gathers = 2 * jumps + moved
    size, prate = probe_rate_for(probes, ws_bytes)
    achieved = ops / seconds
    return {
        "bound": "alu", "kernel": kernel,
        "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
        "frac": achieved / VALU_PEAK_LANE_OPS, "traffic": traffic,
        "peak_measured_probe": probes["valu_lane_ops_per_s"] / 1e12,
        "frac_of_measured_peak": achieved / probes["valu_lane_ops_per_s"],
        "launch_avg_ms": seconds / max(launches, 1) * 1e3, "launches": launches,
        "per_unit": {"ops_per_step": OPS_PER_STEP, "ops_per_jump": OPS_PER_JUMP,
                     "ops_per_walk_base": OPS_PER_WALK_BASE, "ops_per_walk_above": OPS_PER_WALK_ABOVE,
                     "ops_per_rhs_sample": OPS_PER_RHS_SAMPLE, "bytes_per_jump": BYTES_PER_JUMP,
                     "bytes_per_walk_end": 4 * nrhs},
        "memory": {
            # the algorithmic bytes over the HBM peak; the caches serve most of them, and the
            # HBM traffic the counters measured is hbm_GBps_from_counters
            "algorithmic_GBps": nbytes / seconds / 1e9,
            "algorithmic_over_hbm_peak": nbytes / seconds / HBM_PEAK_BPS,
            "hbm_GBps_from_counters": (traffic * launches / seconds / 1e9
                                       if traffic is not None else None),
            "working_set_MB": ws_bytes / 2 ** 20,
            "gathers_per_s": gathers / seconds,
            "probe_table_MB": size / 2 ** 20,
            "probe_gathers_per_s": prate,
            "frac_of_probe_gather_rate": gathers / seconds / prate,
        },
    }


def kernel_sums(stats_list):
    """Summed walk-kernel time, launches, steps, jumps, base-level and other walks."""
    out = {"ms": 0.0, "launches": 0, "steps": 0, "jumps": 0, "walks_base": 0, "walks_above": 0}
    for st, n_rows in stats_list:
        out["ms"] += st["walk_kernel_ms"]
        out["launches"] += st["walk_launches"]
        out["steps"] += st["steps"]
        out["jumps"] += st["total_jumps"]
        out["walks_base"] += st["walks"][0] * n_rows
        out["walks_above"] += sum(st["walks"][1:]) * n_rows
    return out


def kernel_only(args):
    """Two launches of the walk kernel at one level of the benchmark workload."""
    import numpy as np
    import torch

    from paper_1904_12754_amd import api, inputs

    A, t, v = inputs.workload_laplace2d(args.grid)
    plan = api.Plan(A, t, precision="fp32")
    u = torch.as_tensor(v.astype(np.float32), device="cuda")
    lev = plan.l0 + args.level
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, jumps = plan.level_sums(u, lev, 0, args.walks, seed=rep)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        walks = args.walks * A.n
        print(json.dumps({"mode": "kernel", "level": lev, "walks": walks, "steps": walks << lev,
                          "jumps": jumps, "seconds": el, "steps_per_s": (walks << lev) / el}),
              flush=True)
    plan.close()


def _progress(*a):
    print(*a, file=sys.stderr, flush=True)


def _batch_vs_runs(insts, steps, keep_x=False, compare=True):
    """Times one graph replay of the batch of `insts` (four levels from each instance's l0,
    64 * 2^(1.5 (3 - q)) walks per row at level l0 + q, FP32 weights) and, with compare, the
    same work as one fixed-schedule run per instance. keep_x: also return the batch's
    estimates (host)."""
    import numpy as np
    import torch

    from paper_1904_12754_amd import api

    t0 = time.perf_counter()
    plans = [api.Plan(A, t, precision="fp32") for A, t, v in insts]
    us = [torch.as_tensor(v.astype(np.float32), device="cuda") for A, t, v in insts]
    t_plan = time.perf_counter() - t0
    _progress(f"batch of {len(insts)}: plans built in {t_plan:.1f} s")
    walks = np.array([[int(round(64 * 2 ** (1.5 * (3 - q)))) for q in range(4)]
                      for _ in insts], dtype=np.int64)
    t0 = time.perf_counter()
    batch = api.Batch(plans, us, walks, autotune=True)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    _progress(f"batch of {len(insts)}: created and tuned in {t_create:.1f} s")
    batch.launch(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        batch.launch(100 + k)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    _progress(f"batch of {len(insts)}: {steps} replays, {el * 1e3:.1f} ms each")
    st = batch.stats()
    total_steps = sum(x["steps"] for x in st)
    jumps = sum(x["total_jumps"] for x in st)
    xs = [x.cpu().numpy()[:, 0] for x in batch.xs] if keep_x else None
    el_seq = None
    if compare:
        # the same work, one fixed-schedule run per instance
        for b, p in enumerate(plans[:8]):
            p.run(us[b], walks=walks[b], seed=99, instance=b, want_stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b, p in enumerate(plans):
            p.run(us[b], walks=walks[b], seed=100, instance=b, want_stats=False)
        torch.cuda.synchronize()
        el_seq = time.perf_counter() - t0
        _progress(f"batch of {len(insts)}: one run per instance, {el_seq * 1e3:.1f} ms")
    rows = int(sum(A.n for A, _, _ in insts))
    out = {"steps_per_s": total_steps / el, "ms_per_launch": el * 1e3,
           "steps_per_launch": total_steps, "jumps_per_launch": jumps,
           "graph_ms": st[0]["kernel_ms"],
           "one_run_per_instance_ms": None if el_seq is None else el_seq * 1e3,
           "speedup_vs_one_run_per_instance": None if el_seq is None else el_seq / el,
           "rows_total": rows,
           "walks_per_row_per_level": walks[0].tolist(), "batch": batch.info,
           "host_s": {"plans": t_plan, "create_with_autotune": t_create},
           "est_rmse": [math.sqrt(x["est_variance"]) for x in st],
           "_kernel": {"seconds": st[0]["kernel_ms"] * 1e-3, "launches": batch.info["phases"],
                       "steps": total_steps, "jumps": jumps,
                       "walks_base": int(sum(walks[b][0] * A.n for b, (A, _, _) in enumerate(insts))),
                       "walks_above": int(sum(walks[b][1:].sum() * A.n for b, (A, _, _) in enumerate(insts))),
                       "rows_levels": 4 * rows,
                       "ws_bytes": int(sum(A.nnz * 16 + A.n * (32 * 4 + 4) for A, _, _ in insts))}}
    batch.close()
    for p in plans:
        p.close()
    return out, xs


def batch_part(args, probes=None, small=False):
    """The uneven batch: `args.instances` instances (1D/2D Laplacians and Erdos-Renyi graphs,
    n log-uniform in [1e3, 1e5], ||tA||_1 log-uniform in [0.5, 8], v ~ N(0, 1)), four levels
    per instance, in one graph replay; with small=True also a batch of 2048 small instances
    (n log-uniform in [100, 2000]) where one run per instance is dominated by launch and host
    costs. Returns the result and a closure that computes the true errors (CPU)."""
    from paper_1904_12754_amd import inputs

    t0 = time.perf_counter()
    insts = inputs.workload_uneven_batch(args.instances)
    t_gen = time.perf_counter() - t0
    big, xs = _batch_vs_runs(insts, args.steps, keep_x=True, compare=not args.profile_run)
    big["host_s"]["generate"] = t_gen
    k = big.pop("_kernel")
    if probes is not None:
        big["roofline"] = walk_roofline("batch_walks<float,float>", k["seconds"], k["launches"],
                                        k["steps"], k["jumps"], k["walks_base"], k["walks_above"],
                                        k["rows_levels"], 1, k["ws_bytes"], probes)
        big["roofline"]["note"] = ("time = the whole graph (walk phases plus the per-row sums "
                                   "and the combine), so the rates are lower bounds")
    out = {"metric": "walk steps/s", "value": big.pop("steps_per_s"), "unit": "steps/s", **big,
           "config": {"workload": f"{args.instances} uneven instances (1D/2D Laplacian, ER mean "
                                  "degree 8, n in [1e3, 1e5]), 4 levels, FP32 weights, one graph "
                                  "replay"}}
    if small:
        s, _ = _batch_vs_runs(inputs.workload_uneven_batch(2048, nmin=100, nmax=2000), args.steps)
        s.pop("_kernel")
        out["small_instances"] = {"workload": "2048 uneven instances, n in [100, 2000], same "
                                              "schedule", **s}
    est = out.pop("est_rmse")

    def truth():
        import numpy as np

        refs = bench_reference_many(insts)
        errs = np.array([float(np.sqrt(np.mean((x - r) ** 2))) for x, r in zip(xs, refs)])
        ratio = errs / np.maximum(np.array(est), 1e-300)
        return {"true_rmse_median": float(np.median(errs)), "true_rmse_max": float(errs.max()),
                "true_over_est_rmse_median": float(np.median(ratio)),
                "true_over_est_rmse_p95": float(np.quantile(ratio, 0.95)),
                "instances_checked": len(errs),
                "reference": "exp(tA)v per instance in FP64 (truncated Taylor with scaling, "
                             "Al-Mohy & Higham)"}
    return out, truth


def bench_reference_many(insts):
    """FP64 references of many small instances, in threads."""
    from concurrent.futures import ThreadPoolExecutor

    import bench_reference

    with ThreadPoolExecutor(16) as ex:
        return list(ex.map(lambda it: bench_reference.expv_sparse(it[0], it[2], it[1]), insts))


def batch_bench(args):
    if args.profile_run:
        out, _ = batch_part(args)
    else:
        out, truth = batch_part(args, machine_probes(), small=True)
        out["true_error"] = truth()
    print(json.dumps(out), flush=True)


def tc_part(args, probes=None):
    """Total communicability with many right-hand sides: exp(beta A) [1, r_1..r_63] on a
    Barabasi-Albert graph (n = 1e6, m = 5, symmetric 0/1 adjacency stored as FP32),
    beta = 1/d_max, levels l0..l0+4 with 128 walks per row per level, FP32 weights, 64
    right-hand sides carried by every path, in one persistent launch (a batch of this one
    instance replayed from a graph); also timed as five per-level launches of one run, the
    forward scalar estimate of the total communicability, and the forward full vector
    exp(beta A) 1 against the backward run's first column. Returns the result and a closure
    that computes the true errors (CPU)."""
    import numpy as np
    import torch

    from paper_1904_12754_amd import api, inputs

    t0 = time.perf_counter()
    A, beta, U = inputs.workload_ba_tc(n=args.grid if args.grid > 256 else 1_000_000)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = api.Plan(A, beta, precision="fp32", values_dtype=np.float32)
    u = torch.as_tensor(U.astype(np.float32), device="cuda")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    walks = [128] * 5
    plan.run(u, walks=walks, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sts = []
    for k in range(args.steps):
        x, st = plan.run(u, walks=walks, seed=10 + k)
        sts.append(st)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    x_host = x.cpu().numpy()
    tc = float(x_host[:, 0].sum())
    sd_back = math.sqrt(st["est_variance"] * A.n)
    ks = kernel_sums([(s_, A.n) for s_ in sts])
    # the same quantity by the forward scalar representation: walks from uniformly drawn
    # start rows, Algorithm 1 to the backward run's standard deviation
    ones = torch.ones(A.n, dtype=torch.float32, device="cuda")
    plan.functional(ones, ones, walks=[1 << 16] * 5, seed=2)
    # timed over three seeds (one run takes a few ms, so one alone shows the host's jitter);
    # the estimate reported is the first run's
    t_fs = []
    for k in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_f = plan.functional(ones, ones, eps=sd_back, seed=3 + 10 * k, pilot_walks=1 << 16)
        torch.cuda.synchronize()
        t_fs.append(time.perf_counter() - t0)
        if k == 0:
            tc_f, var_f, st_f = res_f
    t_f = sorted(t_fs)[1]
    # the vector exp(beta A) 1 by the forward representation: as many walks per level as the
    # backward run spends on one right-hand side (128 per row), from uniformly drawn rows,
    # deposited at their final states; compared with the backward run's first column
    fwd_walks = [128 * A.n] * 5
    plan.forward(ones, walks=fwd_walks, seed=4)
    t_fws = []
    for k in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res_fw = plan.forward(ones, walks=fwd_walks, seed=5 + 10 * k)
        torch.cuda.synchronize()
        t_fws.append(time.perf_counter() - t0)
        if k == 0:
            xf, vf, st_fw = res_fw
    del res_fw
    t_fw = sorted(t_fws)[1]
    xf_host = xf.cpu().numpy()
    dfb = xf_host - x_host[:, 0]
    fwd = {"seconds": t_fw, "seconds_runs": t_fws, "steps": st_fw["steps"], "walks": fwd_walks,
           "rms_forward_minus_backward": float(np.sqrt(np.mean(dfb * dfb))),
           "rms_expected": math.sqrt(float(vf.mean().item()) + st["est_variance"]),
           "rms_of_x": float(np.sqrt(np.mean(x_host[:, 0] ** 2))),
           "note": "exp(beta A) 1 by walks deposited at their final states (seconds: the median "
                   "of three seeds, the estimate the first's); rms_expected from "
                   "the two estimated variances"}
    # the same five levels as one persistent launch: a batch of this one instance, captured
    # in a graph and replayed
    batch = api.Batch([plan], [u], np.array([walks], dtype=np.int64), autotune=True)
    batch.launch(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        batch.launch(10 + k)
    torch.cuda.synchronize()
    el_b = (time.perf_counter() - t0) / args.steps
    st_b = batch.stats()[0]
    xb_host = batch.xs[0].cpu().numpy()
    tc_b = float(xb_host[:, 0].sum())
    info_b = {k: batch.info[k] for k in ("walks_per_item", "waves_per_cu", "phases", "items")}
    batch.close()
    n_slots = plan.info["n_slots"]
    plan.close()
    del u
    out = {
        "metric": "walk steps/s", "value": st_b["steps"] / el_b, "unit": "steps/s",
        "ms_per_launch": el_b * 1e3, "batch": info_b,
        "rhs_samples_per_s": st_b["steps"] * U.shape[1] / el_b,
        "jumps": st_b["total_jumps"], "steps": st_b["steps"],
        "total_communicability_estimate_batch": tc_b,
        "per_level_runs": {"ms_per_run": el * 1e3, "walk_kernel_ms": st["walk_kernel_ms"],
                           "steps_per_s": st["steps"] / el,
                           "note": "the same walks as five launches (one per level) of one run"},
        "total_communicability_estimate": tc,
        "total_communicability_sd": sd_back,
        "est_rmse": math.sqrt(st["est_variance"]),
        "forward_scalar": {"estimate": tc_f, "sd": math.sqrt(var_f), "seconds": t_f,
                           "seconds_runs": t_fs,
                           "walks": st_f["walks"][:st_f["num_levels"]],
                           "steps": st_f["steps"],
                           "note": "Algorithm 1 on the scalar to the backward run's sd (seconds: "
                                   "the median of three seeds, the estimate the first's)"},
        "forward_full_vector": fwd,
        "config": {"workload": f"Barabasi-Albert n={A.n} m=5, beta=1/d_max={beta:.3e}, "
                               f"{U.shape[1]} right-hand sides (ones + Rademacher), "
                               f"levels {st['l0']}..{st['l0'] + 4}, 128 walks per row per level, "
                               "one persistent launch (graph replay)",
                   "nnz": A.nnz, "d_max": int(round(1 / beta)),
                   "host_s": {"generate": t_gen, "plan": t_plan}},
    }
    # the share of the slot gathers that hot-row staging in LDS could serve: walks start
    # evenly over the rows and mostly stay (beta = 1 / d_max), so a jump leaves row i in
    # proportion to its rate deg_i; the largest rows whose 16-byte slots fit in 64 KB of LDS
    # (64 KB, a workgroup's LDS, and 160 KB, a whole CU's)
    deg = np.sort(np.diff(A.row_ptr))[::-1]
    out_lds = {"note": "jumps leave row i at rate deg_i and the walks start evenly over the rows; "
                       "the hottest rows whose 16-byte alias slots fit in the LDS size"}
    for lds in (64 << 10, 160 << 10):
        k = int(np.searchsorted(np.cumsum(deg), lds // 16, side="right"))
        out_lds[f"{lds >> 10}KB"] = {"rows_that_fit": k,
                                     "share_of_jumps_from_them": float(deg[:k].sum() / deg.sum())}
    if probes is not None:
        R = U.shape[1]
        ws = n_slots * 16 + A.n * 32 + A.n * 4 * R
        out["roofline"] = walk_roofline("level_walks_rhs<float,float>", ks["ms"] * 1e-3,
                                        ks["launches"], ks["steps"], ks["jumps"], ks["walks_base"],
                                        ks["walks_above"], 5 * A.n * len(sts), R, ws, probes)
        out["roofline"]["note"] = "the per-level runs' walk launches (event pairs around each)"
    out["lds_hot_row_staging_bound"] = out_lds

    def truth():
        import bench_reference

        ref = bench_reference.expv_sparse(A, U, beta, threads=16)
        e = x_host - ref
        eb = xb_host - ref
        return {"true_rmse": float(np.sqrt(np.mean(e ** 2))),
                "true_rmse_batch": float(np.sqrt(np.mean(eb ** 2))),
                "true_rmse_column0": float(np.sqrt(np.mean(e[:, 0] ** 2))),
                "forward_full_vector_true_rmse": float(np.sqrt(np.mean((xf_host - ref[:, 0]) ** 2))),
                "total_communicability_exact": float(ref[:, 0].sum()),
                "reference": "exp(beta A) U for all 64 right-hand sides in FP64 (truncated "
                             "Taylor with scaling, Al-Mohy & Higham)"}
    return out, truth


def tc_bench(args):
    if args.profile_run:
        out, _ = tc_part(args)
    else:
        out, truth = tc_part(args, machine_probes())
        out["true_error"] = truth()
    print(json.dumps(out), flush=True)


def learned_part(args):
    """Time to a target RMSE with the learned proposal against the plain jump law, on the 3D
    7-point convection-diffusion operator (m^3 cells, lognormal(0, 0.5) diffusivity,
    uniform(-1, 1) velocity per cell, ||tA||_1 = 4, v = exp(-|x|^2)), FP32 weights,
    Algorithm 1 with the same pilot in both cases, at the target eps, eps / 10 and eps / 30. The
    proposal is trained once (pilot estimate, transition capture, Adam, table build: the
    whole call is timed) and then used for all targets; if the variance judge rejects it, the
    'learned' rows run with the plain law the library fell back to, and say so. At the target
    eps the learned run (training inside Algorithm 1, on its own pilot) is timed whole against
    the plain solve. Returns the result and a closure that computes the true errors (CPU)."""
    import numpy as np
    import torch

    from paper_1904_12754_amd import api, inputs

    t0 = time.perf_counter()
    A, t, v = inputs.workload_convdiff3d(args.cd_grid)
    t_gen = time.perf_counter() - t0
    u = torch.as_tensor(v.astype(np.float32), device="cuda")
    t0 = time.perf_counter()
    plan = api.Plan(A, t, precision="fp32")
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def solve(eps, seed):
        return timed(lambda: plan.run(u, eps=eps, seed=seed, pilot_walks=args.cd_pilot,
                                      max_levels=12))

    def summary(st, el):
        nl = st["num_levels"]
        return {"time_to_rmse_s": el, "steps": st["steps"], "jumps": st["total_jumps"],
                "walks": st["walks"][:nl], "level_var": st["level_var"][:nl],
                "est_rmse": math.sqrt(st["est_variance"] + st["est_bias"] ** 2),
                "steps_per_s": st["steps"] / el}

    solve(args.eps, 1)                                # warm-up: level tables, scratch
    rng = np.random.default_rng(0)
    P0 = _init_params(rng)
    train_opts = dict(seed=3, pilot_walks=32, capture_walks=16,
                      sample_stride=max(1, A.n // 65536), steps=200, batch=4096, lr=1e-2,
                      shrink=10.0, num_levels=1, judge_walks=8)
    (params, tst), t_train = timed(lambda: plan.train_proposal(u, P0, **train_opts))
    accepted = bool(tst["accepted"])
    out = {
        "workload": f"3D 7-point convection-diffusion {args.cd_grid}^3 (n={A.n}, nonsymmetric), "
                    f"lognormal(0,0.5) diffusivity, U(-1,1) velocity, ||tA||_1=4, "
                    f"v=exp(-|x|^2); Algorithm 1 (pilot "
                    f"{args.cd_pilot or 'from the row count: max(2, 2^18 / n)'} walks per row "
                    f"on l0..l0+4); FP32 weights",
        "train_s": t_train,
        "training": {k: tst[k] for k in ("transitions", "held_out", "steps", "best_step",
                                         "train_ms", "first_val_loss", "best_val_loss",
                                         "judge_var_plain", "judge_var_learned", "accepted")},
        "train_options": train_opts,
        "learned_law": "trained proposal" if accepted else
                       "plain law (the variance judge rejected the trained proposal)",
        "targets": [],
        "host_s": {"generate": t_gen, "plan": t_plan},
    }
    xs = []
    for k, eps in enumerate((args.eps, args.eps / 10, args.eps / 30)):
        plan.enable_proposal(False)
        (xp, stp), tp = solve(eps, 100 + k)
        plan.enable_proposal(accepted)
        (xl, stl), tl = solve(eps, 200 + k)
        xp_h = xp.cpu().numpy()[:, 0]
        xl_h = xl.cpu().numpy()[:, 0]
        xs.append((xp_h, xl_h))
        d = xl_h - xp_h
        out["targets"].append({
            "eps": eps, "plain": summary(stp, tp), "learned": summary(stl, tl),
            "speedup_solve": tp / tl, "speedup_incl_training": tp / (tl + t_train),
            # solves with the same trained proposal after which the training has paid off
            "solves_to_amortize_training": t_train / (tp - tl) if tp > tl else None,
            "variance_ratio_l0": stp["level_var"][0] / max(stl["level_var"][0], 1e-300),
            "rms_learned_minus_plain": float(np.sqrt(np.mean(d * d))),
        })
    # the learned run at the target eps: Algorithm 1 whose plain pilot gives the estimate the
    # proposal of l0 is trained on (16 Adam steps on batches of 1024, early stopping), from
    # the network's value-ratio prior alone (zero corrections, alpha = 0.9 sigmoid(3) = 0.857);
    # the variance judge compares the pilot's plain level-l0 walks with the same walks under the
    # proposal. Timed whole, three times each against the plain solve
    P_run = _init_params(np.random.default_rng(0), alpha_logit=3.0)
    run_opts = dict(capture_walks=4, sample_stride=max(1, A.n // 65536), steps=16, batch=1024,
                    lr=1e-2, shrink=10.0)

    def learned_run(seed, train_seed):
        return timed(lambda: plan.run_learned(u, args.eps, P_run, seed=seed, train_seed=train_seed,
                                              pilot_walks=args.cd_pilot, max_levels=12,
                                              **run_opts))

    plan.enable_proposal(False)
    learned_run(400, 0)
    runs, plain_s = [], []
    for rep in range(3):
        plan.enable_proposal(False)
        (_, stp), tp = solve(args.eps, 500 + rep)
        plain_s.append(tp)
        (xr, sr, tr, _), tl = learned_run(401 + rep, rep)
        nl = sr["num_levels"]
        runs.append({"time_s": tl, "train_ms": tr["train_ms"], "accepted": bool(tr["accepted"]),
                     "best_step": tr["best_step"], "transitions": tr["transitions"],
                     "judge_var_plain": tr["judge_var_plain"],
                     "judge_var_learned": tr["judge_var_learned"],
                     "walks": sr["walks"][:nl], "plain_walks": stp["walks"][:stp["num_levels"]],
                     "est_rmse": math.sqrt(sr["est_variance"] + sr["est_bias"] ** 2)})
    xr_h = xr.cpu().numpy()[:, 0]
    out["learned_run"] = {
        "eps": args.eps, "train_options": run_opts, "init": "value-ratio prior, alpha 0.857",
        "runs": runs, "plain_solve_s": plain_s,
        "speedup_incl_training": min(plain_s) / min(r["time_s"] for r in runs),
        "variance_ratio_l0": runs[-1]["judge_var_plain"] / max(runs[-1]["judge_var_learned"], 1e-300),
    }
    plan.close()

    def truth():
        import bench_reference

        ref = bench_reference.expv_sparse(A, v, t)
        out["learned_run"]["true_rmse_last"] = float(np.sqrt(np.mean((xr_h - ref) ** 2)))
        for tg, (xp_h, xl_h) in zip(out["targets"], xs):
            tg["plain"]["true_rmse"] = float(np.sqrt(np.mean((xp_h - ref) ** 2)))
            tg["learned"]["true_rmse"] = float(np.sqrt(np.mean((xl_h - ref) ** 2)))
        return "exp(tA)v in FP64 (truncated Taylor with scaling, Al-Mohy & Higham)"
    return out, truth


def learned_bench(args):
    out, truth = learned_part(args)
    if not args.profile_run:
        out["true_error_reference"] = truth()
    print(json.dumps(out), flush=True)


def classical_bench(args):
    """MLMC against classical (single-level) Monte Carlo at the same accuracy, on workload 2
    restricted to 4096 sampled rows: for each eps, Algorithm 1 gives the finest level L
    whose bias passes its test; classical MC samples the base estimator at that level alone
    (a plan with l0 = L) with M = 2 V_L / eps^2 walks per row (the same variance budget
    eps^2 / 2), V_L from a 1024-walk pilot that is timed with it. Section 4 predicts costs
    of order eps^-2 for MLMC and eps^-5/2 for classical MC."""
    import numpy as np
    import torch

    from paper_1904_12754_amd import api, inputs

    A, t, v = inputs.workload_laplace2d(args.grid)
    rows = np.sort(np.random.default_rng(11).choice(A.n, size=4096, replace=False))
    u = torch.as_tensor(v.astype(np.float32), device="cuda")
    ml = api.Plan(A, t, precision="fp32", rows=rows)
    ml.run(u, eps=1e-2, seed=1, pilot_walks=1024)
    torch.cuda.synchronize()
    out = {"workload": f"2D 5-point Laplacian {args.grid}x{args.grid}, 4096 sampled rows, "
                       f"t=h^2/2, FP32 weights", "targets": []}
    mc_plans = {}
    for k, eps in enumerate((1e-2, 3e-3, 1e-3)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x_ml, st = ml.run(u, eps=eps, seed=100 + k, pilot_walks=1024, max_levels=12)
        torch.cuda.synchronize()
        t_ml = time.perf_counter() - t0
        L = st["l0"] + st["num_levels"] - 1
        if L not in mc_plans:
            mc_plans[L] = api.Plan(A, t, precision="fp32", rows=rows, l0=L)
            mc_plans[L].run(u, walks=[64], seed=1)
        mc = mc_plans[L]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, pst = mc.run(u, walks=[1024], seed=200 + k)
        M = int(math.ceil(2.0 * pst["level_var"][0] / eps ** 2))
        x_mc, mst = mc.run(u, walks=[M], seed=300 + k)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t0
        d = (x_ml - x_mc).cpu().numpy()[:, 0]
        out["targets"].append({
            "eps": eps, "finest_level": L,
            "mlmc": {"time_s": t_ml, "steps": st["steps"], "walks": st["walks"][:st["num_levels"]],
                     "est_rmse": math.sqrt(st["est_variance"] + st["est_bias"] ** 2)},
            "classical": {"time_s": t_mc, "steps": pst["steps"] + mst["steps"], "walks": M,
                          "est_rmse": math.sqrt(mst["est_variance"])},
            "classical_over_mlmc_time": t_mc / t_ml,
            "rms_mlmc_minus_classical": float(np.sqrt(np.mean(d * d))),
        })
    ts = out["targets"]
    le = np.log([t_["eps"] for t_ in ts])
    for key in ("mlmc", "classical"):
        out[f"{key}_cost_slope_vs_eps"] = float(np.polyfit(le, np.log([t_[key]["steps"] for t_ in ts]), 1)[0])
    for p in list(mc_plans.values()) + [ml]:
        p.close()
    return out


def _init_params(rng, alpha_logit=-2.0):
    """Initial weights of the 16-64-64-7 proposal network (flat, FP32): He-scaled hidden
    layers, a zero output layer (no correction to the value-ratio prior) and the mixing
    output at alpha = 0.9 sigmoid(alpha_logit); the default, 0.11, keeps the untrained
    proposal close to the plain law, so that the gain comes from training."""
    import numpy as np

    W1 = rng.normal(size=(16, 64)) * math.sqrt(2.0 / 16)
    W2 = rng.normal(size=(64, 64)) * math.sqrt(2.0 / 64)
    W3 = np.zeros((64, 7))
    b3 = np.zeros(7)
    b3[6] = alpha_logit
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(),
                           b3]).astype(np.float32)


def copy_only(args):
    """A plain device-to-device copy of a known size (the traffic-counter calibration)."""
    import torch

    n = args.bytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for rep in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.copy_(a)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "seconds": el, "GBps": 8 * n / el / 1e9}), flush=True)


def cpu_baseline(A, t, v, l0, walks, target_s, threads=0, min_steps=1.2e9):
    """The oracle (plain FP64 C, OpenMP over rows; `threads` 0 = all of the host's) on a
    bounded sample of the same workload: a random subset of rows with the solve's sample
    sizes scaled down so that the run takes about target_s seconds, and at least min_steps
    walk steps. Returns walk steps per second."""
    import numpy as np

    from oracle import mlmc as orc

    tables = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    threads = threads or orc.max_threads()
    rng = np.random.default_rng(5)
    # calibration on a slice of about 0.1 s of work
    rows = rng.choice(A.n, size=1024, replace=False)
    orc.level_sums(tables, t, l0, l0, 1, v, rows[:64], 0, 64, threads=threads)
    t0 = time.perf_counter()
    orc.level_sums(tables, t, l0, l0, 1, v, rows, 0, 256, threads=threads)
    cal = time.perf_counter() - t0
    speed = 1024 * 256 * (1 << l0) / max(cal, 1e-6)
    steps_full = sum(w * (1 << (l0 + q)) for q, w in enumerate(walks)) * A.n
    target = max(min_steps, target_s * speed)
    frac = min(1.0, target / steps_full)
    n_rows = max(64, min(A.n, int(A.n * math.sqrt(frac))))
    scale = min(1.0, frac * A.n / n_rows)
    rows = np.sort(rng.choice(A.n, size=n_rows, replace=False))
    Ms = [max(1, int(round(w * scale))) for w in walks]
    steps = 0
    t0 = time.perf_counter()
    for q, M in enumerate(Ms):
        orc.level_sums(tables, t, l0 + q, l0, 1, v, rows, 0, M, threads=threads)
        steps += n_rows * M * (1 << (l0 + q))
    el = time.perf_counter() - t0
    return {"value": steps / el, "unit": "walk steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_rows} of {A.n} rows, walks per level {Ms} (the solve's sample "
                      f"sizes x {scale:.2e}), levels {l0}..{l0 + len(Ms) - 1}, FP64, "
                      f"{steps:.3e} steps in {el:.1f} s"}


def config1_part(args):
    """The FP64 1D Dirichlet Laplacian (n = 100, t = 1e-4, v = sin(pi i h) + U(0, 0.1)),
    full vector, 1e4 walks per row at the finest of four levels (coarser levels by the ratio
    2^{1.5}), FP64 weights; error against the dense FP64 matrix exponential."""
    import numpy as np
    import torch

    import bench_reference
    from paper_1904_12754_amd import api, inputs

    A, t, v = inputs.workload_laplace1d()
    exact = bench_reference.expv_dense(A.to_dense(), v, t)
    plan = api.Plan(A, t, precision="fp64")
    u = torch.as_tensor(v, device="cuda")
    walks = [int(round(1e4 * 2 ** (1.5 * (3 - q)))) for q in range(4)]
    plan.run(u, walks=walks, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, st = plan.run(u, walks=walks, seed=2)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    err = x.cpu().numpy()[:, 0] - exact
    plan.close()
    return {"workload": "1D Dirichlet Laplacian n=100, t=1e-4, FP64, levels "
                        f"{st['l0']}..{st['l0'] + 3}, walks per row {walks}",
            "seconds": el, "steps": st["steps"], "steps_per_s": st["steps"] / el,
            "true_rmse_vs_dense_expm": float(np.sqrt(np.mean(err ** 2))),
            "max_abs_error": float(np.abs(err).max()),
            "est_rmse": math.sqrt(st["est_variance"])}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the walk kernel is "
                                   "measured at one GPU's share of the work (--gpus 1)"}))
        sys.exit(2)
    if args.mode == "config1":
        print(json.dumps(config1_part(args)), flush=True)
        return
    if args.mode == "kernel":
        return kernel_only(args)
    if args.mode == "copy":
        return copy_only(args)
    if args.mode == "probe":
        print(json.dumps(machine_probes()), flush=True)
        return
    if args.mode == "batch":
        return batch_bench(args)
    if args.mode == "tc":
        return tc_bench(args)
    if args.mode == "learned":
        return learned_bench(args)
    if args.mode == "classical":
        print(json.dumps(classical_bench(args)), flush=True)
        return
    import numpy as np
    import torch

    import bench_reference
    from paper_1904_12754_amd import api, inputs

    dev = torch.device("cuda:0")
    probes = machine_probes()
    A, t, v = inputs.workload_laplace2d(args.grid)
    x_exact = bench_reference.expv_laplace2d(v, t)
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

    ks = kernel_sums([(s_, plan.n_rows) for s_ in stats])
    steps = ks["steps"]
    jumps = ks["jumps"]
    last = stats[-1]
    xg = x.cpu().numpy()[:, 0]
    true_rmse = float(np.sqrt(np.mean((xg - x_exact) ** 2)))
    walks_total = ks["walks_base"] + ks["walks_above"]
    ws = plan.info["n_slots"] * 16 + A.n * (32 + 4)
    roofline = walk_roofline("level_walks_r1<float,float>", ks["ms"] * 1e-3, ks["launches"], steps,
                             jumps, ks["walks_base"], ks["walks_above"],
                             plan.n_rows * sum(s_["num_levels"] for s_ in stats), 1, ws, probes,
                             traffic=kernel_traffic(walks_total / max(ks["launches"], 1)))
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
            "walk_kernel_share": ks["ms"] * 1e-3 / elapsed,
            "path_decisions": "fp64 + u32 (bit-identical to the FP64 oracle)",
        },
        "roofline": roofline,
        "probes": probes,
    }
    # the same solve to a looser target (outside the timed region)
    if not args.no_loose:
        plan.run(u, eps=1e-2, seed=30_000, pilot_walks=args.pilot, max_levels=12)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(3):
            x2, st2 = plan.run(u, eps=1e-2, seed=31_000 + k, pilot_walks=args.pilot, max_levels=12)
        torch.cuda.synchronize()
        el2 = (time.perf_counter() - t0) / 3
        line["config"]["time_to_rmse_1e-2"] = {
            "seconds": el2, "walks_per_row_per_level": st2["walks"],
            "true_rmse_vs_exact": float(np.sqrt(np.mean((x2.cpu().numpy()[:, 0] - x_exact) ** 2))),
            "steps_per_s": st2["steps"] / el2}
    plan.close()
    del u
    torch.cuda.empty_cache()
    truths = {}
    others = {}
    if not args.no_others:
        others["laplace1d_fp64"] = config1_part(args)
        print("bench: workload 1 done", file=sys.stderr, flush=True)
        others["barabasi_albert_64rhs"], truths["barabasi_albert_64rhs"] = tc_part(args, probes)
        torch.cuda.empty_cache()
        print("bench: workload 3 done", file=sys.stderr, flush=True)
        others["uneven_batch"], truths["uneven_batch"] = batch_part(args, probes)
        torch.cuda.empty_cache()
        print("bench: workload 4 done", file=sys.stderr, flush=True)
    if not args.no_learned:
        line["learned_proposal"], learned_truth = learned_part(args)
        print("bench: workload 5 done", file=sys.stderr, flush=True)
        line["learned_proposal"]["true_error_reference"] = learned_truth()
    for key, fn in truths.items():
        others[key]["true_error"] = fn()
    if others:
        line["other_workloads"] = others
    if not args.no_cpu_baseline:
        cb = cpu_baseline(A, t, v, last["l0"], last["walks"], args.cpu_seconds)
        one = cpu_baseline(A, t, v, last["l0"], last["walks"], args.cpu_seconds / 3, threads=1,
                           min_steps=0)
        cb["one_core"] = {"value": one["value"], "sample": one["sample"]}
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Parity at the benchmark workloads' full sizes, in the launch configurations the benchmark
times: the device computes every row of the plan (or every instance of the batch) with the
benchmark's walk counts, so the chunking, sub-launches and lane packing are those of the
timed runs, and sampled rows are checked against the oracle one by one. Paths are pinned
bit-exact through the per-row sums of the path hashes (or the jump counts), sums within the
FP32 bar relative to each row's absolute mass."""
import sys

import numpy as np
import pytest
import torch

from oracle import mlmc as orc
from paper_1904_12754_amd import inputs

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1904_12754_amd import api as _api
    return _api


def _sample_rows(n, k, seed, extra=()):
    rng = np.random.default_rng(seed)
    rows = set(int(r) for r in rng.choice(n, size=k, replace=False))
    rows.update(int(r) for r in extra)
    return np.array(sorted(rows), dtype=np.int64)


def _check_rows(plan, t, beta, u_dev, u_host, level, M, seed, rows):
    """level_sums of every row on the device; the sampled rows against the oracle."""
    s1, s2, jumps, hs = plan.level_sums(u_dev, level, 0, M, seed=seed, hashes=True)
    # the benchmark's kernel (no path hashes) walks the same paths. With one right-hand side
    # its sums are bit-identical; with several on a screened plan it first screens out the
    # walks that never jump, so its compensated sums add the moved walks in another order
    # and are checked against the oracle like the others
    s1b, s2b, jb = plan.level_sums(u_dev, level, 0, M, seed=seed)
    assert jb == jumps, level
    runs = [(s1, s2)]
    if plan.info["screened"] and u_dev.dim() > 1 and u_dev.shape[1] > 1:
        runs.append((s1b, s2b))
    else:
        assert torch.equal(s1b, s1) and torch.equal(s2b, s2), level
    idx = torch.as_tensor(rows, device=s1.device)
    gh = hs[idx].cpu().numpy().view(np.uint64)
    o = orc.level_sums(t, beta, level, plan.l0, seed, u_host, rows, 0, M)
    assert np.array_equal(gh, o.hash_sum), level
    for a1, a2 in runs:
        g1 = a1[idx].cpu().numpy()
        g2 = a2[idx].cpu().numpy()
        assert np.all(np.abs(g1 - o.sum1) <= TOL32 * (o.mass + 1e-300)), level
        assert np.all(np.abs(g2 - o.sum2) <= 4 * TOL32 * (o.mass2 + 1e-300)), level
    del s1b, s2b
    assert jumps >= int(o.jumps.sum())
    return int(o.jumps.sum())


def test_laplace2d_256_all_rows_sampled(api):
    """2D 5-point Laplacian 256 x 256, t = h^2 / 2, FP32 weights: level l0 with 65536 walks
    per row (items of 4096 walks, 16 per row, as in the benchmark's solve) and levels
    l0 + 1 .. l0 + 4 with 4096 walks per row; 48 random rows plus corners and edges."""
    A, t, v = inputs.workload_laplace2d(256)
    plan = api.Plan(A, t, precision="fp32")
    tables = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    u32 = v.astype(np.float32)
    u_dev = torch.as_tensor(u32, device="cuda")
    rows = _sample_rows(A.n, 48, 31, extra=(0, 255, 256 * 128 + 1, A.n - 1))
    for q, M in enumerate([65536, 4096, 4096, 4096, 4096]):
        lev = plan.l0 + q
        _say(f"laplace2d 256: level {lev}, {M} walks per row, {len(rows)} sampled rows")
        jumps = _check_rows(plan, tables, t, u_dev, u32.astype(np.float64), lev, M, 900 + q, rows)
        assert jumps > 0
    plan.close()


def test_total_communicability_ba_1e6_64_rhs_sampled(api):
    """Barabasi-Albert n = 1e6, m = 5, beta = 1 / d_max, 64 right-hand sides, FP32 weights
    and values, levels l0 .. l0 + 4 with 128 walks per row (the benchmark's run); 32 random
    rows plus the largest hub."""
    A, beta, U = inputs.workload_ba_tc()
    plan = api.Plan(A, beta, precision="fp32", values_dtype=np.float32)
    vals = np.asarray(A.values, dtype=np.float32).astype(np.float64)
    tables = orc.decompose(A.n, A.row_ptr, A.col_idx, vals)
    u32 = np.ascontiguousarray(U.astype(np.float32))
    u_dev = torch.as_tensor(u32, device="cuda")
    hub = int(np.argmax(np.diff(A.row_ptr)))
    rows = _sample_rows(A.n, 32, 32, extra=(hub,))
    for q in range(5):
        lev = plan.l0 + q
        _say(f"BA 1e6 x 64: level {lev}, 128 walks per row, {len(rows)} sampled rows")
        _check_rows(plan, tables, beta, u_dev, u32.astype(np.float64), lev, 128, 500 + q, rows)
    plan.close()


def test_convdiff_128_under_a_proposal_sampled(api):
    """3D convection-diffusion 128^3 (n = 2.1e6), ||tA||_1 = 4, walks under a non-trivial
    proposal (the oracle walks on the device's exported tables), 32 walks per row at levels
    l0 and l0 + 1 (the benchmark's pilot size); 32 random rows plus boundary rows."""
    from oracle import proposal as prop
    A, t, v = inputs.workload_convdiff3d(128)
    plan = api.Plan(A, t, precision="fp32")
    rng = np.random.default_rng(33)
    P = prop.init_params(5)
    P["W3"] *= 20.0
    P["b3"][prop.NS] = 1.0
    xhat = np.abs(v) + 0.1 * np.abs(rng.normal(size=A.n))
    plan.set_proposal(prop.flatten(P).astype(np.float32), xhat, num_levels=2)
    tables = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    u32 = v.astype(np.float32)
    u_dev = torch.as_tensor(u32, device="cuda")
    rows = _sample_rows(A.n, 32, 34, extra=(0, 127, A.n // 2 + 64 * 128 + 64, A.n - 1))
    for q in range(2):
        lev = plan.l0 + q
        thr, alias, ratio, _ = plan.proposal_tables(lev)
        ti = tables.with_proposal(thr, alias, ratio.astype(np.float64))
        del thr, alias, ratio
        _say(f"convdiff 128^3 under a proposal: level {lev}, 32 walks per row, {len(rows)} rows")
        _check_rows(plan, ti, t, u_dev, u32.astype(np.float64), lev, 32, 700 + q, rows)
    plan.close()


def test_uneven_batch_512_sampled(api):
    """The 512-instance uneven batch with the benchmark's schedule (1448, 512, 181, 64 walks
    per row on four levels) in one graph replay with the autotuned shape; 8 instances x 8
    rows against the oracle's fixed-schedule estimate of the same instance number."""
    insts = inputs.workload_uneven_batch(512)
    walks = np.array([[int(round(64 * 2 ** (1.5 * (3 - q)))) for q in range(4)]
                      for _ in insts], dtype=np.int64)
    plans = [api.Plan(A, t, precision="fp32") for A, t, _ in insts]
    us = [torch.as_tensor(v.astype(np.float32), device="cuda") for _, _, v in insts]
    batch = api.Batch(plans, us, walks, autotune=True)
    _say(f"uneven batch 512: {batch.info}")
    seed = 2024
    xs = batch.launch(seed)
    torch.cuda.synchronize()
    sizes = np.array([A.n for A, _, _ in insts])
    order = np.argsort(sizes)
    pick = sorted(set(int(order[k]) for k in (0, 100, 200, 300, 400, 480, 510, 511)))
    for b in pick:
        A, t, v = insts[b]
        rows = _sample_rows(A.n, 8, 40 + b)
        _say(f"  instance {b}: n={A.n} l0={plans[b].l0}, rows {rows.tolist()}")
        tt = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
        res = orc.mlmc_fixed(tt, t, v.astype(np.float32).astype(np.float64), plans[b].l0,
                             plans[b].l0 + 3, walks[b], seed, rows=rows, instance=b)
        xg = xs[b][torch.as_tensor(rows, device=xs[b].device)].cpu().numpy()
        assert np.all(np.abs(xg - res.x) <= TOL32 * res.mass + 1e-300), b
    batch.close()
    for p in plans:
        p.close()

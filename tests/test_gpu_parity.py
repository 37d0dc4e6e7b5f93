"""Parity of the HIP path (through the C-ABI) with the oracle, on identical seeded inputs.

Bars (from the rounding of the two evaluation orders: the oracle multiplies the per-step
factors, the kernel sums exponents and evaluates one exp / expm1):
  - paths: final state, sign, jump count and the FNV path hash are bit-exact;
  - FP64 weights: per-row level sums within 1e-12 of the oracle's, relative to the row's
    absolute mass  sum_w |u_j| (|eta_fine| + |eta_coarse|)  (the scale of the rounding of
    each sample; the oracle multiplies factors, the kernel sums exponents);
  - FP32 weights: within 1e-5 of the same mass.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import mlmc as orc
from oracle import reference
from paper_1904_12754_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1904_12754_amd import api as _api
    return _api


def _tables(A):
    return orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)


def _signed(n, seed, density=0.5, scale=1.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, n)) * (rng.random((n, n)) < density) * scale
    return a


def _check_trace(api, A, beta, precision, levels, rows, walks, seed, l0=None, instance=0):
    plan = api.Plan(A, beta, precision=precision, l0=l0)
    t = _tables(A)
    for lev in levels:
        _say(f"trace n={A.n} prec={precision} level={lev} walks={len(rows)}")
        g = plan.trace(lev, rows, walks, seed=seed, instance=instance)
        o = orc.walk_trace(t, beta, lev, seed, rows, walks, instance=instance)
        assert np.array_equal(g["final_state"].cpu().numpy(), o.final_state)
        assert np.array_equal(g["sign"].cpu().numpy(), o.sign)
        assert np.array_equal(g["jumps"].cpu().numpy(), o.jumps)
        assert np.array_equal(g["hash"].cpu().numpy().view(np.uint64), o.hash)
        lf = g["log_eta_fine"].cpu().numpy()
        ref = np.log(np.abs(o.eta_fine))
        tol = 1e-12 if precision == "fp64" else 1e-5
        assert np.max(np.abs(lf - ref) / (1.0 + np.abs(ref))) < tol
        if lev > 0:
            lc = g["log_eta_coarse"].cpu().numpy()
            refc = np.log(np.abs(o.eta_coarse))
            assert np.max(np.abs(lc - refc) / (1.0 + np.abs(refc))) < tol
        assert o.jumps.sum() > 0
    plan.close()


def test_trace_bit_exact_laplace1d_fp64(api):
    A, t, v = inputs.workload_laplace1d()
    M = 2000
    rows = np.repeat(np.arange(A.n), M // 20)[:M]
    walks = np.arange(M, dtype=np.uint32) * 7919
    _check_trace(api, A, t, "fp64", range(3, 7), rows, walks, seed=123)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_trace_bit_exact_signed_all_levels(api, precision):
    a = _signed(40, 3, density=0.3)
    a[5, :] = 0.0
    a[5, 5] = 0.3                        # absorbing row
    a[7, :] *= 3.0                       # a fast row
    A = inputs.from_dense(a)
    beta = 0.3                           # r_max beta ~ 10: several jumps per step at level 0
    M = 4096
    rng = np.random.default_rng(1)
    rows = rng.integers(0, A.n, size=M)
    walks = rng.integers(0, 2 ** 32, size=M, dtype=np.uint64).astype(np.uint32)
    # levels 0 and 1 have fewer than four steps (partial Philox block)
    _check_trace(api, A, beta, precision, range(0, 7), rows, walks, seed=2 ** 40 + 17, l0=0,
                 instance=9)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("scale", [1e32, 1e-34])
def test_exact_decisions_at_extreme_time_scales(api, precision, scale):
    """e^{beta A} is unchanged when A is scaled by s and beta by 1/s. At these scales dt lies
    outside [2^-100, 2^100], where the kernels' FP32 bounds around dt are switched off and
    every chain decision takes the exact FP64 path: paths bit-exact at levels 0..4 and level
    sums within the bars."""
    a = _signed(40, 3, density=0.3) * scale
    A = inputs.from_dense(a)
    beta = 0.3 / scale
    rng = np.random.default_rng(12)
    rows = rng.integers(0, A.n, size=2048)
    walks = rng.integers(0, 2 ** 32, size=2048, dtype=np.uint64).astype(np.uint32)
    _check_trace(api, A, beta, precision, range(0, 5), rows, walks, seed=4242, l0=0)
    u = rng.normal(size=A.n)
    _check_level_sums(api, A, beta, u, precision, 3, 512, seed=31)
    t = _tables(A)
    l0 = orc.default_l0(t, beta)
    for lev in (0, 4, l0, l0 + 2):
        dt = beta / 2 ** lev
        assert dt < 2.0 ** -100 or dt > 2.0 ** 100, (lev, dt)


def _mass_tol(o_ls, prec):
    return TOL[prec] * (o_ls.mass + 1e-300)


def _check_level_sums(api, A, beta, u, precision, nlev, walks, seed, rows=None,
                      values_dtype=np.float64, walk0=0, hashes_only_check=True):
    """Levels l0 .. l0 + nlev - 1 of the plan."""
    plan = api.Plan(A, beta, precision=precision, rows=rows, values_dtype=values_dtype)
    vals = np.asarray(A.values, dtype=values_dtype).astype(np.float64)
    t = orc.decompose(A.n, A.row_ptr, A.col_idx, vals)
    assert plan.l0 == orc.default_l0(t, beta)
    screened = bool(plan.info["screened"])
    ut = torch.as_tensor(np.ascontiguousarray(u), device="cuda")
    for lev in range(plan.l0, plan.l0 + nlev):
        _say(f"level_sums n={A.n} prec={precision} level={lev} M={walks} R={ut.shape[-1] if ut.dim() > 1 else 1}")
        s1, s2, jumps, hs = plan.level_sums(ut, lev, walk0, walks, seed=seed, hashes=True)
        o = orc.level_sums(t, beta, lev, plan.l0, seed, u, rows, walk0, walks)
        assert jumps == int(o.jumps.sum())
        # the production kernel's paths: per-row sums of the path hashes, bit-exact
        assert np.array_equal(hs.cpu().numpy().view(np.uint64), o.hash_sum)
        runs = [(s1, s2)]
        if hashes_only_check:
            # the kernel without path hashes (the production one) takes the same paths; with
            # several right-hand sides on a screened plan it first screens out the walks that
            # never jump, so its compensated sums add the moved walks in another order
            s1b, s2b, jb = plan.level_sums(ut, lev, walk0, walks, seed=seed)
            assert jb == jumps
            if screened and ut.dim() > 1 and ut.shape[1] > 1:
                runs.append((s1b, s2b))
            else:
                assert torch.equal(s1b, s1) and torch.equal(s2b, s2)
        for a1, a2 in runs:
            g1 = a1.cpu().numpy()
            g2 = a2.cpu().numpy()
            assert np.all(np.abs(g1 - o.sum1) <= _mass_tol(o, precision))
            # sums of squares: the error of each Y^2 is below 2 tol m_w^2
            assert np.all(np.abs(g2 - o.sum2) <= 4 * TOL[precision] * (o.mass2 + 1e-300))
    plan.close()
    return screened


def test_level_sums_fp64_laplace1d_ragged(api):
    A, t, v = inputs.workload_laplace1d()
    _check_level_sums(api, A, t, v, "fp64", 4, 3001, seed=5)


def test_level_sums_fp32_laplace1d(api):
    A, t, v = inputs.workload_laplace1d()
    _check_level_sums(api, A, t, v, "fp32", 4, 2048, seed=6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_level_sums_signed_u32_walk_offset(api, precision):
    a = _signed(60, 11, density=0.2)
    A = inputs.from_dense(a)
    u = np.random.default_rng(2).normal(size=60)
    beta = 0.7
    # walk indices near the top of the 32-bit range
    _check_level_sums(api, A, beta, u, precision, 3, 777, seed=9, walk0=2 ** 32 - 800)


@pytest.mark.parametrize("R", [3, 64, 130])
def test_level_sums_multi_rhs(api, R):
    """Several right-hand sides on a Barabasi-Albert graph at beta = 1/d_max, where few walks
    jump: the plan screens its walks (each walk's steps drawn at its start row first), and
    the screened kernel's sums, jumps and paths are the oracle's."""
    A = inputs.barabasi_albert(3000, 3, seed=4)
    dmax = float(np.diff(A.row_ptr).max())
    beta = 1.0 / dmax
    u = inputs.rhs_ones_rademacher(A.n, R, seed=7)
    rows = np.random.default_rng(3).choice(A.n, size=300, replace=False)
    rows[0] = int(np.argmax(np.diff(A.row_ptr)))            # the hub
    assert _check_level_sums(api, A, beta, u, "fp32", 3, 200, seed=3, rows=rows,
                             values_dtype=np.float32)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_level_sums_multi_rhs_screened_ragged(api, precision):
    """A screened plan (a signed matrix at a small beta) with 5 right-hand sides and 4096 and
    777 walks per row, on levels 0..3 (levels 0 and 1 have fewer steps than a Philox block
    has words)."""
    a = _signed(40, 13, density=0.3)
    A = inputs.from_dense(a)
    u = np.random.default_rng(4).normal(size=(40, 5))
    beta = 0.02
    # the plan's jump probability: the mean over the rows of 1 - exp(-beta r_i)
    r = np.abs(a).sum(axis=1) - np.abs(np.diag(a))
    plan = api.Plan(A, beta, precision=precision)
    assert plan.info["jump_probability"] == pytest.approx(np.mean(-np.expm1(-beta * r)), rel=1e-12)
    assert plan.info["screened"] == 1
    plan.close()
    assert _check_level_sums(api, A, beta, u, precision, 4, 4096, seed=21)
    assert _check_level_sums(api, A, beta, u, precision, 4, 777, seed=22, walk0=5)


def test_level_sums_multi_rhs_screened_full_ranges(api):
    """16384 rows with 4096 walks each: every wave screens one whole 4096-walk range (64
    walks per lane, the most a screened range holds), 3 right-hand sides, FP32 weights."""
    A = inputs.barabasi_albert(16384, 3, seed=8)
    beta = 1.0 / float(np.diff(A.row_ptr).max())
    u = inputs.rhs_ones_rademacher(A.n, 3, seed=9)
    assert _check_level_sums(api, A, beta, u, "fp32", 2, 4096, seed=23, values_dtype=np.float32)


@pytest.mark.parametrize("precision,M", [("fp64", 1), ("fp32", 5), ("fp64", 8), ("fp32", 17),
                                         ("fp32", 32), ("fp64", 40), ("fp32", 63)])
def test_level_sums_few_walks_per_row(api, precision, M):
    """Items of fewer than 64 walks share a wave (groups of 1..32 lanes per row): sums,
    jumps and path hashes per row as the oracle's, on rows that do and do not fill a wave."""
    a = _signed(150, 21, density=0.05, scale=2.0)
    A = inputs.from_dense(a)
    u = np.random.default_rng(5).normal(size=150)
    _check_level_sums(api, A, 0.5, u, precision, 3, M, seed=19, walk0=M * 3)


def test_level_sums_full_size_laplace2d_sampled_rows(api):
    """The 256 x 256 workload at its full size, in the launch configuration of the
    benchmark, on 384 sampled rows (FP32 weights, levels 2..7)."""
    A, t, v = inputs.workload_laplace2d(256)
    rows = np.random.default_rng(8).choice(A.n, size=384, replace=False)
    _check_level_sums(api, A, t, v, "fp32", 6, 256, seed=77, rows=rows)


def test_walk_ranges_split_exactly(api):
    """Walks are addressed by counters: [0, M) = [0, a) + [a, M) in counts and sums."""
    A, t, v = inputs.workload_laplace1d()
    plan = api.Plan(A, t, precision="fp64")
    u = torch.as_tensor(v, device="cuda")
    lev = plan.l0 + 1
    s1, s2, j = plan.level_sums(u, lev, 0, 5000, seed=1)
    a1, a2, ja = plan.level_sums(u, lev, 0, 1234, seed=1)
    b1, b2, jb = plan.level_sums(u, lev, 1234, 5000 - 1234, seed=1)
    assert j == ja + jb
    assert torch.allclose(s1, a1 + b1, rtol=1e-13, atol=1e-15)
    plan.close()


def test_run_fixed_schedule_matches_oracle(api):
    A, t, v = inputs.workload_laplace1d()
    walks = [8000, 4000, 2000, 1000]
    plan = api.Plan(A, t, precision="fp64")
    x, st = plan.run(torch.as_tensor(v, device="cuda"), walks=walks, seed=31)
    tt = _tables(A)
    res = orc.mlmc_fixed(tt, t, v, plan.l0, plan.l0 + 3, walks, seed=31)
    assert st["steps"] == res.steps
    assert st["total_jumps"] == res.jumps
    assert st["walks"] == walks
    xg = x.cpu().numpy()[:, 0]
    assert np.all(np.abs(xg - res.x[:, 0]) <= 1e-12 * res.mass[:, 0])
    plan.close()


@pytest.mark.parametrize("vdtype", [torch.float64, torch.float32])
def test_plan_from_a_device_matrix_equals_the_host_one(api, vdtype):
    """A CSR matrix handed over in device memory builds the same plan as the same arrays on
    the host: identical plan facts and bit-identical estimates; an FP64 run matches the
    oracle."""
    A, t, v = inputs.workload_laplace1d()
    walks = [4000, 2000, 1000]
    ndt = np.float64 if vdtype == torch.float64 else np.float32
    host = api.Plan(A, t, precision="fp64", values_dtype=ndt)

    class DevCSR:
        n = A.n
        row_ptr = torch.as_tensor(np.asarray(A.row_ptr, np.int64), device="cuda")
        col_idx = torch.as_tensor(np.asarray(A.col_idx, np.int32), device="cuda")
        values = torch.as_tensor(np.asarray(A.values, ndt), device="cuda")

    dev = api.Plan(DevCSR, t, precision="fp64")
    assert dev.info == host.info
    u = torch.as_tensor(v, device="cuda")
    xh, sh = host.run(u, walks=walks, seed=5)
    xd, sd = dev.run(u, walks=walks, seed=5)
    assert torch.equal(xh, xd)
    assert sh["total_jumps"] == sd["total_jumps"]
    if vdtype == torch.float64:
        res = orc.mlmc_fixed(_tables(A), t, v, dev.l0, dev.l0 + 2, walks, seed=5)
        assert np.all(np.abs(xd.cpu().numpy()[:, 0] - res.x[:, 0]) <= 1e-12 * res.mass[:, 0])
    host.close()
    dev.close()


def test_diagonal_matrix_and_empty_rows(api):
    d = np.array([-1.0, 0.0, 0.5, 2.0])
    A = inputs.from_dense(np.diag(d))
    u = np.array([1.0, 2.0, -3.0, 0.5])
    plan = api.Plan(A, 0.3, precision="fp64")
    x, st = plan.run(torch.as_tensor(u, device="cuda"), walks=[64, 64, 64], seed=1)
    assert st["total_jumps"] == 0
    assert np.allclose(x.cpu().numpy()[:, 0], np.exp(0.3 * d) * u, rtol=1e-14, atol=0)
    plan.close()
    empty = api.Plan(A, 0.3, precision="fp32", rows=np.zeros(0, np.int64))
    x, st = empty.run(torch.as_tensor(u, device="cuda"), walks=[64, 64], seed=1)
    assert x.shape == (0, 1) and st["steps"] == 0
    empty.close()


def test_adaptive_run_reaches_target(api):
    A, t, v = inputs.workload_laplace1d()
    plan = api.Plan(A, t, precision="fp64")
    eps = 1e-3
    x, st = plan.run(torch.as_tensor(v, device="cuda"), eps=eps, seed=2, pilot_walks=1000)
    assert st["converged"]
    assert st["est_variance"] <= eps * eps / 2 * 1.0001
    exact = reference.laplace1d_exact(v, t)
    rmse = math.sqrt(float(np.mean((x.cpu().numpy()[:, 0] - exact) ** 2)))
    _say(f"adaptive eps={eps}: rmse={rmse:.3e} levels={st['num_levels']} walks={st['walks']}")
    assert rmse < 3 * eps
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adaptive_run_equals_the_oracle_at_its_final_sample_sizes(api, precision):
    """Algorithm 1 adds walks to levels it already sampled: the added walk ranges are summed
    into the accumulators (straight from the kernel when a row's new walks form one chunk,
    through the partials otherwise). Walks are addressed by counters, so the final estimate
    equals the oracle's fixed-schedule estimate at the final sample sizes: same jumps, sums
    within the bars. 16384 rows, so each row's walks of a call form a single item."""
    A, t, v = inputs.workload_laplace2d(128)
    dt = np.float64 if precision == "fp64" else np.float32
    u = v.astype(dt)
    plan = api.Plan(A, t, precision=precision)
    x, st = plan.run(torch.as_tensor(u, device="cuda"), eps=3e-2, seed=12, pilot_walks=200,
                     max_levels=8)
    nl = st["num_levels"]
    walks = st["walks"][:nl]
    _say(f"adaptive {precision}: levels {nl}, walks {walks}")
    assert any(w > 200 for w in walks)          # Algorithm 1 added walks after the pilot
    tt = _tables(A)
    res = orc.mlmc_fixed(tt, t, u.astype(np.float64), plan.l0, plan.l0 + nl - 1, walks, seed=12)
    assert st["total_jumps"] == res.jumps
    xg = x.cpu().numpy()[:, 0]
    assert np.all(np.abs(xg - res.x[:, 0]) <= TOL[precision] * res.mass[:, 0] + 1e-300)
    plan.close()


def test_adaptive_run_takes_the_oracles_levels_and_sample_sizes(api):
    """Algorithm 1's decisions: on a chain whose splitting bias at the pilot's finest level
    is 1.25 eps / sqrt(2) (dense truth; beta r_max = 16, l0 = 0), the FP64 GPU run must add
    the same level as the oracle's driver and end with the same walks per level (a sample
    size may differ by one walk where a rounded optimum falls on an integer), and its
    estimate must equal the oracle's at those sizes within the FP64 bar."""
    A, u = inputs.small_chain(20, 7, False, 0.5, 0.3)
    beta = 16.0
    a = A.to_dense()
    x_true = reference.expm_action(a, u, beta)
    bias4 = math.sqrt(float(np.mean((reference.strang_level(a, u, beta, 4) - x_true) ** 2)))
    eps = bias4 * math.sqrt(2.0) / 1.25
    tt = _tables(A)
    res = orc.mlmc_adaptive(tt, beta, u, eps, seed=5, l0=0, pilot=256)
    want = [st.M for st in res.levels]
    plan = api.Plan(A, beta, precision="fp64", l0=0)
    x, st = plan.run(torch.as_tensor(u, device="cuda"), eps=eps, seed=5, pilot_walks=256)
    nl = st["num_levels"]
    got = list(st["walks"][:nl])
    _say(f"adaptive bias case: gpu levels {nl} walks {got}; oracle levels {len(want)} walks {want}")
    assert st["converged"] and res.converged
    assert nl == len(want) == 6
    assert all(abs(g - w) <= 1 for g, w in zip(got, want)), (got, want)
    ref = res if got == want else orc.mlmc_fixed(tt, beta, u, 0, nl - 1, got, seed=5)
    xg = x.cpu().numpy()[:, 0]
    assert np.all(np.abs(xg - ref.x[:, 0]) <= TOL["fp64"] * ref.mass[:, 0] + 1e-300)
    assert st["est_bias"] <= eps / math.sqrt(2.0)
    plan.close()


def test_classical_single_level_mc_estimates_the_finest_strang_product(api):
    """Classical Monte Carlo is the base estimator at one fine level L: a plan with l0 = L
    and one level. Its expectation is the Strang product x^L, the same as that of MLMC on
    l0..L (section 2.2's telescoping sum), checked here against the dense product row by row
    and against an MLMC run with independent streams."""
    a = _signed(40, 33, density=0.2, scale=0.5)
    A = inputs.from_dense(a)
    beta = 0.6
    u = np.random.default_rng(8).normal(size=40)
    ut = torch.as_tensor(u, device="cuda")
    mlmc_plan = api.Plan(A, beta, precision="fp64")
    L = mlmc_plan.l0 + 3
    mc_plan = api.Plan(A, beta, precision="fp64", l0=L)
    assert mc_plan.l0 == L
    M = 200_000
    x_mc, st_mc = mc_plan.run(ut, walks=[M], seed=3)
    s1, s2, _ = mc_plan.level_sums(ut, L, 0, M, seed=3)
    mean = s1.cpu().numpy()[:, 0] / M
    assert np.allclose(mean, x_mc.cpu().numpy()[:, 0], rtol=1e-13, atol=1e-300)
    se = np.sqrt(np.maximum(s2.cpu().numpy()[:, 0] / M - mean ** 2, 0.0) / M)
    exact_L = reference.strang_level(a, u, beta, L)
    z = (mean - exact_L) / se
    x_ml, st_ml = mlmc_plan.run(ut, walks=[M, M // 4, M // 16, M // 64], seed=4)
    _say(f"classical MC at level {L}: max |z| {np.abs(z).max():.2f}, mean z^2 {np.mean(z * z):.2f}, "
         f"steps {st_mc['steps']:.3e}; MLMC steps {st_ml['steps']:.3e}")
    assert np.abs(z).max() < 5.0 and 0.3 < np.mean(z * z) < 2.0
    d = mean - x_ml.cpu().numpy()[:, 0]
    assert np.sqrt(np.mean(d ** 2)) < 5 * np.sqrt(st_mc["est_variance"] + st_ml["est_variance"])
    assert st_mc["steps"] == M * 40 * (1 << L)
    mc_plan.close()
    mlmc_plan.close()


def test_adaptive_run_with_the_default_pilot_takes_the_oracles_decisions(api):
    """pilot_walks = 0 lets the driver size M0 from the row count (at least 2^18 samples per
    pilot level: 2622 walks per row for 100 rows); with the variance estimate made unbiased
    and the level terms' root mean square freed of the sampling noise, the FP64 GPU run must
    take the oracle's levels and sample sizes (each within one walk) and reach the target."""
    A, t, v = inputs.workload_laplace1d()
    tt = _tables(A)
    eps = 1e-3
    res = orc.mlmc_adaptive(tt, t, v, eps, seed=9, pilot=0)
    want = [st.M for st in res.levels]
    plan = api.Plan(A, t, precision="fp64")
    x, st = plan.run(torch.as_tensor(v, device="cuda"), eps=eps, seed=9, pilot_walks=0)
    nl = st["num_levels"]
    got = list(st["walks"][:nl])
    _say(f"default pilot: gpu levels {nl} walks {got}; oracle walks {want}")
    assert st["converged"] and res.converged
    assert nl == len(want)
    assert all(abs(g - w) <= 1 for g, w in zip(got, want)), (got, want)
    assert min(got) >= 2622
    exact = reference.laplace1d_exact(v, t)
    assert float(np.sqrt(np.mean((x.cpu().numpy()[:, 0] - exact) ** 2))) < 2 * eps
    plan.close()

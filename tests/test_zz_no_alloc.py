"""The allocation-free level sums (mlmc_expv_level_sums_noalloc) against mlmc_expv_level_sums.

Both run the same walks (same items, same kernels); they differ in where the per-(row,
chunk) partial sums of a launch live and therefore in how the walks are split into
launches, so the FP64 chunk sums may be added in another order. Bars:
  - jump counts and the per-row sums of the path hashes: bit-exact (integer sums);
  - sum Y: within tol * sqrt(M * sum Y^2), a bound on the row's absolute mass sum |Y|
    (Cauchy-Schwarz), tol = 1e-12 for FP64 weights and for FP32 weights alike (the per-item
    partials are the same bits in both; only their FP64 additions are reordered);
  - sum Y^2 (a sum of non-negative terms): within tol relative.
The plan's device memory must not grow in an allocation-free call, and a level whose tables
were never built is refused.
"""
import math
import sys

import numpy as np
import pytest
import torch

from paper_1904_12754_amd import inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1904_12754_amd import api as _api
    return _api


def _compare(plan, u, level, walk0, walks, seed):
    _say(f"noalloc vs level_sums: n={plan.n} nrhs={u.shape[1] if u.dim() > 1 else 1} "
         f"level={level} walk0={walk0} walks={walks}")
    before = plan.current_info()["device_bytes"]
    a1, a2, ja, ha = plan.level_sums(u, level, walk0, walks, seed=seed, hashes=True, noalloc=True)
    torch.cuda.synchronize()
    assert plan.current_info()["device_bytes"] == before
    b1, b2, jb, hb = plan.level_sums(u, level, walk0, walks, seed=seed, hashes=True)
    torch.cuda.synchronize()
    assert ja == jb and ja > 0
    assert torch.equal(ha, hb)
    a1, a2, b1, b2 = (t.cpu().numpy() for t in (a1, a2, b1, b2))
    bound = np.sqrt(walks * np.maximum(b2, 0.0))
    assert np.all(np.abs(a1 - b1) <= TOL * bound + 1e-300)
    assert np.all(np.abs(a2 - b2) <= TOL * b2 + 1e-300)
    assert np.any(a1 != 0.0)


def test_noalloc_fp64_many_rhs_then_smaller(api):
    A, t, v = inputs.workload_laplace1d()
    rng = np.random.default_rng(3)
    U = torch.as_tensor(rng.normal(size=(A.n, 256)), device="cuda")
    with api.Plan(A, t, precision="fp64") as plan:
        lev = plan.l0 + 1
        # the level's tables are not built yet: refused, nothing launched
        with pytest.raises(Exception, match="not built"):
            plan.level_sums(U, lev, 0, 64, seed=1, noalloc=True)
        plan.trace(lev, np.zeros(1, np.int64), np.zeros(1, np.uint32), seed=1)   # builds it
        # 256 right-hand sides and 20000 walks per row: the partials of all 157 chunks of
        # the 100 rows exceed the fixed scratch, so the walks run as two launches there
        _compare(plan, U, lev, 5, 20000, seed=7)
        # a second call with a smaller input on the same plan (and the same scratch)
        _compare(plan, U[:, :3], plan.l0, 0, 3001, seed=8)


def test_noalloc_fp32_fresh_plan_then_smaller(api):
    A, t, v = inputs.workload_laplace2d(64)
    u = torch.as_tensor(v.astype(np.float32), device="cuda")
    with api.Plan(A, t, precision="fp32") as plan:
        # a fresh plan has no partial buffer yet; the allocation-free call must not add one
        _compare(plan, u, plan.l0, 0, 4096, seed=11)
        _compare(plan, u, plan.l0, 4096, 100, seed=11)


def test_noalloc_single_chunk_writes_directly(api):
    A, t, v = inputs.workload_laplace2d(32)
    u = torch.as_tensor(v.astype(np.float32), device="cuda")
    rows = np.arange(0, A.n, 3)
    with api.Plan(A, t, precision="fp32", rows=rows) as plan:
        _compare(plan, u, plan.l0, 0, 40, seed=2)

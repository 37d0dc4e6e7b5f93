"""Pins of the oracle's Algorithm 3 (the inhomogeneous system x' = A x + F with constant F,
solved as exp(beta A) u + int_0^beta exp(sA) F ds with the composite Simpson rule over the
walk's grid times). CPU only."""
import numpy as np
import pytest

from oracle import mlmc, reference
from paper_1904_12754_amd import inputs


def _sparse_signed(n, seed, per_row=4, scale=1.0):
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n))
    for i in range(n):
        cols = rng.choice([j for j in range(n) if j != i], size=per_row, replace=False)
        a[i, cols] = rng.normal(size=per_row) * scale
        a[i, i] = rng.normal() * scale
    return a


def test_simpson_weights_integrate_cubics_exactly():
    w = reference.simpson_weights(8)
    x = np.linspace(0.0, 2.0, 9)
    for k in range(4):
        assert abs((2.0 / 8) / 3.0 * np.sum(w * x ** k) - 2.0 ** (k + 1) / (k + 1)) < 1e-12


def test_diagonal_matrix_gives_the_simpson_sum_with_zero_variance():
    """No jumps: every walk returns e^{beta d} u + (dt/3) sum_n w_n e^{n dt d} F, the
    Simpson rule for int_0^beta e^{s d} F ds, within the rule's error bound of the
    integral's closed form F (e^{beta d} - 1) / d."""
    d = np.array([-2.0, 0.0, 0.7, -0.3])
    u = np.array([1.0, -2.0, 0.5, 3.0])
    F = np.array([0.25, 1.5, -1.0, 2.0])
    A = inputs.from_dense(np.diag(d))
    t = mlmc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    beta = 0.9
    for level in (1, 3, 5):
        ls = mlmc.level_sums(t, beta, level, level, 7, u, None, 0, 16, F=F)
        mean = ls.sum1[:, 0] / 16
        assert np.allclose(ls.sum2[:, 0] / 16, mean ** 2, rtol=1e-12)
        N = 1 << level
        dt = beta / N
        w = reference.simpson_weights(N)
        simpson = np.array([dt / 3 * np.sum(w * np.exp(np.arange(N + 1) * dt * di)) * Fi
                            for di, Fi in zip(d, F)])
        assert np.allclose(mean, np.exp(beta * d) * u + simpson, rtol=1e-12, atol=1e-14)
        exact = np.where(d != 0, F * np.expm1(beta * d) / np.where(d != 0, d, 1.0), F * beta)
        bound = beta * dt ** 4 * np.max(np.abs(d)) ** 4 * np.exp(beta * np.abs(d)) * np.abs(F) / 180
        assert np.all(np.abs(simpson - exact) <= bound + 1e-15)


@pytest.mark.parametrize("seed", [3, 4])
def test_level_means_match_the_dense_algorithm3_products(seed):
    """Each level's sample has the expectation of the dense products: the fine sum
    S^N u + (dt/3) sum w_n S^n F at l0 and its difference with level l - 1 above (the
    coarse Simpson sum on even points has the law of the level below)."""
    a = _sparse_signed(9, seed, scale=0.8)
    A = inputs.from_dense(a)
    t = mlmc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    beta = 0.5
    l0 = max(1, mlmc.default_l0(t, beta))
    rng = np.random.default_rng(seed)
    u = rng.normal(size=9)
    F = rng.normal(size=9)
    exact = reference.source_level_means(a, u, F, beta, l0, l0 + 2)
    z = []
    for q, lev in enumerate(range(l0, l0 + 3)):
        ls = mlmc.level_sums(t, beta, lev, l0, 11 + q, u, None, 0, 40_000, F=F)
        M = ls.walks
        mean = ls.sum1[:, 0] / M
        se = np.sqrt(np.maximum(ls.sum2[:, 0] / M - mean ** 2, 0) / M)
        ok = se > 1e-12
        z.append((mean[ok] - exact[q][ok]) / se[ok])
    z = np.concatenate(z)
    assert np.max(np.abs(z)) < 5.0
    assert 0.4 < np.mean(z * z) < 1.8


def test_source_term_alone_converges_to_the_integral():
    """u = 0: MLMC on l0..l0+3 estimates int_0^beta exp(sA) F ds within its error plus the
    O(dt^2) bias of the finest level (1D Laplacian)."""
    n = 30
    A = inputs.laplacian_1d(n)
    a = A.to_dense()
    beta = 0.5 / A.norm1()
    t = mlmc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    l0 = max(1, mlmc.default_l0(t, beta))
    F = np.sin(np.pi * np.arange(1, n + 1) / (n + 1)) + 0.3
    res = mlmc.mlmc_fixed(t, beta, np.zeros(n), l0, l0 + 3, [60_000, 20_000, 8_000, 4_000], 5, F=F)
    exact = reference.inhomogeneous_exact(a, np.zeros(n), F, beta)
    xL = reference.source_level(a, np.zeros(n), F, beta, l0 + 3)
    var = sum(st.var[:, 0] / st.M for st in res.levels)
    err = np.abs(res.x[:, 0] - exact)
    assert np.all(err <= 5 * np.sqrt(var) + 2 * np.abs(xL - exact) + 1e-12)
    assert np.max(np.abs(xL - exact)) < 1e-3 * np.max(np.abs(exact))

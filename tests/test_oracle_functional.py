"""Pins of the oracle's scalar functional (w, exp(beta A) u) by walks from random start rows
(the full-vector representation of section 2.1 summed against w): the start law, and the
level expectations against dense products on A^T. CPU only."""
import numpy as np
import pytest
import scipy.stats

from oracle import mlmc, reference
from paper_1904_12754_amd import inputs


def test_start_rows_follow_abs_u():
    """A = 0: no jumps, eta = 1, so with w = e_k the sum of the samples is sign(u_k) times
    the number of walks started at k: chi-square against M |u_k| / U, never at u_k = 0."""
    u = np.array([1.0, -2.0, 3.0, 0.5, 0.0, 4.0, -1.0])
    n = u.size
    A = inputs.from_dense(np.zeros((n, n)))
    t = mlmc.decompose(n, A.row_ptr, A.col_idx, A.values)
    M = 200_000
    counts = []
    for k in range(n):
        w = np.zeros(n)
        w[k] = 1.0
        fs = mlmc.functional_sums(t, 0.5, 0, 0, 3, u, w, 0, M)
        assert fs.sum1 == np.sign(u[k]) * abs(fs.sum1)
        counts.append(abs(fs.sum1))
    counts = np.array(counts)
    assert counts.sum() == M and counts[4] == 0
    p = np.abs(u) / np.abs(u).sum()
    ok = p > 0
    chi2 = np.sum((counts[ok] - M * p[ok]) ** 2 / (M * p[ok]))
    assert scipy.stats.chi2.sf(chi2, ok.sum() - 1) > 1e-3


@pytest.mark.parametrize("sym", [False, True])
def test_level_means_match_dense_products_on_the_transpose(sym):
    """U * mean of the level samples estimates (u, S^N w) - (u, S'^{N/2} w) with S the
    Strang step of A^T: z-tests over levels l0..l0+2 (nonsymmetric signed A, signed u, w;
    and a symmetric adjacency matrix with u = w = 1, the total communicability)."""
    rng = np.random.default_rng(7 if sym else 8)
    n = 12
    if sym:
        a = (rng.random((n, n)) < 0.35).astype(float)
        a = np.triu(a, 1)
        a = a + a.T
        u = np.ones(n)
        w = np.ones(n)
        beta = 1.0 / a.sum(axis=1).max()
    else:
        a = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.4)
        u = rng.normal(size=n)
        w = rng.normal(size=n)
        beta = 0.3
    AT = inputs.from_dense(a.T)
    tT = mlmc.decompose(n, AT.row_ptr, AT.col_idx, AT.values)
    l0 = mlmc.default_l0(tT, beta)
    xs = [float(u @ reference.strang_level(a.T, w, beta, l)) for l in range(l0, l0 + 3)]
    exact = [xs[0], xs[1] - xs[0], xs[2] - xs[1]]
    z = []
    for q, lev in enumerate(range(l0, l0 + 3)):
        fs = mlmc.functional_sums(tT, beta, lev, l0, 30 + q, u, w, 0, 120_000)
        m = fs.sum1 / fs.walks
        v = max(fs.sum2 / fs.walks - m * m, 0.0)
        se = fs.U * np.sqrt(v / fs.walks)
        if se > 1e-13:
            z.append((fs.U * m - exact[q]) / se)
    assert len(z) >= 2
    assert np.max(np.abs(z)) < 4.5
    est, var = mlmc.functional_fixed(tT, beta, u, w, l0, l0 + 2, [120_000, 40_000, 20_000], 5)
    assert abs(est - xs[2]) < 5 * np.sqrt(var)
    if sym:
        tc = float(np.ones(n) @ reference.expm_action(a, np.ones(n), beta))
        assert abs(est - tc) < 5 * np.sqrt(var) + abs(xs[2] - tc)


def _signed_case(seed, n):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, n)) * (rng.random((n, n)) < 0.4)
    u = rng.normal(size=n)
    AT = inputs.from_dense(a.T)
    tT = mlmc.decompose(n, AT.row_ptr, AT.col_idx, AT.values)
    return rng, a, u, tT


def test_forward_deposits_give_every_functional():
    """The forward representation of the full vector deposits each walk's sample at its
    final state. Against any w the deposits give the scalar functional's samples of the same
    walks: equal jumps and path hashes, and sum_j w_j sum1[j] equal to the functional's sum
    within the rounding of the two summation orders; the deposit counts add up to M."""
    rng, a, u, tT = _signed_case(21, 11)
    beta = 0.3
    l0 = mlmc.default_l0(tT, beta)
    for lev in (l0, l0 + 2):
        fs = mlmc.forward_sums(tT, beta, lev, l0, 44, u, 5, 30_000)
        assert fs.count.sum() == 30_000 and np.all(fs.mass >= np.abs(fs.sum1))
        ws = [rng.normal(size=tT.n), np.ones(tT.n)] + [np.eye(tT.n)[k] for k in (0, 4, 9)]
        for w in ws:
            f = mlmc.functional_sums(tT, beta, lev, l0, 44, u, w, 5, 30_000)
            assert f.jumps == fs.jumps and f.hash_sum == fs.hash_sum
            scale = float(np.abs(w) @ fs.mass) + 1e-300
            assert abs(float(w @ fs.sum1) - f.sum1) <= 1e-12 * scale


def test_forward_level_means_match_dense_strang_products():
    """U sum1[j] / M estimates the level term of ((S^N)^T u)_j = (u, S^N e_j), S the Strang
    step of A^T with the splitting of A^T (the walks' generator; it is not the transpose of
    A's Strang step, as the rates are column sums, and the two agree only in the limit):
    per-entry z-tests at levels l0..l0+2 on a signed nonsymmetric A, and the fixed-schedule
    estimate within 5 sigma of the finest product in every entry."""
    rng, a, u, tT = _signed_case(8, 10)
    beta = 0.3
    l0 = mlmc.default_l0(tT, beta)
    eye = np.eye(tT.n)
    xs = [np.column_stack([reference.strang_level(a.T, eye[j], beta, l) for j in range(tT.n)]).T @ u
          for l in range(l0, l0 + 3)]
    exact = [xs[0], xs[1] - xs[0], xs[2] - xs[1]]
    z = []
    for q, lev in enumerate(range(l0, l0 + 3)):
        fs = mlmc.forward_sums(tT, beta, lev, l0, 60 + q, u, 0, 150_000)
        m = fs.sum1 / fs.walks
        v = np.maximum(fs.sum2 / fs.walks - m * m, 0.0)
        se = fs.U * np.sqrt(v / fs.walks)
        ok = se > 1e-13
        z.extend(((fs.U * m - exact[q])[ok] / se[ok]).tolist())
    assert len(z) >= 20
    assert np.max(np.abs(z)) < 5.0
    est, var = mlmc.forward_fixed(tT, beta, u, l0, l0 + 2, [150_000, 50_000, 20_000], 9)
    assert np.all(np.abs(est - xs[2]) < 5 * np.sqrt(var) + 1e-13)

"""Pins of the oracle's learned-proposal reference (CPU only): analytic gradients against
finite differences, the defensive mixture, and unbiasedness of the importance-sampled MLMC
levels against the dense Strang products for an arbitrary proposal."""
import numpy as np
import pytest

from oracle import mlmc, proposal, reference
from paper_1904_12754_amd import inputs


def _sparse_signed(n, seed, per_row=4):
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n))
    for i in range(n):
        cols = rng.choice([j for j in range(n) if j != i], size=per_row, replace=False)
        a[i, cols] = rng.normal(size=per_row)
        a[i, i] = rng.normal()
    return a


def _batch(seed, B=40):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, proposal.NF))
    deg = rng.integers(1, proposal.NS + 1, size=B)
    valid = np.arange(proposal.NS)[None, :] < deg[:, None]
    p6 = np.where(valid, rng.random((B, proposal.NS)) + 0.05, 0.0)
    p6 /= p6.sum(axis=1, keepdims=True)
    slot = np.array([rng.integers(0, d) for d in deg])
    w = rng.exponential(size=B)
    return X, p6, valid, slot, w


@pytest.mark.parametrize("shrink", [0.0, 0.7])
def test_gradients_match_finite_differences(shrink):
    P = proposal.init_params(3)
    P["b3"][proposal.NS] = 0.3        # away from the tiny-alpha corner
    P["W3"] *= 10.0                   # corrections of order one
    X, p6, valid, slot, w = _batch(4)
    G, L0 = proposal.grads(P, X, p6, valid, slot, w, shrink)
    assert abs(L0 - proposal.loss(P, X, p6, valid, slot, w, shrink)) < 1e-14
    rng = np.random.default_rng(5)
    for key in proposal.ORDER:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in P[key].shape)
            h = 1e-6
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[key][idx] += h
            Pm[key][idx] -= h
            fd = (proposal.loss(Pp, X, p6, valid, slot, w, shrink) -
                  proposal.loss(Pm, X, p6, valid, slot, w, shrink)) / (2 * h)
            assert abs(fd - G[key][idx]) <= 1e-6 * max(1.0, abs(fd)), (key, idx, fd, G[key][idx])


def test_mixture_is_a_law_with_bounded_ratio():
    P = proposal.init_params(7)
    P["b3"][proposal.NS] = 4.0        # alpha near its maximum
    X, p6, valid, slot, w = _batch(8, B=200)
    q = proposal.forward(P, X, p6, valid)["q"]
    assert np.allclose(q.sum(axis=1), 1.0, atol=1e-12)
    assert np.all(q[~valid] == 0.0)
    assert np.all(q[valid] >= (1 - proposal.ALPHA_MAX) * p6[valid] * (1 - 1e-12))


def test_plain_tables_with_unit_ratio_reproduce_the_plain_walks():
    a = _sparse_signed(12, 2)
    C = inputs.from_dense(a)
    t = mlmc.decompose(C.n, C.row_ptr, C.col_idx, C.values)
    ti = t.with_proposal(t.slot_thr, t.slot_alias, np.ones_like(t.slot_probs()))
    u = np.random.default_rng(1).normal(size=12)
    for lev in (2, 3):
        a1 = mlmc.level_sums(t, 0.3, lev, 2, 9, u, None, 0, 500)
        a2 = mlmc.level_sums(ti, 0.3, lev, 2, 9, u, None, 0, 500)
        assert np.array_equal(a1.sum1, a2.sum1) and np.array_equal(a1.hash_sum, a2.hash_sum)


@pytest.mark.parametrize("seed", [11, 12])
def test_importance_sampled_levels_are_unbiased(seed):
    """Any proposal with the jump law's support leaves the level expectations equal to the
    dense Strang products (the IS weights p/q multiply both functionals)."""
    a = _sparse_signed(10, seed)
    C = inputs.from_dense(a)
    t = mlmc.decompose(C.n, C.row_ptr, C.col_idx, C.values)
    beta = 0.4
    l0 = mlmc.default_l0(t, beta)
    rng = np.random.default_rng(seed)
    u = rng.normal(size=10)
    P = proposal.init_params(seed)
    P["W3"] *= 30.0                   # a markedly different law
    P["b3"][proposal.NS] = 2.0
    xhat = rng.normal(size=10)
    levels = []
    for lev in range(l0, l0 + 3):
        q, thr, alias, ratio = proposal.proposal_tables(t, P, xhat, beta, lev, l0)
        assert np.max(np.abs(q - t.slot_probs())) > 0.05
        ti = t.with_proposal(thr, alias, ratio)
        ls = mlmc.level_sums(ti, beta, lev, l0, 21, u, None, 0, 60_000)
        levels.append(ls)
    exact = reference.level_means(a, u, beta, l0, l0 + 2)
    z = []
    for ls, m in zip(levels, exact):
        mean = ls.sum1[:, 0] / ls.walks
        var = np.maximum(ls.sum2[:, 0] / ls.walks - mean ** 2, 0)
        se = np.sqrt(var / ls.walks)
        ok = se > 1e-12
        z.append((mean[ok] - m[ok]) / se[ok])
    z = np.concatenate(z)
    assert np.max(np.abs(z)) < 5.0
    assert 0.4 < np.mean(z * z) < 1.8


def test_zero_correction_gives_the_value_ratio_prior():
    """With the network's outputs 0..5 at zero, softmax(z) is p_s times the value ratio
    (|xhat_j| + delta) / (|xhat_k| + delta), clipped to [e^-8, e^8], normalised over the
    row (without the clip the row's denominator cancels), and alpha = 0.9 sigmoid(b3[6])."""
    a = _sparse_signed(14, 6, per_row=5)
    C = inputs.from_dense(a)
    t = mlmc.decompose(C.n, C.row_ptr, C.col_idx, C.values)
    P = proposal.init_params(1)
    P["W3"][:] = 0.0
    P["b3"][:] = 0.0
    P["b3"][proposal.NS] = 1.3
    xhat = np.random.default_rng(2).normal(size=14)
    xhat[3] = 0.0
    q = proposal.proposal_tables(t, P, xhat, 0.2, 3, 1)[0]
    alpha = proposal.ALPHA_MAX / (1.0 + np.exp(-1.3))
    delta = 1e-6 * np.abs(xhat).max()
    p = t.slot_probs()
    for i in range(14):
        b, e = t.slot_begin[i], t.slot_begin[i + 1]
        ratio = (np.abs(xhat[t.slot_col[b:e]]) + delta) / (abs(xhat[i]) + delta)
        w = p[b:e] * np.clip(ratio, np.exp(-8.0), np.exp(8.0))
        expect = alpha * w / w.sum() + (1.0 - alpha) * p[b:e]
        assert np.allclose(q[b:e], expect, rtol=1e-12, atol=1e-15)


def test_shrinkage_is_the_weighted_square_of_the_corrections():
    """The penalty term alone, for a network whose corrections are known: with W1 = W2 = 0
    and b1 = b2 = 0 the hidden layers are zero, so output s is b3[s] for every row."""
    P = proposal.init_params(9)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        P[k][:] = 0.0
    P["b3"][:] = [0.5, -1.0, 0.25, 2.0, 0.0, 1.5, 0.3]
    X, p6, valid, slot, w = _batch(12, B=30)
    base = proposal.loss(P, X, p6, valid, slot, w, 0.0)
    with_pen = proposal.loss(P, X, p6, valid, slot, w, 0.4)
    per_row = np.array([sum(P["b3"][s] ** 2 for s in range(proposal.NS) if valid[b, s])
                        for b in range(len(w))])
    assert abs((with_pen - base) - 0.4 * (w * per_row).sum() / w.sum()) < 1e-13

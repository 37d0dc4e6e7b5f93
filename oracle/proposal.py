"""FP64 reference of the learned proposal (importance sampling of the jump law).

TEST INFRASTRUCTURE (see oracle/__init__.py).

The walks of the method jump from row k to the column of slot s with the law
p_s = |a_ks| / r_k (section 3, the jump law of the integral form of the backward
equation). Drawing the jump from another law q with the same support and multiplying the
path's functional by p_s / q_s at every jump leaves every level expectation unchanged
(importance sampling), so the MLMC estimator stays unbiased for any such q. The proposal
here is a small MLP of row features:

  features of row k (16): max(log p_s, -20) (6 slots),
                          clip(log((|xhat_{j_s}| + delta) / (|xhat_k| + delta)), -8, 8)
                          (6 slots), r_k dt, d_k dt, |xhat_k| / max|xhat|, (l - l0) / 8,
                          with delta = 1e-6 max|xhat| (slot features 0 past the row's slots)
  MLP: 16 -> 64 (ReLU) -> 64 (ReLU) -> 7
  q_s = alpha softmax_s(z) + (1 - alpha) p_s over the valid slots (s < deg_k <= 6),
        z_s = F_s + F_{6+s} + output s (the log-ratio prior plus the network's correction),
        alpha = ALPHA_MAX * sigmoid(output 6)

(the defensive mixture keeps q_s >= (1 - ALPHA_MAX) p_s, so p / q <= 10). With a
zero correction softmax(z) is p_s (|xhat_{j_s}| + delta) normalised over the row, the
variance-optimal law when the pilot estimate is exact and the walk makes one jump; the
network learns how far to trust it (alpha) and corrections to it. Rows with more
than six off-diagonal entries keep q = p. Training is the cross-entropy method: minimise
the |Y|-weighted negative log-likelihood of the jumps the plain walks took,
  L = - sum_b w_b log q_{s_b}(k_b) / sum_b w_b,  w_b = |Y| of the walk of jump b,
whose minimiser over all laws is q proportional to |Y| p, the variance-optimal proposal,
plus a shrinkage of the network's corrections towards the prior,
  + shrink * sum_b w_b sum_{s valid} (output s)^2 / sum_b w_b,
because the variance is far more sensitive to small logit errors than the loss is.
"""
from __future__ import annotations

import numpy as np

NF, NH, NO, NS = 16, 64, 7, 6
ALPHA_MAX = 0.9
LOG_P_MIN = -20.0       # floor of the log p_s features
LOG_RATIO_MAX = 8.0     # clip of the log value-ratio features


def init_params(seed: int) -> dict:
    """He-scaled normal weights, zero biases; the mixing output starts at alpha ~ 0.1."""
    rng = np.random.default_rng(seed)
    P = {
        "W1": rng.normal(size=(NF, NH)) * np.sqrt(2.0 / NF),
        "b1": np.zeros(NH),
        "W2": rng.normal(size=(NH, NH)) * np.sqrt(2.0 / NH),
        "b2": np.zeros(NH),
        "W3": rng.normal(size=(NH, NO)) * np.sqrt(1.0 / NH) * 0.1,
        "b3": np.zeros(NO),
    }
    P["b3"][NS] = -2.0
    return P


ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(P: dict) -> np.ndarray:
    return np.concatenate([np.asarray(P[k], np.float64).reshape(-1) for k in ORDER])


def unflatten(v) -> dict:
    v = np.asarray(v, np.float64)
    shapes = {"W1": (NF, NH), "b1": (NH,), "W2": (NH, NH), "b2": (NH,), "W3": (NH, NO), "b3": (NO,)}
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = v[o:o + n].reshape(shapes[k])
        o += n
    return out


def features(t, xhat, beta: float, level: int, l0: int):
    """Row features (n x 16), the plain law per slot (n x 6) and the valid-slot mask."""
    n = t.n
    deg = np.asarray(t.deg)
    sb = np.asarray(t.slot_begin)
    p_all = t.slot_probs()
    xabs = np.abs(np.asarray(xhat, np.float64))
    xmax = float(xabs.max()) if xabs.size and xabs.max() > 0 else 1.0
    dt = beta / 2.0 ** level
    F = np.zeros((n, NF))
    p6 = np.zeros((n, NS))
    valid = np.zeros((n, NS), bool)
    eligible = (deg >= 1) & (deg <= NS)
    delta = 1e-6 * xmax
    for s in range(NS):
        ok = eligible & (deg > s)
        idx = sb[:-1][ok] + s
        p6[ok, s] = p_all[idx]
        F[ok, s] = np.maximum(np.log(p_all[idx]), LOG_P_MIN)
        ratio = (xabs[np.asarray(t.slot_col)[idx]] + delta) / (xabs[ok] + delta)
        F[ok, NS + s] = np.clip(np.log(ratio), -LOG_RATIO_MAX, LOG_RATIO_MAX)
        valid[ok, s] = True
    F[:, 12] = np.asarray(t.r) * dt
    F[:, 13] = np.asarray(t.d) * dt
    F[:, 14] = xabs / xmax
    F[:, 15] = (level - l0) / 8.0
    return F, p6, valid, eligible


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def forward(P: dict, X, p6, valid):
    """q (B x 6) and the intermediate values."""
    X = np.asarray(X, np.float64)
    a1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(a2, 0.0)
    o = h2 @ P["W3"] + P["b3"]
    z = np.where(valid, o[:, :NS] + X[:, :NS] + X[:, NS:2 * NS], -np.inf)
    zmax = np.max(np.where(valid, z, -1e300), axis=1, keepdims=True)
    e = np.where(valid, np.exp(z - zmax), 0.0)
    den = e.sum(axis=1, keepdims=True)
    soft = np.where(valid, e / np.where(den > 0, den, 1.0), 0.0)
    sg = _sigmoid(o[:, NS])
    alpha = ALPHA_MAX * sg
    q = alpha[:, None] * soft + (1.0 - alpha[:, None]) * p6
    return {"X": X, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "o": o, "soft": soft,
            "sg": sg, "alpha": alpha, "q": q}


def _penalty(f, valid, w, shrink):
    corr = np.where(valid, f["o"][:, :NS], 0.0)
    return shrink * float((np.asarray(w) * (corr * corr).sum(axis=1)).sum())


def loss(P: dict, X, p6, valid, slot, w, shrink: float = 0.0) -> float:
    f = forward(P, X, p6, valid)
    qs = f["q"][np.arange(len(slot)), slot]
    ce = -(np.asarray(w) * np.log(qs)).sum()
    return float((ce + _penalty(f, valid, w, shrink)) / np.sum(w))


def grads(P: dict, X, p6, valid, slot, w, shrink: float = 0.0):
    """Analytic gradients of `loss` (same keys as P) and the loss value."""
    f = forward(P, X, p6, valid)
    B = len(slot)
    w = np.asarray(w, np.float64)
    W = w.sum()
    rows = np.arange(B)
    qs = f["q"][rows, slot]
    soft, alpha, sg = f["soft"], f["alpha"], f["sg"]
    # d(-w log q_s)/d z_j = -w alpha soft_s (delta_sj - soft_j) / q_s   (valid j); the prior
    # part of z does not depend on the parameters, so dz/d output is the identity
    coef = -(w / W) / qs
    dz = np.zeros((B, NS))
    onehot = np.zeros((B, NS))
    onehot[rows, slot] = 1.0
    dz = coef[:, None] * alpha[:, None] * soft[rows, slot][:, None] * (onehot - soft)
    dz = np.where(valid, dz + 2.0 * shrink * (w / W)[:, None] * f["o"][:, :NS], 0.0)
    # d/d output 6: (soft_s - p_s) * ALPHA_MAX * sg (1 - sg)
    da = coef * (soft[rows, slot] - p6[rows, slot]) * ALPHA_MAX * sg * (1.0 - sg)
    dO = np.concatenate([dz, da[:, None]], axis=1)
    G = {}
    G["W3"] = f["h2"].T @ dO
    G["b3"] = dO.sum(axis=0)
    dh2 = (dO @ P["W3"].T) * (f["a2"] > 0)
    G["W2"] = f["h1"].T @ dh2
    G["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"].T) * (f["a1"] > 0)
    G["W1"] = f["X"].T @ dh1
    G["b1"] = dh1.sum(axis=0)
    return G, float((-(w * np.log(qs)).sum() + _penalty(f, valid, w, shrink)) / W)


def proposal_tables(t, P: dict, xhat, beta: float, level: int, l0: int):
    """Per-slot proposal q for every row (q = p where the row is not eligible)."""
    from . import mlmc

    F, p6, valid, eligible = features(t, xhat, beta, level, l0)
    f = forward(P, F, p6, valid)
    q_slot = t.slot_probs().copy()
    deg = np.asarray(t.deg)
    sb = np.asarray(t.slot_begin)
    for s in range(NS):
        ok = eligible & (deg > s)
        q_slot[sb[:-1][ok] + s] = f["q"][ok, s]
    thr, alias = mlmc.alias_tables(t, q_slot)
    p_slot = t.slot_probs()
    ratio = np.where(q_slot > 0, p_slot / np.where(q_slot > 0, q_slot, 1.0), 1.0)
    return q_slot, thr, alias, ratio

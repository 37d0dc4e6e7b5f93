"""The learned proposal on the GPU, through the C-ABI:
  - BF16 matrix-core inference against an FP32 emulation of the same arithmetic (the MFMA
    operand layout) and against the oracle's FP64 network;
  - the alias tables and likelihood ratios built on the device are exactly the ones the
    oracle builds from the same proposal law;
  - walks under the proposal follow the oracle's paths bit-exactly, and their level sums
    agree with the oracle's within the plain method's bars;
  - the identity proposal reproduces the plain walks bit for bit;
  - the FP32 training gradients match the oracle's analytic FP64 gradients;
  - training on the GPU lowers the estimator variance without moving its mean;
  - the learned run (Algorithm 1 with the proposal trained on its own pilot) judges the
    proposal on exactly the pilot's walks, meets eps against the FP64 reference, and falls
    back to the plain law when the proposal loses.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import mlmc as orc
from oracle import proposal as prop
from oracle import reference as ref
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


def _convdiff(m, seed=3):
    A = inputs.convection_diffusion_3d(m, seed)
    return A, 4.0 / A.norm1(), inputs.rhs_gaussian_bump(m)


def _mixed(n=400, seed=5):
    """Rows of degree 1..12, so that some rows are past the six proposal slots."""
    return inputs.erdos_renyi(n, 5.0, seed)


def _params(seed, scale3=20.0, alpha_logit=1.5):
    P = prop.init_params(seed)
    P["W3"] = P["W3"] * scale3
    P["b3"][prop.NS] = alpha_logit
    return P


def _bf16(x):
    return torch.as_tensor(np.asarray(x, np.float32)).bfloat16().float()


def _kernel_features(t, xhat, beta, level, l0):
    """The network inputs exactly as the device forms them (FP32 arithmetic)."""
    n = t.n
    deg = np.asarray(t.deg)
    sb = np.asarray(t.slot_begin)
    p32 = t.slot_probs().astype(np.float32)
    xabs = np.abs(np.asarray(xhat, np.float64))
    xmax = float(xabs.max()) if xabs.max() > 0 else 1.0
    delta = 1e-6 * xmax
    dt = np.float32(beta / 2.0 ** level)
    F = np.zeros((n, prop.NF), np.float32)
    elig = (deg >= 1) & (deg <= prop.NS)
    col = np.asarray(t.slot_col)
    for s in range(prop.NS):
        ok = elig & (deg > s)
        idx = sb[:-1][ok] + s
        F[ok, s] = np.maximum(np.log(p32[idx].astype(np.float64)), prop.LOG_P_MIN)
        # the device forms the log value ratio as a difference of per-row logarithms
        lr = np.log(xabs[col[idx]] + delta) - np.log(xabs[ok] + delta)
        F[ok, prop.NS + s] = np.clip(lr, -prop.LOG_RATIO_MAX, prop.LOG_RATIO_MAX)
    r = np.asarray(t.r)
    with np.errstate(divide="ignore"):
        F[:, 12] = np.where(r > 0, (1.0 / (1.0 / r)).astype(np.float32) * dt, 0.0)
    F[:, 13] = np.asarray(t.d).astype(np.float32) * dt
    F[:, 14] = xabs / xmax
    F[:, 15] = np.float32(level - l0) / np.float32(8.0)
    return F


def _emulated_q(t, P, xhat, beta, level, l0):
    """q per slot from BF16 inputs, weights and hidden activations with FP32 sums."""
    F = _kernel_features(t, xhat, beta, level, l0)
    W = {k: torch.as_tensor(np.asarray(v, np.float32)) for k, v in P.items()}
    h1 = torch.relu(_bf16(F) @ _bf16(W["W1"]) + W["b1"])
    h2 = torch.relu(_bf16(h1) @ _bf16(W["W2"]) + W["b2"])
    o = (_bf16(h2) @ _bf16(W["W3"]) + W["b3"]).numpy()
    deg = np.asarray(t.deg)
    sb = np.asarray(t.slot_begin)
    p32 = t.slot_probs().astype(np.float32)
    q = p32.copy()
    for i in np.nonzero((deg >= 1) & (deg <= prop.NS))[0]:
        k = deg[i]
        z = o[i, :k] + (F[i, :k] + F[i, prop.NS:prop.NS + k])
        e = np.exp(z - z.max()).astype(np.float32)
        soft = e / e.sum(dtype=np.float32)
        alpha = np.float32(prop.ALPHA_MAX) / (np.float32(1.0) + np.exp(-o[i, prop.NS]))
        q[sb[i]:sb[i] + k] = alpha * soft + (np.float32(1.0) - alpha) * p32[sb[i]:sb[i] + k]
    return q


def _set(plan, P, xhat, nlev):
    plan.set_proposal(prop.flatten(P).astype(np.float32), xhat, num_levels=nlev)


@pytest.mark.parametrize("case", ["convdiff", "mixed"])
def test_inference_and_tables(api, case):
    if case == "convdiff":
        A, beta, _ = _convdiff(9)
    else:
        A = _mixed()
        beta = 0.3
    t = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    rng = np.random.default_rng(17)
    xhat = np.abs(rng.normal(size=A.n)) * (rng.random(A.n) < 0.7)
    P = _params(4, scale3=5.0)
    plan = api.Plan(A, beta, precision="fp32")
    l0 = plan.l0
    _set(plan, P, xhat, 3)
    deg = np.asarray(t.deg)
    sb = np.asarray(t.slot_begin)
    ns = int(sb[-1])
    slot_row = np.repeat(np.arange(A.n), deg)
    elig_slot = (deg[slot_row] <= prop.NS)
    plain_thr, plain_alias = t.slot_thr[:ns], t.slot_alias[:ns]
    for lev in (l0, l0 + 2):
        thr, alias, ratio, q = plan.proposal_tables(lev)
        # (1) against the FP32 emulation of the BF16 arithmetic: the operand layout
        qe = _emulated_q(t, P, xhat, beta, lev, l0)
        d_emul = np.abs(q - qe)
        # (2) against the oracle's FP64 network
        qo = prop.proposal_tables(t, P, xhat, beta, lev, l0)[0]
        d_orc = np.abs(q - qo)
        _say(f"{case} level {lev}: |q - emulated| max {d_emul.max():.2e} "
             f"p99 {np.quantile(d_emul, 0.99):.2e}; |q - fp64| max {d_orc.max():.2e}; "
             f"|q - p| max {np.abs(qo - t.slot_probs()).max():.2f}")
        assert np.quantile(d_emul, 0.99) <= 1e-5
        assert d_emul.max() <= 2e-3
        # BF16 inputs, weights and activations (relative rounding 2^-9 each, three layers)
        assert d_orc.max() <= 0.02
        assert np.abs(qo - t.slot_probs()).max() > 0.1      # a law well away from p
        # rows past six slots keep the plain law and tables
        assert np.array_equal(q[~elig_slot], t.slot_probs()[~elig_slot].astype(np.float32))
        assert np.array_equal(thr[~elig_slot], plain_thr[~elig_slot])
        assert np.array_equal(alias[~elig_slot], plain_alias[~elig_slot])
        # alias tables of the device's q: exactly the oracle's construction
        othr, oal = orc.alias_tables(t, q.astype(np.float64))
        assert np.array_equal(thr[elig_slot], othr[:ns][elig_slot])
        assert np.array_equal(alias[elig_slot], oal[:ns][elig_slot])
        # ratios p/q in FP32
        r32 = t.slot_probs().astype(np.float32) / q
        assert np.array_equal(ratio[elig_slot], r32[elig_slot])
        assert np.all(ratio <= np.float32(1.0 / (1.0 - prop.ALPHA_MAX)) * 1.0001)
        # every row's law sums to one
        sums = np.add.reduceat(q.astype(np.float64), sb[:-1][deg > 0])
        assert np.max(np.abs(sums - 1.0)) < 1e-5
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_walks_under_proposal_match_oracle(api, precision):
    A, beta, v = _convdiff(8)
    t = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    rng = np.random.default_rng(23)
    xhat = np.abs(rng.normal(size=A.n))
    P = _params(9)
    plan = api.Plan(A, beta, precision=precision)
    l0 = plan.l0
    _set(plan, P, xhat, 3)
    u = np.ascontiguousarray(v)
    ut = torch.as_tensor(u, device="cuda")
    for lev in range(l0, l0 + 3):
        thr, alias, ratio, q = plan.proposal_tables(lev)
        ti = t.with_proposal(thr, alias, ratio.astype(np.float64))
        # individual paths
        M = 1500
        rows = rng.integers(0, A.n, size=M)
        walks = (np.arange(M, dtype=np.uint64) * 104729 % (2 ** 32)).astype(np.uint32)
        _say(f"IS trace prec={precision} level={lev}")
        g = plan.trace(lev, rows, walks, seed=71)
        o = orc.walk_trace(ti, beta, lev, 71, rows, walks)
        assert np.array_equal(g["final_state"].cpu().numpy(), o.final_state)
        assert np.array_equal(g["sign"].cpu().numpy(), o.sign)
        assert np.array_equal(g["jumps"].cpu().numpy(), o.jumps)
        assert np.array_equal(g["hash"].cpu().numpy().view(np.uint64), o.hash)
        ref = np.log(np.abs(o.eta_fine))
        lf = g["log_eta_fine"].cpu().numpy()
        assert np.max(np.abs(lf - ref) / (1.0 + np.abs(ref))) < TOL[precision]
        assert o.jumps.sum() > 0
        # and the plain paths are different ones
        o_plain = orc.walk_trace(t, beta, lev, 71, rows, walks)
        assert not np.array_equal(o_plain.hash, o.hash)
        # level sums of the production kernel
        _say(f"IS level sums prec={precision} level={lev}")
        s1, s2, jumps, hs = plan.level_sums(ut, lev, 0, 700, seed=13, hashes=True)
        ol = orc.level_sums(ti, beta, lev, l0, 13, u, None, 0, 700)
        assert jumps == int(ol.jumps.sum())
        assert np.array_equal(hs.cpu().numpy().view(np.uint64), ol.hash_sum)
        assert np.all(np.abs(s1.cpu().numpy() - ol.sum1) <= TOL[precision] * (ol.mass + 1e-300))
        assert np.all(np.abs(s2.cpu().numpy() - ol.sum2) <= 4 * TOL[precision] * (ol.mass2 + 1e-300))
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_identity_proposal_is_the_plain_method(api, precision):
    A, beta, v = _convdiff(8)
    plan = api.Plan(A, beta, precision=precision)
    ut = torch.as_tensor(v, device="cuda")
    l0 = plan.l0
    plain = [plan.level_sums(ut, lev, 0, 900, seed=3, hashes=True) for lev in range(l0, l0 + 3)]
    plan.set_proposal(None, None, num_levels=3)
    ident = [plan.level_sums(ut, lev, 0, 900, seed=3, hashes=True) for lev in range(l0, l0 + 3)]
    for a, b in zip(plain, ident):
        assert a[2] == b[2]
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[3], b[3])
    thr, alias, ratio, q = plan.proposal_tables(l0)
    t = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    ns = int(t.slot_begin[-1])
    assert np.array_equal(thr, t.slot_thr[:ns]) and np.array_equal(alias, t.slot_alias[:ns])
    assert np.all(ratio == 1.0)
    # switching a learned proposal off gives the plain walks again
    _set(plan, _params(2), np.abs(v), 3)
    learned = plan.level_sums(ut, l0 + 1, 0, 900, seed=3, hashes=True)
    assert not torch.equal(learned[3], plain[1][3])
    plan.enable_proposal(False)
    off = plan.level_sums(ut, l0 + 1, 0, 900, seed=3, hashes=True)
    assert torch.equal(off[0], plain[1][0]) and torch.equal(off[3], plain[1][3])
    plan.close()


def test_training_gradients_match_oracle(api):
    A, beta, v = _convdiff(7)
    t = orc.decompose(A.n, A.row_ptr, A.col_idx, A.values)
    plan = api.Plan(A, beta, precision="fp32")
    rng = np.random.default_rng(31)
    xhat = np.abs(rng.normal(size=A.n))
    P = _params(6, scale3=5.0, alpha_logit=0.3)
    P = prop.unflatten(prop.flatten(P).astype(np.float32).astype(np.float64))
    B = 3000
    deg = np.asarray(t.deg)
    rows = rng.integers(0, A.n, size=B)
    slots = np.array([rng.integers(0, d) if d <= prop.NS and d > 0 else -1 for d in deg[rows]],
                     dtype=np.int32)
    slots[:7] = -1                                    # transitions that carry nothing
    w = rng.exponential(size=B).astype(np.float32)
    lev = plan.l0 + 1
    shrink = 0.5
    g, loss = plan.proposal_loss_grad(prop.flatten(P).astype(np.float32), xhat, lev, rows, slots, w,
                                      shrink=shrink)
    # oracle: FP64 network on the FP32 features the device forms
    F = _kernel_features(t, xhat, beta, lev, plan.l0).astype(np.float64)
    _, p6, valid, _ = prop.features(t, xhat, beta, lev, plan.l0)
    keep = slots >= 0
    G, L = prop.grads(P, F[rows[keep]], p6.astype(np.float32).astype(np.float64)[rows[keep]],
                      valid[rows[keep]], slots[keep], w[keep].astype(np.float64), shrink)
    # the oracle normalises by the weights of the kept transitions; the device by all
    L *= w[keep].sum(dtype=np.float64) / w.sum(dtype=np.float64)
    Gf = prop.flatten(G) * (w[keep].sum(dtype=np.float64) / w.sum(dtype=np.float64))
    err = np.abs(g - Gf)
    _say(f"loss gpu {loss:.8f} oracle {L:.8f}; grad max err {err.max():.2e} of max {np.abs(Gf).max():.2e}")
    assert abs(loss - L) <= 1e-5 * abs(L)
    assert err.max() <= 1e-4 * np.abs(Gf).max()
    off = 0
    for k in prop.ORDER:
        n = P[k].size
        assert np.abs(g[off:off + n] - Gf[off:off + n]).max() <= 1e-4 * np.abs(Gf[off:off + n]).max() + 1e-9, k
        off += n
    plan.close()


def test_training_lowers_variance_and_keeps_the_mean(api):
    A, beta, v = _convdiff(12)
    u = torch.as_tensor(np.asarray(v, np.float32), device="cuda")
    plan = api.Plan(A, beta, precision="fp32")
    nlev = 3
    walks = [2048, 512, 128]
    x0, st0 = plan.run(u, walks=walks, seed=101)
    P = prop.init_params(0)
    P["W3"][:] = 0.0                  # no correction to the value-ratio prior, and ...
    P["b3"][:] = 0.0
    P["b3"][prop.NS] = -2.0           # ... alpha = 0.11: close to the plain law
    P0 = prop.flatten(P).astype(np.float32)
    # the untrained proposal, for comparison
    _, t0st = plan.train_proposal(u, P0, seed=5, pilot_walks=256, capture_walks=64, steps=0,
                                  judge_walks=0, num_levels=nlev)
    xi, sti = plan.run(u, walks=walks, seed=303)
    params, tst = plan.train_proposal(u, P0, seed=5, pilot_walks=256, capture_walks=64,
                                      steps=400, batch=4096, lr=1e-2, shrink=10.0,
                                      num_levels=nlev, judge_walks=16)
    _say(f"training: {tst['transitions']} transitions ({tst['held_out']} held out), held-out "
         f"loss {tst['first_val_loss']:.5f} -> {tst['best_val_loss']:.5f} at step "
         f"{tst['best_step']}, {tst['train_ms']:.1f} ms")
    x1, st1 = plan.run(u, walks=walks, seed=202)
    v0 = np.array(st0["level_var"][:nlev])
    v1 = np.array(st1["level_var"][:nlev])
    _say(f"level variances plain {v0} learned {v1}; est var {st0['est_variance']:.3e} -> "
         f"{st1['est_variance']:.3e} (untrained {sti['est_variance']:.3e}); judge "
         f"{tst['judge_var_plain']:.3e} -> {tst['judge_var_learned']:.3e}")
    assert tst["best_val_loss"] <= tst["first_val_loss"]
    assert tst["held_out"] > 1000
    assert tst["accepted"] and tst["judge_var_learned"] < tst["judge_var_plain"]
    # training, not the initialisation, makes the gain
    assert st1["est_variance"] < 0.5 * sti["est_variance"]
    assert st1["est_variance"] < 0.5 * st0["est_variance"]
    # same finite-level estimator, independent samples: the difference is noise
    d = (x1 - x0).cpu().numpy()[:, 0]
    se = np.sqrt((st0["est_variance"] + st1["est_variance"]) / 1.0)
    _say(f"mean |x_learned - x_plain| {np.abs(d).mean():.3e}, pooled se {se:.3e}")
    assert abs(d.mean()) < 5 * se / np.sqrt(A.n) + 1e-12
    plan.close()


def _prior_params(alpha_logit=3.0, slot0=0.0):
    """Zero corrections (the value-ratio prior alone; slot0 adds a constant to the logit of
    every row's first slot) and alpha = 0.9 sigmoid(alpha_logit)."""
    P = prop.init_params(0)
    P["W3"][:] = 0.0
    P["b3"][:] = 0.0
    P["b3"][0] = slot0
    P["b3"][prop.NS] = alpha_logit
    return prop.flatten(P).astype(np.float32)


def _level_var(s1, s2, M):
    """Mean over rows of the unbiased per-walk variance, each row's clamped at 0 (what the
    run's judge reads)."""
    m = s1.double().cpu().numpy()[:, 0] / M
    raw = np.maximum(s2.double().cpu().numpy()[:, 0] / M - m * m, 0.0)
    return float(raw.mean() * M / (M - 1))


def _learned_case(api):
    A, beta, v = _convdiff(16)
    u = torch.as_tensor(np.asarray(v, np.float32), device="cuda")
    exact = ref.expm_action_sparse(A.n, A.row_ptr, A.col_idx, A.values, np.asarray(v, np.float64), beta)
    return A, beta, u, exact


LEARN = dict(pilot_walks=64, capture_walks=64, sample_stride=1, steps=16, batch=1024, lr=1e-2,
             shrink=10.0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_learned_run_trains_on_its_pilot_and_judges(api, precision):
    A, beta, u, exact = _learned_case(api)
    plan = api.Plan(A, beta, precision=precision)
    l0, eps, M0 = plan.l0, 2e-4, LEARN["pilot_walks"]
    xp, stp = plan.run(u, eps=eps, seed=7, pilot_walks=M0, max_levels=12)
    x, st, tst, params = plan.run_learned(u, eps, _prior_params(), seed=7, train_seed=3,
                                          max_levels=12, **LEARN)
    nl = st["num_levels"]
    _say(f"learned run: walks {st['walks'][:nl]} (plain {stp['walks'][:stp['num_levels']]}), "
         f"judge {tst['judge_var_plain']:.3e} -> {tst['judge_var_learned']:.3e}, best step "
         f"{tst['best_step']}, {tst['transitions']} transitions, {tst['train_ms']:.2f} ms")
    assert tst["accepted"] == 1 and tst["judge_var_learned"] < tst["judge_var_plain"]
    # the variance judge read exactly the pilot's level-l0 walks: plain, then the same walk indices
    # under the trained proposal (which the run leaves set and enabled)
    plan.enable_proposal(False)
    s1, s2, _ = plan.level_sums(u, l0, 0, M0, seed=7)
    assert tst["judge_var_plain"] == pytest.approx(_level_var(s1, s2, M0), rel=1e-12)
    plan.enable_proposal(True)
    s1, s2, _ = plan.level_sums(u, l0, 0, M0, seed=7)
    assert tst["judge_var_learned"] == pytest.approx(_level_var(s1, s2, M0), rel=1e-12)
    # the proposal's lower variance shows in the sample size at l0
    assert st["walks"][0] < stp["walks"][0]
    # the dropped plain pilot is counted in the steps, not in the walks
    steps = sum(st["walks"][q] * A.n * 2 ** (l0 + q) for q in range(nl)) + M0 * A.n * 2 ** l0
    assert st["steps"] == steps
    # eps against the FP64 reference
    est = np.sqrt(st["est_variance"] + st["est_bias"] ** 2)
    err = np.sqrt(np.mean((x.cpu().numpy()[:, 0] - exact) ** 2))
    err_p = np.sqrt(np.mean((xp.cpu().numpy()[:, 0] - exact) ** 2))
    _say(f"true rmse learned {err:.3e} (est {est:.3e}), plain {err_p:.3e}, eps {eps}")
    assert st["converged"] and est <= eps and err <= 1.5 * eps
    # reproducible: the same seeds give the same estimate and schedule
    x2, st2, tst2, p2 = plan.run_learned(u, eps, _prior_params(), seed=7, train_seed=3,
                                         max_levels=12, **LEARN)
    assert torch.equal(x, x2) and st2["walks"] == st["walks"]
    assert np.array_equal(params, p2)
    plan.close()


def test_learned_run_falls_back_to_the_plain_law(api):
    A, beta, u, exact = _learned_case(api)
    plan = api.Plan(A, beta, precision="fp32")
    eps, M0 = 2e-4, LEARN["pilot_walks"]
    # a law that sends most jumps to each row's first slot: far worse than the plain law
    bad = _prior_params(alpha_logit=3.0, slot0=8.0)
    x, st, tst, _ = plan.run_learned(u, eps, bad, seed=9, train_seed=3, max_levels=12,
                                     **dict(LEARN, steps=0))
    _say(f"rejected: judge {tst['judge_var_plain']:.3e} -> {tst['judge_var_learned']:.3e}, "
         f"walks {st['walks'][:st['num_levels']]}")
    assert tst["accepted"] == 0 and tst["judge_var_learned"] >= tst["judge_var_plain"]
    # the plain pilot's walks are kept and the proposal is left disabled: a later run is
    # the plain one, bit for bit
    assert st["walks"][0] >= M0
    xa, _ = plan.run(u, walks=[64, 16], seed=11)
    fresh = api.Plan(A, beta, precision="fp32")
    xb, _ = fresh.run(u, walks=[64, 16], seed=11)
    assert torch.equal(xa, xb)
    est = np.sqrt(st["est_variance"] + st["est_bias"] ** 2)
    err = np.sqrt(np.mean((x.cpu().numpy()[:, 0] - exact) ** 2))
    assert st["converged"] and est <= eps and err <= 1.5 * eps
    fresh.close()
    plan.close()


def test_learned_run_refuses_what_it_cannot_do(api):
    """The learned run is adaptive, reads one FP32 right-hand side, trains on a plan over all
    rows and sets tables for level l0 only; each of these is checked before any walk."""
    import ctypes
    from paper_1904_12754_amd import _abi

    A, beta, u, _ = _learned_case(api)
    P = _prior_params()
    plan = api.Plan(A, beta, precision="fp32")
    with pytest.raises(_abi.MLMCError) as e:
        plan.run_learned(u, 0.0, P)                      # not adaptive
    assert e.value.code == _abi.MLMC_ERR_INVALID_ARG
    with pytest.raises(_abi.MLMCError) as e:
        plan.run_learned(u.double(), 1e-3, P)            # FP64 right-hand side
    assert e.value.code == _abi.MLMC_ERR_UNSUPPORTED
    with pytest.raises(_abi.MLMCError) as e:
        plan.run_learned(u, 1e-3, P, capture_walks=0)    # training options out of range
    assert e.value.code == _abi.MLMC_ERR_INVALID_ARG
    # tables for more levels than l0: through the C-ABI, as the binding always asks for one
    lib = _abi.load()
    x = torch.empty((A.n, 1), dtype=torch.float64, device="cuda")
    Pp = np.ascontiguousarray(P, dtype=np.float32)
    opts = _abi.RunOpts(1, 0, 0, None, 1e-3, 0, 12, 0)
    topts = _abi.TrainOpts(0, Pp.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 0, 16, 1, 16,
                           1024, 1e-2, 10.0, 2, 0)
    code = lib.mlmc_expv_run_learned(plan._handle, ctypes.c_void_p(u.data_ptr()),
                                     _abi.MLMC_DTYPE_F32, ctypes.byref(opts), ctypes.byref(topts),
                                     None, ctypes.c_void_p(x.data_ptr()), None, None,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == _abi.MLMC_ERR_INVALID_ARG
    plan.close()
    # a plan over some rows only
    sub = api.Plan(A, beta, precision="fp32", rows=np.arange(0, A.n, 7))
    with pytest.raises(_abi.MLMCError) as e:
        sub.run_learned(u, 1e-3, P)
    assert e.value.code == _abi.MLMC_ERR_UNSUPPORTED
    sub.close()

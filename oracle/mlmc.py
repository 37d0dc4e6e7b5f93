"""ctypes binding of the oracle's C code, the MLMC combine and Algorithm 1.

TEST INFRASTRUCTURE (see oracle/__init__.py): never imported by the product path.

Paper sections followed:
  - the telescoping estimator x^L = E[P_l0] + sum_{l>l0} E[P_l - P_{l-1}] and its
    sample form (section 2.2, the MLMC estimate);
  - m_l and V_l per level from the samples (Algorithm 2's accumulators, read as the
    sample mean and the sample variance mean(Y^2) - mean(Y)^2);
  - Algorithm 1 (pilot run, optimal sample sizes, add a level until the error is
    below epsilon), with the optimal sample size read in Giles' form
    M_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)) and the error test read
    as Giles' variance and bias test with weak order alpha = 2 (the Strang splitting
    order of section 4).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _lib = ctypes.CDLL(path)
        _declare(_lib)
    return _lib


def _p(t):
    return ctypes.POINTER(t)


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_p(ctypes.c_uint32), _p(ctypes.c_uint32), _p(ctypes.c_uint32)]
    L.orc_philox4x32_10.restype = None
    L.orc_log.argtypes = [ctypes.c_double]
    L.orc_log.restype = ctypes.c_double
    L.orc_uniform.argtypes = [ctypes.c_uint32]
    L.orc_uniform.restype = ctypes.c_double
    L.orc_decompose.argtypes = [ctypes.c_int64, _p(ctypes.c_int64), _p(ctypes.c_int32),
                                _p(ctypes.c_double), _p(ctypes.c_double), _p(ctypes.c_double),
                                _p(ctypes.c_double), _p(ctypes.c_int64), _p(ctypes.c_int32),
                                _p(ctypes.c_int32), _p(ctypes.c_uint8), _p(ctypes.c_uint32),
                                _p(ctypes.c_int32)]
    L.orc_decompose.restype = ctypes.c_int
    tables = [_p(ctypes.c_double), _p(ctypes.c_double), _p(ctypes.c_int64), _p(ctypes.c_int32),
              _p(ctypes.c_int32), _p(ctypes.c_uint8), _p(ctypes.c_uint32), _p(ctypes.c_int32),
              _p(ctypes.c_uint32), _p(ctypes.c_int32), _p(ctypes.c_double)]
    L.orc_walk_trace.argtypes = tables + [ctypes.c_double, ctypes.c_int, ctypes.c_uint64,
                                          ctypes.c_uint32, ctypes.c_int64, _p(ctypes.c_int64),
                                          _p(ctypes.c_uint32), _p(ctypes.c_int64),
                                          _p(ctypes.c_int32), _p(ctypes.c_int64),
                                          _p(ctypes.c_uint64), _p(ctypes.c_double),
                                          _p(ctypes.c_double)]
    L.orc_walk_trace.restype = None
    L.orc_level_sums.argtypes = tables + [ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.c_uint32, _p(ctypes.c_double),
                                          _p(ctypes.c_double), ctypes.c_int32, ctypes.c_int64, _p(ctypes.c_int64),
                                          ctypes.c_uint32, ctypes.c_uint32, _p(ctypes.c_double),
                                          _p(ctypes.c_double), _p(ctypes.c_double),
                                          _p(ctypes.c_double), _p(ctypes.c_int64),
                                          _p(ctypes.c_uint64), ctypes.c_int32]
    L.orc_level_sums.restype = None
    L.orc_functional_sums.argtypes = tables[:8] + [
        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
        ctypes.c_int64, _p(ctypes.c_uint32), _p(ctypes.c_int32), _p(ctypes.c_uint8),
        _p(ctypes.c_double), ctypes.c_uint32, ctypes.c_uint32, _p(ctypes.c_double),
        _p(ctypes.c_double), _p(ctypes.c_int64), _p(ctypes.c_uint64)]
    L.orc_functional_sums.restype = None
    L.orc_forward_sums.argtypes = tables[:8] + [
        ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
        ctypes.c_int64, _p(ctypes.c_uint32), _p(ctypes.c_int32), _p(ctypes.c_uint8),
        ctypes.c_uint32, ctypes.c_uint32, _p(ctypes.c_double), _p(ctypes.c_double),
        _p(ctypes.c_double), _p(ctypes.c_int64), _p(ctypes.c_int64), _p(ctypes.c_uint64)]
    L.orc_forward_sums.restype = ctypes.c_int
    L.orc_log_array.argtypes = [ctypes.c_int64, _p(ctypes.c_double), _p(ctypes.c_double)]
    L.orc_log_array.restype = None
    L.orc_philox_array.argtypes = [ctypes.c_int64, _p(ctypes.c_uint32), _p(ctypes.c_uint32),
                                   _p(ctypes.c_uint32)]
    L.orc_philox_array.restype = None
    L.orc_alias_tables.argtypes = [ctypes.c_int64, _p(ctypes.c_int64), _p(ctypes.c_int32),
                                   _p(ctypes.c_double), _p(ctypes.c_uint32), _p(ctypes.c_int32)]
    L.orc_alias_tables.restype = None
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = ctypes.c_int


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(_p(t))


# ----------------------------------------------------------------------------------
# primitives
# ----------------------------------------------------------------------------------
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return out


def log(x: float) -> float:
    return lib().orc_log(float(x))


def log_array(x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    lib().orc_log_array(x.size, _ptr(x, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def philox_array(ctr, key) -> np.ndarray:
    """ctr: (q, 4) uint32, key: (q, 2) uint32 -> (q, 4) uint32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(c)
    lib().orc_philox_array(c.shape[0], _ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                           _ptr(out, ctypes.c_uint32))
    return out


def uniform(w: int) -> float:
    return lib().orc_uniform(int(w))


def max_threads() -> int:
    return lib().orc_max_threads()


# ----------------------------------------------------------------------------------
# decomposition A = D - T (section 2.1)
# ----------------------------------------------------------------------------------
@dataclass
class Tables:
    n: int
    r: np.ndarray
    d: np.ndarray
    inv_r: np.ndarray
    slot_begin: np.ndarray
    deg: np.ndarray
    slot_col: np.ndarray
    slot_sign: np.ndarray
    slot_thr: np.ndarray
    slot_alias: np.ndarray
    # importance sampling: proposal alias tables and per-slot likelihood ratios p/q
    q_thr: np.ndarray | None = None
    q_alias: np.ndarray | None = None
    q_ratio: np.ndarray | None = None

    def args(self):
        nil = lambda t: ctypes.cast(None, _p(t))
        return (_ptr(self.d, ctypes.c_double), _ptr(self.inv_r, ctypes.c_double),
                _ptr(self.slot_begin, ctypes.c_int64), _ptr(self.deg, ctypes.c_int32),
                _ptr(self.slot_col, ctypes.c_int32), _ptr(self.slot_sign, ctypes.c_uint8),
                _ptr(self.slot_thr, ctypes.c_uint32), _ptr(self.slot_alias, ctypes.c_int32),
                nil(ctypes.c_uint32) if self.q_thr is None else _ptr(self.q_thr, ctypes.c_uint32),
                nil(ctypes.c_int32) if self.q_alias is None else _ptr(self.q_alias, ctypes.c_int32),
                nil(ctypes.c_double) if self.q_ratio is None else _ptr(self.q_ratio, ctypes.c_double))

    def slot_probs(self) -> np.ndarray:
        """The plain jump law p per slot (|a_kj| / r_k), recomputed from the tables."""
        return np.asarray(self._p_slot)

    def with_proposal(self, q_thr, q_alias, q_ratio) -> "Tables":
        """The same tables walking under a proposal law (alias tables + ratios p/q)."""
        import copy
        t = copy.copy(self)
        t.q_thr = np.ascontiguousarray(q_thr, dtype=np.uint32)
        t.q_alias = np.ascontiguousarray(q_alias, dtype=np.int32)
        t.q_ratio = np.ascontiguousarray(q_ratio, dtype=np.float64)
        return t


def decompose(n: int, row_ptr, col, val) -> Tables:
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    nnz = int(row_ptr[-1])
    r = np.zeros(n, np.float64)
    d = np.zeros(n, np.float64)
    inv_r = np.zeros(n, np.float64)
    slot_begin = np.zeros(n + 1, np.int64)
    deg = np.zeros(n, np.int32)
    slot_col = np.zeros(max(nnz, 1), np.int32)
    slot_sign = np.zeros(max(nnz, 1), np.uint8)
    slot_thr = np.zeros(max(nnz, 1), np.uint32)
    slot_alias = np.zeros(max(nnz, 1), np.int32)
    rc = lib().orc_decompose(n, _ptr(row_ptr, ctypes.c_int64), _ptr(col, ctypes.c_int32),
                             _ptr(val, ctypes.c_double), _ptr(r, ctypes.c_double),
                             _ptr(d, ctypes.c_double), _ptr(inv_r, ctypes.c_double),
                             _ptr(slot_begin, ctypes.c_int64), _ptr(deg, ctypes.c_int32),
                             _ptr(slot_col, ctypes.c_int32), _ptr(slot_sign, ctypes.c_uint8),
                             _ptr(slot_thr, ctypes.c_uint32), _ptr(slot_alias, ctypes.c_int32))
    if rc != 0:
        raise MemoryError("oracle decomposition failed")
    t = Tables(n, r, d, inv_r, slot_begin, deg, slot_col, slot_sign, slot_thr, slot_alias)
    # plain jump law per slot, |a_kj| / r_k, in CSR slot order
    p_slot = np.zeros(max(int(slot_begin[-1]), 1), np.float64)
    for i in range(n):
        b, e = row_ptr[i], row_ptr[i + 1]
        cols, vals = col[b:e], val[b:e]
        keep = (cols != i) & (vals != 0.0)
        if keep.any():
            p_slot[slot_begin[i]:slot_begin[i + 1]] = np.abs(vals[keep]) / r[i]
    t._p_slot = p_slot
    return t


def alias_tables(t: Tables, prob) -> tuple[np.ndarray, np.ndarray]:
    """Alias tables (thr, alias slot) of an arbitrary per-slot law."""
    prob = np.ascontiguousarray(prob, dtype=np.float64)
    ns = max(int(t.slot_begin[-1]), 1)
    thr = np.zeros(ns, np.uint32)
    alias = np.zeros(ns, np.int32)
    lib().orc_alias_tables(t.n, _ptr(t.slot_begin, ctypes.c_int64), _ptr(t.deg, ctypes.c_int32),
                           _ptr(prob, ctypes.c_double), _ptr(thr, ctypes.c_uint32),
                           _ptr(alias, ctypes.c_int32))
    return thr, alias


def default_l0(tables: Tables, beta: float) -> int:
    """Coarsest level from the paper's practical rule l0 = log2(2 beta d_max) (section 4),
    read with the jump rate r_i = L_ii in place of d_i and rounded up:
    l0 = max(0, ceil(log2(2 beta max_i r_i))), so that dt_l0 * r_max <= 1/2."""
    rmax = float(tables.r.max()) if tables.n else 0.0
    if rmax <= 0.0 or beta <= 0.0:
        return 0
    return max(0, int(math.ceil(math.log2(2.0 * beta * rmax))))


# ----------------------------------------------------------------------------------
# walks and level sums (Algorithm 2)
# ----------------------------------------------------------------------------------
@dataclass
class Trace:
    final_state: np.ndarray
    sign: np.ndarray
    jumps: np.ndarray
    hash: np.ndarray
    eta_fine: np.ndarray
    eta_coarse: np.ndarray


def walk_trace(t: Tables, beta: float, level: int, seed: int, rows, walks, instance: int = 0
               ) -> Trace:
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    walks = np.ascontiguousarray(walks, dtype=np.uint32)
    q = rows.size
    assert walks.size == q
    out = Trace(np.zeros(q, np.int64), np.zeros(q, np.int32), np.zeros(q, np.int64),
                np.zeros(q, np.uint64), np.zeros(q, np.float64), np.zeros(q, np.float64))
    lib().orc_walk_trace(*t.args(), float(beta), int(level), int(seed), int(instance), q,
                         _ptr(rows, ctypes.c_int64), _ptr(walks, ctypes.c_uint32),
                         _ptr(out.final_state, ctypes.c_int64), _ptr(out.sign, ctypes.c_int32),
                         _ptr(out.jumps, ctypes.c_int64), _ptr(out.hash, ctypes.c_uint64),
                         _ptr(out.eta_fine, ctypes.c_double),
                         _ptr(out.eta_coarse, ctypes.c_double))
    return out


@dataclass
class LevelSums:
    sum1: np.ndarray   # (n_rows, R)
    sum2: np.ndarray   # (n_rows, R)
    mass: np.ndarray   # (n_rows, R)  sum_w |u_j| (|eta_fine| + |eta_coarse|)
    mass2: np.ndarray  # (n_rows, R)  sum_w of the square of that magnitude
    jumps: np.ndarray  # (n_rows,)
    hash_sum: np.ndarray  # (n_rows,) uint64: sum of the FNV path hashes mod 2^64
    walks: int
    steps_per_walk: int


def level_sums(t: Tables, beta: float, level: int, l0: int, seed: int, u, rows=None,
               walk0: int = 0, M: int = 1, instance: int = 0, threads: int = 0,
               F=None) -> LevelSums:
    """Algorithm 2's per-row sums at one level; with a source vector F (one right-hand side,
    level >= 1, and levels above l0 need l0 >= 1), Algorithm 3's samples, which add the
    Simpson sums of the source term to each sample."""
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u[:, None]
    u = np.ascontiguousarray(u)
    R = u.shape[1]
    if F is not None:
        F = np.ascontiguousarray(F, dtype=np.float64)
        if R != 1 or F.shape != (t.n,) or level < 1 or (level > l0 and l0 < 1):
            raise ValueError("source term: one right-hand side, n entries, level >= 1, l0 >= 1")
    rows = np.arange(t.n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    nr = rows.size
    s1 = np.zeros((nr, R), np.float64)
    s2 = np.zeros((nr, R), np.float64)
    ms = np.zeros((nr, R), np.float64)
    ms2 = np.zeros((nr, R), np.float64)
    jp = np.zeros(nr, np.int64)
    hs = np.zeros(nr, np.uint64)
    lib().orc_level_sums(*t.args(), float(beta), int(level), int(l0), int(seed), int(instance),
                         _ptr(u, ctypes.c_double),
                         ctypes.cast(None, _p(ctypes.c_double)) if F is None else _ptr(F, ctypes.c_double),
                         R, nr, _ptr(rows, ctypes.c_int64),
                         int(walk0), int(M), _ptr(s1, ctypes.c_double), _ptr(s2, ctypes.c_double),
                         _ptr(ms, ctypes.c_double), _ptr(ms2, ctypes.c_double),
                         _ptr(jp, ctypes.c_int64), _ptr(hs, ctypes.c_uint64), int(threads))
    return LevelSums(s1, s2, ms, ms2, jp, hs, int(M), 1 << int(level))


# ----------------------------------------------------------------------------------
# the MLMC estimator with a fixed schedule (section 2.2)
# ----------------------------------------------------------------------------------
@dataclass
class LevelStats:
    level: int
    M: int
    s1: np.ndarray
    s2: np.ndarray
    mass: np.ndarray
    jumps: int

    @property
    def mean(self) -> np.ndarray:          # m_{l,i}
        return self.s1 / self.M

    @property
    def var(self) -> np.ndarray:           # V_{l,i}, the unbiased per-walk sample variance
        return row_variances(self.s1, self.s2, self.M)


@dataclass
class Result:
    x: np.ndarray                      # (n_rows, R)
    levels: list = field(default_factory=list)
    l0: int = 0
    mass: np.ndarray | None = None     # sum_l mean_w |u|(|eta_f| + |eta_c|)
    steps: int = 0
    jumps: int = 0

    def est_mse(self) -> float:
        """Row-mean estimated variance of the estimator: sum_l mean_i V_{l,i} / M_l."""
        return float(sum(np.mean(L.var) / L.M for L in self.levels))


def mlmc_fixed(t: Tables, beta: float, u, l0: int, L: int, M, seed: int, rows=None,
               instance: int = 0, threads: int = 0, F=None) -> Result:
    """x^L estimate with M[l - l0] walks per row at level l, l = l0..L (with a source vector
    F: Algorithm 3's estimate of exp(beta A) u + int_0^beta exp(sA) F ds)."""
    levels = []
    x = None
    mass = None
    steps = 0
    jumps = 0
    for q, lev in enumerate(range(l0, L + 1)):
        Ml = int(M[q]) if np.ndim(M) else int(M)
        ls = level_sums(t, beta, lev, l0, seed, u, rows, 0, Ml, instance, threads, F=F)
        st = LevelStats(lev, Ml, ls.sum1, ls.sum2, ls.mass, int(ls.jumps.sum()))
        levels.append(st)
        x = st.mean if x is None else x + st.mean
        mass = ls.mass / Ml if mass is None else mass + ls.mass / Ml
        steps += Ml * (1 << lev) * ls.sum1.shape[0]
        jumps += st.jumps
    return Result(x, levels, l0, mass, steps, jumps)


# ----------------------------------------------------------------------------------
# Algorithm 1 (adaptive driver)
# ----------------------------------------------------------------------------------
JUMP_COST = 4.0     # cost model C_l = N_l + JUMP_COST * (mean jumps per walk)
ALPHA = 2.0         # weak order of the Strang splitting


def optimal_M(V, C, eps):
    """Giles' optimal sample sizes for a variance budget eps^2 / 2."""
    V = np.asarray(V, np.float64)
    C = np.asarray(C, np.float64)
    tot = float(np.sum(np.sqrt(V * C)))
    return np.ceil(2.0 * eps ** -2 * np.sqrt(V / C) * tot).astype(np.int64)


def row_variances(s1, s2, M: int) -> np.ndarray:
    """Per-entry sample variance of M samples from their sum and sum of squares (Algorithm 2's
    m_l and m2l, each divided by M once), with the factor M / (M - 1) that makes it unbiased;
    clamped at 0 against rounding."""
    m = s1 / M
    raw = np.maximum(s2 / M - m * m, 0.0)
    return raw * (M / (M - 1.0)) if M > 1 else raw


def level_variance(s1, s2, M: int) -> float:
    """V_l of Algorithm 1 for a vector: the mean over the entries of their per-walk variances."""
    return float(np.mean(row_variances(s1, s2, M)))


def level_term_rms(s1, s2, M: int) -> float:
    """The root mean square over the entries of the level term m_{l,i}, from M-walk means:
    mean_i mhat_i^2 overstates mean_i m_i^2 by the sampling noise mean_i V_{l,i} / M, which
    is taken off (clamped at 0), so that small pilots do not inflate the bias estimate."""
    m = s1 / M
    return math.sqrt(max(float(np.mean(m * m)) - level_variance(s1, s2, M) / M, 0.0))


def bias_estimate(mL: float, mLm1: float) -> float:
    """Extrapolated bias of the finest level, from the RMS level means of the two
    finest levels with weak order alpha."""
    return max(abs(mL), abs(mLm1) / 2.0 ** ALPHA) / (2.0 ** ALPHA - 1.0)


PILOT_SAMPLES = 1 << 18


def default_pilot(n_rows: int, u_shape) -> int:
    """M0 when the caller leaves it to the driver: enough walks per row that every pilot level
    holds at least 2^18 samples over its rows and right-hand sides, and at least 2."""
    R = int(u_shape[1]) if len(u_shape) > 1 else 1
    return max(2, -(-PILOT_SAMPLES // max(1, n_rows * R)))


@dataclass
class _Acc:
    M: int
    s1: np.ndarray
    s2: np.ndarray
    mass: np.ndarray
    jumps: int


def mlmc_adaptive(t: Tables, beta: float, u, eps: float, seed: int, l0: int | None = None,
                  pilot: int = 256, max_levels: int = 20, rows=None, instance: int = 0,
                  threads: int = 0, max_walks: int | None = None, max_iterations: int = 100):
    """Algorithm 1: pilot M0 walks on levels l0..l0+4 (pilot = 0: default_pilot), then
    repeat {optimal M_l; run the extra walks; stop when the error is below eps, else add a
    level}.

    The error is read as two parts: the estimator's variance sum_l V_l / M_l against the
    budget eps^2 / 2, and the extrapolated bias of the finest level against eps / sqrt(2).
    The optimal sample sizes are recomputed from the updated variances, and the missing
    walks run, until they ask for no more walks (so the variance part holds); only then is
    the bias tested, and a failed bias test adds the level L + 1 with M0 walks."""
    if l0 is None:
        l0 = default_l0(t, beta)
    L = l0 + 4
    acc: dict[int, _Acc] = {}

    def run(lev, extra):
        prev = acc.get(lev)
        w0 = prev.M if prev else 0
        ls = level_sums(t, beta, lev, l0, seed, u, rows, w0, extra, instance, threads)
        if prev is None:
            acc[lev] = _Acc(extra, ls.sum1, ls.sum2, ls.mass, int(ls.jumps.sum()))
        else:
            prev.M += extra
            prev.s1 = prev.s1 + ls.sum1
            prev.s2 = prev.s2 + ls.sum2
            prev.mass = prev.mass + ls.mass
            prev.jumps += int(ls.jumps.sum())

    def level_var(lev):          # row-mean per-walk variance of the level's samples
        a = acc[lev]
        return level_variance(a.s1, a.s2, a.M)

    def level_rms(lev):          # root mean square over rows of the level term
        a = acc[lev]
        return level_term_rms(a.s1, a.s2, a.M)

    if pilot == 0:
        pilot = default_pilot(len(rows) if rows is not None else t.n, np.shape(u))
    for lev in range(l0, L + 1):
        run(lev, pilot)
    converged = False
    iterations = 0
    while iterations < max_iterations:
        iterations += 1
        levs = list(range(l0, L + 1))
        nrows = acc[l0].s1.shape[0]
        V = [max(level_var(lev), 1e-300) for lev in levs]
        C = [(1 << lev) + JUMP_COST * acc[lev].jumps / (acc[lev].M * nrows) for lev in levs]
        Mopt = optimal_M(V, C, eps)
        topped = False
        for lev, Mo in zip(levs, Mopt):
            extra = int(Mo) - acc[lev].M
            if max_walks is not None:
                extra = min(extra, max_walks - acc[lev].M)
            if extra > 0:
                run(lev, extra)
                topped = True
        if topped:
            continue                   # the variance part: re-estimate V_l, resize
        var = sum(level_var(lev) / acc[lev].M for lev in levs)
        bias = bias_estimate(level_rms(L), level_rms(L - 1))
        if var <= eps * eps / 2.0 * 1.0000001 and bias <= eps / math.sqrt(2.0):
            converged = True
            break
        if var > eps * eps / 2.0 * 1.0000001 or L - l0 + 1 >= max_levels:
            break                      # walk cap reached, or no level left to add
        L += 1
        run(L, pilot)
    levels = [LevelStats(l, acc[l].M, acc[l].s1, acc[l].s2, acc[l].mass, acc[l].jumps)
              for l in range(l0, L + 1)]
    x = sum(st.mean for st in levels)
    mass = sum(st.mass / st.M for st in levels)
    nrows = levels[0].s1.shape[0]
    steps = sum(st.M * (1 << st.level) * nrows for st in levels)
    res = Result(x, levels, l0, mass, steps, sum(st.jumps for st in levels))
    res.converged = converged
    res.iterations = iterations
    return res


# ----------------------------------------------------------------------------------
# scalar functional (w, exp(beta A) u) by walks from random start rows
# ----------------------------------------------------------------------------------
def start_tables(u):
    """Alias table over rows for the start law |u_l| / U (the construction of the slot
    tables, on one 'row' of n entries), the sign of u per row, and U."""
    u = np.asarray(u, np.float64)
    n = u.size
    U = float(np.cumsum(np.abs(u))[-1]) if n else 0.0      # summed in row order
    one = Tables(1, None, None, None, np.array([0, n], np.int64), np.array([n], np.int32),
                 None, None, None, None)
    thr, alias = alias_tables(one, np.abs(u) / U)
    return thr, alias, (u < 0).astype(np.uint8), U


@dataclass
class FunctionalSums:
    sum1: float
    sum2: float
    jumps: int
    hash_sum: int
    walks: int
    U: float


def functional_sums(tT: Tables, beta: float, level: int, l0: int, seed: int, u, w,
                    walk0: int = 0, M: int = 1, instance: int = 0) -> FunctionalSums:
    """Sums of the samples sign(u_l) w_j (eta_f - eta_c) over walks walk0..walk0+M-1 on the
    tables tT of A^T; the functional's level term is U sum1 / M."""
    thr, alias, neg, U = start_tables(u)
    w = np.ascontiguousarray(w, np.float64)
    s1 = np.zeros(1)
    s2 = np.zeros(1)
    jp = np.zeros(1, np.int64)
    hs = np.zeros(1, np.uint64)
    lib().orc_functional_sums(*tT.args()[:8], float(beta), int(level), int(l0), int(seed),
                              int(instance), int(tT.n), _ptr(thr, ctypes.c_uint32),
                              _ptr(alias, ctypes.c_int32), _ptr(neg, ctypes.c_uint8),
                              _ptr(w, ctypes.c_double), int(walk0), int(M),
                              _ptr(s1, ctypes.c_double), _ptr(s2, ctypes.c_double),
                              _ptr(jp, ctypes.c_int64), _ptr(hs, ctypes.c_uint64))
    return FunctionalSums(float(s1[0]), float(s2[0]), int(jp[0]), int(hs[0]), int(M), U)


@dataclass
class ForwardSums:
    sum1: np.ndarray      # per final state j: sum of the deposits sign(u_l)(eta_f - eta_c)
    sum2: np.ndarray      # and of their squares
    mass: np.ndarray      # sum of |eta_f| (+ |eta_c|) of the deposits at j
    count: np.ndarray     # walks that ended at j
    jumps: int
    hash_sum: int
    walks: int
    U: float


def forward_sums(tT: Tables, beta: float, level: int, l0: int, seed: int, u, walk0: int = 0,
                 M: int = 1, instance: int = 0) -> ForwardSums:
    """The full vector exp(beta A) u by the walks of `functional_sums` (tables tT of A^T):
    each walk deposits its sample at its final state; the level term of x is U sum1 / M."""
    thr, alias, neg, U = start_tables(u)
    n = tT.n
    s1 = np.zeros(n)
    s2 = np.zeros(n)
    ms = np.zeros(n)
    ct = np.zeros(n, np.int64)
    jp = np.zeros(1, np.int64)
    hs = np.zeros(1, np.uint64)
    rc = lib().orc_forward_sums(*tT.args()[:8], float(beta), int(level), int(l0), int(seed),
                                int(instance), int(n), _ptr(thr, ctypes.c_uint32),
                                _ptr(alias, ctypes.c_int32), _ptr(neg, ctypes.c_uint8),
                                int(walk0), int(M), _ptr(s1, ctypes.c_double),
                                _ptr(s2, ctypes.c_double), _ptr(ms, ctypes.c_double),
                                _ptr(ct, ctypes.c_int64), _ptr(jp, ctypes.c_int64),
                                _ptr(hs, ctypes.c_uint64))
    if rc != 0:
        raise MemoryError("orc_forward_sums")
    return ForwardSums(s1, s2, ms, ct, int(jp[0]), int(hs[0]), int(M), U)


def forward_fixed(tT: Tables, beta: float, u, l0: int, L: int, M, seed: int, instance: int = 0):
    """exp(beta A) u with M[q] walks at level l0 + q of the forward representation:
    (estimate, per-entry variance of it)."""
    est = np.zeros(tT.n)
    var = np.zeros(tT.n)
    for q, lev in enumerate(range(l0, L + 1)):
        fs = forward_sums(tT, beta, lev, l0, seed, u, 0, int(M[q]), instance)
        est += fs.U * (fs.sum1 / fs.walks)
        var += fs.U ** 2 * row_variances(fs.sum1, fs.sum2, fs.walks) / fs.walks
    return est, var


def functional_fixed(tT: Tables, beta: float, u, w, l0: int, L: int, M, seed: int,
                     instance: int = 0):
    """(w, exp(beta A) u) with M[q] walks at level l0 + q: (estimate, variance of it)."""
    est = var = 0.0
    for q, lev in enumerate(range(l0, L + 1)):
        fs = functional_sums(tT, beta, lev, l0, seed, u, w, 0, int(M[q]), instance)
        est += fs.U * (fs.sum1 / fs.walks)
        var += fs.U ** 2 * float(row_variances(fs.sum1, fs.sum2, fs.walks)) / fs.walks
    return est, var

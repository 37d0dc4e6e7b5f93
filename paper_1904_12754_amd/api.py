"""Python binding of the mlmc_expv C-ABI (marshalling only; every step of the walks runs
in the library's HIP kernels). PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import check


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _u_args(u: torch.Tensor, n: int):
    if not u.is_cuda:
        raise ValueError("u must be a device tensor")
    if u.dtype not in (torch.float32, torch.float64):
        raise ValueError("u must be float32 or float64")
    if u.dim() == 1:
        u = u[:, None]
    if u.shape[0] != n:
        raise ValueError(f"u has {u.shape[0]} rows, the matrix {n}")
    u = u.contiguous()
    dt = _abi.MLMC_DTYPE_F64 if u.dtype == torch.float64 else _abi.MLMC_DTYPE_F32
    return u, int(u.shape[1]), dt


class Plan:
    """A prepared matrix: A = D - T split, alias tables and step thresholds in HBM.

    A: an object with n, row_ptr, col_idx, values: numpy arrays (host), or device tensors
       (int64 row_ptr, int32 col_idx, float32 or float64 values; values_dtype is then ignored).
    precision: "fp32" (FP32 path weights, compensated FP32 sums, FP64 combine) or "fp64".
    """

    def __init__(self, A, beta: float, precision: str = "fp32", l0: int | None = None,
                 rows=None, values_dtype=np.float64, stream=None):
        self._lib = _abi.load()
        self._handle = ctypes.c_void_p()
        self.n = int(A.n)
        if isinstance(A.row_ptr, torch.Tensor) and A.row_ptr.is_cuda:
            self._row_ptr = A.row_ptr.contiguous()
            self._col_idx = A.col_idx.contiguous()
            self._values = A.values.contiguous()
            if (self._row_ptr.dtype != torch.int64 or self._col_idx.dtype != torch.int32 or
                    self._values.dtype not in (torch.float32, torch.float64) or
                    not (self._col_idx.is_cuda and self._values.is_cuda)):
                raise ValueError("device CSR: int64 row_ptr, int32 col_idx, float32/float64 "
                                 "values, all on the device")
            csr = _abi.CSR(self.n, ctypes.cast(_dev_ptr(self._row_ptr), ctypes.POINTER(ctypes.c_int64)),
                           ctypes.cast(_dev_ptr(self._col_idx), ctypes.POINTER(ctypes.c_int32)),
                           _dev_ptr(self._values),
                           _abi.MLMC_DTYPE_F64 if self._values.dtype == torch.float64
                           else _abi.MLMC_DTYPE_F32, _abi.MLMC_MEMORY_DEVICE)
        else:
            self._row_ptr = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
            self._col_idx = np.ascontiguousarray(A.col_idx, dtype=np.int32)
            self._values = np.ascontiguousarray(A.values, dtype=values_dtype)
            csr = _abi.CSR(self.n, self._row_ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           self._col_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                           ctypes.c_void_p(self._values.ctypes.data),
                           _abi.MLMC_DTYPE_F64 if self._values.dtype == np.float64
                           else _abi.MLMC_DTYPE_F32, _abi.MLMC_MEMORY_HOST)
        prec = {"fp64": _abi.MLMC_PRECISION_FP64, "fp32": _abi.MLMC_PRECISION_FP32}[precision]
        self._rows = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
        opts = _abi.PlanOpts(float(beta), prec, -1 if l0 is None else int(l0),
                             None if self._rows is None else
                             self._rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             0 if self._rows is None else int(self._rows.size))
        check(self._lib.mlmc_expv_plan(ctypes.byref(self._handle), ctypes.byref(csr),
                                       ctypes.byref(opts), _stream_ptr(stream)))
        info = _abi.PlanInfo()
        check(self._lib.mlmc_expv_plan_info(self._handle, ctypes.byref(info)))
        self.n_rows = int(info.n_rows)
        self.l0 = int(info.l0)
        self.beta = float(info.beta)
        self.info = {f: getattr(info, f) for f, _ in _abi.PlanInfo._fields_}

    # ------------------------------------------------------------------------------
    def _source(self, source, u):
        if source is None:
            return None
        if not source.is_cuda or source.dtype != u.dtype or source.numel() != self.n:
            raise ValueError("source must be a device vector of n entries with u's dtype")
        if u.shape[1] != 1:
            raise ValueError("a source term takes one right-hand side")
        return source.contiguous()

    def run(self, u: torch.Tensor, walks=None, eps: float | None = None, seed: int = 0,
            instance: int = 0, pilot_walks: int = 1024, max_levels: int = 20,
            max_walks: int = 0, out: torch.Tensor | None = None, stream=None,
            want_stats: bool = True, allow=(), source: torch.Tensor | None = None):
        """x = exp(beta A) u at the plan's rows (with a source vector F: Algorithm 3's
        exp(beta A) u + int_0^beta exp(sA) F ds). Fixed schedule: walks[q] walks per row at
        level l0 + q. Adaptive (Algorithm 1): eps > 0."""
        u, R, dt = _u_args(u, self.n)
        F = self._source(source, u)
        x = out if out is not None else torch.empty((self.n_rows, R), dtype=torch.float64,
                                                    device=u.device)
        if eps is not None and eps > 0:
            opts = _abi.RunOpts(seed, instance, 0, None, float(eps), int(pilot_walks),
                                int(max_levels), int(max_walks))
            walks_arr = None
        else:
            walks_arr = np.ascontiguousarray(walks, dtype=np.int64)
            opts = _abi.RunOpts(seed, instance, int(walks_arr.size),
                                walks_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0.0,
                                0, 0, 0)
        stats = _abi.Stats() if want_stats else None
        if F is None:
            code = self._lib.mlmc_expv_run(self._handle, _dev_ptr(u), R, dt, ctypes.byref(opts),
                                           _dev_ptr(x), ctypes.byref(stats) if stats else None,
                                           _stream_ptr(stream))
        else:
            code = self._lib.mlmc_expv_run_source(self._handle, _dev_ptr(u), _dev_ptr(F), dt,
                                                  ctypes.byref(opts), _dev_ptr(x),
                                                  ctypes.byref(stats) if stats else None,
                                                  _stream_ptr(stream))
        check(code, allow)
        del walks_arr
        return x, (stats.to_dict() if stats else None)

    def level_sums(self, u: torch.Tensor, level: int, walk0: int, walks: int, seed: int = 0,
                   instance: int = 0, stream=None, hashes: bool = False,
                   source: torch.Tensor | None = None, noalloc: bool = False, out=None,
                   want_jumps: bool = True):
        """Algorithm 2's accumulators at one level (Algorithm 3's with a source vector):
        (sum Y, sum Y^2) per (row, rhs), jumps, and with hashes=True the per-row sum
        (mod 2^64) of the path hashes. noalloc=True calls the allocation-free entry point
        (no source term); out = (s1, s2[, hash_sums]) supplies the output tensors;
        want_jumps=False skips the jump count (no wait for the stream; jumps is None)."""
        u, R, dt = _u_args(u, self.n)
        F = self._source(source, u)
        if out is not None:
            s1, s2 = out[0], out[1]
            hs = out[2] if hashes else None
        else:
            s1 = torch.empty((self.n_rows, R), dtype=torch.float64, device=u.device)
            s2 = torch.empty_like(s1)
            hs = torch.empty(self.n_rows, dtype=torch.int64, device=u.device) if hashes else None
        jumps = ctypes.c_int64()
        jp = ctypes.byref(jumps) if want_jumps else None
        if noalloc:
            if F is not None:
                raise ValueError("the allocation-free level sums take no source term")
            check(self._lib.mlmc_expv_level_sums_noalloc(self._handle, _dev_ptr(u), R, dt, seed,
                                                         instance, level, walk0, walks,
                                                         _dev_ptr(s1), _dev_ptr(s2), jp,
                                                         _dev_ptr(hs) if hashes else None,
                                                         _stream_ptr(stream)))
        elif F is None:
            check(self._lib.mlmc_expv_level_sums(self._handle, _dev_ptr(u), R, dt, seed, instance,
                                                 level, walk0, walks, _dev_ptr(s1), _dev_ptr(s2),
                                                 jp, _dev_ptr(hs) if hashes else None,
                                                 _stream_ptr(stream)))
        else:
            check(self._lib.mlmc_expv_level_sums_source(
                self._handle, _dev_ptr(u), _dev_ptr(F), dt, seed, instance, level, walk0, walks,
                _dev_ptr(s1), _dev_ptr(s2), jp,
                _dev_ptr(hs) if hashes else None, _stream_ptr(stream)))
        nj = int(jumps.value) if want_jumps else None
        if hashes:
            return s1, s2, nj, hs
        return s1, s2, nj

    def trace(self, level: int, rows, walks, seed: int = 0, instance: int = 0, stream=None):
        dev = torch.device("cuda")
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if rows.size and (rows.min() < 0 or rows.max() >= self.n):
            raise ValueError("trace rows must be rows of A")
        rows_t = torch.as_tensor(rows, device=dev)
        walks_t = torch.as_tensor(np.ascontiguousarray(walks, dtype=np.uint32).view(np.int32),
                                  device=dev)
        q = rows_t.numel()
        out = {
            "final_state": torch.empty(q, dtype=torch.int64, device=dev),
            "sign": torch.empty(q, dtype=torch.int32, device=dev),
            "jumps": torch.empty(q, dtype=torch.int64, device=dev),
            "hash": torch.empty(q, dtype=torch.int64, device=dev),
            "log_eta_fine": torch.empty(q, dtype=torch.float64, device=dev),
            "log_eta_coarse": torch.empty(q, dtype=torch.float64, device=dev),
        }
        check(self._lib.mlmc_expv_trace(self._handle, seed, instance, level, q,
                                        _dev_ptr(rows_t), _dev_ptr(walks_t),
                                        *(_dev_ptr(out[k]) for k in ("final_state", "sign",
                                                                     "jumps", "hash",
                                                                     "log_eta_fine",
                                                                     "log_eta_coarse")),
                                        _stream_ptr(stream)))
        return out

    # ---- scalar functional (w, exp(beta A) u) by walks from random start rows ----------
    def _uw(self, u, w):
        if not (u.is_cuda and w.is_cuda) or u.dtype != w.dtype or u.dtype not in (torch.float32, torch.float64):
            raise ValueError("u and w must be device vectors of one float dtype")
        if u.numel() != self.n or w.numel() != self.n:
            raise ValueError("u and w must have n entries")
        dt = _abi.MLMC_DTYPE_F64 if u.dtype == torch.float64 else _abi.MLMC_DTYPE_F32
        return u.contiguous(), w.contiguous(), dt

    def functional(self, u: torch.Tensor, w: torch.Tensor, walks=None, eps: float | None = None,
                   seed: int = 0, instance: int = 0, pilot_walks: int = 1 << 16,
                   max_levels: int = 20, max_walks: int = 0, stream=None, allow=()):
        """(w, exp(beta A) u) with the plan built on A^T (on A when A is symmetric): walks[q]
        total walks at level l0 + q, or Algorithm 1 to eps. Returns (value, variance, stats)."""
        u, w, dt = self._uw(u, w)
        if eps is not None and eps > 0:
            opts = _abi.RunOpts(seed, instance, 0, None, float(eps), int(pilot_walks),
                                int(max_levels), int(max_walks))
            walks_arr = None
        else:
            walks_arr = np.ascontiguousarray(walks, dtype=np.int64)
            opts = _abi.RunOpts(seed, instance, int(walks_arr.size),
                                walks_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0.0,
                                0, 0, 0)
        res = ctypes.c_double()
        var = ctypes.c_double()
        st = _abi.Stats()
        check(self._lib.mlmc_expv_functional(self._handle, _dev_ptr(u), _dev_ptr(w), dt,
                                             ctypes.byref(opts), ctypes.byref(res),
                                             ctypes.byref(var), ctypes.byref(st),
                                             _stream_ptr(stream)), allow)
        del walks_arr
        return float(res.value), float(var.value), st.to_dict()

    def functional_level_sums(self, u: torch.Tensor, w: torch.Tensor, level: int, walk0: int,
                              walks: int, seed: int = 0, instance: int = 0, stream=None):
        """(sum of samples without U, sum of squares, jumps, hash sum, U) of one level."""
        u, w, dt = self._uw(u, w)
        s1, s2, U = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        j = ctypes.c_int64()
        h = ctypes.c_uint64()
        check(self._lib.mlmc_expv_functional_level_sums(
            self._handle, _dev_ptr(u), _dev_ptr(w), dt, seed, instance, level, walk0, walks,
            ctypes.byref(s1), ctypes.byref(s2), ctypes.byref(j), ctypes.byref(h), ctypes.byref(U),
            _stream_ptr(stream)))
        return float(s1.value), float(s2.value), int(j.value), int(h.value), float(U.value)

    # ---- the full vector by the forward representation (same walks, deposited) --------
    def _u_only(self, u):
        if not u.is_cuda or u.dtype not in (torch.float32, torch.float64) or u.numel() != self.n:
            raise ValueError("u must be a device vector of n float32 or float64 entries")
        dt = _abi.MLMC_DTYPE_F64 if u.dtype == torch.float64 else _abi.MLMC_DTYPE_F32
        return u.contiguous(), dt

    def forward(self, u: torch.Tensor, walks=None, eps: float | None = None, seed: int = 0,
                instance: int = 0, pilot_walks: int = 1 << 16, max_levels: int = 20,
                max_walks: int = 0, stream=None, allow=()):
        """exp(beta A) u by the forward representation, the plan built on A^T (on A when A
        is symmetric): walks[q] total walks at level l0 + q, or Algorithm 1 to eps (RMS over
        the entries). Returns (x, per-entry variance, stats)."""
        u, dt = self._u_only(u)
        if eps is not None and eps > 0:
            walks_arr = None
            opts = _abi.RunOpts(seed, instance, 0, None, float(eps), int(pilot_walks),
                                int(max_levels), int(max_walks))
        else:
            walks_arr = np.ascontiguousarray(walks, dtype=np.int64)
            opts = _abi.RunOpts(seed, instance, int(walks_arr.size),
                                walks_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0.0,
                                0, 0, 0)
        x = torch.empty(self.n, dtype=torch.float64, device=u.device)
        var = torch.empty(self.n, dtype=torch.float64, device=u.device)
        st = _abi.Stats()
        check(self._lib.mlmc_expv_forward(self._handle, _dev_ptr(u), dt, ctypes.byref(opts),
                                          _dev_ptr(x), _dev_ptr(var), ctypes.byref(st),
                                          _stream_ptr(stream)), allow)
        del walks_arr
        return x, var, st.to_dict()

    def forward_level_sums(self, u: torch.Tensor, level: int, walk0: int, walks: int,
                           seed: int = 0, instance: int = 0, hashes: bool = False, stream=None):
        """Per-state sums of the deposits (without U) and of their squares (device, n
        doubles each), jumps, hash sum (with hashes) and U, of one level."""
        u, dt = self._u_only(u)
        s1 = torch.empty(self.n, dtype=torch.float64, device=u.device)
        s2 = torch.empty(self.n, dtype=torch.float64, device=u.device)
        j = ctypes.c_int64()
        h = ctypes.c_uint64()
        U = ctypes.c_double()
        check(self._lib.mlmc_expv_forward_level_sums(
            self._handle, _dev_ptr(u), dt, seed, instance, level, walk0, walks, _dev_ptr(s1),
            _dev_ptr(s2), ctypes.byref(j), ctypes.byref(h) if hashes else None, ctypes.byref(U),
            _stream_ptr(stream)))
        return s1, s2, int(j.value), (int(h.value) if hashes else None), float(U.value)

    # ---- learned proposal (importance sampling of the jump law) -----------------------
    @staticmethod
    def _params(params):
        if params is None:
            return None, None
        P = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if P.size != _abi.MLMC_PROPOSAL_PARAMS:
            raise ValueError(f"params must hold {_abi.MLMC_PROPOSAL_PARAMS} floats")
        return P, P.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def _xhat(self, xhat):
        if xhat is None:
            return None, None
        x = torch.as_tensor(xhat, dtype=torch.float64, device="cuda").reshape(-1).contiguous()
        if x.numel() != self.n:
            raise ValueError("xhat must have n entries")
        return x, _dev_ptr(x)

    def set_proposal(self, params=None, xhat=None, num_levels: int = 1, stream=None):
        """Proposal tables for levels l0 .. l0 + num_levels - 1 from the flat parameters
        (W1, b1, W2, b2, W3, b3; None = identity proposal) and a pilot estimate xhat."""
        P, pp = self._params(params)
        x, xp = self._xhat(xhat)
        check(self._lib.mlmc_expv_proposal_set(self._handle, pp, xp, int(num_levels),
                                               _stream_ptr(stream)))
        (stream if stream is not None else torch.cuda.current_stream()).synchronize()
        del P, x

    def enable_proposal(self, on: bool = True):
        check(self._lib.mlmc_expv_proposal_enable(self._handle, 1 if on else 0))

    def proposal_tables(self, level: int, stream=None):
        """(thr uint32, alias slot int32, ratio p/q float32, q float32) per slot, on host."""
        ns = max(int(self.info["n_slots"]), 1)
        dev = torch.device("cuda")
        thr = torch.empty(ns, dtype=torch.int32, device=dev)
        al = torch.empty(ns, dtype=torch.int32, device=dev)
        ratio = torch.empty(ns, dtype=torch.float32, device=dev)
        q = torch.empty(ns, dtype=torch.float32, device=dev)
        check(self._lib.mlmc_expv_proposal_tables(self._handle, int(level), _dev_ptr(thr),
                                                  _dev_ptr(al), _dev_ptr(ratio), _dev_ptr(q),
                                                  _stream_ptr(stream)))
        k = int(self.info["n_slots"])
        return (thr.cpu().numpy().view(np.uint32)[:k], al.cpu().numpy()[:k],
                ratio.cpu().numpy()[:k], q.cpu().numpy()[:k])

    def proposal_loss_grad(self, params, xhat, level: int, rows, slots, weights,
                           shrink: float = 0.0, stream=None):
        """(flat FP32 gradient, loss) of the cross-entropy training loss on given transitions."""
        P, pp = self._params(params)
        x, xp = self._xhat(xhat)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        slots = np.ascontiguousarray(slots, dtype=np.int32)
        weights = np.ascontiguousarray(weights, dtype=np.float32)
        g = np.zeros(_abi.MLMC_PROPOSAL_PARAMS, np.float32)
        loss = ctypes.c_double()
        check(self._lib.mlmc_expv_proposal_loss_grad(
            self._handle, pp, xp, int(level), int(rows.size),
            rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            slots.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            weights.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), float(shrink),
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss),
            _stream_ptr(stream)))
        del P, x
        return g, float(loss.value)

    def train_proposal(self, u: torch.Tensor, init_params, seed: int = 0,
                       pilot_walks: int = 256, capture_walks: int = 64, sample_stride: int = 1,
                       steps: int = 200, batch: int = 4096, lr: float = 1e-3,
                       shrink: float = 1.0, num_levels: int = 1, judge_walks: int = 8,
                       stream=None):
        """Train the proposal on the device and set it; returns (params, stats)."""
        u, R, dt = _u_args(u, self.n)
        if R != 1:
            raise ValueError("training reads one right-hand side")
        P, pp = self._params(init_params)
        out = np.zeros(_abi.MLMC_PROPOSAL_PARAMS, np.float32)
        opts = _abi.TrainOpts(int(seed), pp, int(pilot_walks), int(capture_walks),
                              int(sample_stride), int(steps), int(batch), float(lr),
                              float(shrink), int(num_levels), int(judge_walks))
        st = _abi.TrainStats()
        check(self._lib.mlmc_expv_proposal_train(
            self._handle, _dev_ptr(u), dt, ctypes.byref(opts),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(st),
            _stream_ptr(stream)))
        del P
        return out, st.to_dict()

    def run_learned(self, u: torch.Tensor, eps: float, init_params, seed: int = 0,
                    instance: int = 0, pilot_walks: int = 0, max_levels: int = 20,
                    max_walks: int = 0, train_seed: int = 0, capture_walks: int = 16,
                    sample_stride: int = 1, steps: int = 16, batch: int = 4096,
                    lr: float = 1e-2, shrink: float = 1.0, stream=None, allow=()):
        """Algorithm 1 with the proposal of level l0 trained inside the run on the pilot's
        estimate and judged against the pilot's plain level-l0 walks; returns
        (x, stats, train_stats, params)."""
        u, R, dt = _u_args(u, self.n)
        if R != 1:
            raise ValueError("the learned run reads one right-hand side")
        x = torch.empty((self.n_rows, 1), dtype=torch.float64, device=u.device)
        opts = _abi.RunOpts(seed, instance, 0, None, float(eps), int(pilot_walks),
                            int(max_levels), int(max_walks))
        P, pp = self._params(init_params)
        topts = _abi.TrainOpts(int(train_seed), pp, 0, int(capture_walks), int(sample_stride),
                               int(steps), int(batch), float(lr), float(shrink), 1, 0)
        out = np.zeros(_abi.MLMC_PROPOSAL_PARAMS, np.float32)
        stats = _abi.Stats()
        tst = _abi.TrainStats()
        code = self._lib.mlmc_expv_run_learned(
            self._handle, _dev_ptr(u), dt, ctypes.byref(opts), ctypes.byref(topts),
            out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _dev_ptr(x), ctypes.byref(stats),
            ctypes.byref(tst), _stream_ptr(stream))
        check(code, allow)
        del P
        return x, stats.to_dict(), tst.to_dict(), out

    def current_info(self) -> dict:
        """mlmc_expv_plan_info now (device_bytes grows as levels and buffers are added)."""
        info = _abi.PlanInfo()
        check(self._lib.mlmc_expv_plan_info(self._handle, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in _abi.PlanInfo._fields_}

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self._lib.mlmc_expv_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many plans with fixed level schedules in a few walk launches, captured in a graph.

    plans: list of Plan (one precision); us: list of device tensors (n_b or n_b x R_b, one
    dtype); walks: (count, num_levels) walks per row at levels l0_b + q. Instance b draws
    the streams of instance number b, so its paths are those of plans[b].run(us[b],
    walks=walks[b], instance=b) with the same seed. Without autotune, waves_per_cu picks
    the grid: 0 for one wave per item, else a resident grid of that many waves per CU.
    """

    def __init__(self, plans, us, walks, autotune: bool = True, waves_per_cu: int = 0,
                 stream=None):
        self._lib = _abi.load()
        self._handle = ctypes.c_void_p()
        walks = np.ascontiguousarray(walks, dtype=np.int64)
        count = len(plans)
        if walks.shape[0] != count or len(us) != count:
            raise ValueError("one u and one row of walks per plan")
        self.plans = plans
        self.us = []
        nrhs = []
        dts = set()
        for p, u in zip(plans, us):
            u2, R, dt = _u_args(u, p.n)
            self.us.append(u2)
            nrhs.append(R)
            dts.add(dt)
        if len(dts) != 1:
            raise ValueError("all right-hand sides of a batch must share one dtype")
        self.xs = [torch.empty((p.n_rows, R), dtype=torch.float64, device=self.us[0].device)
                   for p, R in zip(plans, nrhs)]
        self._plan_ptrs = (ctypes.c_void_p * count)(*[p._handle.value for p in plans])
        self._u_ptrs = (ctypes.c_void_p * count)(*[u.data_ptr() for u in self.us])
        self._x_ptrs = (ctypes.c_void_p * count)(*[x.data_ptr() for x in self.xs])
        self._nrhs = (ctypes.c_int32 * count)(*nrhs)
        self._walks = walks
        desc = _abi.BatchDesc(count, self._plan_ptrs, self._u_ptrs, self._nrhs, dts.pop(),
                              self._x_ptrs, int(walks.shape[1]),
                              walks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              1 if autotune else 0, int(waves_per_cu))
        check(self._lib.mlmc_expv_batch_create(ctypes.byref(self._handle), ctypes.byref(desc),
                                               _stream_ptr(stream)))
        info = _abi.BatchInfo()
        check(self._lib.mlmc_expv_batch_info(self._handle, ctypes.byref(info)))
        n = int(info.tune_count)
        self.info = {f: (list(getattr(info, f))[:n] if f.startswith("tune_") and f != "tune_count"
                         else getattr(info, f))
                     for f, _ in _abi.BatchInfo._fields_ if f != "pad"}

    def launch(self, seed: int = 0, stream=None):
        """Replay the captured graph; every x in self.xs is overwritten (asynchronous)."""
        check(self._lib.mlmc_expv_batch_launch(self._handle, seed, _stream_ptr(stream)))
        return self.xs

    def stats(self, stream=None):
        arr = (_abi.Stats * len(self.plans))()
        check(self._lib.mlmc_expv_batch_stats(self._handle, arr, _stream_ptr(stream)))
        return [s.to_dict() for s in arr]

    def close(self):
        if getattr(self, "_handle", None) and self._handle.value:
            self._lib.mlmc_expv_batch_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---- measurement probes (include/mlmc_probe.h) -----------------------------------------
def probe_gather(table: torch.Tensor, log2_records: int, waves_per_cu: int = 16, iters: int = 64,
                 stream=None, lds: bool = False, dependent: bool = False):
    """Random 16-byte gathers from the first 2^log2_records records of `table` (a device
    tensor of at least 16 * 2^log2_records bytes); lds=True gathers from a copy staged in
    each workgroup's LDS, dependent=True makes each lane's gathers serial (one stream whose
    next index takes in the record read). Returns (gathers, seconds) of one timed launch."""
    if not table.is_cuda or table.numel() * table.element_size() < (16 << log2_records):
        raise ValueError("table must be a device tensor of at least 16 * 2^log2_records bytes")
    lib = _abi.load()
    g = ctypes.c_uint64()
    ms = ctypes.c_double()
    mode = (_abi.MLMC_PROBE_LDS if lds else 0) | (_abi.MLMC_PROBE_DEPENDENT if dependent else 0)
    check(lib.mlmc_probe_gather_mode(_dev_ptr(table), int(log2_records), int(waves_per_cu),
                                     int(iters), mode, ctypes.byref(g), ctypes.byref(ms),
                                     _stream_ptr(stream)))
    return int(g.value), ms.value * 1e-3


def probe_valu(waves_per_cu: int = 16, iters: int = 4096, stream=None):
    """Integer VALU issue probe. Returns (lane-instructions, seconds) of one timed launch."""
    lib = _abi.load()
    n = ctypes.c_uint64()
    ms = ctypes.c_double()
    check(lib.mlmc_probe_valu(int(waves_per_cu), int(iters), ctypes.byref(n), ctypes.byref(ms),
                              _stream_ptr(stream)))
    return int(n.value), ms.value * 1e-3

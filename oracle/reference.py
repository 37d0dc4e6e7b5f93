"""Deterministic FP64 references used to pin the oracle.

TEST INFRASTRUCTURE (see oracle/__init__.py).

  expm_action        x = exp(beta A) u by a dense library matrix exponential
                     (scipy.linalg.expm, scaling and squaring with Pade approximants).
  strang_level       x^l = (e^{dt D/2} e^{-dt T} e^{dt D/2})^N u, dt = beta/2^l, N = 2^l:
                     the splitting of section 2.1 evaluated densely. It is the exact
                     expectation of the level-l sample P_l (section 2.2), so
                     m_l = x^l - x^{l-1} is the exact expectation of each level term.
  laplace1d_exact    exp(tA) v for the 1D Dirichlet Laplacian by its sine eigenbasis.
  laplace2d_exact    the same for the 2D 5-point Laplacian (tensor product).
  decomposition      D and T of section 2.1 built densely from A.
  expm_action_sparse x = exp(beta A) u for a sparse A too large to exponentiate densely: the
                     truncated Taylor method with scaling of Al-Mohy & Higham (the reference
                     the paper cites for the action of the matrix exponential), by the library
                     routine scipy.sparse.linalg.expm_multiply, in FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


def decomposition(a: np.ndarray):
    """D = diag(a_ii + L_ii), T with T_ii = L_ii and T_ij = (-1)^sigma_ij L_ij, where
    L_ij = -|a_ij| (j != i) and L_ii = sum_{j != i} |a_ij| (section 2.1)."""
    a = np.asarray(a, np.float64)
    n = a.shape[0]
    off = a - np.diag(np.diag(a))
    L = -np.abs(off)
    Lii = -L.sum(axis=1)
    L = L + np.diag(Lii)
    sigma = (a < 0).astype(np.float64)
    T = np.where(np.eye(n, dtype=bool), L, ((-1.0) ** sigma) * L)
    D = np.diag(np.diag(a) + Lii)
    return D, T


def expm_action(a: np.ndarray, u: np.ndarray, beta: float) -> np.ndarray:
    return scipy.linalg.expm(beta * np.asarray(a, np.float64)) @ np.asarray(u, np.float64)


def strang_operator(a: np.ndarray, beta: float, level: int) -> np.ndarray:
    D, T = decomposition(a)
    N = 1 << level
    dt = beta / N
    half = np.diag(np.exp(np.diag(D) * dt / 2.0))
    S = half @ scipy.linalg.expm(-dt * T) @ half
    return np.linalg.matrix_power(S, N)


def strang_level(a: np.ndarray, u: np.ndarray, beta: float, level: int) -> np.ndarray:
    return strang_operator(a, beta, level) @ np.asarray(u, np.float64)


def simpson_weights(K: int) -> np.ndarray:
    """Composite Simpson weights of the K + 1 points of K (even) intervals: 1, 4, 2, ..., 4, 1."""
    w = np.where(np.arange(K + 1) % 2 == 1, 4.0, 2.0)
    w[0] = w[-1] = 1.0
    return w


def source_level(a: np.ndarray, u: np.ndarray, F: np.ndarray, beta: float, level: int) -> np.ndarray:
    """Expectation of Algorithm 3's fine sample at one level: S^N u + (dt/3) sum_n w_n S^n F,
    S the Strang step at dt = beta / N (the n-step product is the expectation of the fine
    functional at time n dt times F at the state then)."""
    D, T = decomposition(a)
    N = 1 << level
    dt = beta / N
    half = np.diag(np.exp(np.diag(D) * dt / 2.0))
    S = half @ scipy.linalg.expm(-dt * T) @ half
    w = simpson_weights(N)
    acc = np.zeros(len(u))
    v = np.asarray(F, np.float64).copy()
    for n in range(N + 1):
        acc += w[n] * v
        v = S @ v
    return np.linalg.matrix_power(S, N) @ np.asarray(u, np.float64) + dt / 3.0 * acc


def source_level_means(a, u, F, beta: float, l0: int, L: int):
    """Exact expectations of Algorithm 3's MLMC terms at levels l0..L."""
    xs = [source_level(a, u, F, beta, l) for l in range(l0, L + 1)]
    return [xs[0]] + [xs[q] - xs[q - 1] for q in range(1, len(xs))]


def inhomogeneous_exact(a: np.ndarray, u: np.ndarray, F: np.ndarray, beta: float) -> np.ndarray:
    """exp(beta A) u + int_0^beta exp(sA) F ds, by the augmented-matrix exponential
    [[A, F], [0, 0]] (Van Loan), no inverse of A needed."""
    n = a.shape[0]
    big = np.zeros((n + 1, n + 1))
    big[:n, :n] = a
    big[:n, n] = F
    E = scipy.linalg.expm(beta * big)
    return E[:n, :n] @ np.asarray(u, np.float64) + E[:n, n]


def level_means(a: np.ndarray, u: np.ndarray, beta: float, l0: int, L: int):
    """Exact expectations of the MLMC terms: [x^{l0}, x^{l0+1} - x^{l0}, ...]."""
    xs = [strang_level(a, u, beta, l) for l in range(l0, L + 1)]
    return [xs[0]] + [xs[q] - xs[q - 1] for q in range(1, len(xs))]


def _dst_ortho(x, axis=-1):
    return scipy.fft.dst(x, type=1, norm="ortho", axis=axis)


def laplace1d_exact(v: np.ndarray, t: float) -> np.ndarray:
    """exp(tA) v, A = (1/h^2) tridiag(1, -2, 1), h = 1/(n+1): eigenvectors sin(k pi i h),
    eigenvalues -(4/h^2) sin^2(k pi h / 2)."""
    v = np.asarray(v, np.float64)
    n = v.shape[0]
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    lam = -(4.0 / h ** 2) * np.sin(k * np.pi * h / 2.0) ** 2
    return _dst_ortho(np.exp(t * lam) * _dst_ortho(v))


def laplace2d_exact(v: np.ndarray, t: float) -> np.ndarray:
    """exp(tA) v for the m x m 5-point Laplacian in lexicographic order (x fastest)."""
    v = np.asarray(v, np.float64)
    m = int(round(np.sqrt(v.shape[0])))
    h = 1.0 / (m + 1)
    k = np.arange(1, m + 1)
    lam = -(4.0 / h ** 2) * np.sin(k * np.pi * h / 2.0) ** 2
    V = v.reshape(m, m)                      # [y, x]
    C = _dst_ortho(_dst_ortho(V, axis=0), axis=1)
    C = C * np.exp(t * (lam[:, None] + lam[None, :]))
    return _dst_ortho(_dst_ortho(C, axis=1), axis=0).reshape(-1)


def expm_action_sparse(n: int, row_ptr, col_idx, values, u, beta: float) -> np.ndarray:
    """exp(beta A) u for A in CSR form (u: n or n x R), FP64."""
    a = scipy.sparse.csr_matrix((np.asarray(values, np.float64), np.asarray(col_idx),
                                 np.asarray(row_ptr)), shape=(n, n))
    return scipy.sparse.linalg.expm_multiply(beta * a, np.asarray(u, np.float64))

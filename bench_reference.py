"""FP64 reference values of exp(tA) v for the benchmark's workloads, used by bench.py to
state the true error of every result it reports. This is measurement code, not part of the
estimator: the library never calls it, and it shares nothing with the oracle.

  expv_laplace1d / expv_laplace2d   closed forms for the Dirichlet Laplacians by their sine
                                    eigenbases (DST-I): e^{tA} v_k = e^{t lambda_k} v_k
  expv_dense                        a dense scaling-and-squaring exponential (scipy.linalg.expm)
  expv_sparse                       exp(beta A) U for a general sparse A by the truncated Taylor
                                    method with scaling of Al-Mohy & Higham (SIAM J. Sci.
                                    Comput. 33 (2011) 488-511; scipy.sparse.linalg.expm_multiply),
                                    in FP64, columns in parallel threads
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


def _dst(x, axis):
    return scipy.fft.dst(x, type=1, norm="ortho", axis=axis)


def laplacian_eigenvalues(m: int) -> np.ndarray:
    """-(4/h^2) sin^2(k pi h / 2), k = 1..m, h = 1/(m+1): the spectrum of
    (1/h^2) tridiag(1, -2, 1)."""
    h = 1.0 / (m + 1)
    k = np.arange(1, m + 1)
    return -(4.0 / (h * h)) * np.sin(0.5 * np.pi * k * h) ** 2


def expv_laplace1d(v, t: float) -> np.ndarray:
    v = np.asarray(v, np.float64)
    lam = laplacian_eigenvalues(v.shape[0])
    return _dst(np.exp(t * lam) * _dst(v, 0), 0)


def expv_laplace2d(v, t: float) -> np.ndarray:
    """v in lexicographic order on an m x m grid (x index fastest)."""
    v = np.asarray(v, np.float64)
    m = int(round(np.sqrt(v.shape[0])))
    lam = laplacian_eigenvalues(m)
    c = _dst(_dst(v.reshape(m, m), 0), 1) * np.exp(t * (lam[:, None] + lam[None, :]))
    return _dst(_dst(c, 1), 0).reshape(-1)


def expv_dense(a, v, t: float) -> np.ndarray:
    return scipy.linalg.expm(t * np.asarray(a, np.float64)) @ np.asarray(v, np.float64)


def to_scipy(A, scale: float = 1.0) -> scipy.sparse.csr_matrix:
    """An (n, row_ptr, col_idx, values) CSR object as a scipy matrix scaled by `scale`."""
    return scipy.sparse.csr_matrix((np.asarray(A.values, np.float64) * scale,
                                    np.asarray(A.col_idx), np.asarray(A.row_ptr)),
                                   shape=(A.n, A.n))


def expv_sparse(A, U, beta: float, threads: int = 8) -> np.ndarray:
    """exp(beta A) U in FP64 (U: n or n x R); blocks of columns run in parallel threads
    (the sparse products release the interpreter lock)."""
    M = to_scipy(A, beta)
    U = np.asarray(U, np.float64)
    if U.ndim == 1:
        return scipy.sparse.linalg.expm_multiply(M, U)
    R = U.shape[1]
    step = max(1, -(-R // max(1, threads)))
    blocks = [(c, min(R, c + step)) for c in range(0, R, step)]
    with ThreadPoolExecutor(len(blocks)) as ex:
        parts = list(ex.map(lambda b: scipy.sparse.linalg.expm_multiply(M, U[:, b[0]:b[1]]), blocks))
    return np.concatenate(parts, axis=1)

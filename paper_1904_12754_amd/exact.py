"""Exact FP64 values of exp(tA) v for the Dirichlet Laplacians the workloads use, from
their sine eigenbases (DST-I). Used to report the true error of an MLMC estimate; it is
not part of the estimator.
"""
from __future__ import annotations

import numpy as np
import scipy.fft


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

"""The benchmark's FP64 references (bench_reference.py, the values every reported true error
is measured against) pinned against the dense scaling-and-squaring exponential and the
Laplacians' eigenbases. CPU only."""
import numpy as np
import scipy.linalg

import bench_reference as br
from paper_1904_12754_amd import inputs


def _dense(A, U, beta):
    return scipy.linalg.expm(beta * A.to_dense()) @ np.asarray(U, np.float64)


def test_dst_forms_match_the_dense_exponential():
    A = inputs.laplacian_1d(50)
    v = inputs.rhs_sine_noise(50, 3)
    t = 3.0 / A.norm1()
    assert np.max(np.abs(br.expv_laplace1d(v, t) - _dense(A, v, t))) < 1e-13
    A2 = inputs.laplacian_2d(12)
    v2 = np.random.default_rng(2).normal(size=A2.n)
    t2 = 4.0 / A2.norm1()
    assert np.max(np.abs(br.expv_laplace2d(v2, t2) - _dense(A2, v2, t2))) < 1e-13


def test_sparse_reference_matches_the_dense_exponential():
    rng = np.random.default_rng(5)
    a = rng.normal(size=(80, 80)) * (rng.random((80, 80)) < 0.08)
    A = inputs.from_dense(a)
    U = rng.normal(size=(80, 13))                     # several column blocks in threads
    beta = 6.0 / A.norm1()
    x = br.expv_sparse(A, U, beta, threads=4)
    ref = _dense(A, U, beta)
    assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))
    xv = br.expv_sparse(A, U[:, 0], beta)
    assert np.max(np.abs(xv - ref[:, 0])) <= 1e-12 * np.max(np.abs(ref[:, 0]))
    Acd = inputs.convection_diffusion_3d(7, seed=1)
    v = inputs.rhs_gaussian_bump(7)
    t = 4.0 / Acd.norm1()
    ref = _dense(Acd, v, t)
    assert np.max(np.abs(br.expv_sparse(Acd, v, t) - ref)) <= 1e-12 * np.max(np.abs(ref))

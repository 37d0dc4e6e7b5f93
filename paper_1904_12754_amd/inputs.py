"""Seeded synthetic workloads: sparse matrices (CSR) and right-hand sides.

This module holds no arithmetic of the MLMC method. It only builds inputs shaped like
the paper's test problems (section 5: method-of-lines PDE operators and
complex-network adjacency matrices), so that the GPU library, the tests and the
benchmark all read identical bytes. Every generator is deterministic in its seed.

CSR convention: int64 row_ptr (n + 1), int32 col_idx sorted within each row, values
float64 (callers cast to float32 where a workload asks for it).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    values: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n), np.float64)
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        np.add.at(a, (rows, self.col_idx), self.values)
        return a

    def scaled(self, s: float) -> "CSR":
        return CSR(self.n, self.row_ptr, self.col_idx, self.values * s)

    def norm1(self) -> float:
        """max_j sum_i |a_ij| (the induced 1-norm)."""
        colsum = np.zeros(self.n, np.float64)
        np.add.at(colsum, self.col_idx, np.abs(self.values))
        return float(colsum.max()) if self.n else 0.0


def from_coo(n: int, rows, cols, vals) -> CSR:
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    vals = np.asarray(vals, np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    # merge duplicates
    if rows.size:
        key = rows * n + cols
        uniq, start = np.unique(key, return_index=True)
        vals = np.add.reduceat(vals, start)
        rows = uniq // n
        cols = uniq % n
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return CSR(n, row_ptr, cols.astype(np.int32), vals)


def from_dense(a: np.ndarray) -> CSR:
    a = np.asarray(a, np.float64)
    r, c = np.nonzero(a)
    return from_coo(a.shape[0], r, c, a[r, c])


# ----------------------------------------------------------------------------------
# PDE operators (section 5, method of lines)
# ----------------------------------------------------------------------------------
def laplacian_1d(n: int) -> CSR:
    """(1/h^2) tridiag(1, -2, 1), Dirichlet, h = 1/(n+1)."""
    h2 = float(n + 1) ** 2
    i = np.arange(n)
    rows = np.concatenate([i, i[1:], i[:-1]])
    cols = np.concatenate([i, i[1:] - 1, i[:-1] + 1])
    vals = np.concatenate([np.full(n, -2.0 * h2), np.full(n - 1, h2), np.full(n - 1, h2)])
    return from_coo(n, rows, cols, vals)


def laplacian_2d(m: int) -> CSR:
    """5-point Dirichlet Laplacian on an m x m interior grid, lexicographic order,
    h = 1/(m+1)."""
    h2 = float(m + 1) ** 2
    n = m * m
    idx = np.arange(n)
    ix, iy = idx % m, idx // m
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, -4.0 * h2)]
    for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        ok = (ix + dx >= 0) & (ix + dx < m) & (iy + dy >= 0) & (iy + dy < m)
        rows.append(idx[ok])
        cols.append(idx[ok] + dx + dy * m)
        vals.append(np.full(int(ok.sum()), h2))
    return from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def convection_diffusion_3d(m: int, seed: int, extent: float = 4.0,
                            log_kappa_sigma: float = 0.5) -> CSR:
    """Cell-centred 7-point operator for div(kappa grad u) + b . grad u on [-e, e]^3 with
    homogeneous Dirichlet data, m^3 unknowns, h = 2e/(m+1). Per cell: kappa =
    exp(N(0, sigma^2)), velocity b with components U(-1, 1). Face diffusivity is the
    harmonic mean of the two cells; convection is by central differences (so the
    matrix is nonsymmetric and may have off-diagonals of either sign)."""
    rng = np.random.default_rng(seed)
    n = m ** 3
    h = 2.0 * extent / (m + 1)
    kappa = np.exp(rng.normal(0.0, log_kappa_sigma, size=n))
    b = rng.uniform(-1.0, 1.0, size=(n, 3))
    idx = np.arange(n)
    coords = (idx % m, (idx // m) % m, idx // (m * m))
    strides = (1, m, m * m)
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for axis in range(3):
        c = coords[axis]
        for sgn in (1, -1):
            ok = (c + sgn >= 0) & (c + sgn < m)
            nb = idx + sgn * strides[axis]
            # face diffusivity: harmonic mean (boundary face: the cell's own kappa)
            kf = np.where(ok, 2.0 * kappa * kappa[np.where(ok, nb, idx)] /
                          (kappa + kappa[np.where(ok, nb, idx)]), kappa)
            diff = kf / (h * h)
            conv = sgn * b[:, axis] / (2.0 * h)
            diag -= diff
            rows.append(idx[ok])
            cols.append(nb[ok])
            vals.append((diff + conv)[ok])
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    return from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# ----------------------------------------------------------------------------------
# networks (section 5, total communicability)
# ----------------------------------------------------------------------------------
def barabasi_albert(n: int, m: int, seed: int) -> CSR:
    """Preferential attachment by the repeated-endpoint list (V. Batagelj, U. Brandes,
    Phys. Rev. E 71, 036113, 2005): a seed clique on m+1 nodes, then each new node v
    adds m edges whose far endpoints are copies of uniformly chosen earlier list
    entries (probability proportional to degree). The pointer chains are resolved in
    vectorised passes. Self-loops and repeated edges are dropped, giving a symmetric
    0/1 adjacency."""
    rng = np.random.default_rng(seed)
    m0 = m + 1
    ci, cj = np.triu_indices(m0, 1)
    n_seed_edges = ci.size
    n_new = max(n - m0, 0)
    E = n_seed_edges + n_new * m
    lst = np.empty(2 * E, np.int64)
    lst[0:2 * n_seed_edges:2] = ci
    lst[1:2 * n_seed_edges:2] = cj
    e = np.arange(n_seed_edges, E)
    src = m0 + (e - n_seed_edges) // m
    lst[2 * e] = src
    # far endpoint of edge e: copy of a uniformly chosen entry among the entries laid
    # down before node src started adding edges
    first_of_node = n_seed_edges + (src - m0) * m
    ptr = (rng.random(e.size) * (2 * first_of_node)).astype(np.int64)
    target = np.full(e.size, -1, np.int64)
    pos = ptr.copy()
    done = (pos % 2) == 0
    target[done] = lst[pos[done]]
    while not done.all():
        todo = ~done
        pidx = pos[todo]
        # odd position 2k+1 belongs to edge k; its value is either a seed entry or the
        # far endpoint chosen for edge k
        k = pidx // 2
        seed_edge = k < n_seed_edges
        newpos = pidx.copy()
        vals = np.full(pidx.size, -1, np.int64)
        vals[seed_edge] = lst[pidx[seed_edge]]
        newpos[~seed_edge] = ptr[k[~seed_edge] - n_seed_edges]
        resolved = seed_edge | (newpos % 2 == 0)
        vals[~seed_edge & resolved] = lst[newpos[~seed_edge & resolved]]
        t_idx = np.nonzero(todo)[0]
        target[t_idx[resolved]] = vals[resolved]
        done[t_idx[resolved]] = True
        pos[t_idx[~resolved]] = newpos[~resolved]
    lst[2 * e + 1] = target
    a = lst[0::2]
    b = lst[1::2]
    keep = a != b
    a, b = a[keep], b[keep]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    key = np.unique(rows * n + cols)
    rows, cols = key // n, key % n
    return from_coo(n, rows, cols, np.ones(rows.size))


def erdos_renyi(n: int, mean_degree: float, seed: int) -> CSR:
    """G(n, p) with p = mean_degree / (n - 1), symmetric 0/1 adjacency, sampled by
    drawing the number of edges and then uniform pairs (repeats dropped)."""
    rng = np.random.default_rng(seed)
    n_pairs = n * (n - 1) // 2
    p = mean_degree / max(n - 1, 1)
    k = rng.binomial(n_pairs, p)
    a = rng.integers(0, n, size=int(k * 1.05) + 16)
    b = rng.integers(0, n, size=a.size)
    keep = a != b
    a, b = a[keep], b[keep]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = np.unique(lo * n + hi)[:k]
    lo, hi = key // n, key % n
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    return from_coo(n, rows, cols, np.ones(rows.size))


# ----------------------------------------------------------------------------------
# right-hand sides
# ----------------------------------------------------------------------------------
def rhs_sine_noise(n: int, seed: int, noise: float = 0.1) -> np.ndarray:
    """v_i = sin(pi i h) + U(0, noise), i = 1..n, h = 1/(n+1)."""
    rng = np.random.default_rng(seed)
    i = np.arange(1, n + 1)
    return np.sin(np.pi * i / (n + 1)) + rng.uniform(0.0, noise, size=n)


def rhs_normal(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(size=n)


def rhs_ones_rademacher(n: int, R: int, seed: int) -> np.ndarray:
    """n x R, row major: column 0 all ones, columns 1..R-1 Rademacher +-1."""
    rng = np.random.default_rng(seed)
    u = np.empty((n, R), np.float64)
    u[:, 0] = 1.0
    if R > 1:
        u[:, 1:] = rng.integers(0, 2, size=(n, R - 1)) * 2.0 - 1.0
    return u


def rhs_gaussian_bump(m: int, extent: float = 4.0) -> np.ndarray:
    """v_i = exp(-|x_i|^2) at the cell centres of the m^3 grid on [-e, e]^3."""
    h = 2.0 * extent / (m + 1)
    c = -extent + h * np.arange(1, m + 1)
    x, y, z = c[None, None, :], c[None, :, None], c[:, None, None]
    return np.exp(-(x * x + y * y + z * z)).reshape(-1)


# ----------------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------------
DATA_SEED = 20190429


def workload_laplace1d():
    """1D Dirichlet Laplacian, n = 100, t = 1e-4, v = sin(pi i h) + U(0, 0.1)."""
    A = laplacian_1d(100)
    return A, 1e-4, rhs_sine_noise(100, DATA_SEED)


def workload_laplace2d(m: int = 256):
    """2D 5-point Laplacian on m x m, t = h^2/2 (so ||tA||_1 = 4), v ~ N(0, 1)."""
    A = laplacian_2d(m)
    h = 1.0 / (m + 1)
    return A, h * h / 2.0, rhs_normal(m * m, DATA_SEED + 1)


def workload_ba_tc(n: int = 1_000_000, m: int = 5, R: int = 64):
    """Barabasi-Albert adjacency, beta = 1/d_max, R right-hand sides (ones + Rademacher)."""
    A = barabasi_albert(n, m, DATA_SEED + 2)
    dmax = float(np.diff(A.row_ptr).max())
    return A, 1.0 / dmax, rhs_ones_rademacher(n, R, DATA_SEED + 3)


def workload_uneven_batch(count: int = 512, nmin: int = 1000, nmax: int = 100_000,
                          seed: int = DATA_SEED + 4):
    """`count` instances: type uniform over {1D Laplacian, 2D Laplacian, ER(mean deg 8)},
    n log-uniform in [nmin, nmax], t = c / ||A||_1 with c log-uniform in [0.5, 8],
    v ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        kind = int(rng.integers(0, 3))
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        c = float(np.exp(rng.uniform(np.log(0.5), np.log(8.0))))
        if kind == 0:
            A = laplacian_1d(n)
        elif kind == 1:
            side = max(2, int(round(np.sqrt(n))))
            A = laplacian_2d(side)
        else:
            A = erdos_renyi(n, 8.0, int(rng.integers(0, 2 ** 31)))
        t = c / A.norm1()
        v = rng.normal(size=A.n)
        out.append((A, t, v))
    return out


def small_chain(n: int, seed: int, signed: bool, density: float, d_spread: float):
    """A small dense-ish matrix for pins of the level structure: off-diagonal entries
    U(-1, 1) (signed) or U(0.3, 1) (positive) kept with probability `density`, scaled so
    that the largest off-diagonal absolute row sum is 1, and a diagonal chosen so that the
    row's diagonal weight a_ii + sum_{j != i} |a_ij| is U(-d_spread, d_spread); right-hand
    side U(-1, 1) (signed) or U(0.5, 1.5). Returns (CSR, u); a time beta makes beta the
    largest jump rate times beta."""
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, (n, n)) if signed else rng.uniform(0.3, 1.0, (n, n))
    off = off * (rng.uniform(size=(n, n)) < density)
    np.fill_diagonal(off, 0.0)
    rowabs = np.abs(off).sum(axis=1)
    off = off / rowabs.max()
    weight = rng.uniform(-d_spread, d_spread, n)
    a = off + np.diag(weight - np.abs(off).sum(axis=1))
    u = rng.uniform(-1.0, 1.0, n) if signed else rng.uniform(0.5, 1.5, n)
    return from_dense(a), u


def workload_convdiff3d(m: int = 128):
    """3D 7-point convection-diffusion, m^3 cells on [-4, 4]^3, ||tA||_1 = 4,
    v = exp(-|x|^2)."""
    A = convection_diffusion_3d(m, DATA_SEED + 5)
    t = 4.0 / A.norm1()
    return A, t, rhs_gaussian_bump(m)

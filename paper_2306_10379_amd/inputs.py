"""Seeded synthetic inputs shared by the device solver, the tests and the benchmark.

This module builds problems and starting blocks only; it holds none of the
eigensolver's arithmetic. Everything is deterministic from an integer seed
(NumPy's counter-based Philox bit generator).

Matrices are returned as :class:`CSR` (full symmetric storage, sorted column
indices, int32 indices, float64 values).

Families (the paper's workloads and their synthetic stand-ins):

* ``laplacian_2d`` / ``laplacian_3d`` -- standard finite-difference Laplacians
  with zero Dirichlet boundary (5- and 7-point stencils, unit mesh scaling:
  diagonal 4 or 6, off-diagonals -1), lexicographic row order, as used in the
  paper's Laplacian experiments (Sec. 6.2 and the FD3D matrix of Sec. 6.3).
* ``schrodinger_2d`` -- H = -Delta_h + V on the unit square with h = 1/(N+1)
  and V a sum of Gaussian wells sampled at the grid nodes.
* ``spiked_sparse`` -- a sparse symmetric random matrix with uniform-random
  columns (a stand-in for the SuiteSparse matrices of Sec. 6.3, which are not
  available here), with a few diagonal spikes that create a dominant subspace.
* ``start_block`` -- i.i.d. N(0,1) entries, the starting block before
  orthonormalization (the paper leaves the distribution of X0 open).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    """Counter-based generator (Philox) keyed by ``seed``."""
    return np.random.Generator(np.random.Philox(key=int(seed)))


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32 (or int64 when nnz >= 2**31), length n+1
    colind: np.ndarray  # int32, length nnz, sorted within each row
    vals: np.ndarray    # float64, length nnz

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.vals, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        d[rows, self.colind] = self.vals
        return d


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Sort (row, col) pairs, sum duplicates and return a CSR."""
    rows = rows.astype(np.int64)
    cols = cols.astype(np.int64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if vals.size else vals
    r = (uniq // n).astype(np.int64)
    c = (uniq % n).astype(np.int32)
    counts = np.bincount(r, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] < 2**31:
        rowptr = rowptr.astype(np.int32)
    return CSR(n=n, rowptr=rowptr, colind=c, vals=summed.astype(np.float64))


def _stencil(dims: tuple[int, ...], diag: float, off: float, shift: np.ndarray | None = None) -> CSR:
    """Dirichlet finite-difference stencil on a tensor grid, lexicographic order
    (the first dimension varies fastest)."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    rows = [idx]
    cols = [idx]
    dvals = np.full(n, diag, dtype=np.float64)
    if shift is not None:
        dvals = dvals + shift
    vals = [dvals]
    stride = 1
    for axis, d in enumerate(dims):
        c = coords[axis]
        for step in (-1, 1):
            ok = (c + step >= 0) & (c + step < d)
            rows.append(idx[ok])
            cols.append(idx[ok] + step * stride)
            vals.append(np.full(int(ok.sum()), off, dtype=np.float64))
        stride *= d
    return _from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def laplacian_2d(nx: int, ny: int | None = None) -> CSR:
    """5-point Dirichlet Laplacian on an nx-by-ny grid (diagonal 4, off-diagonal -1)."""
    return _stencil((nx, ny if ny is not None else nx), 4.0, -1.0)


def laplacian_3d(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """7-point Dirichlet Laplacian on an nx-by-ny-by-nz grid (diagonal 6, off-diagonal -1)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return _stencil((nx, ny, nz), 6.0, -1.0)


@dataclass
class Wells:
    """Gaussian wells V(x) = sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2)) on the unit square."""
    amp: np.ndarray      # (m,)
    width: np.ndarray    # (m,)
    centre: np.ndarray   # (m, 2)

    def sample(self, N: int) -> np.ndarray:
        h = 1.0 / (N + 1)
        t = h * np.arange(1, N + 1)
        x, y = np.meshgrid(t, t, indexing="xy")  # x varies fastest along a row of the grid
        v = np.zeros((N, N))
        for a, w, c in zip(self.amp, self.width, self.centre):
            v += a * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2) / (2.0 * w * w))
        return v.reshape(-1)

    def as_vector(self) -> np.ndarray:
        return np.concatenate([self.amp, self.width, self.centre.reshape(-1)])


def random_wells(seed: int, count: int | tuple[int, int] = (1, 6),
                 amp: tuple[float, float] = (-20.0, 0.0),
                 width: tuple[float, float] = (0.02, 0.2)) -> Wells:
    g = rng(seed)
    m = int(count) if np.isscalar(count) else int(g.integers(count[0], count[1] + 1))
    return Wells(amp=g.uniform(amp[0], amp[1], m), width=g.uniform(width[0], width[1], m),
                 centre=g.uniform(0.0, 1.0, (m, 2)))


def schrodinger_2d(N: int, wells: Wells | None) -> CSR:
    """H = -Delta_h + V on the unit square, N-by-N interior nodes, h = 1/(N+1)."""
    h2 = float(N + 1) ** 2
    v = wells.sample(N) if wells is not None else np.zeros(N * N)
    A = _stencil((N, N), 4.0, -1.0)
    A.vals *= h2
    # add V on the diagonal
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    diag = np.nonzero(rows == A.colind)[0]
    A.vals[diag] += v
    return A


def moving_well_sequence(N: int, steps: int, seed: int = 0, depth: float = -15.0, width: float = 0.08,
                         start=(0.35, 0.4), velocity=(0.01, 0.005)):
    """Schroedinger operators H_t = -Laplacian + V_t, t = 0 .. steps-1, on one N x N grid
    (one sparsity pattern): a fixed random background of wells plus one Gaussian well of the
    given depth and width whose centre moves by `velocity` per step (a slowly varying
    sequence, as in self-consistent field iterations or time stepping)."""
    bg = random_wells(seed, count=3, amp=(-8.0, 0.0))
    mats = []
    for t in range(steps):
        c = np.array([[start[0] + t * velocity[0], start[1] + t * velocity[1]]])
        w = Wells(amp=np.concatenate([bg.amp, [depth]]), width=np.concatenate([bg.width, [width]]),
                  centre=np.concatenate([bg.centre, c]))
        mats.append(schrodinger_2d(N, w))
    return mats


def magnetic_lattice(N: int, flux: float = 0.1, seed: int = 0, disorder: float = 0.5):
    """Complex Hermitian test operator: the 5-point Laplacian on an N x N grid with Peierls
    phases of a uniform magnetic field (Landau gauge: the bond (x, y) -> (x + 1, y) carries
    exp(2 pi i flux y)), plus a random on-site potential U(-disorder, disorder) that lifts
    degeneracies. Returns a scipy CSR complex128 matrix, sorted indices."""
    import scipy.sparse as sps
    g = rng(seed)
    n = N * N
    idx = np.arange(n)
    x, y = idx % N, idx // N
    rows, cols, vals = [idx], [idx], [4.0 + g.uniform(-disorder, disorder, n)]
    ok = x < N - 1
    t = -np.exp(2j * np.pi * flux * y[ok])
    rows += [idx[ok], idx[ok] + 1]
    cols += [idx[ok] + 1, idx[ok]]
    vals += [t, np.conj(t)]
    ok = y < N - 1
    rows += [idx[ok], idx[ok] + N]
    cols += [idx[ok] + N, idx[ok]]
    vals += [-np.ones(ok.sum()), -np.ones(ok.sum())]
    A = sps.csr_matrix((np.concatenate(vals).astype(np.complex128), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n, n))
    A.sort_indices()
    return A


def schrodinger_batch(count: int = 512, seed: int = 2024, sides: tuple[int, int] = (32, 160),
                      blocks: tuple[int, int] = (4, 32), wells: tuple[int, int] = (1, 6)):
    """A batch of 2D Schroedinger operators H = -Laplacian + V of uneven sizes: grid side N
    uniform in `sides`, block size p uniform in `blocks`, V a sum of `wells` Gaussian wells
    (depth U(-20, 0), width U(0.02, 0.2), centre U([0,1]^2)); each with its own N(0,1)
    start block. Returns (mats, X0s, ps)."""
    g = rng(seed)
    mats, X0s, ps = [], [], []
    for i in range(count):
        N = int(g.integers(sides[0], sides[1] + 1))
        p = int(g.integers(blocks[0], blocks[1] + 1))
        A = schrodinger_2d(N, random_wells(seed * 10_000 + i, count=wells))
        mats.append(A)
        ps.append(p)
        X0s.append(start_block(A.n, p, seed * 10_000 + 5_000 + i))
    return mats, X0s, ps


def spiked_sparse(n: int, half_degree: int, p: int, seed: int, gap: float = 1e-3,
                  spike_max: float = 3.0) -> CSR:
    """Sparse symmetric random matrix with uniform-random columns plus diagonal spikes.

    Each row draws ``half_degree`` uniform columns j != i with N(0,1)/sqrt(2*half_degree)
    values; the matrix is B + B^T, so about 2*half_degree off-diagonals per row and a bulk
    spectrum near [-2, 2]. ``p`` seeded rows get diagonal spikes theta with theta + 1/theta
    above the bulk edge 2: the smallest spike puts its outlier ``gap`` above the edge and the
    others are spread up to ``spike_max``.
    """
    g = rng(seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), half_degree)
    cols = g.integers(0, n - 1, size=rows.shape[0], dtype=np.int64)
    cols = cols + (cols >= rows)  # uniform over j != i
    vals = g.standard_normal(rows.shape[0]) / np.sqrt(2.0 * half_degree)
    # theta + 1/theta = 2 + gap  ->  theta = (t + sqrt(t^2 - 4)) / 2
    t = 2.0 + gap
    theta_lo = 0.5 * (t + np.sqrt(t * t - 4.0))
    spikes = np.sort(np.concatenate([[theta_lo], g.uniform(theta_lo, spike_max, p - 1)]))[::-1]
    where = g.choice(n, size=p, replace=False)
    r = np.concatenate([rows, cols, where])
    c = np.concatenate([cols, rows, where])
    v = np.concatenate([vals, vals, spikes])
    return _from_coo(n, r, c, v)


def random_symmetric_dense(n: int, seed: int, spectrum: np.ndarray | None = None) -> np.ndarray:
    """Dense symmetric matrix Q diag(spectrum) Q^T with a Haar-like orthogonal Q (small tests)."""
    g = rng(seed)
    q, r = np.linalg.qr(g.standard_normal((n, n)))
    q = q * np.sign(np.diag(r))
    s = g.standard_normal(n) if spectrum is None else np.asarray(spectrum, dtype=np.float64)
    return (q * s) @ q.T


def dense_to_csr(a: np.ndarray, drop: float = 0.0) -> CSR:
    n = a.shape[0]
    r, c = np.nonzero(np.abs(a) > drop)
    return _from_coo(n, r, c, a[r, c])


def start_block(n: int, p: int, seed: int) -> np.ndarray:
    """n-by-p block of i.i.d. N(0,1) entries (row-major float64)."""
    return rng(seed).standard_normal((n, p))

"""Seeded synthetic inputs shaped like the paper's workloads.

The paper measures on SuiteSparse matrices (its Table 1: n from 1.2M to 8.3M,
4 to 58 nonzeros per row, from circuit simulation, CFD, FEM and porous-media
problems).  Those matrices are not available here, so these generators stand
in for them: power-law random patterns for the circuit-like matrices and 3D
stencils for the PDE matrices, at the same scale.

This module is shared by the GPU library's tests/benchmarks and by the CPU
oracle's tests.  It only builds inputs (index patterns, coefficients, random
vectors); it performs none of the operations under test -- no products, no
solves.  Right-hand sides of the form b = A x* are therefore computed by the
caller with whichever SpMV it is allowed to use.

Every random draw comes from numpy's counter-based Philox generator seeded
with an explicit integer, so the same seed yields the same bytes everywhere.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MATRIX_SEED = 2103
VECTOR_SEED = 10116
SERVING_SEED = 355


@dataclass
class CSRMatrix:
    """Host CSR matrix: int32 row pointers and column indices, FP64 values."""
    n: int
    ncols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def to_dense(self) -> np.ndarray:
        """Dense copy, for tiny matrices only."""
        M = np.zeros((self.n, self.ncols))
        rows = np.repeat(np.arange(self.n), self.row_lengths())
        M[rows, self.col] = self.val
        return M


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


def uniform_vector(n: int, seed: int = VECTOR_SEED, lo=-1.0, hi=1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=n)


def _from_dense_mask(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> CSRMatrix:
    """Rows of `cols`/`vals` (shape [n, k]) whose columns ascend along axis 1."""
    n = cols.shape[0]
    counts = mask.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return CSRMatrix(n, n, rowptr.astype(np.int32), col, val)


def _stencil(dims, offsets, coeff) -> CSRMatrix:
    """Dirichlet-truncated stencil on a regular grid in natural ordering
    (x fastest).  `offsets` must ascend in linear offset so that columns come
    out sorted; `coeff(off)` gives the coefficient for an offset tuple."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    grids = np.meshgrid(*[np.arange(d) for d in reversed(dims)], indexing="ij")
    coords = [g.reshape(-1) for g in reversed(grids)]  # coords[0] = x (fastest)
    strides = [int(np.prod(dims[:d])) for d in range(len(dims))]
    k = len(offsets)
    cols = np.empty((n, k), np.int64)
    vals = np.empty((n, k), np.float64)
    mask = np.ones((n, k), bool)
    idx = np.arange(n, dtype=np.int64)
    for j, off in enumerate(offsets):
        lin = sum(o * s for o, s in zip(off, strides))
        cols[:, j] = idx + lin
        vals[:, j] = coeff(off)
        for d, o in enumerate(off):
            if o:
                c = coords[d] + o
                mask[:, j] &= (c >= 0) & (c < dims[d])
    return _from_dense_mask(cols, vals, mask)


def _sorted_offsets(ndim, reach):
    rng_ = range(-reach, reach + 1)
    if ndim == 2:
        offs = [(dx, dy) for dy in rng_ for dx in rng_]
    else:
        offs = [(dx, dy, dz) for dz in rng_ for dy in rng_ for dx in rng_]
    return offs  # z, y, x nesting = ascending linear offset


def poisson2d(m: int) -> CSRMatrix:
    """5-point Laplacian on an m x m grid: 4 on the diagonal, -1 off it."""
    offs = [o for o in _sorted_offsets(2, 1) if sum(abs(v) for v in o) <= 1]
    return _stencil((m, m), offs, lambda o: 4.0 if o == (0, 0) else -1.0)


def poisson3d(N: int) -> CSRMatrix:
    """7-point Laplacian on an N^3 grid: 6 on the diagonal, -1 off it."""
    offs = [o for o in _sorted_offsets(3, 1) if sum(abs(v) for v in o) <= 1]
    return _stencil((N, N, N), offs, lambda o: 6.0 if o == (0, 0, 0) else -1.0)


def stencil27(N: int) -> CSRMatrix:
    """27-point stencil on an N^3 grid: 26 on the diagonal, -1 for every other
    point of the 3x3x3 neighbourhood, truncated at the Dirichlet boundary
    (nnz = (3N-2)^3)."""
    offs = _sorted_offsets(3, 1)
    return _stencil((N, N, N), offs, lambda o: 26.0 if o == (0, 0, 0) else -1.0)


def convdiff3d(N: int, c: float = 10.0) -> CSRMatrix:
    """First-order upwind discretisation of -Lap(u) + c (u_x + u_y + u_z) on
    the unit cube, mesh width h = 1/(N+1), scaled by h^2: diagonal 6 + 3ch,
    upwind neighbour (offset -1 along an axis) -(1 + ch), downwind -1."""
    h = 1.0 / (N + 1)
    offs = [o for o in _sorted_offsets(3, 1) if sum(abs(v) for v in o) <= 1]

    def coeff(o):
        if o == (0, 0, 0):
            return 6.0 + 3.0 * c * h
        return -(1.0 + c * h) if min(o) < 0 else -1.0

    return _stencil((N, N, N), offs, coeff)


def zipf_lengths(n: int, s: float, kmax: int, g: np.random.Generator) -> np.ndarray:
    """Row lengths L = min(K, kmax) with K ~ Zipf(s), P(K=k) = k^-s / zeta(s)."""
    return np.minimum(g.zipf(s, size=n), kmax).astype(np.int64)


def zipf_random(n: int, s: float = 2.0, kmax: int = 4096, seed: int = MATRIX_SEED,
                ncols: int | None = None) -> CSRMatrix:
    """Power-law random pattern: Zipf(s) row lengths clipped to [1, kmax],
    distinct sorted columns uniform in [0, ncols), values U[-1, 1]."""
    ncols = n if ncols is None else ncols
    g = rng(seed)
    L = np.minimum(zipf_lengths(n, s, kmax, g), ncols)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(L, out=rowptr[1:])
    nnz = int(rowptr[-1])
    rows = np.repeat(np.arange(n, dtype=np.int64), L)
    cols = g.integers(0, ncols, size=nnz, dtype=np.int64)
    # sort within rows; redraw duplicates until every row's columns are distinct
    while True:
        key = rows * ncols + cols
        order = np.argsort(key, kind="stable")
        key = key[order]
        cols = cols[order]
        dup = np.zeros(nnz, bool)
        dup[1:] = key[1:] == key[:-1]
        nd = int(dup.sum())
        if nd == 0:
            break
        cols[dup] = g.integers(0, ncols, size=nd, dtype=np.int64)
    val = g.uniform(-1.0, 1.0, size=nnz)
    return CSRMatrix(n, ncols, rowptr.astype(np.int32), cols.astype(np.int32), val)


def _coo_to_sorted_csr(n, rows, cols, vals) -> CSRMatrix:
    """Sort triplets by (row, col) and sum duplicates in input order."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    r = (uniq // n).astype(np.int64)
    c = (uniq % n).astype(np.int32)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rowptr[1:])
    return CSRMatrix(n, n, rowptr.astype(np.int32), c, summed.astype(np.float64))


def random_spd(n: int, s: float = 2.0, kmax: int = 4096, seed: int = MATRIX_SEED) -> CSRMatrix:
    """Symmetric positive definite matrix from the power-law pattern:
    S = (A + A^T)/2 with the diagonal removed, then d_i = 1.1 * sum_j |s_ij|
    (d_i = 1 for an empty row).  SPD by symmetry and strict diagonal
    dominance (Gershgorin)."""
    A = zipf_random(n, s, kmax, seed)
    rows = np.repeat(np.arange(n, dtype=np.int64), A.row_lengths())
    cols = A.col.astype(np.int64)
    r = np.concatenate([rows, cols])
    c = np.concatenate([cols, rows])
    v = np.concatenate([A.val * 0.5, A.val * 0.5])
    off = r != c
    r, c, v = r[off], c[off], v[off]
    absum = np.bincount(r, weights=np.abs(v), minlength=n)
    d = np.where(absum > 0, 1.1 * absum, 1.0)
    r = np.concatenate([r, np.arange(n, dtype=np.int64)])
    c = np.concatenate([c, np.arange(n, dtype=np.int64)])
    v = np.concatenate([v, d])
    return _coo_to_sorted_csr(n, r, c, v)


def random_spd_small(n: int, cond: float, seed: int) -> np.ndarray:
    """Dense SPD matrix Q diag(lam) Q^T with eigenvalues log-spaced in
    [1, cond] (for tiny finite-termination tests)."""
    g = rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.logspace(0.0, np.log10(cond), n)
    M = (Q * lam) @ Q.T
    return 0.5 * (M + M.T)


def dense_to_csr(M: np.ndarray, drop_zeros: bool = True) -> CSRMatrix:
    n, m = M.shape
    mask = M != 0 if drop_zeros else np.ones_like(M, bool)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    rr, cc = np.nonzero(mask)
    return CSRMatrix(n, m, rowptr.astype(np.int32), cc.astype(np.int32),
                     M[rr, cc].astype(np.float64))


def serving_system(m: int, seed: int) -> CSRMatrix:
    """Weighted Dirichlet 5-point Laplacian on an m x m grid: every interior
    edge gets a weight U[0.5, 1.5] (same on both sides), each of the 4m
    boundary edges adds a weight U[0.5, 1.5] to its cell's diagonal, and the
    whole diagonal is shifted by one sigma ~ U[0, 1].  SPD."""
    g = rng(seed)
    n = m * m
    wx = g.uniform(0.5, 1.5, size=(m, m - 1))  # edge (y,x)-(y,x+1)
    wy = g.uniform(0.5, 1.5, size=(m - 1, m))  # edge (y,x)-(y+1,x)
    ghost = g.uniform(0.5, 1.5, size=4 * m)    # left, right, bottom, top sides
    sigma = g.uniform(0.0, 1.0)
    diag = np.zeros((m, m))
    diag[:, :-1] += wx
    diag[:, 1:] += wx
    diag[:-1, :] += wy
    diag[1:, :] += wy
    diag[:, 0] += ghost[:m]
    diag[:, -1] += ghost[m:2 * m]
    diag[0, :] += ghost[2 * m:3 * m]
    diag[-1, :] += ghost[3 * m:]
    diag += sigma
    # columns ascend: south (i-m), west (i-1), self, east (i+1), north (i+m)
    idx = np.arange(n, dtype=np.int64).reshape(m, m)
    cols = np.stack([idx - m, idx - 1, idx, idx + 1, idx + m], axis=-1).reshape(n, 5)
    vals = np.zeros((m, m, 5))
    mask = np.zeros((m, m, 5), bool)
    vals[1:, :, 0] = -wy
    mask[1:, :, 0] = True
    vals[:, 1:, 1] = -wx
    mask[:, 1:, 1] = True
    vals[:, :, 2] = diag
    mask[:, :, 2] = True
    vals[:, :-1, 3] = -wx
    mask[:, :-1, 3] = True
    vals[:-1, :, 4] = -wy
    mask[:-1, :, 4] = True
    return _from_dense_mask(cols, vals.reshape(n, 5), mask.reshape(n, 5))


@dataclass
class ServingRequest:
    rid: int
    arrival: float   # seconds after the stream start
    m: int           # grid side; n = m*m
    seed: int        # seed of the system and of its right-hand side


def serving_stream(count: int, rate: float, seed: int = SERVING_SEED,
                   m_lo: int = 8, m_hi: int = 96) -> list[ServingRequest]:
    """Poisson arrivals at `rate` requests/s (rate <= 0: all at t = 0), grid
    sides uniform in [m_lo, m_hi]."""
    g = rng(seed)
    ms = g.integers(m_lo, m_hi + 1, size=count)
    seeds = g.integers(1, 2**31 - 1, size=count)
    # arrival times last, so that the systems do not depend on the rate
    if rate > 0:
        t = np.cumsum(g.exponential(1.0 / rate, size=count))
    else:
        t = np.zeros(count)
    return [ServingRequest(i, float(t[i]), int(ms[i]), int(seeds[i])) for i in range(count)]


def serving_rhs(n: int, seed: int) -> np.ndarray:
    """Right-hand side of a served system: U[-1, 1] entries."""
    return rng(seed + 7919).uniform(-1.0, 1.0, size=n)


# ---------------------------------------------------------------------------
# directed graphs, stored by in-links (row j lists the sources of the edges
# i -> j, sorted and distinct), every stored value 1
# ---------------------------------------------------------------------------
def inlinks(n: int, src, dst) -> CSRMatrix:
    """In-link CSR of the edge list (repeated edges and self-loops kept once)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    key = np.unique(dst * n + src)
    rows, cols = key // n, key % n
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    return CSRMatrix(n, n, rowptr, cols.astype(np.int32), np.ones(len(cols)))


def cycle_graph(n: int) -> CSRMatrix:
    i = np.arange(n)
    return inlinks(n, i, (i + 1) % n)


def star_graph(m: int) -> CSRMatrix:
    """Hub 0 and leaves 1..m: every leaf links to the hub, the hub to every leaf."""
    leaves = np.arange(1, m + 1)
    return inlinks(m + 1, np.concatenate([leaves, np.zeros(m, np.int64)]),
                   np.concatenate([np.zeros(m, np.int64), leaves]))


def random_graph(n: int, p: float, seed: int) -> CSRMatrix:
    """Each ordered pair (i, j), i != j, is an edge with probability p."""
    g = rng(seed)
    a = g.random((n, n)) < p
    np.fill_diagonal(a, False)
    src, dst = np.nonzero(a)
    return inlinks(n, src, dst)


def powerlaw_graph(n: int, s: float = 1.79, kmax: int = 4096, seed: int = MATRIX_SEED) -> CSRMatrix:
    """In-degrees Zipf(s) clipped to [1, kmax] and sources uniform: the
    power-law pattern of zipf_random read as in-links."""
    Z = zipf_random(n, s, kmax, seed)
    return CSRMatrix(Z.n, Z.ncols, Z.rowptr, Z.col, np.ones(Z.nnz))


def unsorted_rows(n, ncols, max_len, seed, integer=True, dup_rate=0.4, empty_every=5):
    """A row-grouped coordinate list (rowptr, col, val): each row's columns in
    random order with repeats (about dup_rate of the entries repeat a column
    of the row); integer values in [-8, 8] or uniform in [-1, 1]; every
    empty_every-th row empty."""
    g = rng(seed)
    rows_c, rows_v, lens = [], [], []
    for i in range(n):
        L = 0 if (empty_every and i % empty_every == 0) else int(g.integers(1, max_len + 1))
        base = g.choice(ncols, size=min(ncols, max(1, int(np.ceil(L * (1 - dup_rate))))),
                        replace=False)
        c = g.choice(base, size=L, replace=True) if L else np.zeros(0, np.int64)
        v = (g.integers(-8, 9, L).astype(float) if integer else g.uniform(-1, 1, L))
        rows_c.append(c)
        rows_v.append(v)
        lens.append(L)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    return (rp.astype(np.int32), np.concatenate(rows_c).astype(np.int32),
            np.concatenate(rows_v))

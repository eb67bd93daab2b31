"""Seeded synthetic SPD grid problems shared by the oracle, the tests and the benchmark.

This module only builds inputs: stencil matrices in CSR form, grid coordinates and
right-hand sides drawn from numpy's PCG64 generator.  It holds none of the solver's
arithmetic.  Vertices are numbered x-fastest, ``v = i + nx*(j + ny*k)``, and the
coordinate of a vertex is its integer cell index.

Matrices follow the finite-difference discretisation of div(a grad u) used in the
paper's experiments (Section 4.1.1): the diagonal holds the sum of the face
coefficients of a cell and each off-diagonal entry is minus the coefficient of the
shared face.  Dirichlet boundary faces carry the cell's own coefficient (the paper
gives only interior faces; this is the reading used here), and no h^2 factor is
applied since the preconditioner is scale invariant.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class GridProblem:
    n: int
    rowptr: np.ndarray  # int64, n+1
    colind: np.ndarray  # int32, nnz, sorted within a row, diagonal included
    values: np.ndarray  # float64, nnz
    coords: np.ndarray  # float64, n x dim, row-major
    dim: int
    shape: tuple

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.colind, self.rowptr), shape=(self.n, self.n))


def _assemble(shape, face):
    """CSR of the stencil whose face coefficients are ``face[d]`` (one array per axis).

    ``face[d]`` has the grid shape with one extra layer along axis d (reversed axis
    order, i.e. arrays are indexed [k, j, i]); entry m along that axis is the face
    between cells m-1 and m, so entries 0 and n_d are boundary faces.
    """
    dim = len(shape)
    n = int(np.prod(shape))
    grid_shape = tuple(reversed(shape))  # (nz, ny, nx) / (ny, nx)
    idx = np.arange(n, dtype=np.int64).reshape(grid_shape)
    diag = np.zeros(grid_shape)
    rows = []
    cols = []
    vals = []
    for d in range(dim):
        ax = dim - 1 - d  # numpy axis of coordinate d
        f = face[d]
        lo = np.take(f, np.arange(0, grid_shape[ax]), axis=ax)
        hi = np.take(f, np.arange(1, grid_shape[ax] + 1), axis=ax)
        diag += lo + hi
        inner = np.take(f, np.arange(1, grid_shape[ax]), axis=ax)  # interior faces
        a = np.take(idx, np.arange(0, grid_shape[ax] - 1), axis=ax)
        b = np.take(idx, np.arange(1, grid_shape[ax]), axis=ax)
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
        vals += [-inner.ravel(), -inner.ravel()]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    coords = np.stack(np.meshgrid(*[np.arange(s, dtype=np.float64) for s in reversed(shape)],
                                  indexing="ij")[::-1], axis=-1).reshape(n, dim)
    return GridProblem(n=n, rowptr=rowptr, colind=c.astype(np.int32), values=v.astype(np.float64),
                       coords=np.ascontiguousarray(coords), dim=dim, shape=tuple(shape))


def _const_faces(shape):
    grid_shape = tuple(reversed(shape))
    dim = len(shape)
    faces = []
    for d in range(dim):
        ax = dim - 1 - d
        fs = list(grid_shape)
        fs[ax] += 1
        faces.append(np.ones(fs))
    return faces


def laplacian(shape) -> GridProblem:
    """Constant-coefficient 5-point (2D) or 7-point (3D) Laplacian with Dirichlet boundary."""
    return _assemble(tuple(int(s) for s in shape), _const_faces(shape))


def variable_coefficient(shape, rng: np.random.Generator, log10_lo: float, log10_hi: float) -> GridProblem:
    """Cell coefficients 10**U(lo, hi) drawn from ``rng``; faces take the harmonic mean.

    Boundary faces take the coefficient of the cell they bound.
    """
    shape = tuple(int(s) for s in shape)
    grid_shape = tuple(reversed(shape))
    c = 10.0 ** rng.uniform(log10_lo, log10_hi, grid_shape)
    dim = len(shape)
    faces = []
    for d in range(dim):
        ax = dim - 1 - d
        n_ax = grid_shape[ax]
        c0 = np.take(c, np.arange(0, n_ax - 1), axis=ax)
        c1 = np.take(c, np.arange(1, n_ax), axis=ax)
        inner = 2.0 * c0 * c1 / (c0 + c1)
        first = np.take(c, [0], axis=ax)
        last = np.take(c, [n_ax - 1], axis=ax)
        faces.append(np.concatenate([first, inner, last], axis=ax))
    return _assemble(shape, faces)


def _harmonic_faces(c):
    """Face coefficients of a cell-coefficient array c (numpy axes reversed from the
    grid axes): harmonic mean of the two cells inside, the cell's own value on the
    boundary."""
    dim = c.ndim
    faces = []
    for d in range(dim):
        ax = dim - 1 - d
        n_ax = c.shape[ax]
        c0 = np.take(c, np.arange(0, n_ax - 1), axis=ax)
        c1 = np.take(c, np.arange(1, n_ax), axis=ax)
        inner = 2.0 * c0 * c1 / (c0 + c1)
        first = np.take(c, [0], axis=ax)
        last = np.take(c, [n_ax - 1], axis=ax)
        faces.append(np.concatenate([first, inner, last], axis=ax))
    return faces


def high_contrast_field(shape, rng: np.random.Generator, rho: float) -> np.ndarray:
    """Quantized high-contrast cell field of Sec. 4.1.1, in any dimension: a random
    U(0,1) array, smoothed by convolution with a unit-width Gaussian (standard
    deviation one cell, reflected at the boundary), then rho where the smoothed
    value is >= 0.5 and 1/rho elsewhere.  Returned with numpy axes reversed from the
    grid axes ([k, j, i])."""
    from scipy.ndimage import gaussian_filter
    grid_shape = tuple(reversed(tuple(int(s) for s in shape)))
    a_hat = gaussian_filter(rng.random(grid_shape), sigma=1.0, mode="reflect")
    return np.where(a_hat >= 0.5, float(rho), 1.0 / float(rho))


def high_contrast(shape, rng: np.random.Generator, rho: float) -> GridProblem:
    """The high-contrast operator of Sec. 4.1.1 (5-point in 2D, 7-point in 3D): cell
    coefficients from high_contrast_field, faces by harmonic mean.  rho = 1 gives the
    constant-coefficient Laplacian."""
    shape = tuple(int(s) for s in shape)
    return _assemble(shape, _harmonic_faces(high_contrast_field(shape, rng, rho)))


def knn_graph_laplacian(n: int, k: int, rng: np.random.Generator, shift: float = 0.1) -> GridProblem:
    """An irregular SPD matrix without usable geometry: the graph Laplacian of the
    symmetric k-nearest-neighbour graph of n random points in the unit cube, plus
    shift * I.  The points only build the edges; the returned coords are all zero,
    so an analysis must use the graph."""
    from scipy.spatial import cKDTree
    pts = rng.random((n, 3))
    _, nb = cKDTree(pts).query(pts, k + 1)
    rows = np.repeat(np.arange(n), k)
    cols = nb[:, 1:].ravel()
    a = np.concatenate([rows, cols])
    b = np.concatenate([cols, rows])
    pairs = np.unique(np.stack([a, b], axis=1), axis=0)
    deg = np.bincount(pairs[:, 0], minlength=n).astype(np.float64)
    r = np.concatenate([pairs[:, 0], np.arange(n)])
    c = np.concatenate([pairs[:, 1], np.arange(n)])
    v = np.concatenate([-np.ones(len(pairs)), deg + shift])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return GridProblem(n=n, rowptr=rowptr, colind=c.astype(np.int32), values=v, coords=np.zeros((n, 3)), dim=3,
                       shape=(n,))


def permuted(p: GridProblem, rng: np.random.Generator) -> GridProblem:
    """The same operator with its vertices renumbered by a random permutation (P A P^T),
    coordinates permuted along."""
    perm = rng.permutation(p.n)           # new vertex i is old vertex perm[i]
    inv = np.empty(p.n, dtype=np.int64)
    inv[perm] = np.arange(p.n)
    A = p.scipy().tocsr()[perm][:, perm].tocsr()
    A.sort_indices()
    return GridProblem(n=p.n, rowptr=A.indptr.astype(np.int64), colind=A.indices.astype(np.int32),
                       values=A.data.astype(np.float64), coords=np.ascontiguousarray(p.coords[perm]), dim=p.dim,
                       shape=p.shape)


def rhs(rng: np.random.Generator, n: int, nrhs: int) -> np.ndarray:
    """Right-hand sides b ~ N(0,1), returned column-major as an (n, nrhs) Fortran array."""
    return np.asfortranarray(rng.standard_normal((nrhs, n)).T)


# The workloads of the benchmark configurations.
def config_problem(name: str):
    """Return (problem, b, levels) for a named workload.

    c1: 2D 64x64 Laplacian, 6 levels, 1 RHS (seed 1).
    c2: 3D 32^3 Laplacian, 9 levels, 1 RHS (seed 2).
    c3: 3D 64^3 variable coefficients 10^U(-3,3), 10 levels, 1 RHS (seed 3).
    c4: 3D 128^3 Laplacian, 13 levels, 8 RHS (seed 4).
    c5_<j>: problem j of the batched workload (see batched_problem).
    """
    if name == "c1":
        p = laplacian((64, 64))
        return p, rhs(np.random.default_rng(1), p.n, 1), 6
    if name == "c2":
        p = laplacian((32, 32, 32))
        return p, rhs(np.random.default_rng(2), p.n, 1), 9
    if name == "c3":
        rng = np.random.default_rng(3)
        p = variable_coefficient((64, 64, 64), rng, -3.0, 3.0)
        return p, rhs(rng, p.n, 1), 10
    if name == "c4":
        p = laplacian((128, 128, 128))
        return p, rhs(np.random.default_rng(4), p.n, 8), 13
    if name.startswith("c5_"):
        return batched_problem(int(name[3:]))
    if name.startswith("x4_"):
        return sweep_problem(name)
    if name.startswith("x1_"):
        return contrast2d_problem(name)
    raise KeyError(name)


def contrast2d_problem(name: str):
    """A point of the 2D variant comparison of Sec. 4.1.1: "x1_<n>_rho<rho>" is the
    n x n 5-point operator with the high-contrast field of contrast rho (rho = 1: the
    Laplacian), seed 1000 + n, one RHS from seed 7, depth 1 + ceil(log2(n^2 / 512))."""
    body = name[3:]
    n_s, rho_s = body.split("_rho")
    n, rho = int(n_s), float(rho_s)
    p = high_contrast((n, n), np.random.default_rng(1000 + n), rho)
    return p, rhs(np.random.default_rng(7), p.n, 1), levels_for(p.n)


def sweep_problem(name: str):
    """A point of the 3D size sweep of Sec. 4.2: "x4_<n>_rho<rho>" is the n^3 grid with
    the high-contrast field of contrast rho (rho = 1: the Laplacian), seed 40000 + n,
    one RHS drawn next from the same generator, depth 1 + ceil(log2(n^3 / 512))."""
    body = name[3:]
    n_s, rho_s = body.split("_rho")
    n, rho = int(n_s), float(rho_s)
    rng = np.random.default_rng(40000 + n)
    p = high_contrast((n, n, n), rng, rho)
    return p, rhs(rng, p.n, 1), levels_for(p.n)


def levels_for(n: int) -> int:
    """Tree depth giving leaves of about 512 vertices: 1 + ceil(log2(n / 512)), at least 2."""
    return max(2, 1 + int(np.ceil(np.log2(max(n, 1) / 512.0))))


def batched_problem(j: int, count: int = 256, seed: int = 5, nrhs: int = 16):
    """Problem j of the batched workload: grid edges U{24..48} per axis (one draw of
    count x 3 edges from seed), cell coefficients 10^U(-2,2) and nrhs right-hand
    sides from seed * 1000 + j; depth from the grid size."""
    edges = np.random.default_rng(seed).integers(24, 49, (count, 3))
    rng = np.random.default_rng(seed * 1000 + j)
    p = variable_coefficient(tuple(int(e) for e in edges[j]), rng, -2.0, 2.0)
    return p, rhs(rng, p.n, nrhs), levels_for(p.n)


def batched_problems(count: int = 256, seed: int = 5, nrhs: int = 16):
    """The batched workload: grid edges U{24..48} per axis, coefficients 10^U(-2,2)."""
    for j in range(count):
        yield batched_problem(j, count, seed, nrhs)

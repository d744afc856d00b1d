"""Seeded generators for the sparse systems the solvers are exercised on.

The paper evaluates on SuiteSparse matrices (Section IV-A, Table II), which are
not available here.  These generators are synthetic stand-ins with the same
kind of structure: stencil operators whose non-zeros cluster on a few
exponents, operators whose coefficients spread over several decades, and a
power-law matrix with very uneven row lengths.  Every generator is a pure
function of its arguments (numpy ``default_rng(seed)`` draws only).

All matrices are returned as :class:`CSR` with int32 ``indptr``/``indices``
(column indices sorted ascending inside each row) and float64 ``data``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """A square or rectangular FP64 CSR matrix."""

    n_rows: int
    n_cols: int
    indptr: np.ndarray  # int32 [n_rows + 1]
    indices: np.ndarray  # int32 [nnz]
    data: np.ndarray  # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr),
                             shape=(self.n_rows, self.n_cols))

    @staticmethod
    def from_scipy(m: sp.spmatrix, name: str = "") -> "CSR":
        m = sp.csr_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        if m.nnz >= 2**31:
            raise ValueError("nnz does not fit int32 row pointers")
        return CSR(m.shape[0], m.shape[1],
                   np.ascontiguousarray(m.indptr, dtype=np.int32),
                   np.ascontiguousarray(m.indices, dtype=np.int32),
                   np.ascontiguousarray(m.data, dtype=np.float64), name)


def _from_banded(n: int, cols: np.ndarray, vals: np.ndarray, valid: np.ndarray,
                 name: str) -> CSR:
    """Build CSR from per-row slots given in ascending column order."""
    counts = valid.sum(axis=1).astype(np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return CSR(n, n, indptr.astype(np.int32),
               np.ascontiguousarray(cols[valid], dtype=np.int32),
               np.ascontiguousarray(vals[valid], dtype=np.float64), name)


def poisson2d(N: int) -> CSR:
    """2-D 5-point Laplacian on an N x N grid, Dirichlet boundary.

    Row ``r = i + N*j`` (i fastest); diagonal 4, neighbours -1.
    """
    n = N * N
    r = np.arange(n, dtype=np.int64)
    i = r % N
    j = r // N
    cols = np.stack([r - N, r - 1, r, r + 1, r + N], axis=1)
    vals = np.tile(np.array([-1.0, -1.0, 4.0, -1.0, -1.0]), (n, 1))
    valid = np.stack([j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1], axis=1)
    return _from_banded(n, cols, vals, valid, f"poisson2d_{N}")


def diffusion3d(N: int, seed: int, decades: float = 4.0) -> CSR:
    """3-D 7-point variable-coefficient diffusion on an N^3 grid.

    Every cell face (boundary faces included) carries its own coefficient
    ``kappa = 10**U(-decades/2, decades/2)``.  Off-diagonals are ``-kappa`` of
    the shared face and the diagonal is the sum of the cell's six face
    coefficients, so the operator is symmetric and, through the boundary
    faces, positive definite.  Row ``r = i + N*(j + N*k)``.
    """
    rng = np.random.default_rng(seed)
    lo, hi = -decades / 2.0, decades / 2.0
    kx = 10.0 ** rng.uniform(lo, hi, size=(N, N, N + 1))  # [k, j, i-face]
    ky = 10.0 ** rng.uniform(lo, hi, size=(N, N + 1, N))  # [k, j-face, i]
    kz = 10.0 ** rng.uniform(lo, hi, size=(N + 1, N, N))  # [k-face, j, i]
    diag = (kx[:, :, :-1] + kx[:, :, 1:]) + (ky[:, :-1, :] + ky[:, 1:, :]) \
        + (kz[:-1] + kz[1:])
    n = N ** 3
    r = np.arange(n, dtype=np.int64)
    i = r % N
    j = (r // N) % N
    k = r // (N * N)
    cols = np.stack([r - N * N, r - N, r - 1, r, r + 1, r + N, r + N * N], axis=1)
    vals = np.stack([-kz[:-1].ravel(), -ky[:, :-1, :].ravel(), -kx[:, :, :-1].ravel(),
                     diag.ravel(),
                     -kx[:, :, 1:].ravel(), -ky[:, 1:, :].ravel(), -kz[1:].ravel()], axis=1)
    valid = np.stack([k > 0, j > 0, i > 0, np.ones(n, bool),
                      i < N - 1, j < N - 1, k < N - 1], axis=1)
    return _from_banded(n, cols, vals, valid, f"diffusion3d_{N}_s{seed}")


def layered3d(N: int, seed: int, contrast: float = 8.0, local: float = 1.0,
              layers: int = 16) -> CSR:
    """3-D 7-point diffusion in a layered medium, N^3 grid.

    The grid is cut along k (the slowest row index) into ``layers`` slabs of
    equal thickness; slab q has the level ``c_q ~ U(-contrast/2, contrast/2)``
    (decades) and every cell face inside it the coefficient
    ``10**(c_q + U(-local/2, local/2))``; a face between two slabs takes the
    lower level of the two.  Off-diagonals are ``-kappa`` of the shared face, the
    diagonal the sum of the cell's six faces (boundary faces included), so the
    operator is symmetric positive definite.  Contiguous rows share a slab,
    so the exponents of a block of rows spread over ``local`` decades plus
    the diagonal while the whole matrix spans ``contrast + local``.
    """
    rng = np.random.default_rng(seed)
    level = rng.uniform(-contrast / 2.0, contrast / 2.0, size=layers)
    slab = (np.arange(N) * layers) // N                       # slab of each k plane
    lev_k = level[slab]                                      # [k]
    lev_kface = np.empty(N + 1)
    lev_kface[0], lev_kface[N] = lev_k[0], lev_k[-1]
    lev_kface[1:N] = np.minimum(lev_k[:-1], lev_k[1:])
    lo, hi = -local / 2.0, local / 2.0
    kx = 10.0 ** (lev_k[:, None, None] + rng.uniform(lo, hi, size=(N, N, N + 1)))
    ky = 10.0 ** (lev_k[:, None, None] + rng.uniform(lo, hi, size=(N, N + 1, N)))
    kz = 10.0 ** (lev_kface[:, None, None] + rng.uniform(lo, hi, size=(N + 1, N, N)))
    diag = (kx[:, :, :-1] + kx[:, :, 1:]) + (ky[:, :-1, :] + ky[:, 1:, :]) \
        + (kz[:-1] + kz[1:])
    n = N ** 3
    r = np.arange(n, dtype=np.int64)
    i = r % N
    j = (r // N) % N
    k = r // (N * N)
    cols = np.stack([r - N * N, r - N, r - 1, r, r + 1, r + N, r + N * N], axis=1)
    vals = np.stack([-kz[:-1].ravel(), -ky[:, :-1, :].ravel(), -kx[:, :, :-1].ravel(),
                     diag.ravel(),
                     -kx[:, :, 1:].ravel(), -ky[:, 1:, :].ravel(), -kz[1:].ravel()], axis=1)
    valid = np.stack([k > 0, j > 0, i > 0, np.ones(n, bool),
                      i < N - 1, j < N - 1, k < N - 1], axis=1)
    return _from_banded(n, cols, vals, valid, f"layered3d_{N}_s{seed}")


def block_sample_rows(n_rows: int, block_rows: int, seed: int) -> np.ndarray:
    """One uniformly drawn row of each block of ``block_rows`` rows (the last
    block may be shorter): the random rows whose exponents stand for their
    block's when the shared exponents are chosen by sampling."""
    rng = np.random.default_rng(seed)
    n_blocks = -(-n_rows // block_rows)
    start = np.arange(n_blocks, dtype=np.int64) * block_rows
    size = np.minimum(block_rows, n_rows - start)
    return (start + np.floor(rng.random(n_blocks) * size).astype(np.int64)).astype(np.int32)


def convdiff2d(N: int, seed: int, peclet: float = 10.0) -> CSR:
    """2-D convection-diffusion, first-order upwind 5-point stencil, N x N.

    Scaled by h^2/nu: diagonal ``4 + Pe*(|cos t| + |sin t|)``, the upwind
    neighbour along each axis ``-(1 + Pe*|w_axis|)``, the downwind one ``-1``.
    The wind angle ``t ~ U[0, 2*pi)`` is drawn from ``seed``; ``Pe`` is the
    cell Peclet number.  Nonsymmetric; Dirichlet boundary (neighbours outside
    the grid are dropped).
    """
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi)
    wx, wy = math.cos(theta), math.sin(theta)
    cx_up, cy_up = -(1.0 + peclet * abs(wx)), -(1.0 + peclet * abs(wy))
    west = cx_up if wx > 0 else -1.0
    east = -1.0 if wx > 0 else cx_up
    south = cy_up if wy > 0 else -1.0
    north = -1.0 if wy > 0 else cy_up
    d = 4.0 + peclet * (abs(wx) + abs(wy))
    n = N * N
    r = np.arange(n, dtype=np.int64)
    i = r % N
    j = r // N
    cols = np.stack([r - N, r - 1, r, r + 1, r + N], axis=1)
    vals = np.tile(np.array([south, west, d, east, north]), (n, 1))
    valid = np.stack([j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1], axis=1)
    out = _from_banded(n, cols, vals, valid, f"convdiff2d_{N}_s{seed}")
    return out


def powerlaw(n: int, seed: int, zipf_s: float = 2.0, max_off: int = 9999,
             decades: float = 6.0, diag_factor: float = 1.1) -> CSR:
    """Symmetric positive definite matrix with power-law row lengths.

    A helper matrix B gets ``o_i = min(max_off, Z_i + 1)`` off-diagonal
    entries in row i, ``Z_i ~ Zipf(zipf_s)``, in uniformly drawn columns other
    than i, with values ``N(0,1) * 10**U(-decades/2, decades/2)``.  Then
    ``A = B + B^T`` (coincident entries summed) and the diagonal is
    ``diag_factor`` times the absolute row sum, which makes A strictly
    diagonally dominant and hence SPD.
    """
    rng = np.random.default_rng(seed)
    z = rng.zipf(zipf_s, size=n)
    o = np.minimum(max_off, z + 1).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), o)
    cols = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    cols += (cols >= rows)
    lo, hi = -decades / 2.0, decades / 2.0
    vals = rng.standard_normal(rows.size) * 10.0 ** rng.uniform(lo, hi, size=rows.size)
    B = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    del rows, cols, vals
    A = (B + B.T).tocsr()
    del B
    A.sum_duplicates()
    absrow = np.asarray(abs(A).sum(axis=1)).ravel()
    A = (A + sp.diags(diag_factor * absrow + (absrow == 0), format="csr")).tocsr()
    return CSR.from_scipy(A, f"powerlaw_{n}_s{seed}")


def random_sparse(n_rows: int, n_cols: int, seed: int, mean_row: float = 6.0,
                  empty_frac: float = 0.0, long_rows: int = 0, long_len: int = 0,
                  exp_spread: float = 8.0) -> CSR:
    """Unstructured test matrix: Poisson row lengths, optional empty rows and
    a few very long rows, values with a chosen spread of binary exponents."""
    rng = np.random.default_rng(seed)
    lens = rng.poisson(mean_row, size=n_rows).astype(np.int64)
    if empty_frac > 0:
        lens[rng.random(n_rows) < empty_frac] = 0
    if long_rows > 0:
        pick = rng.choice(n_rows, size=min(long_rows, n_rows), replace=False)
        lens[pick] = min(long_len, n_cols)
    lens = np.minimum(lens, n_cols)
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    cols = np.empty(int(indptr[-1]), dtype=np.int64)
    for r in np.nonzero(lens)[0]:
        c = rng.choice(n_cols, size=int(lens[r]), replace=False) if lens[r] > 64 \
            else np.unique(rng.integers(0, n_cols, size=int(lens[r])))
        if c.size < lens[r]:  # rare duplicate draws for short rows: top up
            extra = np.setdiff1d(np.arange(n_cols), c)[: int(lens[r]) - c.size]
            c = np.concatenate([c, extra])
        cols[indptr[r]:indptr[r + 1]] = np.sort(c)
    vals = rng.standard_normal(cols.size) * np.exp2(
        rng.uniform(-exp_spread / 2, exp_spread / 2, size=cols.size))
    return CSR(n_rows, n_cols, indptr.astype(np.int32), cols.astype(np.int32),
               vals.astype(np.float64), f"random_{n_rows}x{n_cols}_s{seed}")


def diagonal(n: int, seed: int, exp_spread: float = 16.0) -> CSR:
    """Diagonal matrix with positive values over a spread of binary exponents
    (one non-zero per row: a 1024-non-zero tile spans 1024 rows)."""
    rng = np.random.default_rng(seed)
    vals = np.exp2(rng.uniform(-exp_spread / 2, exp_spread / 2, size=n)) * rng.uniform(1, 2, size=n)
    idx = np.arange(n, dtype=np.int32)
    indptr = np.arange(n + 1, dtype=np.int32)
    return CSR(n, n, indptr, idx, vals.astype(np.float64), f"diagonal_{n}_s{seed}")


def fixed_rows(n_rows: int, n_cols: int, row_len: int, seed: int, exp_spread: float = 8.0) -> CSR:
    """Every row holds exactly `row_len` distinct random columns (so the
    number of non-zeros is n_rows * row_len exactly)."""
    rng = np.random.default_rng(seed)
    cols = np.stack([np.sort(rng.choice(n_cols, size=row_len, replace=False)) for _ in range(n_rows)])
    vals = rng.standard_normal(cols.size) * np.exp2(
        rng.uniform(-exp_spread / 2, exp_spread / 2, size=cols.size))
    indptr = (np.arange(n_rows + 1) * row_len).astype(np.int32)
    return CSR(n_rows, n_cols, indptr, cols.reshape(-1).astype(np.int32), vals.astype(np.float64),
               f"fixed_{n_rows}x{n_cols}_r{row_len}_s{seed}")


def rhs_from_solution(A: CSR, seed: int):
    """``x_true ~ U[-1, 1]`` from ``seed`` and ``b = A @ x_true`` in FP64."""
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(-1.0, 1.0, size=A.n_cols)
    b = A.to_scipy() @ x_true
    return x_true, np.ascontiguousarray(b, dtype=np.float64)


def serving_stream(seed: int, count: int = 2000, n_lo: float = 1e3, n_hi: float = 1e6,
                   rate: float = 1.0, decades: float = 4.0) -> List[Dict]:
    """Poisson-arrival stream of SPD stencil systems.

    Each request has ``n = 10**U(log10 n_lo, log10 n_hi)`` unknowns, is a 2-D
    5-point or 3-D 7-point variable-coefficient diffusion operator with
    probability 1/2 each (grid side ``round(n**(1/2))`` or ``round(n**(1/3))``),
    and arrives after an ``Exp(rate)`` gap (seconds).
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for q in range(count):
        t += rng.exponential(1.0 / rate)
        n = 10.0 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))
        dim = 2 if rng.random() < 0.5 else 3
        side = max(2, int(round(n ** (1.0 / dim))))
        out.append({"id": q, "arrival": t, "dim": dim, "side": side,
                    "seed": int(rng.integers(0, 2**31 - 1)), "decades": decades})
    return out


def diffusion2d(N: int, seed: int, decades: float = 4.0) -> CSR:
    """2-D 5-point variable-coefficient diffusion (serving requests)."""
    rng = np.random.default_rng(seed)
    lo, hi = -decades / 2.0, decades / 2.0
    kx = 10.0 ** rng.uniform(lo, hi, size=(N, N + 1))  # [j, i-face]
    ky = 10.0 ** rng.uniform(lo, hi, size=(N + 1, N))  # [j-face, i]
    diag = (kx[:, :-1] + kx[:, 1:]) + (ky[:-1] + ky[1:])
    n = N * N
    r = np.arange(n, dtype=np.int64)
    i = r % N
    j = r // N
    cols = np.stack([r - N, r - 1, r, r + 1, r + N], axis=1)
    vals = np.stack([-ky[:-1].ravel(), -kx[:, :-1].ravel(), diag.ravel(),
                     -kx[:, 1:].ravel(), -ky[1:].ravel()], axis=1)
    valid = np.stack([j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1], axis=1)
    return _from_banded(n, cols, vals, valid, f"diffusion2d_{N}_s{seed}")


def serving_request_matrix(req: Dict) -> CSR:
    if req["dim"] == 2:
        return diffusion2d(req["side"], req["seed"], req["decades"])
    return diffusion3d(req["side"], req["seed"], req["decades"])


# Named workloads.  Sizes follow the evaluation configurations; ``small``
# variants keep the same structure at sizes a sequential oracle handles in
# seconds.
CONFIGS = {
    "poisson2d_64": lambda seed=0: poisson2d(64),
    "diffusion3d_128": lambda seed=0: diffusion3d(128, seed),
    "convdiff2d_1024": lambda seed=0: convdiff2d(1024, seed),
    "powerlaw_4m": lambda seed=0: powerlaw(4_000_000, seed),
    "layered3d_128": lambda seed=0: layered3d(128, seed),
    # reduced instances (same recipes)
    "diffusion3d_24": lambda seed=0: diffusion3d(24, seed),
    "diffusion3d_48": lambda seed=0: diffusion3d(48, seed),
    "convdiff2d_64": lambda seed=0: convdiff2d(64, seed),
    "convdiff2d_128": lambda seed=0: convdiff2d(128, seed),
    "powerlaw_50k": lambda seed=0: powerlaw(50_000, seed),
    "layered3d_24": lambda seed=0: layered3d(24, seed),
}


def make_config(name: str, seed: int = 0) -> CSR:
    return CONFIGS[name](seed)

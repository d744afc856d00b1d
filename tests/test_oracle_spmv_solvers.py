"""Pins of the oracle's SpMV operators, CG, GMRES and stepped controller.

Pins come from library routines on tiny cases (dense numpy products and
solves, least squares over an explicit Krylov basis), closed forms (Poisson
eigenpairs, CG's finite termination on few distinct eigenvalues, the window
metrics of constant and geometric residual sequences) and the fact that an
exactly representable stencil makes the stepped solver identical to FP64.
"""
import math

import numpy as np
import pytest

import oracle as O
from workloads import (convdiff2d, diffusion3d, poisson2d, random_sparse,
                       rhs_from_solution)


def dense(A, vals=None):
    D = np.zeros((A.n_rows, A.n_cols))
    v = A.data if vals is None else vals
    for r in range(A.n_rows):
        for j in range(A.indptr[r], A.indptr[r + 1]):
            D[r, A.indices[j]] += v[j]
    return D


# ------------------------------------------------------------------ SpMV ---
@pytest.mark.parametrize("seed", [0, 1])
def test_spmv_against_dense_product(seed):
    A = random_sparse(90, 70, seed, mean_row=5, empty_frac=0.1, long_rows=2, long_len=60,
                      exp_spread=40)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    x = np.random.default_rng(seed).standard_normal(A.n_cols)
    y64 = O.csr_spmv(A.indptr, A.indices, A.data, x)
    assert np.allclose(y64, dense(A) @ x, rtol=1e-13, atol=1e-13 * np.abs(dense(A)).sum())
    for s in (1, 2, 3):
        D = dense(A, O.decode(enc, s))
        ys = O.gse_spmv(A.indptr, enc, s, x)
        ref = D @ x
        scale = np.abs(D) @ np.abs(x)
        assert np.all(np.abs(ys - ref) <= 1e-14 * scale + 1e-300)
        rows = np.array([0, 5, 17, 89, 42], np.int32)
        assert np.array_equal(O.gse_spmv_rows(rows, A.indptr, enc, s, x), ys[rows])
    # empty rows give exact zeros
    empty = np.nonzero(np.diff(A.indptr) == 0)[0]
    assert empty.size > 0 and np.all(O.gse_spmv(A.indptr, enc, 1, x)[empty] == 0.0)


def test_spmv_format_bound_componentwise():
    """|y_s - y| <= sum_j 2^(SEM_j-1023-W_s)|x_j| + gamma_n sum|a_ij x_j|."""
    A = random_sparse(200, 200, 3, mean_row=8, exp_spread=50)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    x = np.random.default_rng(3).standard_normal(A.n_cols)
    y = dense(A) @ x
    absy = np.abs(dense(A)) @ np.abs(x)
    sem = enc.sem.astype(np.int64)
    for s, W in ((1, 15), (2, 31), (3, 63)):
        ys = O.gse_spmv(A.indptr, enc, s, x)
        grid = np.exp2((sem[enc.col_idx >> 29] - 1023 - W).astype(float))
        bound = np.zeros(A.n_rows)
        for r in range(A.n_rows):
            js = slice(A.indptr[r], A.indptr[r + 1])
            bound[r] = np.sum(grid[js] * np.abs(x[A.indices[js]]))
        nmax = np.diff(A.indptr).max()
        bound += 2 * nmax * 2.0**-53 * absy
        assert np.all(np.abs(ys - y) <= bound)


@pytest.mark.parametrize("N", [8, 31])
def test_poisson_eigenpairs(N):
    A = poisson2d(N)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    assert list(enc.eta) == [0.0, 0.0, 0.0]
    i = np.arange(1, N + 1)
    for p, q in ((1, 1), (2, 5), (N, N - 1)):
        lam = 4 - 2 * math.cos(p * math.pi / (N + 1)) - 2 * math.cos(q * math.pi / (N + 1))
        v = np.outer(np.sin(i * q * math.pi / (N + 1)), np.sin(i * p * math.pi / (N + 1))).ravel()
        for s in (1, 2, 3):
            y = O.gse_spmv(A.indptr, enc, s, v)
            assert np.linalg.norm(y - lam * v) <= 1e-13 * np.linalg.norm(lam * v)


# ------------------------------------------------------------ controller ---
def test_window_metrics_constant_sequence_triggers_c3():
    resid = np.full(400, 0.25)  # exact in binary: the mean is exact
    rsd, nd, rd = O.window_metrics(resid, 300, 250)
    assert rsd == 0.0 and nd == 0 and rd == 0.0
    p = O.make_params(preset="paper_cg", l=300, m=50)
    assert O.precision_trigger(resid, 300, p) == 3
    assert O.precision_trigger(resid, 325, p) == 0  # off the check grid
    assert O.precision_trigger(resid, 350, p) == 3


@pytest.mark.parametrize("q", [0.99, 0.9, 0.5])
def test_window_metrics_geometric_closed_form(q):
    t, j = 250, 600
    resid = q ** np.arange(j + 1, dtype=float)
    rsd, nd, rd = O.window_metrics(resid, j, t)
    a = q ** (j - t)
    mu = a * (1 - q**t) / (t * (1 - q))
    m2 = a * a * (1 - q ** (2 * t)) / (t * (1 - q * q))
    assert nd == t
    assert rd == pytest.approx(1 - q ** (t - 1), rel=1e-12)
    assert rsd == pytest.approx(math.sqrt(max(m2 - mu * mu, 0.0)) / mu, rel=1e-6)


def test_conditions_hand_sequences():
    p = O.make_params(preset="paper_cg", l=20, t=10, m=5, rsd_limit=0.5, ndec_limit=6,
                      reldec_limit=0.45)
    # steady slow decrease: nDec = 10 >= 6, relDec small -> C2
    slow = 1.0 - 0.001 * np.arange(40)
    assert O.precision_trigger(slow, 25, p) == 2
    # fast decrease: nDec = 10, relDec = 1 - 0.5^9 > 0.45 -> no switch
    fast = 0.5 ** np.arange(40, dtype=float)
    assert O.precision_trigger(fast, 25, p) == 0
    # wild oscillation with few decreases: large RSD, nDec < 6 -> C1
    osc = np.array([1.0, 10.0, 10.0, 100.0, 100.0] * 8)
    rsd, nd, rd = O.window_metrics(osc, 25, 10)
    assert nd < 6 and rsd > 0.5
    assert O.precision_trigger(osc, 25, p) == 1
    # rising sequence: nDec = 0 and RSD small -> C3
    rise = 1.0 + 0.001 * np.arange(40)
    assert O.precision_trigger(rise, 25, p) == 3
    # t/2 rule: nDec = 5 of t = 10 -> counts as ">= t/2" under rule 1
    half = np.array([1.0, 0.999] * 20)
    p2 = O.make_params(preset="paper_cg", l=20, t=10, m=5, rsd_limit=0.5, ndec_limit=6,
                       reldec_limit=0.45, ndec_rule=1)
    _, nd, rd = O.window_metrics(half, 25, 10)
    assert nd == 5
    assert O.precision_trigger(half, 25, p2) == 2
    assert O.precision_trigger(half, 25, p) == 0  # 5 < 6, RSD tiny, nDec > 0


# ------------------------------------------------------------------- CG ---
def tiny_spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    D = M @ M.T + n * np.eye(n)
    import scipy.sparse as sp
    from workloads import CSR
    return CSR.from_scipy(sp.csr_matrix(D)), D


@pytest.mark.parametrize("n", [1, 3, 12])
def test_cg_tiny_against_dense_solve(n):
    A, D = tiny_spd(n, n)
    b = np.random.default_rng(n).standard_normal(n)
    x_ref = np.linalg.solve(D, b)
    r = O.cg(A.indptr, b, O.make_params(fixed_segments=-1, max_iter=200, tol=1e-13),
             A.indices, A.data)
    assert r.status == O.OK
    assert np.allclose(r.x, x_ref, rtol=1e-10, atol=1e-12)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    r = O.cg(A.indptr, b, O.make_params(max_iter=400, tol=1e-12), A.indices, A.data, enc)
    assert r.status == O.OK and r.relres_true <= 1e-12
    assert np.allclose(r.x, x_ref, rtol=1e-9, atol=1e-11)


def test_cg_finite_termination_distinct_eigenvalues():
    """b spanning m eigenvectors with distinct eigenvalues: CG converges in m
    iterations in exact arithmetic; in FP64 the residual falls by at least
    nine orders of magnitude exactly at step m."""
    N = 20
    A = poisson2d(N)
    i = np.arange(1, N + 1)
    vecs = []
    for p, q in ((1, 1), (1, 2), (3, 3), (5, 2)):  # lambda distinct
        vecs.append(np.outer(np.sin(i * q * np.pi / (N + 1)),
                             np.sin(i * p * np.pi / (N + 1))).ravel())
    for m in (1, 2, 4):
        b = sum(vecs[:m])
        r = O.cg(A.indptr, b, O.make_params(fixed_segments=-1, max_iter=50, tol=1e-9),
                 A.indices, A.data)
        assert r.status == O.OK and r.iters == m, (m, r.iters)
        assert r.hist[m - 1] > 1e-3


def test_stepped_cg_identical_to_fp64_on_exact_stencil():
    A = poisson2d(40)
    _, b = rhs_from_solution(A, 0)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    r64 = O.cg(A.indptr, b, O.make_params(fixed_segments=-1, max_iter=3000), A.indices, A.data)
    rst = O.cg(A.indptr, b, O.make_params(max_iter=3000), A.indices, A.data, enc)
    assert r64.iters == rst.iters and rst.iters_per_seg == (rst.iters, 0, 0)
    assert np.array_equal(r64.x, rst.x)
    assert np.array_equal(r64.hist, rst.hist)


def test_stepped_cg_reaches_tolerance_on_variable_coefficients():
    A = diffusion3d(12, 1)
    x_true, b = rhs_from_solution(A, 1)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    assert enc.eta[0] > 0
    for mode in (0, 1):
        r = O.cg(A.indptr, b, O.make_params(max_iter=5000, switch_mode=mode), A.indices,
                 A.data, enc)
        assert r.status == O.OK and r.relres_true <= 1e-10
        assert r.iters_per_seg[0] > 0 and r.switch_iter[0] > 0
        assert r.switch_trigger[0] in (1, 2, 3, 4, 5)
        assert np.linalg.norm(r.x - x_true) <= 1e-6 * np.linalg.norm(x_true)
        # the switch points are where the segment count steps up by one
        steps = np.nonzero(np.diff(r.seg_hist[1:]))[0]
        assert np.all(np.diff(r.seg_hist[1:])[steps] == 1)


def test_cg_breakdown_on_indefinite_fp64():
    import scipy.sparse as sp
    from workloads import CSR
    A = CSR.from_scipy(sp.csr_matrix(np.diag([1.0, -1.0])))
    r = O.cg(A.indptr, np.array([1.0, 1.0]), O.make_params(fixed_segments=-1, max_iter=10),
             A.indices, A.data)
    assert r.status == O.ERR_BREAKDOWN


# ---------------------------------------------------------------- GMRES ---
def tiny_nonsym(n, seed):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((n, n)) + n * np.eye(n)
    import scipy.sparse as sp
    from workloads import CSR
    return CSR.from_scipy(sp.csr_matrix(D)), D


@pytest.mark.parametrize("orth", [0, 1, 2])
@pytest.mark.parametrize("n", [2, 7, 12])
def test_gmres_full_restart_is_exact(n, orth):
    A, D = tiny_nonsym(n, n + 10)
    b = np.random.default_rng(n).standard_normal(n)
    p = O.make_params(fixed_segments=-1, max_iter=n, restart=n, preset="paper_gmres",
                      tol=1e-12, orth=orth)
    r = O.gmres(A.indptr, b, p, A.indices, A.data)
    assert r.iters <= n
    assert np.allclose(r.x, np.linalg.solve(D, b), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("orth", [0, 1, 2])
def test_gmres_residual_is_krylov_minimum(orth):
    """After j steps of one cycle the estimate |g_{j+1}| equals
    min over z in K_j(A, b) of ||b - A z|| (least squares on a basis)."""
    n = 30
    A, D = tiny_nonsym(n, 4)
    b = np.random.default_rng(5).standard_normal(n)
    for j in (1, 3, 6, 11):
        p = O.make_params(fixed_segments=-1, max_iter=j, restart=30, preset="paper_gmres",
                          tol=1e-30, orth=orth)
        r = O.gmres(A.indptr, b, p, A.indices, A.data)
        K = np.stack([np.linalg.matrix_power(D, k) @ b for k in range(j)], axis=1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(D @ Q, b, rcond=None)
        best = np.linalg.norm(b - D @ Q @ y)
        assert r.hist[j] * np.linalg.norm(b) == pytest.approx(best, rel=1e-8)
        assert np.linalg.norm(b - D @ r.x) == pytest.approx(best, rel=1e-8)


def test_stepped_gmres_reaches_tolerance():
    A = convdiff2d(40, 2)
    x_true, b = rhs_from_solution(A, 2)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    for orth in (0, 1, 2):
        p = O.make_params(max_iter=15000, preset="paper_gmres", orth=orth)
        r = O.gmres(A.indptr, b, p, A.indices, A.data, enc)
        assert r.status == O.OK and r.relres_true <= 1e-10
        assert r.iters_per_seg[0] > 0
        r64 = O.gmres(A.indptr, b, O.make_params(max_iter=15000, preset="paper_gmres",
                                                 fixed_segments=-1, orth=orth),
                      A.indices, A.data)
        assert r64.status == O.OK and r64.relres_true <= 1e-10


@pytest.mark.parametrize("n", [3, 5, 9])
def test_dcgs2_exact_in_fewer_steps_than_the_cycle(n):
    """A cycle longer than the system: the Krylov space is exhausted after n
    steps (the delayed second pass finds a zero norm) and the solve is exact."""
    A, D = tiny_nonsym(n, n + 3)
    b = np.random.default_rng(n + 1).standard_normal(n)
    p = O.make_params(fixed_segments=-1, max_iter=60, restart=30, preset="paper_gmres",
                      tol=1e-14, orth=2)
    r = O.gmres(A.indptr, b, p, A.indices, A.data)
    assert r.iters <= n
    assert np.allclose(r.x, np.linalg.solve(D, b), rtol=1e-9, atol=1e-11)


def test_dcgs2_follows_cgs2():
    """The delayed second pass changes only the order in which the same
    Krylov quantities are formed: over restarted cycles of a nonsymmetric
    operator (FP64 and the stepped GSE operators) the residual estimates of
    every iteration agree with those of CGS2 to rounding, with the same
    iteration counts and switch points."""
    A = convdiff2d(40, 3)
    x_true, b = rhs_from_solution(A, 3)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    for fs in (-1, 0):
        res = []
        for orth in (1, 2):
            p = O.make_params(max_iter=15000, preset="paper_gmres", orth=orth, fixed_segments=fs)
            res.append(O.gmres(A.indptr, b, p, A.indices, A.data, enc))
        c, d = res
        assert c.status == d.status == O.OK
        assert c.iters == d.iters and c.switch_iter == d.switch_iter
        assert c.iters_per_seg == d.iters_per_seg
        k = c.iters + 1
        np.testing.assert_allclose(d.hist[:k], c.hist[:k], rtol=1e-6)
        assert np.linalg.norm(d.x - c.x) <= 1e-8 * np.linalg.norm(c.x)

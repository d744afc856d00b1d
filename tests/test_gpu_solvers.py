"""GPU parity of the stepped CG and GMRES solvers against the oracle.

Solves are iterations, so several results are correct: both sides must reach
the true relative residual ||b - A x|| / ||b|| <= 1e-10 (checked again here
in FP64 on the host), agree on the solution within the accuracy the
tolerance allows (relative difference <= 1e-6 for these well-conditioned
systems), and take iteration counts within 10 % of each other.  Where the
operator is exact (Poisson: integer stencil, eta_1 = 0) the stepped GPU
solve never leaves one segment and follows the GPU FP64 solve to rounding:
the operators give identical products, and only the grouping of the dot
products' partial sums (each format runs at its own occupancy) may differ.
"""
import numpy as np
import pytest

import oracle as O
from workloads import CSR, convdiff2d, diffusion2d, diffusion3d, poisson2d, rhs_from_solution

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(A: CSR):
    return (torch.from_numpy(A.indptr).to(DEV), torch.from_numpy(A.indices).to(DEV),
            torch.from_numpy(A.data).to(DEV))


def true_relres(A: CSR, x, b):
    r = b - A.to_scipy() @ x
    return np.linalg.norm(r) / np.linalg.norm(b)


def gpu_solve(kind, A: CSR, b, method, fixed=0, max_iter=5000, switch_mode=1, x0=None,
              record=True, rv=-1, launch_mode=0, restart=None, **ctrl):
    rp, ci, va = to_dev(A)
    p = G.gse_default_params(method)
    p.max_iter = max_iter
    if restart is not None:
        p.restart = restart
    for k, v in ctrl.items():  # controller parameters (l, t, m, floor_c, ndec_limit, ...)
        setattr(p, k, v)
    p.fixed_segments = fixed
    p.switch_mode = switch_mode
    p.launch_mode = launch_mode
    p.record_history = 1 if record else 0
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV) if x0 is None else \
        torch.from_numpy(x0).to(DEV)
    bd = torch.from_numpy(b).to(DEV)
    if kind == "gse":
        M = G.GseMatrix(rp, ci, va, A.n_cols)
        if rv != -1:
            M.plan(1024, rv)  # the same schedule as the FP64 operator below
        fn = G.gse_cg if method == G.CG else G.gse_gmres
        rep = fn(M.A, bd, x, p, ws)
    else:
        M = G.CsrMatrix(rp, ci, va, A.n_cols, tile_nnz=1024, rv_lanes=rv)
        fn = G.gse_csr_cg if method == G.CG else G.gse_csr_gmres
        rep = fn(M.M, bd, x, p, ws)
    torch.cuda.synchronize()
    hist = seg = None
    if record:
        hist, seg = G.gse_solve_history(ws, rep.iters + 1)
    return rep, x.cpu().numpy(), hist, seg


def gmres_orth(restart=30):
    """The oracle's Gram-Schmidt variant matching the library default:
    delayed CGS2 (2) for restarts up to 32, CGS2 (1) beyond."""
    return 2 if restart <= 32 else 1


def oracle_params(method, fixed=0, max_iter=5000, switch_mode=1, restart=30):
    preset = "paper_cg" if method == G.CG else "paper_gmres"
    return O.make_params(tol=1e-10, max_iter=max_iter, restart=restart, fixed_segments=fixed,
                         preset=preset, switch_mode=switch_mode, orth=gmres_orth(restart))


def test_cg_fp64_poisson_matches_oracle():
    A = poisson2d(64)
    x_true, b = rhs_from_solution(A, 0)
    rep, x, hist, _ = gpu_solve("csr", A, b, G.CG)
    ref = O.cg(A.indptr, b, oracle_params(G.CG, fixed=-1), A.indices, A.data)
    assert rep.status == G.OK and ref.status == O.OK
    assert abs(rep.iters - ref.iters) <= 2
    assert rep.relres_true <= 1e-10 and true_relres(A, x, b) <= 1e-10
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    n = min(len(hist), len(ref.hist))
    assert np.allclose(hist[:n], ref.hist[:n], rtol=1e-6, atol=1e-13)


def test_stepped_cg_follows_fp64_on_exact_stencil():
    A = poisson2d(64)
    _, b = rhs_from_solution(A, 1)
    for rv in (-1, 8):
        r64, x64, h64, _ = gpu_solve("csr", A, b, G.CG, rv=rv)
        rst, xst, hst, sst = gpu_solve("gse", A, b, G.CG, rv=rv)
        assert r64.status == G.OK and rst.status == G.OK
        assert rst.iters == r64.iters and list(rst.iters_per_seg) == [rst.iters, 0, 0]
        assert np.all(sst[1:] == 1)
        assert np.linalg.norm(xst - x64) <= 1e-12 * np.linalg.norm(x64)
        assert np.allclose(hst, h64, rtol=1e-9, atol=0)
        if rv == 8:  # the row-vector schedule's grid does not depend on the format
            assert np.array_equal(xst, x64) and np.array_equal(hst, h64)


def test_spmv_products_identical_across_formats_on_exact_stencil():
    """Each row sum has a fixed order, so formats that decode to the same
    values give the same bits, whatever kernel or occupancy."""
    A = poisson2d(64)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    C = G.CsrMatrix(rp, ci, va, A.n_cols)
    x = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, A.n_cols)).to(DEV)
    y64 = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    C.spmv(x, y64)
    for s in (1, 2, 3):
        ys = torch.empty_like(y64)
        M.spmv(s, x, ys)
        torch.cuda.synchronize()
        assert torch.equal(ys, y64)


@pytest.mark.parametrize("switch_mode", [0, 1, 2])
def test_stepped_cg_variable_coefficients(switch_mode):
    A = diffusion3d(20, 3)
    x_true, b = rhs_from_solution(A, 3)
    rep, x, hist, seg = gpu_solve("gse", A, b, G.CG, switch_mode=switch_mode)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    ref = O.cg(A.indptr, b, oracle_params(G.CG, switch_mode=switch_mode), A.indices, A.data,
               enc)
    assert rep.status == G.OK and ref.status == O.OK
    assert rep.relres_true <= 1e-10 and true_relres(A, x, b) <= 1e-10
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10)
    assert rep.iters_per_seg[0] > 0 and rep.switch_iter[0] > 0
    # segment history steps up by one at the switches and matches the report
    d = np.diff(seg[1:])
    assert np.all((d == 0) | (d == 1))
    assert [int((seg[1:] == s).sum()) for s in (1, 2, 3)] == list(rep.iters_per_seg)
    assert abs(rep.switch_iter[0] - ref.switch_iter[0]) <= 3


def test_fixed_segments_cg():
    A = diffusion3d(12, 4)
    _, b = rhs_from_solution(A, 4)
    rep3, x3, _, _ = gpu_solve("gse", A, b, G.CG, fixed=3)
    assert rep3.status == G.OK and list(rep3.iters_per_seg) == [0, 0, rep3.iters]
    rep1, x1, _, _ = gpu_solve("gse", A, b, G.CG, fixed=1, max_iter=400)
    # with the head only the true residual floors near eta_1, far above 1e-10
    assert rep1.status == G.NOT_CONVERGED and rep1.relres_true > 1e-8


@pytest.mark.parametrize("kind", ["csr", "gse"])
def test_gmres_convdiff_matches_oracle(kind):
    A = convdiff2d(48, 2)
    x_true, b = rhs_from_solution(A, 2)
    rep, x, hist, seg = gpu_solve(kind, A, b, G.GMRES, max_iter=15000)
    if kind == "csr":
        ref = O.gmres(A.indptr, b, oracle_params(G.GMRES, fixed=-1, max_iter=15000), A.indices,
                      A.data)
    else:
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        ref = O.gmres(A.indptr, b, oracle_params(G.GMRES, max_iter=15000), A.indices, A.data,
                      enc)
    assert rep.status == G.OK and ref.status == O.OK, (rep.as_dict(), ref.status)
    assert rep.relres_true <= 1e-10 and true_relres(A, x, b) <= 1e-10
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(5, ref.iters // 10)


def test_gmres_first_cycle_residuals_match_oracle():
    """Within one cycle the GMRES residual estimates follow the oracle's
    (CGS2 on both sides) to rounding."""
    A = convdiff2d(32, 5)
    _, b = rhs_from_solution(A, 5)
    rep, x, hist, _ = gpu_solve("csr", A, b, G.GMRES, max_iter=30)
    ref = O.gmres(A.indptr, b, oracle_params(G.GMRES, fixed=-1, max_iter=30), A.indices, A.data)
    assert rep.iters == ref.iters == 30
    assert np.allclose(hist[:31], ref.hist[:31], rtol=1e-8, atol=1e-15)


@pytest.mark.parametrize("restart", [1, 2, 3, 4, 8, 32, 33])
def test_gmres_short_and_boundary_restarts_first_cycles(restart):
    """The delayed CGS2's edge steps (a cycle of one to four columns, the
    last basis tier at 32) and the first CGS2 restart past it (33): the
    residual estimates of the first cycles follow the oracle's same variant
    to rounding, on FP64 and on the head-only operator."""
    A = convdiff2d(40, 9)
    _, b = rhs_from_solution(A, 9)
    cycles = 3 * restart
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    for kind, fixed in (("csr", -1), ("gse", 1)):
        rep, x, hist, _ = gpu_solve(kind, A, b, G.GMRES, fixed=max(fixed, 0), max_iter=cycles,
                                    restart=restart)
        ref = O.gmres(A.indptr, b, oracle_params(G.GMRES, fixed=fixed, max_iter=cycles,
                                                 restart=restart),
                      A.indices, A.data, enc if kind == "gse" else None)
        assert rep.iters == ref.iters == cycles, (kind, rep.iters, ref.iters)
        np.testing.assert_allclose(hist[:cycles + 1], ref.hist[:cycles + 1], rtol=1e-8,
                                   atol=1e-15)
        assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("restart", [5, 17, 45, 60])
def test_gmres_restart_lengths_match_oracle(restart):
    """Every restart length runs its own Gram-Schmidt instantiations (basis
    counts rounded up to 4, up to 60) and update kernel: the residual
    estimates of the first cycle follow the oracle's CGS2 to rounding, and
    the restarted solve converges with the oracle's solution."""
    A = convdiff2d(40, 9)  # no restart length converges inside one cycle
    _, b = rhs_from_solution(A, 9)
    rep, x, hist, _ = gpu_solve("csr", A, b, G.GMRES, max_iter=restart, restart=restart)
    ref = O.gmres(A.indptr, b, oracle_params(G.GMRES, fixed=-1, max_iter=restart, restart=restart),
                  A.indices, A.data)
    assert rep.iters == ref.iters == restart
    assert np.allclose(hist[:restart + 1], ref.hist[:restart + 1], rtol=1e-8, atol=1e-15)
    rep, x, _, _ = gpu_solve("gse", A, b, G.GMRES, max_iter=15000, restart=restart)
    assert rep.status == G.OK and true_relres(A, x, b) <= 1e-10
    ref = O.gmres(A.indptr, b, oracle_params(G.GMRES, max_iter=15000, restart=restart), A.indices,
                  A.data, O.encode(A.indptr, A.indices, A.data, A.n_cols))
    assert ref.status == O.OK
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_gmres_small_dense_exact_within_one_cycle():
    """n <= restart: the Krylov space is the whole space after n steps, so
    GMRES ends with ||w|| = 0 (or below the tolerance) inside the first cycle
    -- the one-workgroup launches and the lucky-breakdown path."""
    import scipy.sparse as sp
    rng = np.random.default_rng(11)
    for n in (1, 3, 12, 29):
        D = rng.standard_normal((n, n)) + n * np.eye(n)  # nonsymmetric, well conditioned
        A = CSR.from_scipy(sp.csr_matrix(D))
        b = rng.standard_normal(n)
        rep, x, _, _ = gpu_solve("gse", A, b, G.GMRES, fixed=3, restart=30)
        assert rep.status == G.OK, (n, rep.as_dict())
        assert rep.iters <= n
        assert np.allclose(x, np.linalg.solve(D, b), rtol=1e-8, atol=1e-10)


def _tridiag(n, seed):
    """1-D variable-coefficient diffusion plus a small shift (rows of at
    most 3 non-zeros; CG converges in ~160 iterations)."""
    import scipy.sparse as sp
    k = 10.0 ** np.random.default_rng(seed).uniform(-1, 1, n + 1)
    main = k[:-1] + k[1:] + 0.05 * k[:-1].mean()
    off = -k[1:-1]
    return CSR.from_scipy(sp.diags([off, main, off], [-1, 0, 1], format="csr"))


@pytest.mark.parametrize("name", ["poisson_400", "tridiag_1500", "diff2d_4096", "diff3d_4096"])
def test_small_system_cg_matches_oracle(name):
    """Systems of at most 4096 rows with rows of at most 8 non-zeros run
    all their iterations in one workgroup (one, two or four rows per thread;
    4, 6 or 8 register slots per row): stepped GSE and FP64 CG against the
    oracle."""
    A = {"poisson_400": lambda: poisson2d(20), "tridiag_1500": lambda: _tridiag(1500, 4),
         "diff2d_4096": lambda: diffusion2d(64, 4), "diff3d_4096": lambda: diffusion3d(16, 4)}[name]()
    _, b = rhs_from_solution(A, 4)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    for kind in ("gse", "csr"):
        rep, x, hist, seg = gpu_solve(kind, A, b, G.CG)
        if kind == "gse":
            ref = O.cg(A.indptr, b, oracle_params(G.CG), A.indices, A.data, enc)
        else:
            ref = O.cg(A.indptr, b, oracle_params(G.CG, fixed=-1), A.indices, A.data)
        assert rep.status == G.OK and ref.status == O.OK, (kind, rep.as_dict())
        assert rep.relres_true <= 1e-10 and true_relres(A, x, b) <= 1e-10
        assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
        assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10)
        if kind == "gse":
            assert list(rep.iters_per_seg) == [int((seg[1:] == s).sum()) for s in (1, 2, 3)]
            assert abs(rep.switch_iter[0] - ref.switch_iter[0]) <= 3


def test_small_system_conditions_on_the_check_grid():
    """A short check grid (l = 20, t = m = 10, no floor trigger): Conditions
    1-3 are evaluated inside the one-workgroup loop and switch the segment
    count where the oracle's controller does."""
    A = diffusion2d(40, 5)
    _, b = rhs_from_solution(A, 5)
    ctrl = dict(l=20, t=10, m=10, ndec_limit=6, floor_c=0.0)
    rep, x, hist, seg = gpu_solve("gse", A, b, G.CG, **ctrl)
    ref = O.cg(A.indptr, b, O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg", switch_mode=1,
                                          orth=1, **ctrl),
               A.indices, A.data, O.encode(A.indptr, A.indices, A.data, A.n_cols))
    assert rep.status == G.OK and ref.status == O.OK
    assert true_relres(A, x, b) <= 1e-10
    assert list(rep.switch_iter) == list(ref.switch_iter)
    assert list(rep.switch_trigger) == list(ref.switch_trigger)
    assert rep.switch_trigger[0] in (1, 2, 3)  # Conditions 1-3, not the floor or tolerance
    # the residual histories agree to the rounding CG accumulates over ~50
    # iterations and a residual replacement (different reduction trees)
    assert np.allclose(hist[: rep.switch_iter[1] + 1], ref.hist[: rep.switch_iter[1] + 1],
                       rtol=1e-6, atol=0)


def test_cg_small_dense_and_edge_cases():
    import scipy.sparse as sp
    rng = np.random.default_rng(7)
    for n in (1, 5, 12):
        Mx = rng.standard_normal((n, n))
        D = Mx @ Mx.T + n * np.eye(n)
        A = CSR.from_scipy(sp.csr_matrix(D))
        b = rng.standard_normal(n)
        rep, x, _, _ = gpu_solve("gse", A, b, G.CG, fixed=3)
        assert rep.status == G.OK
        assert np.allclose(x, np.linalg.solve(D, b), rtol=1e-8, atol=1e-10)
    # b = 0 -> x = 0
    A = poisson2d(8)
    rep, x, _, _ = gpu_solve("gse", A, np.zeros(A.n_rows), G.CG, x0=np.ones(A.n_rows))
    assert rep.status == G.OK and np.all(x == 0)
    # indefinite: breakdown with all segments
    Ai = CSR.from_scipy(sp.csr_matrix(np.diag([1.0, -1.0, 2.0])))
    rep, _, _, _ = gpu_solve("gse", Ai, np.ones(3), G.CG, fixed=3)
    assert rep.status == G.ERR_BREAKDOWN
    rep, _, _, _ = gpu_solve("csr", Ai, np.ones(3), G.CG)
    assert rep.status == G.ERR_BREAKDOWN


def test_solver_argument_errors():
    A = poisson2d(8)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    p = G.gse_default_params(G.CG)
    ws = torch.empty(1024, dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    b = torch.ones(A.n_rows, dtype=torch.float64, device=DEV)
    with pytest.raises(G.GseError) as ei:
        G.gse_cg(M.A, b, x, p, ws)
    assert ei.value.status == G.ERR_NOMEM
    p.start_segments = 4
    ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    with pytest.raises(G.GseError) as ei:
        G.gse_cg(M.A, b, x, p, ws)
    assert ei.value.status == G.ERR_ARG


@pytest.mark.parametrize("method", [G.CG, G.GMRES])
def test_graph_replay_matches_direct_launches(method):
    """Iterations replayed from HIP graphs give the same bits as direct
    launches, solve after solve, with eager work on the device in between."""
    A = diffusion3d(14, 6) if method == G.CG else convdiff2d(40, 6)
    _, b = rhs_from_solution(A, 6)
    kw = dict(max_iter=5000 if method == G.CG else 15000)
    rd, xd, hd, _ = gpu_solve("gse", A, b, method, launch_mode=1, **kw)
    for _ in range(3):
        junk = torch.randn(1 << 20, device=DEV).sum()  # unrelated eager work
        rg, xg, hg, _ = gpu_solve("gse", A, b, method, launch_mode=0, **kw)
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert rg.status == rd.status == G.OK
        assert rg.iters == rd.iters and list(rg.iters_per_seg) == list(rd.iters_per_seg)
        assert np.array_equal(xg, xd)
        assert np.array_equal(hg, hd)


@pytest.mark.parametrize("k", [2, 16, 64])
def test_stepped_cg_with_other_table_sizes(k):
    """Stepped CG on tables of k = 2, 16, 64 shared exponents (slot index of
    1, 4, 6 bits) against the oracle's CG on the same encoding; a 1600-row
    system whose index is wider than 3 bits runs the multi-launch path."""
    for A in (diffusion3d(18, 7), diffusion2d(40, 8)):
        _, b = rhs_from_solution(A, 7)
        rp, ci, va = to_dev(A)
        M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=k)
        p = G.gse_default_params(G.CG)
        p.switch_mode = 0
        ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                         dtype=torch.uint8, device=DEV)
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
        rep = G.gse_cg(M.A, torch.from_numpy(b).to(DEV), x, p, ws)
        torch.cuda.synchronize()
        xs = x.cpu().numpy()
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=k)
        ref = O.cg(A.indptr, b, O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg",
                                              switch_mode=0, orth=1), A.indices, A.data, enc)
        assert rep.status == G.OK and ref.status == O.OK, (k, rep.as_dict())
        assert rep.relres_true <= 1e-10 and true_relres(A, xs, b) <= 1e-10
        assert np.linalg.norm(xs - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
        assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10)


def test_batch_with_other_table_sizes():
    """Batched CG on systems encoded with k = 4 and k = 32 (2- and 5-bit slot
    indices) side by side: each against the oracle's CG."""
    systems = [(diffusion3d(12, 9), 4), (diffusion2d(50, 10), 32)]
    keep, triples = [], []
    p = G.gse_default_params(G.CG)
    p.switch_mode = 0
    for A, k in systems:
        _, b = rhs_from_solution(A, 9)
        rp, ci, va = to_dev(A)
        M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=k)
        bd = torch.from_numpy(b).to(DEV)
        xd = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
        keep.append((M, bd, xd, b))
        triples.append((M.A, bd, xd))
    ws = torch.empty(G.gse_batch_workspace(triples, p), dtype=torch.uint8, device=DEV)
    reps = G.gse_batch_cg(triples, p, ws)
    torch.cuda.synchronize()
    for (A, k), rep, (_, _, xd, b) in zip(systems, reps, keep):
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=k)
        ref = O.cg(A.indptr, b, O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg",
                                              switch_mode=0, orth=1), A.indices, A.data, enc)
        xs = xd.cpu().numpy()
        assert rep.status == G.OK and ref.status == O.OK
        assert true_relres(A, xs, b) <= 1e-10
        assert np.linalg.norm(xs - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
        assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10)


def test_stepped_cg_with_the_index_in_the_value():
    """Stepped CG (multi-launch; the one-workgroup loop keeps the column
    layout) and batched CG on encodings with the slot in the value word,
    against the oracle's CG on the same layout."""
    A = diffusion2d(40, 12)
    _, b = rhs_from_solution(A, 12)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols, idx_layout=G.IDX_VALUE)
    p = G.gse_default_params(G.CG)
    p.switch_mode = 0
    ws = torch.empty(G.gse_solver_workspace(G.CG, A.n_rows, A.nnz, 30, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    bd = torch.from_numpy(b).to(DEV)
    rep = G.gse_cg(M.A, bd, x, p, ws)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, layout=1)
    ref = O.cg(A.indptr, b, O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg",
                                          switch_mode=0, orth=1), A.indices, A.data, enc)
    xs = x.cpu().numpy()
    assert rep.status == G.OK and ref.status == O.OK
    assert true_relres(A, xs, b) <= 1e-10
    assert np.linalg.norm(xs - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10)
    xb = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    wsb = torch.empty(G.gse_batch_workspace([(M.A, bd, xb)], p), dtype=torch.uint8, device=DEV)
    rb, = G.gse_batch_cg([(M.A, bd, xb)], p, wsb)
    torch.cuda.synchronize()
    assert rb.status == G.OK
    assert np.linalg.norm(xb.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("method", [G.CG, G.GMRES], ids=["cg", "gmres"])
def test_graphs_kept_across_solves(method):
    """A second solve with the same operand, workspace and vectors replays the
    graphs the first one captured: same bits, same report.  A different
    matrix on the same workspace and vectors captures its own and still
    matches the oracle."""
    A = diffusion3d(24, 5)
    x_true, b = rhs_from_solution(A, 6)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    p = G.gse_default_params(method)
    p.max_iter = 5000
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    bd = torch.from_numpy(b).to(DEV)
    fn = G.gse_cg if method == G.CG else G.gse_gmres
    runs = []
    for _ in range(3):
        x.zero_()
        rep = fn(M.A, bd, x, p, ws)
        torch.cuda.synchronize()
        runs.append((rep.as_dict(), x.cpu().numpy().copy()))
    for r, xs in runs[1:]:
        assert r["iters"] == runs[0][0]["iters"] and r["switch_iter"] == runs[0][0]["switch_iter"]
        assert np.array_equal(xs, runs[0][1])
    # another operator (other coefficients, same shape) on the same buffers
    A2 = diffusion3d(24, 7)
    b2 = A2.to_scipy() @ x_true
    rp2, ci2, va2 = to_dev(A2)
    M2 = G.GseMatrix(rp2, ci2, va2, A2.n_cols)
    bd.copy_(torch.from_numpy(b2))
    x.zero_()
    rep = fn(M2.A, bd, x, p, ws)
    torch.cuda.synchronize()
    assert rep.status == G.OK
    assert true_relres(A2, x.cpu().numpy(), b2) <= 1e-10


def test_gmres_gram_schmidt_variants():
    """orth = 1 (CGS2) and 2 (DCGS2, the default up to restart 32) against
    the oracle's same variant on the stepped 64^2 convection-diffusion
    system: iteration counts, per-segment counts and switch points equal,
    solutions within 1e-8; orth 0 is DCGS2 at restart 30 and CGS2 at
    restart 40, bit for bit; DCGS2 past restart 32 and unknown values are
    refused."""
    A = convdiff2d(64, 4)
    _, b = rhs_from_solution(A, 4)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    runs = {}
    for orth, restart in ((1, 30), (2, 30), (0, 30), (0, 40), (1, 40)):
        rep, x, hist, _ = gpu_solve("gse", A, b, G.GMRES, restart=restart, orth=orth,
                                    max_iter=15000)
        runs[(orth, restart)] = (rep, x, hist)
        if orth == 0:
            continue
        prm = O.make_params(tol=1e-10, max_iter=15000, restart=restart, preset="paper_gmres",
                            orth=orth)
        ref = O.gmres(A.indptr, b, prm, A.indices, A.data, enc)
        assert rep.status == G.OK and ref.status == O.OK, (orth, restart)
        assert rep.iters == ref.iters and list(rep.switch_iter) == list(ref.switch_iter)
        assert list(rep.iters_per_seg) == list(ref.iters_per_seg)
        assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
        k = rep.iters + 1
        np.testing.assert_allclose(hist[:k], ref.hist[:k], rtol=1e-6)
    for same, other in (((0, 30), (2, 30)), ((0, 40), (1, 40))):
        assert np.array_equal(runs[same][1], runs[other][1])
        assert np.array_equal(runs[same][2], runs[other][2])
    for orth, restart in ((2, 40), (3, 30), (-1, 30)):
        with pytest.raises(G.GseError) as e:
            gpu_solve("gse", A, b, G.GMRES, restart=restart, orth=orth)
        assert e.value.status == G.ERR_ARG

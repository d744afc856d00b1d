"""GPU parity of the FP16 / BF16 comparators (Section IV-C, IV-D.3) against
the oracle: the 16-bit words bit-exact (one round to nearest even per value,
overflow to infinity counted), eta_h against the host, the 16-bit SpMV
within 1e-12 of the oracle's (the widened values are exact on both sides,
only the summation order may differ) on every schedule, and CG / GMRES on
the fixed 16-bit operator against the oracle's."""
import numpy as np
import pytest

import oracle as O
from workloads import CSR, convdiff2d, diffusion3d, powerlaw, random_sparse, rhs_from_solution

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")
FMTS = [(G.LP_FP16, O.LP_FP16), (G.LP_BF16, O.LP_BF16)]


def to_dev(A: CSR):
    return (torch.from_numpy(A.indptr).to(DEV), torch.from_numpy(A.indices).to(DEV),
            torch.from_numpy(A.data).to(DEV))


def matrices():
    return {"diffusion3d_20": lambda: diffusion3d(20, 1),
            "powerlaw_20k": lambda: powerlaw(20_000, 2),
            "random_wide": lambda: random_sparse(3000, 2500, 5, mean_row=4, empty_frac=0.2,
                                                 long_rows=6, long_len=2400, exp_spread=60),
            "convdiff2d_48": lambda: convdiff2d(48, 3)}


@pytest.mark.parametrize("fmt", FMTS, ids=["fp16", "bf16"])
@pytest.mark.parametrize("name", list(matrices()))
def test_lp_conversion_and_spmv_match_oracle(name, fmt):
    gfmt, ofmt = fmt
    A = matrices()[name]()
    rp, ci, va = to_dev(A)
    M = G.LpMatrix(rp, ci, va, A.n_cols, fmt=gfmt)
    want, over = O.lp_convert(A.data, ofmt)
    assert np.array_equal(M.values(), want)
    assert M.M.overflow == over
    wide = np.array([O.lp_widen(h, ofmt) for h in want])
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    with np.errstate(invalid="ignore", over="ignore"):
        d = np.zeros(A.n_rows)
        a = np.zeros(A.n_rows)
        np.add.at(d, rows, np.abs(A.data - wide))
        np.add.at(a, rows, np.abs(A.data))
        eta = d.max() / a.max()
    if np.isfinite(eta):
        assert M.M.eta == pytest.approx(eta, rel=1e-12, abs=1e-300)
    else:
        assert not np.isfinite(M.M.eta)
    if over:
        return  # infinities in the operator: no finite product to compare
    x = np.random.default_rng(gfmt).uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    ref = O.lp_spmv(A.indptr, A.indices, want, ofmt, x)
    scale = np.zeros(A.n_rows)
    np.add.at(scale, rows, np.abs(wide * x[A.indices]))
    for sched in ((1024, -1), (2048, 0), (4096, 0), (2048, 8)):
        M.plan(*sched)
        M.spmv(xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        assert np.all(np.abs(y - ref) <= 1e-12 * scale + 1e-300), (name, sched)


def test_fp16_overflow_is_counted():
    """Values past 65504 round to infinity in FP16 (the overflow of
    Section IV-D.2) and are counted; BF16 holds them."""
    A = diffusion3d(8, 0)
    big = A.data * 1e5  # off-diagonals up to ~1e7: beyond binary16
    rp, ci, _ = to_dev(A)
    vb = torch.from_numpy(big).to(DEV)
    M16 = G.LpMatrix(rp, ci, vb, A.n_cols, fmt=G.LP_FP16)
    _, want = O.lp_convert(big, O.LP_FP16)
    assert want > 0 and M16.M.overflow == want and not np.isfinite(M16.M.eta)
    Mb = G.LpMatrix(rp, ci, vb, A.n_cols, fmt=G.LP_BF16)
    assert Mb.M.overflow == 0 and np.isfinite(Mb.M.eta)


def _solve(method, A, b, gfmt, ofmt, restart=30):
    rp, ci, va = to_dev(A)
    M = G.LpMatrix(rp, ci, va, A.n_cols, fmt=gfmt)
    p = G.gse_default_params(method)
    p.max_iter = 15000 if method == G.GMRES else 5000
    p.restart = restart
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    fn = G.gse_lp_gmres if method == G.GMRES else G.gse_lp_cg
    rep = fn(M.M, torch.from_numpy(b).to(DEV), x, p, ws)
    torch.cuda.synchronize()
    plane, _ = O.lp_convert(A.data, ofmt)
    prm = O.make_params(tol=1e-10, max_iter=p.max_iter, restart=restart, fixed_segments=O.S_LP,
                        preset="paper_gmres" if method == G.GMRES else "paper_cg",
                        orth=2 if restart <= 32 else 1)
    osolve = O.gmres if method == G.GMRES else O.cg
    ref = osolve(A.indptr, b, prm, A.indices, A.data, lp=(plane, ofmt))
    return rep, x.cpu().numpy(), ref


@pytest.mark.parametrize("fmt", FMTS, ids=["fp16", "bf16"])
def test_lp_cg_matches_oracle(fmt):
    A = diffusion3d(18, 4, decades=2.0)
    _, b = rhs_from_solution(A, 4)
    rep, x, ref = _solve(G.CG, A, b, *fmt)
    assert rep.status == G.OK and ref.status == O.OK, rep.as_dict()
    assert rep.relres_true <= 1e-10  # on its own operator
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10)
    assert list(rep.iters_per_seg) == [0, 0, rep.iters]


@pytest.mark.parametrize("fmt", FMTS, ids=["fp16", "bf16"])
def test_lp_gmres_matches_oracle(fmt):
    A = convdiff2d(40, 6)
    _, b = rhs_from_solution(A, 6)
    rep, x, ref = _solve(G.GMRES, A, b, *fmt)
    assert rep.status == G.OK and ref.status == O.OK, rep.as_dict()
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(5, ref.iters // 10)


def test_lp_cg_with_an_overflowed_operator_stops():
    """An FP16 operator holding infinities gives a non-finite p.Ap at once:
    the solve reports a breakdown, as the oracle's does."""
    A = diffusion3d(8, 0)
    big = A.data * 1e5
    _, b = rhs_from_solution(A, 0)
    B = CSR(A.n_rows, A.n_cols, A.indptr, A.indices, big, A.name + "_x1e5")
    rep, x, ref = _solve(G.CG, B, b, G.LP_FP16, O.LP_FP16)
    assert rep.status == G.ERR_BREAKDOWN and ref.status == O.ERR_BREAKDOWN

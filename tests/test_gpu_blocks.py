"""GPU parity of the sampled tables (Section III-B.1, sampling): per row
block, and one table from the pooled drawn rows.

gse_encode_blocks against the oracle's encode_blocks on the same seeded
inputs and the same drawn rows: the block tables, the four planes and
exact_frac bit-exact, eta within 1e-12 relative.  The SpMV (row-vector
schedule, every lane width) against the oracle's block SpMV within 1e-12
relative, norm-wise and componentwise (the values are exact on both sides;
only the summation order differs).  CG and GMRES on block matrices: both
sides reach the true residual 1e-10, solutions within 1e-6, iteration counts
within 10 %.  gse_encode_sampled against the oracle's encode_sampled: the
table, planes and exact_frac bit-exact, eta within 1e-12, the SpMV as above.
"""
import numpy as np
import pytest

import oracle as O
from workloads import (CSR, block_sample_rows, diffusion3d, layered3d, powerlaw, random_sparse,
                       rhs_from_solution)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(A: CSR):
    return (torch.from_numpy(A.indptr).to(DEV), torch.from_numpy(A.indices).to(DEV),
            torch.from_numpy(A.data).to(DEV))


CASES = {
    # ragged last block (700 = 5 * 128 + 60), exponents over 30 binades
    "random_700_R128": (lambda: random_sparse(700, 500, 3, mean_row=5, exp_spread=30.0), 128),
    # empty rows, a block size that is no power of two
    "random_empty_R130": (lambda: random_sparse(1000, 1000, 4, mean_row=7, empty_frac=0.2,
                                                exp_spread=12.0), 130),
    "layered_10_R200": (lambda: layered3d(10, 5, contrast=12.0), 200),
    "diffusion3d_24_R4096": (lambda: diffusion3d(24, 0), 4096),
    # long rows (up to a few hundred non-zeros) across block boundaries
    "powerlaw_20k_R1000": (lambda: powerlaw(20_000, 2), 1000),
    # fewer rows than one block
    "tiny_R128": (lambda: random_sparse(5, 5, 8, mean_row=2), 128),
}


def encode_both(A, R, k=8, sampled=False, layout=G.IDX_AUTO, seed=1):
    sr = block_sample_rows(A.n_rows, R, seed) if sampled else None
    olay = {G.IDX_AUTO: -1, G.IDX_COLUMN: 0, G.IDX_VALUE: 1}[layout]
    enc = O.encode_blocks(A.indptr, A.indices, A.data, A.n_cols, num_exp=k, block_rows=R,
                          sample_rows=sr, layout=olay)
    rp, ci, va = to_dev(A)
    srd = None if sr is None else torch.from_numpy(sr).to(DEV)
    M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=k, idx_layout=layout, block_rows=R,
                    sample_rows=srd)
    return enc, M


def check_encode(name, A, enc, M):
    stride = M.A.block_stride
    assert stride == 1 << enc.idx_bits and M.A.block_rows == enc.block_rows
    got = M.block_tables()
    assert np.array_equal(got, enc.block_sem[:, :stride]), name
    assert not enc.block_sem[:, stride:].any()
    assert M.A.num_used == max(int((t > 0).sum()) for t in enc.block_sem) if A.n_rows else True
    for g, w, what in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2),
                          ("col_idx", "head", "tail1", "tail2")):
        assert np.array_equal(g, w), (name, what, np.nonzero(g != w)[0][:5])
    assert M.A.exact_frac == enc.exact_frac
    for s in range(3):
        assert M.eta[s] == pytest.approx(enc.eta[s], rel=1e-12, abs=1e-300)
    assert M.A.idx_layout == (G.IDX_VALUE if enc.layout == 1 else G.IDX_COLUMN)


def _check_close(got, ref, scale, tol=1e-12):
    assert np.all(np.abs(got - ref) <= tol * scale + 1e-300)
    nr = np.linalg.norm(ref)
    if nr > 0:
        assert np.linalg.norm(got - ref) <= tol * nr + 1e-300


def check_spmv(A, enc, M, lanes=(0,)):
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.full((A.n_rows,), np.nan, dtype=torch.float64, device=DEV)
    for L in lanes:
        M.plan(1024, L)  # L = 0: the row-tile ring on rows of <= 8 non-zeros
        assert M.A.rv_lanes == L
        for s in (1, 2, 3):
            M.spmv(s, xd, yd)
            torch.cuda.synchronize()
            y = yd.cpu().numpy()
            ref = O.gse_spmv(A.indptr, enc, s, x)
            dec = O.decode_blocks(A.indptr, enc, s)
            scale = np.zeros(A.n_rows)
            np.add.at(scale, np.repeat(np.arange(A.n_rows), np.diff(A.indptr)),
                      np.abs(dec * x[A.indices]))
            _check_close(y, ref, scale)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("sampled", [False, True], ids=["exact", "sampled"])
def test_encode_and_spmv(name, sampled):
    make, R = CASES[name]
    A = make()
    enc, M = encode_both(A, R, sampled=sampled)
    check_encode(name, A, enc, M)
    check_spmv(A, enc, M, lanes=(0, 1, 4, 16, 64))


@pytest.mark.parametrize("k", [1, 2, 3, 5, 16, 64])
def test_table_sizes(k):
    A = random_sparse(1500, 1200, 9, mean_row=6, exp_spread=40.0)
    for sampled in (False, True):
        enc, M = encode_both(A, 256, k=k, sampled=sampled, seed=k)
        check_encode(f"k{k}", A, enc, M)
        check_spmv(A, enc, M, lanes=(0, 8))


def test_index_in_value_layout():
    A = layered3d(8, 3, contrast=10.0)
    for k in (3, 8):
        enc, M = encode_both(A, 128, k=k, sampled=True, layout=G.IDX_VALUE)
        assert enc.layout == 1
        check_encode("value", A, enc, M)
        check_spmv(A, enc, M, lanes=(0, 2))


def test_autotune_picks_lanes():
    A = powerlaw(20_000, 3)
    enc, M = encode_both(A, 512)
    x = torch.ones(A.n_cols, dtype=torch.float64, device=DEV)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    M.autotune(1, x, y, reps=3)
    assert M.A.rv_lanes in (1, 2, 4, 8, 16, 32, 64)  # long rows: no row-tile ring
    check_spmv(A, enc, M, lanes=(M.A.rv_lanes,))
    # short rows: the row-tile ring is a candidate too
    A = layered3d(12, 1)
    enc, M = encode_both(A, 256)
    assert M.A.rv_lanes == 0  # default: the row-tile ring
    x = torch.ones(A.n_cols, dtype=torch.float64, device=DEV)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    M.autotune(2, x, y, reps=3)
    check_spmv(A, enc, M, lanes=(M.A.rv_lanes,))


def test_full_size_layered_128_sampled_rows():
    """The benchmark's block workload (layered medium, 128^3, 4096-row blocks,
    drawn rows) in the launch configuration the benchmark times: every table
    and every plane against the oracle, and the SpMV on sampled rows."""
    A = layered3d(128, 0)
    R = 4096
    enc, M = encode_both(A, R, sampled=True, seed=0)
    check_encode("layered3d_128", A, enc, M)
    x = np.random.default_rng(5).uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    rows = np.random.default_rng(6).choice(A.n_rows, size=2000, replace=False).astype(np.int32)
    rows = np.concatenate([rows, [0, R - 1, R, A.n_rows - 1]]).astype(np.int32)
    for s in (1, 2, 3):
        M.spmv(s, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()[rows]
        ref = O.gse_spmv_rows(rows, A.indptr, enc, s, x)
        dec = O.decode_blocks(A.indptr, enc, s)
        scale = np.array([np.abs(dec[A.indptr[r]:A.indptr[r + 1]] *
                                 x[A.indices[A.indptr[r]:A.indptr[r + 1]]]).sum() for r in rows])
        _check_close(y, ref, scale)


# ---- one table from the pooled drawn rows (gse_encode_sampled) ----------

def encode_pooled(A, R, k=8, layout=G.IDX_AUTO, seed=1):
    sr = block_sample_rows(A.n_rows, R, seed)
    olay = {G.IDX_AUTO: -1, G.IDX_COLUMN: 0, G.IDX_VALUE: 1}[layout]
    enc = O.encode_sampled(A.indptr, A.indices, A.data, A.n_cols, num_exp=k, block_rows=R,
                           sample_rows=sr, layout=olay)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=k, idx_layout=layout, block_rows=R,
                    sample_rows=torch.from_numpy(sr).to(DEV), pooled=True)
    return enc, M


def check_pooled(name, A, enc, M, k):
    assert M.A.block_rows == 0 and M.A.block_stride == 0
    want = np.zeros(64, np.int16)
    want[:min(k, 64)] = enc.sem[:min(k, 64)]
    assert np.array_equal(np.array(list(M.A.sem), np.int16), want), name
    assert M.A.num_used == int((want > 0).sum())
    for g, w, what in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2),
                          ("col_idx", "head", "tail1", "tail2")):
        assert np.array_equal(g, w), (name, what, np.nonzero(g != w)[0][:5])
    assert M.A.exact_frac == enc.exact_frac
    for s in range(3):
        assert M.eta[s] == pytest.approx(enc.eta[s], rel=1e-12, abs=1e-300)
    assert M.A.idx_layout == (G.IDX_VALUE if enc.layout == 1 else G.IDX_COLUMN)


def check_pooled_spmv(A, enc, M):
    x = np.random.default_rng(8).uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.full((A.n_rows,), np.nan, dtype=torch.float64, device=DEV)
    for s in (1, 2, 3):
        M.spmv(s, xd, yd)
        torch.cuda.synchronize()
        ref = O.gse_spmv(A.indptr, enc, s, x)
        dec = O.decode(enc, s)
        scale = np.zeros(A.n_rows)
        np.add.at(scale, np.repeat(np.arange(A.n_rows), np.diff(A.indptr)),
                  np.abs(dec * x[A.indices]))
        _check_close(yd.cpu().numpy(), ref, scale)


@pytest.mark.parametrize("name", list(CASES))
def test_pooled_table(name):
    make, R = CASES[name]
    A = make()
    enc, M = encode_pooled(A, R)
    check_pooled(name, A, enc, M, 8)
    check_pooled_spmv(A, enc, M)


@pytest.mark.parametrize("k", [1, 2, 5, 16, 64])
def test_pooled_table_sizes(k):
    # exponents over 40 binades: the drawn rows miss much of the range
    A = random_sparse(3000, 2500, 11, mean_row=6, exp_spread=40.0)
    for R in (1, 128, 1000):
        enc, M = encode_pooled(A, R, k=k, seed=k + R)
        check_pooled(f"k{k}_R{R}", A, enc, M, k)
    check_pooled_spmv(A, enc, M)


def test_pooled_index_in_value():
    A = layered3d(8, 3, contrast=10.0)
    enc, M = encode_pooled(A, 128, k=5, layout=G.IDX_VALUE)
    assert enc.layout == 1
    check_pooled("value", A, enc, M, 5)
    check_pooled_spmv(A, enc, M)


def test_pooled_full_size_layered_128():
    """The benchmark's block workload at full size with 4096-row blocks: the
    table, every plane, exact_frac and eta against the oracle."""
    A = layered3d(128, 0)
    enc, M = encode_pooled(A, 4096, seed=0)
    check_pooled("layered3d_128", A, enc, M, 8)


def test_pooled_errors():
    A = random_sparse(600, 600, 2, mean_row=5)
    rp, ci, va = to_dev(A)
    sr = block_sample_rows(A.n_rows, 128, 0)
    sr[3] -= 128  # a row of the previous block
    with pytest.raises(G.GseError) as e:
        G.GseMatrix(rp, ci, va, A.n_cols, block_rows=128, sample_rows=torch.from_numpy(sr).to(DEV),
                    pooled=True)
    assert e.value.status == G.ERR_ARG
    # the drawn rows hold only zeros and the added maximum (exponent field
    # 10) is below the normal grid: a range error, as in the oracle
    indptr = np.array([0, 2, 4] + [4] * 127, dtype=np.int32)
    data = np.array([0.0, 0.0, 2.0 ** -1013, 2.0 ** -1014])
    T = CSR(129, 2, indptr, np.array([0, 1, 0, 1], np.int32), data, "tiny")
    sr = torch.tensor([0, 128], dtype=torch.int32, device=DEV)
    rp, ci, va = to_dev(T)
    for pooled in (False, True):
        with pytest.raises(G.GseError) as e:
            G.GseMatrix(rp, ci, va, 2, block_rows=128, sample_rows=sr, pooled=pooled)
        assert e.value.status == G.ERR_RANGE


def test_pooled_table_in_cg():
    """The pooled table is an ordinary one-table matrix: the stepped CG on it
    against the oracle's CG on the same planes."""
    A = layered3d(16, 2, contrast=3.0, layers=4)
    x_true, b = rhs_from_solution(A, 3)
    enc, M = encode_pooled(A, 256, seed=4)
    rep, x = gpu_solve(M, A, b, G.CG)
    prm = O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg")
    ref = O.cg(A.indptr, b, prm, A.indices, A.data, enc)
    assert rep.status == G.OK and ref.status == O.OK
    assert rep.relres_true <= 1e-10
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10), (rep.iters, ref.iters)


def test_pooled_table_in_the_batched_solver():
    """The batched solver takes a pooled-table matrix like any one-table
    matrix: its CG against the oracle's CG on the oracle's pooled encoding."""
    A = layered3d(14, 5, contrast=3.0, layers=4)
    _, b = rhs_from_solution(A, 6)
    enc, M = encode_pooled(A, 512, seed=2)
    p = G.gse_default_params(G.CG)
    p.max_iter = 5000
    bd = torch.from_numpy(b).to(DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    ws = torch.empty(G.gse_batch_workspace([(M.A, bd, x)], p), dtype=torch.uint8, device=DEV)
    rep, = G.gse_batch_cg([(M.A, bd, x)], p, ws)
    torch.cuda.synchronize()
    ref = O.cg(A.indptr, b, O.make_params(tol=1e-10, max_iter=5000, preset="paper_cg"),
               A.indices, A.data, enc)
    xs = x.cpu().numpy()
    assert rep.status == G.OK and ref.status == O.OK
    assert np.linalg.norm(b - A.to_scipy() @ xs) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(xs - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10), (rep.iters, ref.iters)


def gpu_solve(M, A, b, method, switch_mode=2, max_iter=5000):
    p = G.gse_default_params(method)
    p.max_iter = max_iter
    p.switch_mode = switch_mode
    ws = torch.empty(G.gse_solver_workspace(method, A.n_rows, A.nnz, p.restart, p.max_iter),
                     dtype=torch.uint8, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    fn = G.gse_cg if method == G.CG else G.gse_gmres
    rep = fn(M.A, torch.from_numpy(b).to(DEV), x, p, ws)
    torch.cuda.synchronize()
    return rep, x.cpu().numpy()


@pytest.mark.parametrize("method", [G.CG, G.GMRES], ids=["cg", "gmres"])
@pytest.mark.parametrize("sampled", [False, True], ids=["exact", "sampled"])
def test_solvers_on_block_tables(method, sampled):
    # three decades between slabs: conditioned well enough for both solvers
    # to reach 1e-10 within the caps (eight decades stall FP64 CG too)
    A = layered3d(16, 2, contrast=3.0, layers=4)
    x_true, b = rhs_from_solution(A, 3)
    enc, M = encode_both(A, 256, sampled=sampled, seed=4)
    rep, x = gpu_solve(M, A, b, method)
    preset = "paper_cg" if method == G.CG else "paper_gmres"
    prm = O.make_params(tol=1e-10, max_iter=5000, preset=preset, orth=2)
    fn = O.cg if method == G.CG else O.gmres
    ref = fn(A.indptr, b, prm, A.indices, A.data, enc)
    assert rep.status == G.OK and ref.status == O.OK
    r = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    assert rep.relres_true <= 1e-10 and r <= 1e-10
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    assert abs(rep.iters - ref.iters) <= max(3, ref.iters // 10), (rep.iters, ref.iters)
    assert rep.iters_per_seg[0] > 0  # the head-only operator ran


def test_errors():
    A = random_sparse(600, 600, 2, mean_row=5)
    rp, ci, va = to_dev(A)
    with pytest.raises(G.GseError) as e:
        G.GseMatrix(rp, ci, va, A.n_cols, block_rows=64)
    assert e.value.status == G.ERR_ARG
    sr = block_sample_rows(A.n_rows, 128, 0)
    sr[2] += 128  # a row of the next block
    with pytest.raises(G.GseError) as e:
        G.GseMatrix(rp, ci, va, A.n_cols, block_rows=128, sample_rows=torch.from_numpy(sr).to(DEV))
    assert e.value.status == G.ERR_ARG
    # the batched solver takes one table per matrix
    M = G.GseMatrix(rp, ci, va, A.n_cols, block_rows=128)
    b = torch.ones(A.n_rows, dtype=torch.float64, device=DEV)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device=DEV)
    p = G.gse_default_params(G.CG)
    with pytest.raises(G.GseError) as e:
        G.gse_batch_workspace([(M.A, b, x)], p)
    assert e.value.status == G.ERR_ARG

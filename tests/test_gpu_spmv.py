"""GPU parity: encoder planes bit-exact, SpMV within tolerance of the oracle.

Every case runs the HIP library through its C ABI (ctypes binding) and the
oracle on the same seeded inputs.  Tolerances:
  * planes, shared-exponent table, slot indices: bit-exact;
  * SpMV at every segment count: the decoded values are exact on both sides,
    only the summation order may differ, so the result must agree with the
    oracle's same-s result within 1e-12 relative (norm-wise and, scaled by
    sum |a_ij x_j|, componentwise);
  * eta_s (a sum of rounded differences): 1e-12 relative.
"""
import numpy as np
import pytest

import oracle as O
from workloads import (CSR, convdiff2d, diagonal, diffusion3d, fixed_rows, poisson2d, powerlaw,
                       random_sparse, rhs_from_solution)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - collected on the CPU machine too
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


def to_dev(A: CSR):
    return (torch.from_numpy(A.indptr).to(DEV), torch.from_numpy(A.indices).to(DEV),
            torch.from_numpy(A.data).to(DEV))


def cases():
    return {
        "poisson2d_64": lambda: poisson2d(64),
        "diffusion3d_24": lambda: diffusion3d(24, 0),
        "convdiff2d_64": lambda: convdiff2d(64, 1),
        "powerlaw_20k": lambda: powerlaw(20_000, 2),
        "random_empty_long": lambda: random_sparse(3000, 2500, 5, mean_row=4, empty_frac=0.2,
                                                   long_rows=6, long_len=2400, exp_spread=60),
        "random_ragged": lambda: random_sparse(1777, 1901, 6, mean_row=9, exp_spread=20),
        "one_row_long": lambda: random_sparse(1, 9000, 7, mean_row=1, long_rows=1, long_len=8999),
        "tiny": lambda: random_sparse(3, 3, 8, mean_row=2),
        # tiles spanning more rows than the ring stages row pointers for
        "diagonal_3000": lambda: diagonal(3000, 10),
        "sparse_many_empty": lambda: random_sparse(6000, 6000, 9, mean_row=0.6, exp_spread=12),
        # non-zeros an exact multiple of the tile: the look-ahead past the end
        "fixed_rows_512x8": lambda: fixed_rows(512, 700, 8, 11),
        # every row exactly as long as the row-tile batch (the fullest staged
        # window for B = 3, 5, 7) and a last tile of fewer than 192 rows
        "fixed_rows_1000x3": lambda: fixed_rows(1000, 1200, 3, 12),
        "fixed_rows_777x5": lambda: fixed_rows(777, 800, 5, 13),
        "fixed_rows_1111x7": lambda: fixed_rows(1111, 1500, 7, 14),
        "fixed_rows_500x6": lambda: fixed_rows(500, 640, 6, 15),
        # ragged short rows with many empty ones and a wide exponent spread, on
        # either side of the row-tile ring's limit (longest row 7 and 9)
        "random_rows_max7": lambda: random_sparse(2023, 2100, 23, mean_row=1.5, empty_frac=0.3,
                                                  exp_spread=30),
        "random_rows_max9": lambda: random_sparse(2021, 2100, 21, mean_row=2, empty_frac=0.2,
                                                  exp_spread=30),
    }


@pytest.fixture(scope="module", params=list(cases()))
def case(request):
    A = cases()[request.param]()
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    return request.param, A, enc, M


def test_encode_bit_exact(case):
    name, A, enc, M = case
    assert M.sem == [int(s) for s in enc.sem], name
    for got, want, what in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2),
                               ("col_idx", "head", "tail1", "tail2")):
        assert np.array_equal(got, want), (name, what, np.nonzero(got != want)[0][:5])
    assert M.A.exact_frac == enc.exact_frac
    for s in range(3):
        assert M.eta[s] == pytest.approx(enc.eta[s], rel=1e-12, abs=1e-300)


def _check_close(got, ref, scale, tol=1e-12):
    assert np.all(np.abs(got - ref) <= tol * scale + 1e-300)
    nr = np.linalg.norm(ref)
    if nr > 0:
        assert np.linalg.norm(got - ref) <= tol * nr + 1e-300


SCHEDULES = [(1024, 0), (2048, 0), (4096, 0), (2048, 1), (2048, 2), (2048, 8), (2048, 64)]


@pytest.mark.parametrize("sched", SCHEDULES, ids=[f"t{t}_rv{r}" for t, r in SCHEDULES])
def test_spmv_all_segments(case, sched):
    name, A, enc, M = case
    tile, rv = sched
    M.plan(tile, rv)
    assert M.A.rv_lanes == rv and M.A.tile_nnz == tile
    rng = np.random.default_rng(tile + rv)
    x = rng.uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.full((A.n_rows,), np.nan, dtype=torch.float64, device=DEV)
    for s in (1, 2, 3):
        M.spmv(s, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        ref = O.gse_spmv(A.indptr, enc, s, x)
        dec = O.decode(enc, s)
        scale = np.zeros(A.n_rows)
        np.add.at(scale, np.repeat(np.arange(A.n_rows), np.diff(A.indptr)),
                  np.abs(dec * x[A.indices]))
        _check_close(y, ref, scale)
    M.plan()


@pytest.mark.parametrize("sched", [(1024, 0), (4096, 0), (2048, 4), (2048, 16)])
def test_csr64_spmv(case, sched):
    name, A, enc, M = case
    rp, ci, va = to_dev(A)
    C64 = G.CsrMatrix(rp, ci, va, A.n_cols, tile_nnz=sched[0], rv_lanes=sched[1])
    x = np.random.default_rng(3).uniform(-1, 1, A.n_cols)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    C64.spmv(torch.from_numpy(x).to(DEV), yd)
    torch.cuda.synchronize()
    ref = O.csr_spmv(A.indptr, A.indices, A.data, x)
    scale = np.zeros(A.n_rows)
    np.add.at(scale, np.repeat(np.arange(A.n_rows), np.diff(A.indptr)),
              np.abs(A.data * x[A.indices]))
    _check_close(yd.cpu().numpy(), ref, scale)


def test_spmv_deterministic_and_x_ones(case):
    """Two launches give identical bits; with x = 1 (Section IV-A protocol)
    the row sums of the decoded matrix."""
    name, A, enc, M = case
    xd = torch.ones(A.n_cols, dtype=torch.float64, device=DEV)
    y1 = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    y2 = torch.empty_like(y1)
    M.spmv(1, xd, y1)
    M.spmv(1, xd, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    ref = O.gse_spmv(A.indptr, enc, 1, np.ones(A.n_cols))
    assert np.allclose(y1.cpu().numpy(), ref, rtol=1e-12, atol=1e-300)


def test_reused_table_and_errors():
    A = diffusion3d(10, 3)
    rp, ci, va = to_dev(A)
    M1 = G.GseMatrix(rp, ci, va, A.n_cols)
    B = diffusion3d(10, 4)  # same recipe, other draw: reuse the first table
    rpb, cib, vab = to_dev(B)
    sem = [s for s in M1.sem if s]
    M2 = G.GseMatrix(rpb, cib, vab, B.n_cols, num_exp=len(sem), sem_in=sem)
    enc = O.encode(B.indptr, B.indices, B.data, B.n_cols, num_exp=len(sem),
                   sem_in=np.array(sem, np.int16))
    assert M2.sem[: len(sem)] == sem
    for got, want in zip(M2.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2)):
        assert np.array_equal(got, want)
    # non-finite value
    bad = va.clone()
    bad[5] = float("nan")
    with pytest.raises(G.GseError) as ei:
        G.GseMatrix(rp, ci, bad, A.n_cols)
    assert ei.value.status == G.ERR_NONFINITE
    # a reused table that does not cover a value
    big = va.clone()
    big[7] = 1e30
    with pytest.raises(G.GseError) as ei:
        G.GseMatrix(rp, ci, big, A.n_cols, num_exp=len(sem), sem_in=sem)
    assert ei.value.status == G.ERR_RANGE
    # bad segment count
    x = torch.ones(A.n_cols, dtype=torch.float64, device=DEV)
    y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    with pytest.raises(G.GseError) as ei:
        M1.spmv(4, x, y)
    assert ei.value.status == G.ERR_ARG


def test_empty_matrix():
    A = CSR(5, 5, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0), "empty")
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, 5)
    x = torch.ones(5, dtype=torch.float64, device=DEV)
    y = torch.full((5,), 7.0, dtype=torch.float64, device=DEV)
    M.spmv(2, x, y)
    torch.cuda.synchronize()
    assert torch.equal(y, torch.zeros_like(y))


def test_default_schedule_choice():
    """The default is the tile schedule with 1024 non-zeros per tile."""
    for A in (diffusion3d(16, 0), poisson2d(32), powerlaw(20_000, 2)):
        rp, ci, va = to_dev(A)
        M = G.GseMatrix(rp, ci, va, A.n_cols)
        assert M.A.rv_lanes == 0 and M.A.tile_nnz == 1024, A.name
        assert M.A.max_row_nnz == int(np.diff(A.indptr).max())


def test_full_size_diffusion3d_128_sampled():
    """The 128^3 operator at full size, in the launch configuration the
    benchmark times (default schedule): the whole planes bit-exact, sampled
    rows of y against the oracle row by row."""
    A = diffusion3d(128, 0)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols)
    assert M.A.rv_lanes == 0
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
    assert M.sem == [int(s) for s in enc.sem]
    for got, want in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2)):
        assert np.array_equal(got, want)
    x, _ = rhs_from_solution(A, 5)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    rows = np.unique(np.concatenate([np.random.default_rng(1).integers(0, A.n_rows, 20000),
                                     [0, 1, A.n_rows - 1]])).astype(np.int32)
    for s in (1, 2, 3):
        M.spmv(s, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()[rows]
        ref = O.gse_spmv_rows(rows, A.indptr, enc, s, x)
        assert np.allclose(y, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_autotune_picks_a_candidate_and_stays_exact():
    for A in (diffusion3d(24, 1), powerlaw(20_000, 3)):
        rp, ci, va = to_dev(A)
        M = G.GseMatrix(rp, ci, va, A.n_cols)
        enc = O.encode(A.indptr, A.indices, A.data, A.n_cols)
        x = np.random.default_rng(0).uniform(-1, 1, A.n_cols)
        xd = torch.from_numpy(x).to(DEV)
        yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
        for s in (1, 3):
            M.autotune(s, xd, yd, reps=3)
            assert (M.A.tile_nnz, M.A.rv_lanes) in {(1024, 0), (2048, 0), (4096, 0)} | {
                (1024, L) for L in (1, 2, 4, 8, 16, 32, 64)}
            first = (M.A.tile_nnz, M.A.rv_lanes)
            M.autotune(s, xd, yd, reps=3)  # cached: same choice
            assert (M.A.tile_nnz, M.A.rv_lanes) == first
            M.spmv(s, xd, yd)
            torch.cuda.synchronize()
            ref = O.gse_spmv(A.indptr, enc, s, x)
            assert np.allclose(yd.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        C64 = G.CsrMatrix(rp, ci, va, A.n_cols)
        C64.autotune(xd, yd, reps=3)
        C64.spmv(xd, yd)
        torch.cuda.synchronize()
        ref = O.csr_spmv(A.indptr, A.indices, A.data, x)
        assert np.allclose(yd.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def row_mix_matrix(lengths, seed):
    """CSR with the given row lengths, distinct random columns in [0, n) and
    N(0,1) values."""
    rng = np.random.default_rng(seed)
    n = len(lengths)
    indptr = np.zeros(n + 1, dtype=np.int32)
    indptr[1:] = np.cumsum(lengths)
    cols = [np.sort(rng.choice(n, size=int(k), replace=False)) for k in lengths]
    indices = np.concatenate(cols).astype(np.int32)
    data = rng.standard_normal(indptr[-1])
    return CSR(n, n, indptr, indices, data, "row_mix")


def test_autotune_cache_keys_carry_the_row_length_signature(tmp_path, monkeypatch):
    """Two matrices of the same size, non-zero count and longest row but a
    different mix of row lengths (all rows of 4, against half of 2 and half
    of 6) are tuned separately: the cache file gets two keys that differ in
    the row-length classes, and a second call on the first matrix is served
    from the cache (no new key)."""
    n = 8192
    a = np.full(n, 4)
    b = np.where(np.arange(n) % 2 == 0, 2, 6)
    for L in (a, b):  # one row of 8 and one empty row, the rest as given
        L[0], L[1] = 8, 0
    assert a.sum() == b.sum() and a.max() == b.max() == 8
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GSE_AUTOTUNE_CACHE", str(path))
    keys = []
    for L, seed in ((a, 0), (b, 1), (a, 0)):
        A = row_mix_matrix(L, seed)
        rp, ci, va = to_dev(A)
        C64 = G.CsrMatrix(rp, ci, va, A.n_cols)
        x = torch.ones(A.n_cols, dtype=torch.float64, device=DEV)
        y = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
        C64.autotune(x, y, reps=2)
        C64.spmv(x, y)
        torch.cuda.synchronize()
        ref = O.csr_spmv(A.indptr, A.indices, A.data, np.ones(A.n_cols))
        assert np.allclose(y.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        keys = [line.split()[0] for line in path.read_text().splitlines()]
    assert len(keys) == 2 and keys[0] != keys[1], keys
    # classes under half a per mille (the empty row, the row of 8) are left out
    assert "_r3.1000" in keys[0] and "_r2.500-3.500" in keys[1], keys


@pytest.mark.parametrize("num_exp", [1, 3, 5])
@pytest.mark.parametrize("name", ["diffusion3d_24", "powerlaw_20k", "random_ragged",
                                  "convdiff2d_64"])
def test_computed_tables_of_fewer_exponents(name, num_exp):
    """Tables of k = 1, 3, 5 shared exponents computed on the device (the k
    most frequent, the maximum forced into the last slot): table, planes and
    eta equal the oracle's, and SpMV at every segment count agrees."""
    A = cases()[name]()
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=num_exp)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=num_exp)
    assert M.sem == [int(s) for s in enc.sem] and M.A.num_used <= num_exp
    for got, want in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2)):
        assert np.array_equal(got, want), (name, num_exp)
    assert M.A.exact_frac == enc.exact_frac
    for s in range(3):
        assert M.eta[s] == pytest.approx(enc.eta[s], rel=1e-12, abs=1e-300)
    x = np.random.default_rng(num_exp).uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    for s in (1, 2, 3):
        M.spmv(s, xd, yd)
        torch.cuda.synchronize()
        ref = O.gse_spmv(A.indptr, enc, s, x)
        dec = O.decode(enc, s)
        scale = np.zeros(A.n_rows)
        np.add.at(scale, np.repeat(np.arange(A.n_rows), np.diff(A.indptr)),
                  np.abs(dec * x[A.indices]))
        _check_close(yd.cpu().numpy(), ref, scale)


@pytest.mark.parametrize("k", [2, 4, 16, 32, 64])
@pytest.mark.parametrize("name", ["powerlaw_20k", "random_empty_long", "diffusion3d_24"])
def test_index_width_follows_the_table_size(name, k):
    """k shared exponents put a ceil(log2 k)-bit slot index in the column word
    (Section III-B.1, III-C.1; the k sweep of Section IV-B): table, planes,
    eta bit-exact against the oracle and SpMV at every segment count on the
    default schedule, the general tiles and the row-vector schedule."""
    A = cases()[name]()
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=k)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=k)
    assert M.A.idx_bits == enc.idx_bits == O.index_bits(k)
    assert M.sem == [int(s) for s in enc.sem]
    for got, want in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2)):
        assert np.array_equal(got, want), (name, k)
    for s in range(3):
        assert M.eta[s] == pytest.approx(enc.eta[s], rel=1e-12, abs=1e-300)
    x = np.random.default_rng(k).uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    dec = {s: O.decode(enc, s) for s in (1, 2, 3)}
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    for sched in ((1024, -1), (2048, 0), (2048, 8)):
        M.plan(*sched)
        for s in (1, 2, 3):
            M.spmv(s, xd, yd)
            torch.cuda.synchronize()
            ref = O.gse_spmv(A.indptr, enc, s, x)
            scale = np.zeros(A.n_rows)
            np.add.at(scale, rows, np.abs(dec[s] * x[A.indices]))
            _check_close(yd.cpu().numpy(), ref, scale)


@pytest.mark.parametrize("k", [2, 8, 16, 64])
@pytest.mark.parametrize("name", ["powerlaw_20k", "random_empty_long", "diffusion3d_24"])
def test_index_in_value_layout(name, k):
    """The slot index in the value word (Algorithm 1's EI_bit, the fallback
    of Section III-C.1): planes bit-exact against the oracle's layout 1, and
    SpMV at every segment count (W_s = 15 - b, 31 - b, 63 - b) on the default
    schedule, the general tiles and the row-vector schedule."""
    A = cases()[name]()
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=k, layout=1)
    rp, ci, va = to_dev(A)
    M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=k, idx_layout=G.IDX_VALUE)
    assert M.A.idx_layout == G.IDX_VALUE and enc.layout == 1
    assert M.sem == [int(s) for s in enc.sem]
    for got, want in zip(M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2)):
        assert np.array_equal(got, want), (name, k)
    for s in range(3):
        assert M.eta[s] == pytest.approx(enc.eta[s], rel=1e-12, abs=1e-300)
    x = np.random.default_rng(k + 1).uniform(-1, 1, A.n_cols)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.empty(A.n_rows, dtype=torch.float64, device=DEV)
    dec = {s: O.decode(enc, s) for s in (1, 2, 3)}
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    for sched in ((1024, -1), (2048, 0), (2048, 8)):
        M.plan(*sched)
        for s in (1, 2, 3):
            M.spmv(s, xd, yd)
            torch.cuda.synchronize()
            ref = O.gse_spmv(A.indptr, enc, s, x)
            scale = np.zeros(A.n_rows)
            np.add.at(scale, rows, np.abs(dec[s] * x[A.indices]))
            _check_close(yd.cpu().numpy(), ref, scale)


def test_wide_matrix_moves_the_index_into_the_value():
    """k = 64 leaves 26 column bits (67,108,864 columns); a matrix with more
    columns is encoded with the index in the value by default, and its SpMV
    (x of 537 MB) matches the oracle on every row."""
    import scipy.sparse as sp
    n_cols = (1 << 26) + 12345
    rng = np.random.default_rng(26)
    n_rows, per = 3000, 7
    cols = np.sort(rng.choice(n_cols, size=(n_rows, per), replace=True), axis=1)
    cols[:, -1] = n_cols - 1 - rng.integers(0, 100, n_rows)  # the far end of x
    cols = np.sort(cols, axis=1)
    vals = rng.standard_normal((n_rows, per)) * np.exp2(rng.integers(-30, 30, (n_rows, per)))
    M = sp.csr_matrix((vals.ravel(), cols.ravel(), np.arange(0, n_rows * per + 1, per)),
                      shape=(n_rows, n_cols))
    M.sum_duplicates()
    A = CSR.from_scipy(M)
    enc = O.encode(A.indptr, A.indices, A.data, A.n_cols, num_exp=64)
    assert enc.layout == 1
    rp, ci, va = to_dev(A)
    G_M = G.GseMatrix(rp, ci, va, A.n_cols, num_exp=64)
    assert G_M.A.idx_layout == G.IDX_VALUE
    for got, want in zip(G_M.planes(), (enc.col_idx, enc.head, enc.tail1, enc.tail2)):
        assert np.array_equal(got, want)
    x = torch.linspace(-1.0, 1.0, n_cols, dtype=torch.float64, device=DEV)
    y = torch.empty(n_rows, dtype=torch.float64, device=DEV)
    xh = x.cpu().numpy()
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.indptr))
    for s in (1, 3):
        G_M.spmv(s, x, y)
        torch.cuda.synchronize()
        ref = O.gse_spmv(A.indptr, enc, s, xh)
        scale = np.zeros(A.n_rows)  # rows sum values over 60 binades: cancellation
        np.add.at(scale, rows, np.abs(O.decode(enc, s) * xh[A.indices]))
        _check_close(y.cpu().numpy(), ref, scale)

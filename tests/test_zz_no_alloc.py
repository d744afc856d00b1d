"""gse_encode_static (scratch in a static device array, no allocation) against
gse_encode (caller workspace): identical planes, table, eta, coverage and
plan, on two calls in a row, the second with a smaller matrix, so that the
second call runs on the scratch record the first one left behind."""
import numpy as np
import pytest

from workloads import diffusion3d, powerlaw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2411_04686_amd import gse as G  # noqa: E402

DEV = torch.device("cuda:0")


def _static_encoded(rp, ci, va, n_cols, num_exp=8, sem_in=None):
    """Planes and record of gse_encode_static on caller-owned planes."""
    n_rows = rp.numel() - 1
    nnz = va.numel()
    pad = G.gse_pad(nnz)
    bufs = dict(col_idx=torch.empty(max(pad, 1), dtype=torch.int32, device=DEV),
                head=torch.empty(max(pad, 1), dtype=torch.int16, device=DEV),
                tail1=torch.empty(max(pad, 1), dtype=torch.int16, device=DEV),
                tail2=torch.empty(max(pad, 1), dtype=torch.int32, device=DEV))
    cap = G.gse_tile_entries(nnz)
    tile_row = torch.empty(cap, dtype=torch.int32, device=DEV)
    A = G.gse_matrix()
    A.col_idx = bufs["col_idx"].data_ptr()
    A.head = bufs["head"].data_ptr()
    A.tail1 = bufs["tail1"].data_ptr()
    A.tail2 = bufs["tail2"].data_ptr()
    A.tile_row = tile_row.data_ptr()
    A.tile_cap = cap
    G.gse_encode_static(rp, ci, va, n_rows, n_cols, nnz, num_exp, sem_in, A)
    torch.cuda.synchronize()
    planes = tuple(bufs[k][:nnz].cpu().numpy().view(dt) for k, dt in
                   (("col_idx", "uint32"), ("head", "uint16"), ("tail1", "uint16"),
                    ("tail2", "uint32")))
    return A, planes, tile_row.cpu().numpy()


def _compare(A_csr, num_exp=8, sem_in=None):
    rp = torch.from_numpy(A_csr.indptr).to(DEV)
    ci = torch.from_numpy(A_csr.indices).to(DEV)
    va = torch.from_numpy(A_csr.data).to(DEV)
    S, planes, tiles = _static_encoded(rp, ci, va, A_csr.n_cols, num_exp, sem_in)
    W = G.GseMatrix(rp, ci, va, A_csr.n_cols, num_exp=num_exp, sem_in=sem_in)
    torch.cuda.synchronize()
    for got, want in zip(planes, W.planes()):
        assert np.array_equal(got, want)
    assert list(S.sem) == list(W.A.sem) and S.num_used == W.A.num_used
    assert list(S.eta) == list(W.A.eta) and S.exact_frac == W.A.exact_frac
    assert (S.n_tiles, S.tile_nnz, S.rv_lanes, S.max_row_nnz) == \
        (W.A.n_tiles, W.A.tile_nnz, W.A.rv_lanes, W.A.max_row_nnz)
    nt = S.n_tiles + 1
    assert np.array_equal(tiles[:nt], W.tile_row[:nt].cpu().numpy())
    return S


def test_static_scratch_size_is_stated():
    assert G.gse_encode_static_scratch_bytes() == 16384
    assert G.gse_encode_workspace(1 << 20, 1 << 10) <= 16384


def test_static_encode_matches_workspace_encode_twice_shrinking():
    # first call: a power-law matrix (many exponents, eta > 0, long rows)
    S1 = _compare(powerlaw(60000, 1))
    assert S1.eta[0] > 0.0
    # second call, smaller: the record left by the first must not leak in
    S2 = _compare(diffusion3d(10, 2))
    assert S2.nnz < S1.nnz and S2.eta[0] > 0.0
    # a reused table and k = 3 on the same scratch
    A = diffusion3d(6, 3)
    S3 = _compare(A, num_exp=3)
    _compare(A, num_exp=3, sem_in=[int(v) for v in list(S3.sem)[:3]])

"""The C ABI without a GPU: the library loads, exports every entry point that
include/gse.h declares, and rejects bad arguments on the host before any
launch (no compute call needs a device here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gse.h")
LIB = os.path.join(ROOT, "paper_2411_04686_amd", "libgse.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(gse_[a-z_0-9]+)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libgse.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("gse_encode", "gse_spmv", "gse_cg", "gse_gmres", "gse_plan", "gse_csr_spmv",
                 "gse_solver_workspace", "gse_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    import importlib
    import sys
    sys.path.insert(0, ROOT)
    g = importlib.import_module("paper_2411_04686_amd.gse")
    assert set(declared()) <= set(g.exported_symbols())


def test_host_side_helpers(lib):
    lib.gse_pad.restype = C.c_int64
    lib.gse_pad.argtypes = [C.c_int64]
    assert [lib.gse_pad(n) for n in (0, 1, 16, 17)] == [0, 16, 16, 32]
    lib.gse_tile_entries.restype = C.c_int32
    lib.gse_tile_entries.argtypes = [C.c_int64]
    assert lib.gse_tile_entries(0) == 3 and lib.gse_tile_entries(1025) == 4
    lib.gse_status_str.restype = C.c_char_p
    assert lib.gse_status_str(0) == b"ok" and lib.gse_status_str(-5) == b"breakdown"
    ws = C.c_size_t()
    assert lib.gse_encode_workspace(C.c_int64(1000), 10, C.byref(ws)) == 0 and ws.value > 8192
    assert lib.gse_solver_workspace(0, 100, C.c_int64(500), 30, 100, C.byref(ws)) == 0
    cg_bytes = ws.value
    assert lib.gse_solver_workspace(1, 100, C.c_int64(500), 30, 100, C.byref(ws)) == 0
    assert ws.value > cg_bytes  # GMRES adds the Krylov basis
    assert lib.gse_solver_workspace(1, 100, C.c_int64(500), 0, 100, C.byref(ws)) == -1


def test_default_params_are_the_paper_presets(lib):
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_04686_amd.gse import gse_params
    p = gse_params()
    assert lib.gse_default_params(0, C.byref(p)) == 0
    assert (p.l, p.t, p.m, p.ndec_limit) == (3000, 250, 500, 130)
    assert (p.rsd_limit, p.reldec_limit, p.max_iter) == (0.5, 0.45, 5000)
    assert lib.gse_default_params(1, C.byref(p)) == 0
    assert (p.l, p.t, p.m, p.ndec_limit, p.restart) == (9000, 300, 1500, 80, 30)
    assert (p.rsd_limit, p.reldec_limit, p.max_iter) == (0.03, 0.08, 15000)
    assert p.tol == 1e-10
    assert lib.gse_default_params(7, C.byref(p)) == -1


def test_argument_errors_without_launch(lib):
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_04686_amd.gse import gse_matrix
    lib.gse_last_error.restype = C.c_char_p
    assert lib.gse_spmv(None, 1, None, None, None) == -1
    A = gse_matrix()
    # planes not set
    assert lib.gse_encode(C.c_void_p(16), None, None, 0, 0, C.c_int64(0), 8, None, C.byref(A),
                          None, C.c_size_t(0), None) == -1
    # num_exp out of range
    assert lib.gse_encode(C.c_void_p(16), None, None, 0, 0, C.c_int64(0), 65, None, C.byref(A),
                          None, C.c_size_t(0), None) == -1
    # too many columns for a 29-bit column field when the index must stay there
    A.idx_layout = 1  # GSE_IDX_COLUMN
    assert lib.gse_encode(C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 1, 2**29 + 1,
                          C.c_int64(1), 8, None, C.byref(A), None, C.c_size_t(0), None) == -3
    assert b"2^29" in lib.gse_last_error()
    # by default such a matrix keeps the index in the value: no range error
    # (it fails only later, on the planes this test never set)
    A.idx_layout = 0  # GSE_IDX_AUTO
    assert lib.gse_encode(C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 1, 2**29 + 1,
                          C.c_int64(1), 8, None, C.byref(A), None, C.c_size_t(0), None) == -1
    # schedule missing -> spmv refuses
    A.row_ptr = A.col_idx = A.head = A.tail1 = A.tail2 = A.tile_row = 256
    assert lib.gse_spmv(C.byref(A), 1, C.c_void_p(256), C.c_void_p(256), None) == -1
    # copy needs 16-byte multiples
    assert lib.gse_stream_copy(C.c_void_p(16), C.c_void_p(32), C.c_size_t(17), None) == -1


def test_column_limit_follows_the_index_width(lib):
    """k = 64 leaves 26 column bits: with the index forced into the column
    word a wider matrix is refused on the host before any device work (the
    device pointers are never touched)."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_04686_amd import gse as G
    L = G.lib()
    A = G.gse_matrix()
    fake = C.c_void_p(256)
    A.idx_layout = 1  # the index forced into the column word
    for k, n_cols, want in ((64, (1 << 26) + 1, -3), (16, (1 << 28) + 1, -3), (0, 10, -1),
                            (65, 10, -1)):
        st = L.gse_encode(fake, fake, fake, 1, n_cols, 1, k, None, C.byref(A), fake, 1 << 20,
                          None)
        assert st == want, (k, n_cols, st)


def test_block_tables_host_side(lib):
    """Per-row-block tables: the size query and the host checks of
    gse_encode_blocks (refused before any device work)."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_04686_amd import gse as G
    L = G.lib()
    assert G.gse_block_table_entries(1000, 128, 8) == 8 * 8
    assert G.gse_block_table_entries(1024, 128, 5) == 8 * 8
    assert G.gse_block_table_entries(1025, 128, 64) == 9 * 64
    assert G.gse_block_table_entries(300, 128, 1) == 3
    assert G.gse_block_table_entries(0, 128, 8) == 0
    assert G.gse_block_table_entries(10, 0, 8) == 0 and G.gse_block_table_entries(10, 128, 65) == 0
    fake = C.c_void_p(256)
    A = G.gse_matrix()
    A.col_idx = A.head = A.tail1 = A.tail2 = A.tile_row = 256
    A.tile_cap = 1 << 20
    # blocks below the minimum, then a NULL table buffer: argument errors
    st = L.gse_encode_blocks(fake, fake, fake, 1000, 1000, 5000, 8, 64, None, C.byref(A), fake,
                             1 << 20, None)
    assert st == -1 and b"block_rows" in L.gse_last_error()
    st = L.gse_encode_blocks(fake, fake, fake, 1000, 1000, 5000, 8, 128, None, C.byref(A), fake,
                             1 << 20, None)
    assert st == -1 and b"block_sem" in L.gse_last_error()
    # a matrix that claims block tables it does not have is refused
    A.num_exp, A.idx_bits, A.idx_layout = 8, 3, 1
    A.row_ptr = 256
    A.tile_nnz, A.n_tiles, A.nnz = 1024, 1, 10
    A.block_rows, A.block_stride = 128, 8
    assert L.gse_spmv(C.byref(A), 1, fake, fake, None) == -1
    assert b"per-block" in L.gse_last_error()


def test_pooled_sample_host_side(lib):
    """gse_encode_sampled refuses a block size below one and a missing list of
    drawn rows before any device work."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_04686_amd import gse as G
    L = G.lib()
    fake = C.c_void_p(256)
    A = G.gse_matrix()
    A.col_idx = A.head = A.tail1 = A.tail2 = A.tile_row = 256
    A.tile_cap = 1 << 20
    st = L.gse_encode_sampled(fake, fake, fake, 1000, 1000, 5000, 8, 0, fake, C.byref(A), fake,
                              1 << 20, None)
    assert st == -1 and b"block_rows" in L.gse_last_error()
    st = L.gse_encode_sampled(fake, fake, fake, 1000, 1000, 5000, 8, 256, None, C.byref(A), fake,
                              1 << 20, None)
    assert st == -1 and b"sample_rows" in L.gse_last_error()


def test_spmv_refuses_overlapping_vectors(lib):
    """x and y of one product may not share memory: refused on the host."""
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_04686_amd import gse as G
    L = G.lib()
    A = G.gse_matrix()
    A.n_rows = A.n_cols = 100
    A.nnz = 500
    A.num_exp, A.idx_bits, A.idx_layout = 8, 3, 1
    A.row_ptr = A.col_idx = A.head = A.tail1 = A.tail2 = A.tile_row = 256
    A.tile_cap, A.tile_nnz, A.n_tiles = 8, 1024, 1
    base = 1 << 20
    # x spans 800 bytes, y 800: any shared byte is refused
    for x, y in ((base, base + 400), (base + 400, base), (base, base + 799), (base, base)):
        st = L.gse_spmv(C.byref(A), 1, C.c_void_p(x), C.c_void_p(y), None)
        assert st == -1 and b"overlap" in L.gse_last_error(), (x, y)

"""ctypes front-end of the CPU oracle (TEST INFRASTRUCTURE).

The oracle is the plain, sequential FP64 definition of what the GPU library
computes: the group-shared-exponent encoder and decoder (Section III-B,
Algorithm 1), the segment SpMV operators (Algorithm 2 and its two wider
variants), the stepped controller (Section III-D, Eqs. 3-6, Conditions 1-3)
and CG / GMRES(m).  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never imports, links or calls it.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

from . import build as _build

_LIB = None

OK, NOT_CONVERGED = 0, 2
ERR_ARG, ERR_NONFINITE, ERR_RANGE, ERR_BREAKDOWN = -1, -2, -3, -5
TRIG_NAMES = {0: "none", 1: "C1", 2: "C2", 3: "C3", 4: "floor", 5: "tol", 6: "breakdown"}


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("max_restarts", C.c_int32), ("start_segments", C.c_int32),
                ("fixed_segments", C.c_int32), ("l", C.c_int32), ("t", C.c_int32),
                ("m", C.c_int32), ("rsd_limit", C.c_double), ("ndec_limit", C.c_int32),
                ("reldec_limit", C.c_double), ("ndec_rule", C.c_int32),
                ("floor_c", C.c_double), ("switch_mode", C.c_int32), ("orth", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32),
                ("iters_per_seg", C.c_int32 * 3), ("switch_iter", C.c_int32 * 2),
                ("switch_trigger", C.c_int32 * 2), ("relres_recursive", C.c_double),
                ("relres_true", C.c_double)]


class Matrix(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("col_idx", C.c_void_p), ("head", C.c_void_p),
                ("tail1", C.c_void_p), ("tail2", C.c_void_p), ("sem64", C.c_void_p),
                ("eta3", C.c_void_p), ("idx_bits", C.c_int32), ("layout", C.c_int32),
                ("lp_val", C.c_void_p), ("lp_fmt", C.c_int32), ("block_sem", C.c_void_p),
                ("block_rows", C.c_int32)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        L.or_index_bits.restype = C.c_int
        L.or_index_bits.argtypes = [C.c_int]
        L.or_exponent_histogram.restype = C.c_int64
        L.or_exponent_histogram.argtypes = [P, C.c_int64, P]
        L.or_select_shared_exponents.restype = C.c_int
        L.or_select_shared_exponents.argtypes = [P, C.c_int, P]
        L.or_encode_values.restype = C.c_int
        L.or_encode_values.argtypes = [P, P, C.c_int64, P, C.c_int, C.c_int, P, P, P, P]
        L.or_encode.restype = C.c_int
        L.or_encode.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int64, C.c_int, C.c_int, P,
                                P, P, P, P, P, P, P, P]
        L.or_decode_one.restype = C.c_double
        L.or_decode_one.argtypes = [C.c_uint32, C.c_uint16, C.c_uint16, C.c_uint32, P, C.c_int,
                                    C.c_int, C.c_int]
        L.or_encode_blocks.restype = C.c_int
        L.or_encode_blocks.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int64, C.c_int, C.c_int,
                                       C.c_int32, P, P, P, P, P, P, P, P, P]
        L.or_encode_sampled.restype = C.c_int
        L.or_encode_sampled.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int64, C.c_int, C.c_int,
                                        C.c_int32, P, P, P, P, P, P, P, P, P]
        L.or_gse_spmv_blocks.restype = None
        L.or_gse_spmv_blocks.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int32, C.c_int, C.c_int,
                                         C.c_int, P, P]
        L.or_decode.restype = None
        L.or_decode.argtypes = [P, P, P, P, C.c_int64, P, C.c_int, C.c_int, C.c_int, P]
        L.or_lp_round.restype = C.c_uint16
        L.or_lp_round.argtypes = [C.c_double, C.c_int, P]
        L.or_lp_widen.restype = C.c_double
        L.or_lp_widen.argtypes = [C.c_uint16, C.c_int]
        L.or_lp_convert.restype = C.c_int64
        L.or_lp_convert.argtypes = [P, C.c_int64, C.c_int, P]
        L.or_lp_spmv.restype = None
        L.or_lp_spmv.argtypes = [C.c_int32, P, P, P, C.c_int, P, P]
        L.or_csr_spmv.restype = None
        L.or_csr_spmv.argtypes = [C.c_int32, P, P, P, P, P]
        L.or_gse_spmv.restype = None
        L.or_gse_spmv.argtypes = [C.c_int32, P, P, P, P, P, P, C.c_int, C.c_int, C.c_int, P, P]
        L.or_gse_spmv_rows.restype = None
        L.or_gse_spmv_rows.argtypes = [P, C.c_int32, P, P, P, P, P, P, C.c_int, C.c_int, C.c_int,
                                       P, P]
        L.or_window_metrics.restype = None
        L.or_window_metrics.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.or_precision_trigger.restype = C.c_int
        L.or_precision_trigger.argtypes = [P, C.c_int32, C.POINTER(Params)]
        L.or_cg.restype = C.c_int
        L.or_cg.argtypes = [C.POINTER(Matrix), P, P, C.POINTER(Params), C.POINTER(Report), P, P]
        L.or_gmres.restype = C.c_int
        L.or_gmres.argtypes = [C.POINTER(Matrix), P, P, C.POINTER(Params), C.POINTER(Report), P, P]
        _LIB = L
    return _LIB


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


# ---------------------------------------------------------------- format ---
def exponent_histogram(val):
    val = _c(val, np.float64)
    hist = np.zeros(2048, dtype=np.uint32)
    nonfinite = lib().or_exponent_histogram(_p(val), val.size, _p(hist))
    return hist, int(nonfinite)


MAX_EXP = 64


def index_bits(num_exp: int) -> int:
    """Slot-index width for a table of num_exp shared exponents."""
    return lib().or_index_bits(num_exp)


def _table(sem):
    """A shared-exponent table padded to the oracle's 64 entries."""
    t = np.zeros(MAX_EXP, np.int16)
    a = np.asarray(sem, dtype=np.int16).ravel()
    t[:a.size] = a
    return t


def select_shared_exponents(hist, num_exp: int = 8):
    """The table (first num_exp of 64 entries returned, at least 8)."""
    hist = _c(hist, np.uint32)
    sem = np.zeros(MAX_EXP, dtype=np.int16)
    rc = lib().or_select_shared_exponents(_p(hist), num_exp, _p(sem))
    if rc < 0:
        raise OracleError(rc, "select_shared_exponents")
    return sem[:max(8, num_exp)].copy()


@dataclasses.dataclass
class Encoded:
    sem: np.ndarray        # int16[max(8, k)]: the table, unused entries 0
    col_idx: np.ndarray    # uint32[nnz]
    head: np.ndarray       # uint16[nnz]
    tail1: np.ndarray      # uint16[nnz]
    tail2: np.ndarray      # uint32[nnz]
    eta: np.ndarray        # float64[3]
    exact_frac: float
    idx_bits: int = 3      # slot-index width
    layout: int = 0        # 0: slot in the column word, 1: in the value (head's top bits)

    @property
    def table(self):
        return _table(self.sem)

    def column(self):
        if self.layout == 1:
            return self.col_idx.copy()
        return self.col_idx & np.uint32(0xFFFFFFFF >> self.idx_bits)

    def slot(self):
        if self.idx_bits == 0:
            return np.zeros_like(self.col_idx)
        if self.layout == 1:
            return ((self.head >> np.uint16(15 - self.idx_bits)) &
                    np.uint16((1 << self.idx_bits) - 1)).astype(np.uint32)
        return self.col_idx >> np.uint32(32 - self.idx_bits)


def encode_values(val, col, sem, idx_bits: int = 3, layout: int = 0):
    val = _c(val, np.float64)
    col = _c(col, np.int32)
    sem = _table(sem)
    nnz = val.size
    ci = np.empty(nnz, np.uint32)
    h = np.empty(nnz, np.uint16)
    t1 = np.empty(nnz, np.uint16)
    t2 = np.empty(nnz, np.uint32)
    rc = lib().or_encode_values(_p(val), _p(col), nnz, _p(sem), idx_bits, layout, _p(ci), _p(h),
                                _p(t1), _p(t2))
    if rc < 0:
        raise OracleError(rc, "encode_values")
    return ci, h, t1, t2


def encode(indptr, indices, data, n_cols: int, num_exp: int = 8, sem_in=None,
           layout: int = -1) -> Encoded:
    """layout: 0 slot in the column word, 1 in the value, -1 the column word
    unless n_cols needs more than its 32 - idx_bits bits."""
    indptr = _c(indptr, np.int32)
    indices = _c(indices, np.int32)
    data = _c(data, np.float64)
    n_rows = indptr.size - 1
    nnz = data.size
    sem = np.zeros(MAX_EXP, np.int16)
    ci = np.empty(max(nnz, 1), np.uint32)
    h = np.empty(max(nnz, 1), np.uint16)
    t1 = np.empty(max(nnz, 1), np.uint16)
    t2 = np.empty(max(nnz, 1), np.uint32)
    eta = np.zeros(3, np.float64)
    ef = C.c_double(0.0)
    si = None if sem_in is None else _c(sem_in, np.int16)
    if si is not None and si.size < num_exp:
        raise OracleError(ERR_ARG, "sem_in holds fewer than num_exp entries")
    lo = C.c_int(0)
    rc = lib().or_encode(_p(indptr), _p(indices), _p(data), n_rows, n_cols, nnz, num_exp, layout,
                         _p(si), _p(sem), _p(ci), _p(h), _p(t1), _p(t2), _p(eta),
                         C.addressof(ef), C.addressof(lo))
    if rc < 0:
        raise OracleError(rc, "encode")
    return Encoded(sem[:max(8, num_exp)].copy(), ci[:nnz], h[:nnz], t1[:nnz], t2[:nnz], eta,
                   ef.value, index_bits(num_exp), lo.value)


@dataclasses.dataclass
class EncodedBlocks(Encoded):
    """Planes with one table per block of ``block_rows`` rows (Section
    III-B.1, sampling); ``block_sem[b]`` is block b's table (64 entries)."""
    block_sem: np.ndarray = None   # int16[n_blocks, 64]
    block_rows: int = 0

    def table_of_rows(self, indptr):
        """The table each non-zero is read with: int16[nnz, 64]."""
        n_rows = np.asarray(indptr).size - 1
        blk = np.arange(n_rows) // self.block_rows
        return self.block_sem[np.repeat(blk, np.diff(np.asarray(indptr)))]


def encode_blocks(indptr, indices, data, n_cols: int, num_exp: int = 8, block_rows: int = 256,
                  sample_rows=None, layout: int = -1) -> EncodedBlocks:
    """Per-row-block tables; ``sample_rows`` (one row of each block, drawn by
    the caller) picks each table from that row's exponents, None from all of
    the block's values."""
    indptr = _c(indptr, np.int32)
    indices = _c(indices, np.int32)
    data = _c(data, np.float64)
    n_rows = indptr.size - 1
    nnz = data.size
    n_blocks = -(-n_rows // block_rows) if block_rows > 0 else 0
    bs = np.zeros((max(n_blocks, 1), MAX_EXP), np.int16)
    ci = np.empty(max(nnz, 1), np.uint32)
    h = np.empty(max(nnz, 1), np.uint16)
    t1 = np.empty(max(nnz, 1), np.uint16)
    t2 = np.empty(max(nnz, 1), np.uint32)
    eta = np.zeros(3, np.float64)
    ef = C.c_double(0.0)
    lo = C.c_int(0)
    sr = None if sample_rows is None else _c(sample_rows, np.int32)
    if sr is not None and sr.size < n_blocks:
        raise OracleError(ERR_ARG, "sample_rows holds fewer rows than there are blocks")
    rc = lib().or_encode_blocks(_p(indptr), _p(indices), _p(data), n_rows, n_cols, nnz, num_exp,
                                layout, block_rows, _p(sr), _p(bs), _p(ci), _p(h), _p(t1), _p(t2),
                                _p(eta), C.addressof(ef), C.addressof(lo))
    if rc < 0:
        raise OracleError(rc, "encode_blocks")
    return EncodedBlocks(np.zeros(max(8, num_exp), np.int16), ci[:nnz], h[:nnz], t1[:nnz],
                         t2[:nnz], eta, ef.value, index_bits(num_exp), lo.value,
                         bs[:n_blocks].copy(), block_rows)


def encode_sampled(indptr, indices, data, n_cols: int, num_exp: int = 8, block_rows: int = 256,
                   sample_rows=None, layout: int = -1) -> Encoded:
    """One table for the matrix from the pooled counts of the drawn rows
    (one per block of ``block_rows`` rows), the largest exponent added."""
    indptr = _c(indptr, np.int32)
    indices = _c(indices, np.int32)
    data = _c(data, np.float64)
    n_rows = indptr.size - 1
    nnz = data.size
    sem = np.zeros(MAX_EXP, np.int16)
    ci = np.empty(max(nnz, 1), np.uint32)
    h = np.empty(max(nnz, 1), np.uint16)
    t1 = np.empty(max(nnz, 1), np.uint16)
    t2 = np.empty(max(nnz, 1), np.uint32)
    eta = np.zeros(3, np.float64)
    ef = C.c_double(0.0)
    lo = C.c_int(0)
    sr = None if sample_rows is None else _c(sample_rows, np.int32)
    n_blocks = -(-n_rows // block_rows) if block_rows > 0 else 0
    if sr is not None and sr.size < n_blocks:
        raise OracleError(ERR_ARG, "sample_rows holds fewer rows than there are blocks")
    rc = lib().or_encode_sampled(_p(indptr), _p(indices), _p(data), n_rows, n_cols, nnz, num_exp,
                                 layout, block_rows, _p(sr), _p(sem), _p(ci), _p(h), _p(t1),
                                 _p(t2), _p(eta), C.addressof(ef), C.addressof(lo))
    if rc < 0:
        raise OracleError(rc, "encode_sampled")
    return Encoded(sem[:max(8, num_exp)].copy(), ci[:nnz], h[:nnz], t1[:nnz], t2[:nnz], eta,
                   ef.value, index_bits(num_exp), lo.value)


def decode_blocks(indptr, enc: EncodedBlocks, s: int):
    """Every value read with s segments and the table of its row's block."""
    indptr = _c(indptr, np.int32)
    out = np.empty(enc.head.size, np.float64)
    for b in range(enc.block_sem.shape[0]):
        j0 = int(indptr[min(b * enc.block_rows, indptr.size - 1)])
        j1 = int(indptr[min((b + 1) * enc.block_rows, indptr.size - 1)])
        table = _c(enc.block_sem[b], np.int16)
        seg = np.empty(max(j1 - j0, 1), np.float64)
        ci, h, t1, t2 = (_c(a[j0:j1], a.dtype) for a in (enc.col_idx, enc.head, enc.tail1,
                                                            enc.tail2))
        lib().or_decode(_p(ci), _p(h), _p(t1), _p(t2), j1 - j0, _p(table), enc.idx_bits,
                        enc.layout, s, _p(seg))
        out[j0:j1] = seg[:j1 - j0]
    return out


def decode(enc: Encoded, s: int):
    out = np.empty(enc.head.size, np.float64)
    lib().or_decode(_p(enc.col_idx), _p(enc.head), _p(enc.tail1), _p(enc.tail2),
                    enc.head.size, _p(enc.table), enc.idx_bits, enc.layout, s, _p(out))
    return out


def decode_one(col_word: int, head: int, tail1: int, tail2: int, sem, s: int,
               idx_bits: int = 3, layout: int = 0) -> float:
    table = _table(sem)
    return lib().or_decode_one(col_word, head, tail1, tail2, _p(table), idx_bits, layout, s)


# ------------------------------------------------- FP16 / BF16 comparators ---
LP_FP16, LP_BF16 = 1, 2
S_LP = -2  # fixed_segments value that selects the 16-bit operator


def lp_round(v: float, fmt: int):
    """(bits, overflowed) of one value rounded to FP16 / BF16."""
    over = C.c_int(0)
    h = lib().or_lp_round(float(v), fmt, C.addressof(over))
    return int(h), bool(over.value)


def lp_widen(h: int, fmt: int) -> float:
    return lib().or_lp_widen(int(h), fmt)


def lp_convert(val, fmt: int):
    """(uint16 plane, number of overflows)."""
    val = _c(val, np.float64)
    out = np.empty(max(val.size, 1), np.uint16)
    n = lib().or_lp_convert(_p(val), val.size, fmt, _p(out))
    return out[:val.size], int(n)


def lp_spmv(indptr, indices, val16, fmt: int, x):
    indptr = _c(indptr, np.int32)
    indices = _c(indices, np.int32)
    val16 = _c(val16, np.uint16)
    x = _c(x, np.float64)
    y = np.empty(indptr.size - 1, np.float64)
    lib().or_lp_spmv(indptr.size - 1, _p(indptr), _p(indices), _p(val16), fmt, _p(x), _p(y))
    return y


# ------------------------------------------------------------------ SpMV ---
def csr_spmv(indptr, indices, data, x):
    indptr = _c(indptr, np.int32)
    indices = _c(indices, np.int32)
    data = _c(data, np.float64)
    x = _c(x, np.float64)
    y = np.empty(indptr.size - 1, np.float64)
    lib().or_csr_spmv(indptr.size - 1, _p(indptr), _p(indices), _p(data), _p(x), _p(y))
    return y


def gse_spmv(indptr, enc: Encoded, s: int, x):
    indptr = _c(indptr, np.int32)
    x = _c(x, np.float64)
    y = np.empty(indptr.size - 1, np.float64)
    if isinstance(enc, EncodedBlocks):
        bs = _c(enc.block_sem, np.int16)
        lib().or_gse_spmv_blocks(indptr.size - 1, _p(indptr), _p(enc.col_idx), _p(enc.head),
                                 _p(enc.tail1), _p(enc.tail2), _p(bs), enc.block_rows,
                                 enc.idx_bits, enc.layout, s, _p(x), _p(y))
        return y
    table = enc.table
    lib().or_gse_spmv(indptr.size - 1, _p(indptr), _p(enc.col_idx), _p(enc.head),
                      _p(enc.tail1), _p(enc.tail2), _p(table), enc.idx_bits, enc.layout, s, _p(x),
                      _p(y))
    return y


def gse_spmv_rows(rows, indptr, enc: Encoded, s: int, x):
    rows = _c(rows, np.int32)
    indptr = _c(indptr, np.int32)
    x = _c(x, np.float64)
    y = np.empty(rows.size, np.float64)
    if isinstance(enc, EncodedBlocks):  # each row with its block's table
        blk = rows // enc.block_rows
        for b in np.unique(blk):
            sel = np.nonzero(blk == b)[0]
            part = _c(rows[sel], np.int32)
            out = np.empty(part.size, np.float64)
            table = _c(enc.block_sem[b], np.int16)
            lib().or_gse_spmv_rows(_p(part), part.size, _p(indptr), _p(enc.col_idx),
                                   _p(enc.head), _p(enc.tail1), _p(enc.tail2), _p(table),
                                   enc.idx_bits, enc.layout, s, _p(x), _p(out))
            y[sel] = out
        return y
    table = enc.table
    lib().or_gse_spmv_rows(_p(rows), rows.size, _p(indptr), _p(enc.col_idx), _p(enc.head),
                           _p(enc.tail1), _p(enc.tail2), _p(table), enc.idx_bits, enc.layout, s,
                           _p(x), _p(y))
    return y


# ------------------------------------------------------------ controller ---
PRESETS = {
    # Section IV-D.1 (CG: l=3000, t=250, m=500, RSD 0.50, nDec 130, relDec 0.45)
    "paper_cg": dict(l=3000, t=250, m=500, rsd_limit=0.50, ndec_limit=130, reldec_limit=0.45),
    # Section IV-D.1 (GMRES: l=9000, t=300, m=1500, RSD 0.03, nDec 80, relDec 0.08)
    "paper_gmres": dict(l=9000, t=300, m=1500, rsd_limit=0.03, ndec_limit=80,
                        reldec_limit=0.08),
}


def make_params(tol=1e-10, max_iter=5000, restart=30, max_restarts=500, start_segments=1,
                fixed_segments=0, preset="paper_cg", ndec_rule=0, floor_c=10.0,
                switch_mode=2, orth=0, **over) -> Params:
    d = dict(PRESETS[preset])
    d.update(over)
    return Params(tol, max_iter, restart, max_restarts, start_segments, fixed_segments,
                  d["l"], d["t"], d["m"], d["rsd_limit"], d["ndec_limit"], d["reldec_limit"],
                  ndec_rule, floor_c, switch_mode, orth)


def window_metrics(resid, j: int, t: int):
    resid = _c(resid, np.float64)
    rsd = C.c_double()
    nd = C.c_int32()
    rd = C.c_double()
    lib().or_window_metrics(_p(resid), j, t, C.addressof(rsd), C.addressof(nd), C.addressof(rd))
    return rsd.value, nd.value, rd.value


def precision_trigger(resid, j: int, params: Params) -> int:
    resid = _c(resid, np.float64)
    return lib().or_precision_trigger(_p(resid), j, C.byref(params))


# --------------------------------------------------------------- solvers ---
@dataclasses.dataclass
class SolveResult:
    x: np.ndarray
    status: int
    iters: int
    iters_per_seg: tuple
    switch_iter: tuple
    switch_trigger: tuple
    relres_recursive: float
    relres_true: float
    hist: np.ndarray
    seg_hist: np.ndarray


def _matrix(indptr, indices=None, data=None, enc: Optional[Encoded] = None, lp=None):
    keep = [indptr, indices, data]
    m = Matrix()
    m.n_rows = indptr.size - 1
    m.row_ptr = _p(indptr)
    m.col = _p(indices)
    m.val = _p(data)
    if enc is not None:
        m.col_idx, m.head, m.tail1, m.tail2 = (_p(enc.col_idx), _p(enc.head), _p(enc.tail1),
                                               _p(enc.tail2))
        table = enc.table
        m.sem64 = _p(table)
        m.eta3 = _p(enc.eta)
        m.idx_bits = enc.idx_bits
        m.layout = enc.layout
        keep.extend([enc, table])
        if isinstance(enc, EncodedBlocks):
            bs = _c(enc.block_sem, np.int16)
            m.block_sem = _p(bs)
            m.block_rows = enc.block_rows
            keep.append(bs)
    if lp is not None:  # (uint16 plane, fmt)
        plane = _c(lp[0], np.uint16)
        m.lp_val = _p(plane)
        m.lp_fmt = int(lp[1])
        keep.append(plane)
    return m, keep


def _solve(fn, indptr, b, params: Params, indices=None, data=None, enc=None, x0=None, lp=None):
    indptr = _c(indptr, np.int32)
    indices = None if indices is None else _c(indices, np.int32)
    data = None if data is None else _c(data, np.float64)
    b = _c(b, np.float64)
    x = np.zeros(indptr.size - 1, np.float64) if x0 is None else _c(x0, np.float64).copy()
    cap = params.max_iter + 2
    hist = np.full(cap, np.nan)
    seg = np.zeros(cap, np.int32)
    m, keep = _matrix(indptr, indices, data, enc, lp)
    rep = Report()
    fn(C.byref(m), _p(b), _p(x), C.byref(params), C.byref(rep), _p(hist), _p(seg))
    del keep
    return SolveResult(x, rep.status, rep.iters, tuple(rep.iters_per_seg),
                       tuple(rep.switch_iter), tuple(rep.switch_trigger),
                       rep.relres_recursive, rep.relres_true, hist[: rep.iters + 1],
                       seg[: rep.iters + 1])


def cg(indptr, b, params: Params, indices=None, data=None, enc=None, x0=None,
       lp=None) -> SolveResult:
    """CG; ``params.fixed_segments == -1`` runs on the FP64 CSR values, -2 on
    the 16-bit values ``lp = (plane, fmt)``."""
    return _solve(lib().or_cg, indptr, b, params, indices, data, enc, x0, lp)


def gmres(indptr, b, params: Params, indices=None, data=None, enc=None, x0=None,
          lp=None) -> SolveResult:
    """Restarted GMRES(params.restart); ``fixed_segments == -1`` runs on FP64,
    -2 on the 16-bit values ``lp``."""
    return _solve(lib().or_gmres, indptr, b, params, indices, data, enc, x0, lp)

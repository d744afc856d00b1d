"""Python binding of libgse (ctypes).  Argument marshalling only.

Every function of the C ABI (``include/gse.h``) is exposed under the same
name; arguments are torch tensors on the GPU (their ``data_ptr()`` is passed)
and the current torch stream.  All computation happens in the HIP library:
if ``libgse.so`` has not been built this module raises on import of the
library, there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgse.so")

OK, PENDING, NOT_CONVERGED = 0, 1, 2
ERR_ARG, ERR_NONFINITE, ERR_RANGE, ERR_NOMEM = -1, -2, -3, -4
ERR_BREAKDOWN, ERR_HIP, ERR_TICKET = -5, -6, -7
CG, GMRES = 0, 1
TRIGGERS = {0: "none", 1: "C1", 2: "C2", 3: "C3", 4: "floor", 5: "tol", 6: "breakdown"}
MAX_EXP = 8


class GseError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libgse status {status}: {msg}")
        self.status = status


class gse_matrix(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("nnz", C.c_int64),
                ("num_exp", C.c_int32), ("num_used", C.c_int32), ("idx_bits", C.c_int32),
                ("idx_layout", C.c_int32), ("sem", C.c_int16 * 64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("head", C.c_void_p),
                ("tail1", C.c_void_p), ("tail2", C.c_void_p), ("tile_row", C.c_void_p),
                ("tile_cap", C.c_int32), ("tile_nnz", C.c_int32), ("n_tiles", C.c_int32),
                ("rv_lanes", C.c_int32), ("max_row_nnz", C.c_int32),
                ("eta", C.c_double * 3), ("exact_frac", C.c_double),
                ("block_rows", C.c_int32), ("block_stride", C.c_int32),
                ("block_sem", C.c_void_p)]


class gse_csr(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("tile_row", C.c_void_p), ("tile_cap", C.c_int32), ("tile_nnz", C.c_int32),
                ("n_tiles", C.c_int32), ("rv_lanes", C.c_int32), ("max_row_nnz", C.c_int32)]


class gse_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("start_segments", C.c_int32), ("fixed_segments", C.c_int32),
                ("l", C.c_int32), ("t", C.c_int32), ("m", C.c_int32),
                ("rsd_limit", C.c_double), ("ndec_limit", C.c_int32),
                ("reldec_limit", C.c_double), ("ndec_rule", C.c_int32),
                ("floor_c", C.c_double), ("switch_mode", C.c_int32),
                ("record_history", C.c_int32), ("launch_mode", C.c_int32), ("orth", C.c_int32)]


class gse_report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("iters_per_seg", C.c_int32 * 3),
                ("switch_iter", C.c_int32 * 2), ("switch_trigger", C.c_int32 * 2),
                ("relres_recursive", C.c_double), ("relres_true", C.c_double),
                ("time_ms", C.c_double)]

    def as_dict(self):
        return {"status": self.status, "iters": self.iters,
                "iters_per_seg": list(self.iters_per_seg), "switch_iter": list(self.switch_iter),
                "switch_trigger": [TRIGGERS.get(t, t) for t in self.switch_trigger],
                "relres_recursive": self.relres_recursive, "relres_true": self.relres_true,
                "time_ms": self.time_ms}


class gse_system(C.Structure):
    _fields_ = [("A", C.c_void_p), ("M", C.c_void_p), ("b", C.c_void_p), ("x", C.c_void_p)]


FMT_GSE, FMT_CSR64 = 0, 1


class gse_lp_matrix(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("nnz", C.c_int64),
                ("fmt", C.c_int32), ("pad", C.c_int32), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("tile_row", C.c_void_p),
                ("tile_cap", C.c_int32), ("tile_nnz", C.c_int32), ("n_tiles", C.c_int32),
                ("rv_lanes", C.c_int32), ("max_row_nnz", C.c_int32), ("pad2", C.c_int32),
                ("overflow", C.c_int64), ("eta", C.c_double)]


class gse_request(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("b", C.c_void_p), ("x", C.c_void_p),
                ("format", C.c_int32), ("num_exp", C.c_int32), ("x0_given", C.c_int32),
                ("params", gse_params)]


class gse_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("running", C.c_int64), ("admitted", C.c_int64),
                ("completed", C.c_int64), ("arena_bytes", C.c_int64), ("arena_used", C.c_int64),
                ("arena_peak", C.c_int64), ("arena_largest_free", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# name -> (restype, argtypes)
_P = C.c_void_p
_SIGS = {
    "gse_pad": (C.c_int64, [C.c_int64]),
    "gse_tile_entries": (C.c_int32, [C.c_int64]),
    "gse_encode_workspace": (C.c_int32, [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "gse_encode": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int64, C.c_int32, _P,
                               C.POINTER(gse_matrix), _P, C.c_size_t, _P]),
    "gse_encode_static": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                      _P, C.POINTER(gse_matrix), _P]),
    "gse_encode_static_scratch_bytes": (C.c_size_t, []),
    "gse_encode_blocks": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                      C.c_int32, _P, C.POINTER(gse_matrix), _P, C.c_size_t, _P]),
    "gse_block_table_entries": (C.c_int64, [C.c_int32, C.c_int32, C.c_int32]),
    "gse_encode_sampled": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                       C.c_int32, _P, C.POINTER(gse_matrix), _P, C.c_size_t, _P]),
    "gse_plan": (C.c_int32, [C.POINTER(gse_matrix), C.c_int32, C.c_int32, _P]),
    "gse_csr_plan": (C.c_int32, [C.POINTER(gse_csr), C.c_int32, C.c_int32, _P]),
    "gse_spmv": (C.c_int32, [C.POINTER(gse_matrix), C.c_int32, _P, _P, _P]),
    "gse_autotune": (C.c_int32, [C.POINTER(gse_matrix), C.c_int32, _P, _P, C.c_int32, _P]),
    "gse_csr_autotune": (C.c_int32, [C.POINTER(gse_csr), _P, _P, C.c_int32, _P]),
    "gse_csr_spmv": (C.c_int32, [C.POINTER(gse_csr), _P, _P, _P]),
    "gse_lp_workspace": (C.c_int32, [C.POINTER(C.c_size_t)]),
    "gse_lp_convert": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int64, C.c_int32,
                                   C.POINTER(gse_lp_matrix), _P, C.c_size_t, _P]),
    "gse_lp_plan": (C.c_int32, [C.POINTER(gse_lp_matrix), C.c_int32, C.c_int32, _P]),
    "gse_lp_spmv": (C.c_int32, [C.POINTER(gse_lp_matrix), _P, _P, _P]),
    "gse_lp_cg": (C.c_int32, [C.POINTER(gse_lp_matrix), _P, _P, C.POINTER(gse_params),
                              C.POINTER(gse_report), _P, C.c_size_t, _P]),
    "gse_lp_gmres": (C.c_int32, [C.POINTER(gse_lp_matrix), _P, _P, C.POINTER(gse_params),
                                 C.POINTER(gse_report), _P, C.c_size_t, _P]),
    "gse_default_params": (C.c_int32, [C.c_int32, C.POINTER(gse_params)]),
    "gse_solver_workspace": (C.c_int32, [C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_int32,
                                         C.POINTER(C.c_size_t)]),
    "gse_cg": (C.c_int32, [C.POINTER(gse_matrix), _P, _P, C.POINTER(gse_params),
                           C.POINTER(gse_report), _P, C.c_size_t, _P]),
    "gse_gmres": (C.c_int32, [C.POINTER(gse_matrix), _P, _P, C.POINTER(gse_params),
                              C.POINTER(gse_report), _P, C.c_size_t, _P]),
    "gse_csr_cg": (C.c_int32, [C.POINTER(gse_csr), _P, _P, C.POINTER(gse_params),
                               C.POINTER(gse_report), _P, C.c_size_t, _P]),
    "gse_csr_gmres": (C.c_int32, [C.POINTER(gse_csr), _P, _P, C.POINTER(gse_params),
                                  C.POINTER(gse_report), _P, C.c_size_t, _P]),
    "gse_solve_history": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "gse_batch_workspace": (C.c_int32, [C.c_int32, _P, C.POINTER(gse_params),
                                        C.POINTER(C.c_size_t)]),
    "gse_batch_cg": (C.c_int32, [C.c_int32, _P, C.POINTER(gse_params), _P, _P, C.c_size_t, _P]),
    "gse_batch_history": (C.c_int32, [_P, C.c_int32, C.c_int32, _P, _P, _P]),
    "gse_solver_create": (C.c_int32, [_P, C.c_size_t, C.c_int32, _P, C.POINTER(C.c_void_p)]),
    "gse_solver_footprint": (C.c_int32, [C.POINTER(gse_request), C.POINTER(C.c_size_t),
                                         C.POINTER(C.c_size_t)]),
    "gse_solver_submit": (C.c_int32, [_P, C.POINTER(gse_request), C.POINTER(C.c_uint64)]),
    "gse_solver_poll": (C.c_int32, [_P, C.c_uint64, C.POINTER(gse_report)]),
    "gse_solver_stats": (C.c_int32, [_P, C.POINTER(gse_server_stats)]),
    "gse_solver_destroy": (C.c_int32, [_P]),
    "gse_stream_copy": (C.c_int32, [_P, _P, C.c_size_t, _P]),
    "gse_stream_reduce8": (C.c_int32, [_P, _P, C.c_size_t, _P]),
    "gse_status_str": (C.c_char_p, [C.c_int32]),
    "gse_last_error": (C.c_char_p, []),
}


def lib():
    """Load libgse.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(status: int, what: str) -> int:
    if status < 0:
        raise GseError(status, f"{what}: {lib().gse_last_error().decode()}")
    return status


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


# ----------------------------------------------------------- raw C names ---
def gse_pad(nnz: int) -> int:
    return lib().gse_pad(nnz)


def gse_tile_entries(nnz: int) -> int:
    return lib().gse_tile_entries(nnz)


def gse_encode_workspace(nnz: int, n_rows: int) -> int:
    out = C.c_size_t()
    _check(lib().gse_encode_workspace(nnz, n_rows, C.byref(out)), "gse_encode_workspace")
    return out.value


def gse_encode(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, sem_in, A: gse_matrix, ws,
               stream=None) -> int:
    si = None
    if sem_in is not None:
        arr = (C.c_int16 * len(sem_in))(*[int(s) for s in sem_in])
        si = C.cast(arr, C.c_void_p)
    return _check(lib().gse_encode(_ptr(row_ptr), _ptr(col), _ptr(val), n_rows, n_cols, nnz,
                                   num_exp, si, C.byref(A), _ptr(ws), ws.numel() * ws.element_size(),
                                   _stream(stream)), "gse_encode")


def gse_encode_blocks(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, block_rows, sample_rows,
                      A: gse_matrix, ws, stream=None) -> int:
    return _check(lib().gse_encode_blocks(_ptr(row_ptr), _ptr(col), _ptr(val), n_rows, n_cols, nnz,
                                          num_exp, block_rows, _ptr(sample_rows), C.byref(A),
                                          _ptr(ws), ws.numel() * ws.element_size(),
                                          _stream(stream)), "gse_encode_blocks")


def gse_encode_sampled(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, block_rows, sample_rows,
                       A: gse_matrix, ws, stream=None) -> int:
    return _check(lib().gse_encode_sampled(_ptr(row_ptr), _ptr(col), _ptr(val), n_rows, n_cols,
                                           nnz, num_exp, block_rows, _ptr(sample_rows),
                                           C.byref(A), _ptr(ws), ws.numel() * ws.element_size(),
                                           _stream(stream)), "gse_encode_sampled")


def gse_block_table_entries(n_rows: int, block_rows: int, num_exp: int) -> int:
    return int(lib().gse_block_table_entries(n_rows, block_rows, num_exp))


def gse_encode_static(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, sem_in, A: gse_matrix,
                      stream=None) -> int:
    si = None
    if sem_in is not None:
        arr = (C.c_int16 * len(sem_in))(*[int(s) for s in sem_in])
        si = C.cast(arr, C.c_void_p)
    return _check(lib().gse_encode_static(_ptr(row_ptr), _ptr(col), _ptr(val), n_rows, n_cols, nnz,
                                          num_exp, si, C.byref(A), _stream(stream)),
                  "gse_encode_static")


def gse_encode_static_scratch_bytes() -> int:
    return lib().gse_encode_static_scratch_bytes()


LP_FP16, LP_BF16 = 1, 2
IDX_AUTO, IDX_COLUMN, IDX_VALUE = 0, 1, 2


def gse_lp_workspace() -> int:
    out = C.c_size_t()
    _check(lib().gse_lp_workspace(C.byref(out)), "gse_lp_workspace")
    return out.value


def gse_lp_convert(row_ptr, col, val, n_rows, n_cols, nnz, fmt, M: gse_lp_matrix, ws,
                   stream=None) -> int:
    return _check(lib().gse_lp_convert(_ptr(row_ptr), _ptr(col), _ptr(val), n_rows, n_cols, nnz,
                                       fmt, C.byref(M), _ptr(ws), ws.numel() * ws.element_size(),
                                       _stream(stream)), "gse_lp_convert")


def gse_lp_plan(M: gse_lp_matrix, tile_nnz: int, rv_lanes: int = -1, stream=None) -> int:
    return _check(lib().gse_lp_plan(C.byref(M), tile_nnz, rv_lanes, _stream(stream)),
                  "gse_lp_plan")


def gse_lp_spmv(M: gse_lp_matrix, x, y, stream=None) -> int:
    return _check(lib().gse_lp_spmv(C.byref(M), _ptr(x), _ptr(y), _stream(stream)), "gse_lp_spmv")


def gse_plan(A: gse_matrix, tile_nnz: int, rv_lanes: int = -1, stream=None) -> int:
    return _check(lib().gse_plan(C.byref(A), tile_nnz, rv_lanes, _stream(stream)), "gse_plan")


def gse_csr_plan(M: gse_csr, tile_nnz: int, rv_lanes: int = -1, stream=None) -> int:
    return _check(lib().gse_csr_plan(C.byref(M), tile_nnz, rv_lanes, _stream(stream)),
                  "gse_csr_plan")


def gse_spmv(A: gse_matrix, k_segments: int, x: torch.Tensor, y: torch.Tensor, stream=None) -> int:
    return _check(lib().gse_spmv(C.byref(A), k_segments, _ptr(x), _ptr(y), _stream(stream)),
                  "gse_spmv")


def gse_autotune(A: gse_matrix, k_segments: int, x: torch.Tensor, y: torch.Tensor, reps: int = 5,
                 stream=None) -> int:
    return _check(lib().gse_autotune(C.byref(A), k_segments, _ptr(x), _ptr(y), reps,
                                     _stream(stream)), "gse_autotune")


def gse_csr_autotune(M: gse_csr, x: torch.Tensor, y: torch.Tensor, reps: int = 5,
                     stream=None) -> int:
    return _check(lib().gse_csr_autotune(C.byref(M), _ptr(x), _ptr(y), reps, _stream(stream)),
                  "gse_csr_autotune")


def gse_csr_spmv(M: gse_csr, x: torch.Tensor, y: torch.Tensor, stream=None) -> int:
    return _check(lib().gse_csr_spmv(C.byref(M), _ptr(x), _ptr(y), _stream(stream)),
                  "gse_csr_spmv")


def gse_default_params(method: int) -> gse_params:
    p = gse_params()
    _check(lib().gse_default_params(method, C.byref(p)), "gse_default_params")
    return p


def gse_solver_workspace(method: int, n_rows: int, nnz: int, restart: int, max_iter: int) -> int:
    out = C.c_size_t()
    _check(lib().gse_solver_workspace(method, n_rows, nnz, restart, max_iter, C.byref(out)),
           "gse_solver_workspace")
    return out.value


def _solve(fn, name, A, b, x, p, ws, stream):
    rep = gse_report()
    st = fn(C.byref(A), _ptr(b), _ptr(x), C.byref(p), C.byref(rep), _ptr(ws),
            ws.numel() * ws.element_size(), _stream(stream))
    if st < 0 and st != ERR_BREAKDOWN:
        _check(st, name)
    return rep


def gse_cg(A, b, x, p, ws, stream=None) -> gse_report:
    return _solve(lib().gse_cg, "gse_cg", A, b, x, p, ws, stream)


def gse_gmres(A, b, x, p, ws, stream=None) -> gse_report:
    return _solve(lib().gse_gmres, "gse_gmres", A, b, x, p, ws, stream)


def gse_csr_cg(M, b, x, p, ws, stream=None) -> gse_report:
    return _solve(lib().gse_csr_cg, "gse_csr_cg", M, b, x, p, ws, stream)


def gse_csr_gmres(M, b, x, p, ws, stream=None) -> gse_report:
    return _solve(lib().gse_csr_gmres, "gse_csr_gmres", M, b, x, p, ws, stream)


def gse_lp_cg(M, b, x, p, ws, stream=None) -> gse_report:
    return _solve(lib().gse_lp_cg, "gse_lp_cg", M, b, x, p, ws, stream)


def gse_lp_gmres(M, b, x, p, ws, stream=None) -> gse_report:
    return _solve(lib().gse_lp_gmres, "gse_lp_gmres", M, b, x, p, ws, stream)


def gse_solve_history(ws, cap: int, stream=None):
    import numpy as np
    hist = np.zeros(cap, np.float64)
    seg = np.zeros(cap, np.int32)
    _check(lib().gse_solve_history(_ptr(ws), cap, C.c_void_p(hist.ctypes.data),
                                   C.c_void_p(seg.ctypes.data), _stream(stream)),
           "gse_solve_history")
    return hist, seg


def _systems(systems):
    """systems: list of (matrix, b, x) with matrix a gse_matrix or gse_csr record."""
    arr = (gse_system * len(systems))()
    for i, (mat, b, x) in enumerate(systems):
        if isinstance(mat, gse_matrix):
            arr[i].A = C.addressof(mat)
        else:
            arr[i].M = C.addressof(mat)
        arr[i].b = b.data_ptr()
        arr[i].x = x.data_ptr()
    return arr


def gse_batch_workspace(systems, p: gse_params) -> int:
    arr = _systems(systems)
    out = C.c_size_t()
    _check(lib().gse_batch_workspace(len(systems), C.cast(arr, C.c_void_p), C.byref(p),
                                     C.byref(out)), "gse_batch_workspace")
    return out.value


def gse_batch_cg(systems, p: gse_params, ws: torch.Tensor, stream=None):
    """Solve every (matrix, b, x) together; returns the list of reports."""
    arr = _systems(systems)
    reps = (gse_report * len(systems))()
    st = lib().gse_batch_cg(len(systems), C.cast(arr, C.c_void_p), C.byref(p),
                            C.cast(reps, C.c_void_p), _ptr(ws), ws.numel() * ws.element_size(),
                            _stream(stream))
    if st < 0 and st != ERR_BREAKDOWN:
        _check(st, "gse_batch_cg")
    return list(reps)


def gse_batch_history(ws, index: int, cap: int, stream=None):
    import numpy as np
    hist = np.zeros(cap, np.float64)
    seg = np.zeros(cap, np.int32)
    _check(lib().gse_batch_history(_ptr(ws), index, cap, C.c_void_p(hist.ctypes.data),
                                   C.c_void_p(seg.ctypes.data), _stream(stream)),
           "gse_batch_history")
    return hist, seg


def gse_solver_create(arena: torch.Tensor, max_slots: int, stream=None):
    out = C.c_void_p()
    _check(lib().gse_solver_create(_ptr(arena), arena.numel() * arena.element_size(), max_slots,
                                   _stream(stream), C.byref(out)), "gse_solver_create")
    return out


def gse_solver_footprint(rq: gse_request):
    res, tr = C.c_size_t(), C.c_size_t()
    _check(lib().gse_solver_footprint(C.byref(rq), C.byref(res), C.byref(tr)),
           "gse_solver_footprint")
    return res.value, tr.value


def gse_solver_submit(server, rq: gse_request) -> int:
    t = C.c_uint64()
    _check(lib().gse_solver_submit(server, C.byref(rq), C.byref(t)), "gse_solver_submit")
    return t.value


def gse_solver_poll(server, ticket: int):
    """None while pending, else the report (the ticket is retired)."""
    rep = gse_report()
    st = _check(lib().gse_solver_poll(server, ticket, C.byref(rep)), "gse_solver_poll")
    return None if st == PENDING else rep


def gse_solver_stats(server) -> gse_server_stats:
    out = gse_server_stats()
    _check(lib().gse_solver_stats(server, C.byref(out)), "gse_solver_stats")
    return out


def gse_solver_destroy(server) -> None:
    _check(lib().gse_solver_destroy(server), "gse_solver_destroy")


class Request:
    """Host arrays of one server request.  The server reads them (and writes
    ``x``) until the ticket completes, so keep this object alive until then."""

    def __init__(self, A, b, fmt: int = FMT_GSE, params: Optional[gse_params] = None,
                 x0=None, num_exp: int = 8):
        import numpy as np
        # private copies: the server reads them until the request completes
        self.row_ptr = np.array(A.indptr, dtype=np.int32)
        self.col = np.array(A.indices, dtype=np.int32)
        self.val = np.array(A.data, dtype=np.float64)
        self.b = np.array(b, dtype=np.float64)
        self.x = np.zeros(A.n_rows) if x0 is None else np.array(x0, dtype=np.float64)
        rq = gse_request()
        rq.n_rows = A.n_rows
        rq.nnz = int(self.val.size)
        rq.row_ptr = self.row_ptr.ctypes.data
        rq.col = self.col.ctypes.data
        rq.val = self.val.ctypes.data
        rq.b = self.b.ctypes.data
        rq.x = self.x.ctypes.data
        rq.format = fmt
        rq.num_exp = num_exp
        rq.x0_given = 0 if x0 is None else 1
        rq.params = params if params is not None else gse_default_params(CG)
        self.rq = rq


def gse_stream_reduce8(src: torch.Tensor, dst: torch.Tensor, n_out: int, stream=None) -> int:
    return _check(lib().gse_stream_reduce8(_ptr(src), _ptr(dst), n_out, _stream(stream)),
                  "gse_stream_reduce8")


def gse_stream_copy(src: torch.Tensor, dst: torch.Tensor, nbytes: int, stream=None) -> int:
    return _check(lib().gse_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)),
                  "gse_stream_copy")


# -------------------------------------------------------- tensor holders ---
def _alloc(n, dtype, device):
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


class GseMatrix:
    """Device planes of one encoded matrix plus its ``gse_matrix`` record."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n_cols: int,
                 num_exp: int = 8, sem_in=None, stream=None, idx_layout: int = IDX_AUTO,
                 block_rows: int = 0, sample_rows: torch.Tensor = None, pooled: bool = False):
        """block_rows > 0: one table per block of that many rows
        (gse_encode_blocks), chosen from the device rows ``sample_rows``
        (one per block) or, when None, from each block's values.  pooled:
        one table for the whole matrix from the pooled exponents of the drawn
        rows (gse_encode_sampled; block_rows and sample_rows required)."""
        dev = row_ptr.device
        n_rows = row_ptr.numel() - 1
        nnz = val.numel()
        pad = gse_pad(nnz)
        self.row_ptr = row_ptr
        self.col_idx = _alloc(pad, torch.int32, dev)
        self.head = _alloc(pad, torch.int16, dev)
        self.tail1 = _alloc(pad, torch.int16, dev)
        self.tail2 = _alloc(pad, torch.int32, dev)
        cap = gse_tile_entries(nnz)
        self.tile_row = _alloc(cap, torch.int32, dev)
        self.ws = _alloc(gse_encode_workspace(nnz, n_rows), torch.uint8, dev)
        A = gse_matrix()
        A.col_idx = self.col_idx.data_ptr()
        A.head = self.head.data_ptr()
        A.tail1 = self.tail1.data_ptr()
        A.tail2 = self.tail2.data_ptr()
        A.tile_row = self.tile_row.data_ptr()
        A.tile_cap = cap
        A.idx_layout = idx_layout
        self.A = A
        if pooled:
            if sem_in is not None or sample_rows is None or not block_rows:
                raise ValueError("the pooled table needs block_rows and sample_rows, and no sem_in")
            gse_encode_sampled(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, block_rows,
                               sample_rows, A, self.ws, stream)
        elif block_rows:
            if sem_in is not None:
                raise ValueError("per-block tables are chosen by the encoder (no sem_in)")
            self.block_sem = _alloc(max(gse_block_table_entries(n_rows, block_rows, num_exp), 1),
                                    torch.int16, dev)
            A.block_sem = self.block_sem.data_ptr()
            gse_encode_blocks(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, block_rows,
                              sample_rows, A, self.ws, stream)
        else:
            gse_encode(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, sem_in, A, self.ws, stream)

    @property
    def n_rows(self):
        return self.A.n_rows

    @property
    def nnz(self):
        return self.A.nnz

    @property
    def sem(self):
        return list(self.A.sem)[:max(8, self.A.num_exp)]

    @property
    def eta(self):
        return list(self.A.eta)

    def block_tables(self):
        """int16 [n_blocks, 2^idx_bits] host copy of the per-block tables."""
        stride = self.A.block_stride
        n = gse_block_table_entries(self.A.n_rows, self.A.block_rows, self.A.num_exp)
        return self.block_sem[:n].cpu().numpy().reshape(-1, stride)

    def planes(self):
        """(col_idx u32, head u16, tail1 u16, tail2 u32) as numpy arrays (host copy)."""
        n = self.nnz
        return (self.col_idx[:n].cpu().numpy().view("uint32"),
                self.head[:n].cpu().numpy().view("uint16"),
                self.tail1[:n].cpu().numpy().view("uint16"),
                self.tail2[:n].cpu().numpy().view("uint32"))

    def plan(self, tile_nnz: int = 1024, rv_lanes: int = -1, stream=None):
        gse_plan(self.A, tile_nnz, rv_lanes, stream)

    def autotune(self, k_segments: int, x: torch.Tensor, y: torch.Tensor, reps: int = 5,
                 stream=None):
        gse_autotune(self.A, k_segments, x, y, reps, stream)

    def spmv(self, k_segments: int, x: torch.Tensor, y: torch.Tensor, stream=None):
        gse_spmv(self.A, k_segments, x, y, stream)


class LpMatrix:
    """Device planes of one FP16 / BF16 comparator matrix plus its
    ``gse_lp_matrix`` record."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n_cols: int,
                 fmt: int = LP_FP16, stream=None):
        dev = row_ptr.device
        n_rows = row_ptr.numel() - 1
        nnz = val.numel()
        pad = gse_pad(nnz)
        self.row_ptr = row_ptr
        self.col = _alloc(pad, torch.int32, dev)
        self.val = _alloc(pad, torch.int16, dev)
        cap = gse_tile_entries(nnz)
        self.tile_row = _alloc(cap, torch.int32, dev)
        self.ws = _alloc(gse_lp_workspace(), torch.uint8, dev)
        M = gse_lp_matrix()
        M.col = self.col.data_ptr()
        M.val = self.val.data_ptr()
        M.tile_row = self.tile_row.data_ptr()
        M.tile_cap = cap
        self.M = M
        gse_lp_convert(row_ptr, col, val, n_rows, n_cols, nnz, fmt, M, self.ws, stream)

    @property
    def n_rows(self):
        return self.M.n_rows

    def values(self):
        """The 16-bit words (uint16, host copy)."""
        return self.val[:self.M.nnz].cpu().numpy().view("uint16")

    def plan(self, tile_nnz: int = 1024, rv_lanes: int = -1, stream=None):
        gse_lp_plan(self.M, tile_nnz, rv_lanes, stream)

    def spmv(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        gse_lp_spmv(self.M, x, y, stream)


class CsrMatrix:
    """Padded device copy of an FP64 CSR matrix for the baseline operators."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, n_cols: int,
                 tile_nnz: int = 1024, rv_lanes: int = -1, stream=None):
        dev = row_ptr.device
        nnz = val.numel()
        pad = gse_pad(nnz)
        self.row_ptr = row_ptr
        self.col = torch.zeros(max(pad, 1), dtype=torch.int32, device=dev)
        self.val = torch.zeros(max(pad, 1), dtype=torch.float64, device=dev)
        if nnz:
            self.col[:nnz].copy_(col)
            self.val[:nnz].copy_(val)
        cap = gse_tile_entries(nnz)
        self.tile_row = _alloc(cap, torch.int32, dev)
        M = gse_csr()
        M.n_rows = row_ptr.numel() - 1
        M.n_cols = n_cols
        M.nnz = nnz
        M.row_ptr = row_ptr.data_ptr()
        M.col = self.col.data_ptr()
        M.val = self.val.data_ptr()
        M.tile_row = self.tile_row.data_ptr()
        M.tile_cap = cap
        self.M = M
        gse_csr_plan(M, tile_nnz, rv_lanes, stream)

    def plan(self, tile_nnz: int = 1024, rv_lanes: int = -1, stream=None):
        gse_csr_plan(self.M, tile_nnz, rv_lanes, stream)

    def autotune(self, x: torch.Tensor, y: torch.Tensor, reps: int = 5, stream=None):
        gse_csr_autotune(self.M, x, y, reps, stream)

    def spmv(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        gse_csr_spmv(self.M, x, y, stream)

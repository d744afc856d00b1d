// api.hip -- the extern "C" entry points of libgse: host-side validation,
// status mapping and the host part of encode / plan / SpMV.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "batch.h"
#include "gse_internal.h"

namespace gse {

thread_local char g_err[512] = "";

gse_status fail(gse_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

const char* last_error_text() { return g_err; }

gse_status hip_fail(hipError_t e, const char* where) {
  return fail(GSE_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Whether the byte ranges [a, a + na) and [b, b + nb) share a byte.
bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

// The SpMV's vectors: x [n_cols] and y [n_rows] FP64, not overlapping.
gse_status check_spmv_vectors(int32_t n_rows, int32_t n_cols, const double* x, const double* y) {
  if ((n_cols > 0 && !x) || (n_rows > 0 && !y)) return fail(GSE_ERR_ARG, "NULL vector");
  if (ranges_overlap(x, sizeof(double) * (size_t)n_cols, y, sizeof(double) * (size_t)n_rows))
    return fail(GSE_ERR_ARG, "x and y overlap");
  return GSE_OK;
}

int64_t pad_nnz(int64_t nnz) { return (nnz + kPadTo - 1) / kPadTo * kPadTo; }

bool valid_tile(int32_t t) { return t == kWG * 4 || t == kWG * 8 || t == kWG * 16; }

bool valid_rv(int32_t L) { return L == 0 || (L >= 1 && L <= 64 && (L & (L - 1)) == 0); }

// Default schedule: the tile schedule, which measured faster than the
// row-vector one on every matrix family here (both formats).  gse_autotune
// times the alternatives on the matrix itself.
int32_t auto_rv(int64_t nnz, int32_t n_rows, int32_t max_row) {
  (void)nnz;
  (void)n_rows;
  (void)max_row;
  return 0;
}

// Default schedule for per-block tables: the row-tile ring (rv_lanes 0 with
// 1024-non-zero tiles) when no row holds more than eight non-zeros, else the
// row-vector schedule with the power of two nearest above half the mean row
// length (1 .. 64) lanes per row.
int32_t block_lanes(int64_t nnz, int32_t n_rows, int32_t max_row) {
  if (max_row <= 8 && nnz >= kDefaultTile) return 0;
  const int64_t half = n_rows > 0 ? (nnz + 2 * (int64_t)n_rows - 1) / (2 * (int64_t)n_rows) : 1;
  int32_t L = 1;
  while (L < 64 && L < half) L *= 2;
  return L;
}

// Tile table for tile_nnz plus the longest row; picks the schedule.
gse_status plan_common(const int32_t* row_ptr, int32_t n_rows, int64_t nnz, int32_t* tile_row,
                       int32_t tile_cap, int32_t tile_nnz, int32_t rv_lanes, hipStream_t st,
                       int32_t* out_tiles, int32_t* out_rv, int32_t* out_maxrow) {
  if (!valid_tile(tile_nnz)) return fail(GSE_ERR_ARG, "tile_nnz %d not supported", tile_nnz);
  if (rv_lanes != -1 && !valid_rv(rv_lanes))
    return fail(GSE_ERR_ARG, "rv_lanes %d not supported", rv_lanes);
  const int32_t nt = n_tiles_for(nnz, tile_nnz);
  if (tile_cap < nt + 2) return fail(GSE_ERR_NOMEM, "tile_row holds %d < %d", tile_cap, nt + 2);
  int* scratch = tile_row + (tile_cap - 1);  // never part of a tile table
  hipError_t e = launch_plan(row_ptr, n_rows, (int32_t)nnz, tile_nnz, nt, tile_row, st);
  if (e == hipSuccess) e = launch_rowmax(row_ptr, n_rows, scratch, st);
  int32_t maxrow = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&maxrow, scratch, sizeof maxrow, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "plan");
  *out_tiles = nt;
  *out_maxrow = maxrow;
  *out_rv = (rv_lanes == -1) ? auto_rv(nnz, n_rows, maxrow) : rv_lanes;
  return GSE_OK;
}

SpmvOperand operand_of(const gse_matrix* A) {
  SpmvOperand o{};
  o.row_ptr = A->row_ptr;
  o.tile_row = A->tile_row;
  o.col = A->col_idx;
  o.head = A->head;
  o.tail1 = A->tail1;
  o.tail2 = A->tail2;
  o.val = nullptr;
  o.n_rows = A->n_rows;
  o.n_tiles = A->n_tiles;
  o.tile_nnz = A->tile_nnz;
  o.nnz = (int32_t)A->nnz;
  o.rv_lanes = A->rv_lanes;
  o.max_row = A->max_row_nnz;
  o.split = col_split(A->idx_bits, A->idx_layout == GSE_IDX_VALUE);
  for (int i = 0; i < GSE_MAX_EXP; ++i) o.sem[i] = A->sem[i];
  if (A->block_rows > 0) {
    o.block_sem = A->block_sem;
    o.block_rows = A->block_rows;
    o.block_stride = A->block_stride;
  }
  return o;
}

SpmvOperand operand_of(const gse_csr* M) {
  SpmvOperand o{};
  o.row_ptr = M->row_ptr;
  o.tile_row = M->tile_row;
  o.col = reinterpret_cast<const uint32_t*>(M->col);
  o.head = nullptr;
  o.tail1 = nullptr;
  o.tail2 = nullptr;
  o.val = M->val;
  o.n_rows = M->n_rows;
  o.n_tiles = M->n_tiles;
  o.tile_nnz = M->tile_nnz;
  o.nnz = (int32_t)M->nnz;
  o.rv_lanes = M->rv_lanes;
  o.max_row = M->max_row_nnz;
  o.split = col_split(0);
  for (int i = 0; i < GSE_MAX_EXP; ++i) o.sem[i] = 0;
  return o;
}

gse_status check_matrix(const gse_matrix* A) {
  if (!A) return fail(GSE_ERR_ARG, "matrix is NULL");
  if (!A->row_ptr || !A->col_idx || !A->head || !A->tail1 || !A->tail2 || !A->tile_row)
    return fail(GSE_ERR_ARG, "matrix has a NULL device buffer");
  if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) return fail(GSE_ERR_ARG, "negative size");
  if (A->nnz > kMaxNnz) return fail(GSE_ERR_RANGE, "nnz %lld exceeds the limit", (long long)A->nnz);
  if (A->num_exp < 1 || A->num_exp > GSE_MAX_EXP || A->idx_bits != index_bits(A->num_exp) ||
      (A->idx_layout != GSE_IDX_COLUMN && A->idx_layout != GSE_IDX_VALUE))
    return fail(GSE_ERR_ARG, "matrix has no valid shared-exponent table (call gse_encode)");
  if (!valid_tile(A->tile_nnz) || A->n_tiles != n_tiles_for(A->nnz, A->tile_nnz) ||
      A->tile_cap < A->n_tiles + 2 || !valid_rv(A->rv_lanes))
    return fail(GSE_ERR_ARG, "matrix has no valid SpMV schedule (call gse_encode / gse_plan)");
  if (A->block_rows != 0 &&
      (A->block_rows < GSE_MIN_BLOCK_ROWS || !A->block_sem ||
       A->block_stride != (1 << A->idx_bits)))
    return fail(GSE_ERR_ARG, "matrix has no valid per-block tables (call gse_encode_blocks)");
  return GSE_OK;
}

gse_status check_csr(const gse_csr* M) {
  if (!M) return fail(GSE_ERR_ARG, "matrix is NULL");
  if (!M->row_ptr || !M->col || !M->val || !M->tile_row)
    return fail(GSE_ERR_ARG, "matrix has a NULL device buffer");
  if (M->n_rows < 0 || M->n_cols < 0 || M->nnz < 0) return fail(GSE_ERR_ARG, "negative size");
  if (M->nnz > kMaxNnz) return fail(GSE_ERR_RANGE, "nnz exceeds the limit");
  if (!aligned16(M->col) || !aligned16(M->val))
    return fail(GSE_ERR_ARG, "col/val must be 16-byte aligned");
  if (!valid_tile(M->tile_nnz) || M->n_tiles != n_tiles_for(M->nnz, M->tile_nnz) ||
      M->tile_cap < M->n_tiles + 2 || !valid_rv(M->rv_lanes))
    return fail(GSE_ERR_ARG, "matrix has no valid SpMV schedule (call gse_csr_plan)");
  return GSE_OK;
}

// Validation, the encoder launches and the host part of gse_encode, on a
// scratch record `ws` of at least gse_encode_workspace() bytes.
// Checks shared by the encoders; on success *layout is the slot layout.
gse_status check_encode(const int32_t* row_ptr, const int32_t* col, const double* val,
                        int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                        const gse_matrix* A, void* ws, size_t ws_bytes, int* layout_out) {
  if (!A) return fail(GSE_ERR_ARG, "matrix is NULL");
  if (!row_ptr || (nnz > 0 && (!col || !val))) return fail(GSE_ERR_ARG, "NULL CSR array");
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(GSE_ERR_ARG, "negative size");
  if (num_exp < 1 || num_exp > GSE_MAX_EXP) return fail(GSE_ERR_ARG, "num_exp must be 1..64");
  if (nnz > kMaxNnz) return fail(GSE_ERR_RANGE, "nnz %lld exceeds the limit", (long long)nnz);
  const int ib = index_bits(num_exp);
  const bool too_wide = (int64_t)n_cols > (int64_t(1) << (32 - ib));
  int layout = A->idx_layout;
  if (layout == GSE_IDX_AUTO) layout = too_wide ? GSE_IDX_VALUE : GSE_IDX_COLUMN;
  if (layout != GSE_IDX_COLUMN && layout != GSE_IDX_VALUE)
    return fail(GSE_ERR_ARG, "idx_layout must be GSE_IDX_AUTO, GSE_IDX_COLUMN or GSE_IDX_VALUE");
  if (layout == GSE_IDX_COLUMN && too_wide)
    return fail(GSE_ERR_RANGE, "n_cols exceeds 2^%d (the column field left by a %d-bit slot index)",
                32 - ib, ib);
  if (!A->col_idx || !A->head || !A->tail1 || !A->tail2 || !A->tile_row)
    return fail(GSE_ERR_ARG, "matrix planes / tile_row not set");
  if (!aligned16(A->col_idx) || !aligned16(A->head) || !aligned16(A->tail1) || !aligned16(A->tail2))
    return fail(GSE_ERR_ARG, "planes must be 16-byte aligned");
  if (A->tile_cap < gse_tile_entries(nnz))
    return fail(GSE_ERR_NOMEM, "tile_row holds %d < %d entries", A->tile_cap, gse_tile_entries(nnz));
  size_t need = 0;
  gse_encode_workspace(nnz, n_rows, &need);
  if (!ws || ws_bytes < need) return fail(GSE_ERR_NOMEM, "encode workspace needs %zu bytes", need);
  if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(GSE_ERR_ARG, "workspace must be 256-byte aligned");
  *layout_out = layout;
  return GSE_OK;
}

// The per-row-block encoder (Section III-B.1, sampling): validation,
// launches, read-back, default plan.
gse_status encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                         int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                         int32_t block_rows, const int32_t* sample_rows, gse_matrix* A, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  int layout = 0;
  gse_status cs = check_encode(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, A, ws, ws_bytes,
                               &layout);
  if (cs != GSE_OK) return cs;
  if (block_rows < GSE_MIN_BLOCK_ROWS)
    return fail(GSE_ERR_ARG, "block_rows must be at least %d", GSE_MIN_BLOCK_ROWS);
  if (!A->block_sem) return fail(GSE_ERR_ARG, "block_sem is NULL");
  EncodeScratch* sc = reinterpret_cast<EncodeScratch*>(ws);
  A->n_rows = n_rows;
  A->n_cols = n_cols;
  A->nnz = nnz;
  A->num_exp = num_exp;
  A->idx_bits = index_bits(num_exp);
  A->idx_layout = layout;
  A->row_ptr = row_ptr;
  A->block_rows = block_rows;
  A->block_stride = 1 << A->idx_bits;
  hipError_t e = launch_encode_blocks(row_ptr, col, val, n_rows, (int32_t)nnz, num_exp, sample_rows,
                                      A, sc, st);
  if (e != hipSuccess) return hip_fail(e, "gse_encode_blocks launch");
  EncodeScratch h;
  e = hipMemcpyAsync(&h, sc, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_encode_blocks");
  int32_t nt, rv, mr;
  gse_status ps = plan_common(row_ptr, n_rows, nnz, A->tile_row, A->tile_cap, kDefaultTile, 0, st,
                              &nt, &rv, &mr);
  if (ps != GSE_OK) return ps;
  A->tile_nnz = kDefaultTile;
  A->n_tiles = nt;
  A->rv_lanes = block_lanes(nnz, n_rows, mr);
  A->max_row_nnz = mr;
  for (int i = 0; i < GSE_MAX_EXP; ++i) A->sem[i] = 0;
  A->num_used = h.used;
  A->exact_frac = nnz ? (double)h.covered / (double)nnz : 1.0;
  double nrm[4];
  for (int i = 0; i < 4; ++i) memcpy(&nrm[i], &h.norm_bits[i], sizeof(double));
  for (int s = 0; s < 3; ++s) A->eta[s] = nrm[0] > 0.0 ? nrm[s + 1] / nrm[0] : 0.0;
  if (h.nonfinite) return fail(GSE_ERR_NONFINITE, "%d non-finite values", h.nonfinite);
  if (h.range_err & 4) return fail(GSE_ERR_ARG, "a sample row lies outside its block");
  if (h.range_err & 1) return fail(GSE_ERR_RANGE, "a shared exponent is below 63");
  if (h.range_err & 2) return fail(GSE_ERR_RANGE, "a value has no larger shared exponent in the table");
  return GSE_OK;
}

// Shared part of the one-table encoders: the fields of A the launches need.
static void set_global_fields(const int32_t* row_ptr, int32_t n_rows, int32_t n_cols, int64_t nnz,
                              int32_t num_exp, int layout, gse_matrix* A) {
  A->n_rows = n_rows;
  A->n_cols = n_cols;
  A->nnz = nnz;
  A->num_exp = num_exp;
  A->idx_bits = index_bits(num_exp);
  A->idx_layout = layout;
  A->row_ptr = row_ptr;
  A->block_rows = 0;
  A->block_stride = 0;
}

// Shared part of the one-table encoders after the launches: read the
// scratch record back, plan the default SpMV schedule, fill the host fields
// of A, report the encoder's errors.
static gse_status finish_global(const int32_t* row_ptr, int32_t n_rows, int64_t nnz,
                                gse_matrix* A, const EncodeScratch* sc, hipStream_t st,
                                const char* what) {
  EncodeScratch h;
  hipError_t e = hipMemcpyAsync(&h, sc, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, what);
  int32_t nt, rv, mr;
  gse_status ps = plan_common(row_ptr, n_rows, nnz, A->tile_row, A->tile_cap, kDefaultTile, -1, st,
                              &nt, &rv, &mr);
  if (ps != GSE_OK) return ps;
  A->tile_nnz = kDefaultTile;
  A->n_tiles = nt;
  A->rv_lanes = rv;
  A->max_row_nnz = mr;
  for (int i = 0; i < GSE_MAX_EXP; ++i) A->sem[i] = h.sem[i];
  A->num_used = h.used;
  A->exact_frac = nnz ? (double)h.covered / (double)nnz : 1.0;
  double nrm[4];
  for (int i = 0; i < 4; ++i) memcpy(&nrm[i], &h.norm_bits[i], sizeof(double));
  for (int s = 0; s < 3; ++s) A->eta[s] = nrm[0] > 0.0 ? nrm[s + 1] / nrm[0] : 0.0;
  if (h.nonfinite) return fail(GSE_ERR_NONFINITE, "%d non-finite values", h.nonfinite);
  if (h.range_err & 4) return fail(GSE_ERR_ARG, "a sample row lies outside its block");
  if (h.range_err & 1) return fail(GSE_ERR_RANGE, "a shared exponent is below 63");
  if (h.range_err & 2) return fail(GSE_ERR_RANGE, "a value has no larger shared exponent in the table");
  return GSE_OK;
}

gse_status encode_matrix(const int32_t* row_ptr, const int32_t* col, const double* val,
                         int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                         const int16_t* sem_in, gse_matrix* A, void* ws, size_t ws_bytes,
                         hipStream_t st) {
  int layout = 0;
  gse_status cs = check_encode(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, A, ws, ws_bytes,
                               &layout);
  if (cs != GSE_OK) return cs;
  if (sem_in) {
    for (int i = 0; i < num_exp; ++i) {
      if (sem_in[i] < 64 || sem_in[i] > 2047)
        return fail(GSE_ERR_RANGE, "shared exponent %d out of range", (int)sem_in[i]);
      for (int k = 0; k < i; ++k)
        if (sem_in[k] == sem_in[i]) return fail(GSE_ERR_ARG, "duplicate shared exponent");
    }
  }
  EncodeScratch* sc = reinterpret_cast<EncodeScratch*>(ws);
  set_global_fields(row_ptr, n_rows, n_cols, nnz, num_exp, layout, A);
  hipError_t e = launch_encode(row_ptr, col, val, n_rows, (int32_t)nnz, num_exp, sem_in, A, sc, st);
  if (e != hipSuccess) return hip_fail(e, "gse_encode launch");
  return finish_global(row_ptr, n_rows, nnz, A, sc, st, "gse_encode");
}

// One table from the pooled exponents of one drawn row per block
// (Section III-B.1, sampling).
static gse_status encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                                 int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                                 int32_t block_rows, const int32_t* sample_rows, gse_matrix* A,
                                 void* ws, size_t ws_bytes, hipStream_t st) {
  int layout = 0;
  gse_status cs = check_encode(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, A, ws, ws_bytes,
                               &layout);
  if (cs != GSE_OK) return cs;
  if (block_rows < 1) return fail(GSE_ERR_ARG, "block_rows must be positive");
  if (!sample_rows) return fail(GSE_ERR_ARG, "sample_rows is NULL");
  EncodeScratch* sc = reinterpret_cast<EncodeScratch*>(ws);
  set_global_fields(row_ptr, n_rows, n_cols, nnz, num_exp, layout, A);
  hipError_t e = launch_encode_sampled(row_ptr, col, val, n_rows, (int32_t)nnz, num_exp, block_rows,
                                       sample_rows, A, sc, st);
  if (e != hipSuccess) return hip_fail(e, "gse_encode_sampled launch");
  return finish_global(row_ptr, n_rows, nnz, A, sc, st, "gse_encode_sampled");
}

}  // namespace gse

using namespace gse;

extern "C" {

int64_t gse_pad(int64_t nnz) { return nnz < 0 ? 0 : pad_nnz(nnz); }

int32_t gse_tile_entries(int64_t nnz) { return n_tiles_for(nnz < 0 ? 0 : nnz, kMinTile) + 2; }

const char* gse_last_error(void) { return g_err; }

const char* gse_status_str(gse_status s) {
  switch (s) {
    case GSE_OK: return "ok";
    case GSE_PENDING: return "pending";
    case GSE_NOT_CONVERGED: return "not converged";
    case GSE_ERR_ARG: return "invalid argument";
    case GSE_ERR_NONFINITE: return "non-finite value";
    case GSE_ERR_RANGE: return "out of range";
    case GSE_ERR_NOMEM: return "workspace too small";
    case GSE_ERR_BREAKDOWN: return "breakdown";
    case GSE_ERR_HIP: return "HIP error";
    case GSE_ERR_TICKET: return "unknown ticket";
    default: return "unknown status";
  }
}

gse_status gse_encode_workspace(int64_t nnz, int32_t n_rows, size_t* ws_bytes) {
  if (!ws_bytes || nnz < 0 || n_rows < 0) return fail(GSE_ERR_ARG, "bad arguments");
  *ws_bytes = (sizeof(EncodeScratch) + 255) / 256 * 256;
  return GSE_OK;
}

gse_status gse_plan(gse_matrix* A, int32_t tile_nnz, int32_t rv_lanes, void* stream) {
  if (!A || !A->row_ptr || !A->tile_row) return fail(GSE_ERR_ARG, "bad matrix");
  if (A->nnz < 0 || A->nnz > kMaxNnz || A->n_rows < 0) return fail(GSE_ERR_RANGE, "bad sizes");
  int32_t nt, rv, mr;
  gse_status s = plan_common(A->row_ptr, A->n_rows, A->nnz, A->tile_row, A->tile_cap, tile_nnz,
                             rv_lanes, (hipStream_t)stream, &nt, &rv, &mr);
  if (s != GSE_OK) return s;
  A->tile_nnz = tile_nnz;
  A->n_tiles = nt;
  A->rv_lanes = rv;
  if (A->block_rows > 0 && rv_lanes == -1) A->rv_lanes = block_lanes(A->nnz, A->n_rows, mr);
  A->max_row_nnz = mr;
  return GSE_OK;
}

gse_status gse_csr_plan(gse_csr* M, int32_t tile_nnz, int32_t rv_lanes, void* stream) {
  if (!M || !M->row_ptr || !M->tile_row) return fail(GSE_ERR_ARG, "bad matrix");
  if (M->nnz < 0 || M->nnz > kMaxNnz || M->n_rows < 0) return fail(GSE_ERR_RANGE, "bad sizes");
  int32_t nt, rv, mr;
  gse_status s = plan_common(M->row_ptr, M->n_rows, M->nnz, M->tile_row, M->tile_cap, tile_nnz,
                             rv_lanes, (hipStream_t)stream, &nt, &rv, &mr);
  if (s != GSE_OK) return s;
  M->tile_nnz = tile_nnz;
  M->n_tiles = nt;
  M->rv_lanes = rv;
  M->max_row_nnz = mr;
  return GSE_OK;
}

gse_status gse_encode(const int32_t* row_ptr, const int32_t* col, const double* val, int32_t n_rows,
                      int32_t n_cols, int64_t nnz, int32_t num_exp, const int16_t* sem_in,
                      gse_matrix* A, void* ws, size_t ws_bytes, void* stream) {
  return encode_matrix(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, sem_in, A, ws, ws_bytes,
                       (hipStream_t)stream);
}

gse_status gse_encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                             int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                             int32_t block_rows, const int32_t* sample_rows, gse_matrix* A,
                             void* ws, size_t ws_bytes, void* stream) {
  return encode_blocks(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, block_rows, sample_rows, A,
                       ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                              int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                              int32_t block_rows, const int32_t* sample_rows, gse_matrix* A,
                              void* ws, size_t ws_bytes, void* stream) {
  return encode_sampled(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, block_rows, sample_rows, A,
                        ws, ws_bytes, (hipStream_t)stream);
}

int64_t gse_block_table_entries(int32_t n_rows, int32_t block_rows, int32_t num_exp) {
  if (n_rows < 0 || block_rows < 1 || num_exp < 1 || num_exp > GSE_MAX_EXP) return 0;
  const int64_t n_blocks = ((int64_t)n_rows + block_rows - 1) / block_rows;
  return n_blocks * ((int64_t)1 << index_bits(num_exp));
}

gse_status gse_autotune(gse_matrix* A, int32_t k_segments, const double* x, double* y,
                        int32_t reps, void* stream) {
  gse_status s = check_matrix(A);
  if (s != GSE_OK) return s;
  if (k_segments < 1 || k_segments > 3) return fail(GSE_ERR_ARG, "k_segments must be 1..3");
  if (!x || !y || reps < 1) return fail(GSE_ERR_ARG, "x, y and reps >= 1 are required");
  if (A->n_rows == 0) return GSE_OK;
  int32_t t, rv, nt;
  s = autotune(k_segments, k_segments, operand_of(A), A->row_ptr, A->tile_row, A->tile_cap,
               A->max_row_nnz, x, y, reps, (hipStream_t)stream, &t, &rv, &nt);
  if (s != GSE_OK) return s;
  A->tile_nnz = t;
  A->rv_lanes = rv;
  A->n_tiles = nt;
  return GSE_OK;
}

gse_status gse_csr_autotune(gse_csr* M, const double* x, double* y, int32_t reps, void* stream) {
  gse_status s = check_csr(M);
  if (s != GSE_OK) return s;
  if (!x || !y || reps < 1) return fail(GSE_ERR_ARG, "x, y and reps >= 1 are required");
  if (M->n_rows == 0) return GSE_OK;
  int32_t t, rv, nt;
  s = autotune(kCsr64, 0, operand_of(M), M->row_ptr, M->tile_row, M->tile_cap, M->max_row_nnz, x,
               y, reps, (hipStream_t)stream, &t, &rv, &nt);
  if (s != GSE_OK) return s;
  M->tile_nnz = t;
  M->rv_lanes = rv;
  M->n_tiles = nt;
  return GSE_OK;
}

gse_status gse_spmv(const gse_matrix* A, int32_t k_segments, const double* x, double* y, void* stream) {
  gse_status s = check_matrix(A);
  if (s != GSE_OK) return s;
  if (k_segments < 1 || k_segments > 3) return fail(GSE_ERR_ARG, "k_segments must be 1..3");
  s = check_spmv_vectors(A->n_rows, A->n_cols, x, y);
  if (s != GSE_OK) return s;
  if (A->n_rows == 0) return GSE_OK;
  SpmvEpilogue ep{};
  ep.epi = kEpiPlain;
  hipError_t e = launch_spmv(k_segments, operand_of(A), x, y, ep, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gse_spmv");
  return GSE_OK;
}

gse_status gse_csr_spmv(const gse_csr* M, const double* x, double* y, void* stream) {
  gse_status s = check_csr(M);
  if (s != GSE_OK) return s;
  s = check_spmv_vectors(M->n_rows, M->n_cols, x, y);
  if (s != GSE_OK) return s;
  if (M->n_rows == 0) return GSE_OK;
  SpmvEpilogue ep{};
  ep.epi = kEpiPlain;
  hipError_t e = launch_spmv(kCsr64, operand_of(M), x, y, ep, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gse_csr_spmv");
  return GSE_OK;
}

gse_status gse_default_params(int32_t method, gse_params* p) {
  if (!p || (method != GSE_CG && method != GSE_GMRES)) return fail(GSE_ERR_ARG, "bad arguments");
  memset(p, 0, sizeof *p);
  p->tol = 1e-10;
  p->restart = 30;
  p->start_segments = 1;
  p->fixed_segments = 0;
  p->ndec_rule = 0;
  p->floor_c = 10.0;
  p->switch_mode = 2;  // p kept after a switch unless the replacement moves ||r|| by 2x
  p->record_history = 0;
  if (method == GSE_CG) {  // Section IV-A (cap) and IV-D.1 (controller)
    p->max_iter = 5000;
    p->l = 3000;
    p->t = 250;
    p->m = 500;
    p->rsd_limit = 0.50;
    p->ndec_limit = 130;
    p->reldec_limit = 0.45;
  } else {
    p->max_iter = 30 * 500;
    p->l = 9000;
    p->t = 300;
    p->m = 1500;
    p->rsd_limit = 0.03;
    p->ndec_limit = 80;
    p->reldec_limit = 0.08;
  }
  return GSE_OK;
}

gse_status gse_solver_workspace(int32_t method, int32_t n_rows, int64_t nnz, int32_t restart,
                                int32_t max_iter, size_t* ws_bytes) {
  if (!ws_bytes || n_rows < 0 || nnz < 0 || max_iter < 0 ||
      (method != GSE_CG && method != GSE_GMRES) || (method == GSE_GMRES && restart < 1))
    return fail(GSE_ERR_ARG, "bad arguments");
  *ws_bytes = solver_workspace_bytes(method, n_rows, nnz, restart, max_iter);
  return GSE_OK;
}

static gse_status check_solve(int32_t n_rows, int32_t n_cols, const double* b, double* x,
                              const gse_params* p, gse_report* rep, const void* ws, int method) {
  if (!p || !rep) return fail(GSE_ERR_ARG, "params / report is NULL");
  if (n_rows != n_cols) return fail(GSE_ERR_ARG, "the matrix must be square");
  if (n_rows > 0 && (!b || !x)) return fail(GSE_ERR_ARG, "NULL vector");
  if (!aligned16(x)) return fail(GSE_ERR_ARG, "x must be 16-byte aligned");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u))
    return fail(GSE_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (!(p->tol > 0.0) || p->max_iter < 0) return fail(GSE_ERR_ARG, "tol must be > 0, max_iter >= 0");
  if (p->start_segments < 1 || p->start_segments > 3 || p->fixed_segments < 0 || p->fixed_segments > 3)
    return fail(GSE_ERR_ARG, "segment counts must be 1..3 (fixed: 0..3)");
  if (p->l < 0 || p->t < 1 || p->m < 0) return fail(GSE_ERR_ARG, "controller needs l >= 0, t >= 1, m >= 0");
  if (method == GSE_GMRES && p->restart < 1) return fail(GSE_ERR_ARG, "restart must be >= 1");
  return GSE_OK;
}

gse_status gse_cg(const gse_matrix* A, const double* b, double* x, const gse_params* p,
                  gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  gse_status s = check_matrix(A);
  if (s == GSE_OK) s = check_solve(A->n_rows, A->n_cols, b, x, p, rep, ws, GSE_CG);
  if (s != GSE_OK) return s;
  return cg_gse(A, operand_of(A), b, x, p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_csr_cg(const gse_csr* M, const double* b, double* x, const gse_params* p,
                      gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  gse_status s = check_csr(M);
  if (s == GSE_OK) s = check_solve(M->n_rows, M->n_cols, b, x, p, rep, ws, GSE_CG);
  if (s != GSE_OK) return s;
  return cg_csr(operand_of(M), b, x, p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_gmres(const gse_matrix* A, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  gse_status s = check_matrix(A);
  if (s == GSE_OK) s = check_solve(A->n_rows, A->n_cols, b, x, p, rep, ws, GSE_GMRES);
  if (s != GSE_OK) return s;
  return gmres_gse(A, operand_of(A), b, x, p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_csr_gmres(const gse_csr* M, const double* b, double* x, const gse_params* p,
                         gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  gse_status s = check_csr(M);
  if (s == GSE_OK) s = check_solve(M->n_rows, M->n_cols, b, x, p, rep, ws, GSE_GMRES);
  if (s != GSE_OK) return s;
  return gmres_csr(operand_of(M), b, x, p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_lp_cg(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  gse_status s = check_lp(M);
  if (s == GSE_OK) s = check_solve(M->n_rows, M->n_cols, b, x, p, rep, ws, GSE_CG);
  if (s != GSE_OK) return s;
  return cg_lp(M, b, x, p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_lp_gmres(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                        gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  gse_status s = check_lp(M);
  if (s == GSE_OK) s = check_solve(M->n_rows, M->n_cols, b, x, p, rep, ws, GSE_GMRES);
  if (s != GSE_OK) return s;
  return gmres_lp(M, b, x, p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_solve_history(const void* ws, int32_t cap, double* hist, int32_t* seg, void* stream) {
  if (!ws || cap < 0 || (cap > 0 && (!hist || !seg))) return fail(GSE_ERR_ARG, "bad arguments");
  if (cap == 0) return GSE_OK;
  return solve_history(ws, cap, hist, seg, (hipStream_t)stream);
}

static gse_status batch_descs(int32_t n_sys, const gse_system* sys, const gse_params* p,
                              std::vector<BatchSystemDesc>* out) {
  if (n_sys < 1 || !sys || !p) return fail(GSE_ERR_ARG, "bad arguments");
  if (!(p->tol > 0.0) || p->max_iter < 0) return fail(GSE_ERR_ARG, "tol must be > 0, max_iter >= 0");
  if (p->start_segments < 1 || p->start_segments > 3 || p->fixed_segments < 0 || p->fixed_segments > 3)
    return fail(GSE_ERR_ARG, "segment counts must be 1..3 (fixed: 0..3)");
  if (p->l < 0 || p->t < 1 || p->m < 0) return fail(GSE_ERR_ARG, "controller needs l >= 0, t >= 1, m >= 0");
  out->clear();
  for (int i = 0; i < n_sys; ++i) {
    const gse_system& y = sys[i];
    if ((y.A == nullptr) == (y.M == nullptr))
      return fail(GSE_ERR_ARG, "system %d: give exactly one of A and M", i);
    BatchSystemDesc d{};
    BatchSlot& B = d.slot;
    gse_status s;
    if (y.A) {
      s = check_matrix(y.A);
      if (s != GSE_OK) return s;
      const gse_matrix* A = y.A;
      if (A->n_rows != A->n_cols || A->n_rows < 1)
        return fail(GSE_ERR_ARG, "system %d: the matrix must be square and non-empty", i);
      if (A->block_rows != 0)
        return fail(GSE_ERR_ARG, "system %d: per-block tables are not taken by the batched solver", i);
      B.row_ptr = A->row_ptr;
      B.tile_row = A->tile_row;
      B.col = A->col_idx;
      B.head = A->head;
      B.tail1 = A->tail1;
      B.tail2 = A->tail2;
      B.n_rows = A->n_rows;
      B.n_tiles = A->n_tiles;
      B.fmt = 1;
      B.max_row = A->max_row_nnz;
      B.split = col_split(A->idx_bits, A->idx_layout == GSE_IDX_VALUE);
      for (int k = 0; k < GSE_MAX_EXP; ++k) B.sem[k] = A->sem[k];
      B.nnz = (int32_t)A->nnz;
      B.tile_nnz = A->tile_nnz;
      B.rv_lanes = A->rv_lanes;
      d.eta = A->eta;
    } else {
      s = check_csr(y.M);
      if (s != GSE_OK) return s;
      const gse_csr* M = y.M;
      if (M->n_rows != M->n_cols || M->n_rows < 1)
        return fail(GSE_ERR_ARG, "system %d: the matrix must be square and non-empty", i);
      B.row_ptr = M->row_ptr;
      B.tile_row = M->tile_row;
      B.col = reinterpret_cast<const uint32_t*>(M->col);
      B.val = M->val;
      B.n_rows = M->n_rows;
      B.n_tiles = M->n_tiles;
      B.fmt = 0;
      B.max_row = M->max_row_nnz;
      B.split = col_split(0);
      B.nnz = (int32_t)M->nnz;
      B.tile_nnz = M->tile_nnz;
      B.rv_lanes = M->rv_lanes;
      d.eta = nullptr;
    }
    if (!y.b || !y.x || !aligned16(y.x)) return fail(GSE_ERR_ARG, "system %d: bad b / x", i);
    B.b = y.b;
    B.x = y.x;
    d.n_rows = B.n_rows;
    d.n_tiles = B.n_tiles;
    out->push_back(d);
  }
  return GSE_OK;
}

gse_status gse_batch_workspace(int32_t n_sys, const gse_system* sys, const gse_params* p,
                               size_t* ws_bytes) {
  if (!ws_bytes) return fail(GSE_ERR_ARG, "ws_bytes is NULL");
  std::vector<BatchSystemDesc> d;
  gse_status s = batch_descs(n_sys, sys, p, &d);
  if (s != GSE_OK) return s;
  *ws_bytes = batch_workspace_bytes(n_sys, d.data(), p->max_iter);
  return GSE_OK;
}

gse_status gse_batch_cg(int32_t n_sys, const gse_system* sys, const gse_params* p,
                        gse_report* rep, void* ws, size_t ws_bytes, void* stream) {
  std::vector<BatchSystemDesc> d;
  gse_status s = batch_descs(n_sys, sys, p, &d);
  if (s != GSE_OK) return s;
  if (!rep) return fail(GSE_ERR_ARG, "reports are NULL");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u))
    return fail(GSE_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  return batch_cg(n_sys, d.data(), p, rep, ws, ws_bytes, (hipStream_t)stream);
}

gse_status gse_batch_history(const void* ws, int32_t index, int32_t cap, double* hist,
                             int32_t* seg, void* stream) {
  if (!ws || cap < 0 || (cap > 0 && (!hist || !seg))) return fail(GSE_ERR_ARG, "bad arguments");
  if (cap == 0) return GSE_OK;
  return batch_history(ws, index, cap, hist, seg, (hipStream_t)stream);
}

gse_status gse_stream_reduce8(const double* src, double* dst, size_t n_out, void* stream) {
  if (!src || !dst || !aligned16(src) || !aligned16(dst))
    return fail(GSE_ERR_ARG, "reduce needs 16-byte aligned buffers");
  if (n_out == 0) return GSE_OK;
  hipError_t e = launch_stream_reduce8(src, dst, n_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gse_stream_reduce8");
  return GSE_OK;
}

gse_status gse_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || (bytes & 15u) || !aligned16(src) || !aligned16(dst))
    return fail(GSE_ERR_ARG, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
  if (bytes == 0) return GSE_OK;
  hipError_t e = launch_stream_copy(src, dst, bytes, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gse_stream_copy");
  return GSE_OK;
}

}  // extern "C"

// gse_internal.h -- device helpers and launcher declarations shared by the
// translation units of libgse (never installed; the public ABI is gse.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gse.h"

namespace gse {

constexpr int kWG = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kWG / 64;
constexpr int kMinTile = 1024;      // smallest tile_nnz the schedule may use
constexpr int kDefaultTile = 1024;
constexpr int kExtra = 256;         // look-ahead elements staged for a crossing row
constexpr int kPadTo = 16;          // planes hold nnz rounded up to this
constexpr int kShortRow = 24;       // rows up to this length: one thread, serial sum
constexpr int kSpec = 16;           // look-ahead non-zeros loaded before the row lookup
constexpr int kRowStage = 1024;     // row pointers staged in LDS per tile
constexpr int kRvBatch = 8;         // row-vector schedule: rows per lane group in flight
constexpr int64_t kMaxNnz = (int64_t(1) << 31) - (int64_t(1) << 16);

// Format identifiers for the SpMV templates: 1..3 = GSE-SEM with s segments,
// 0 = plain FP64 CSR values, 4 / 5 = the FP16 / BF16 comparators (one 16-bit
// value per non-zero in the head plane, bare column words).
constexpr int kCsr64 = 0;
constexpr int kFp16 = 4;
constexpr int kBf16 = 5;

// Planes a format reads besides the column words: 0 the FP64 values, 1 the
// 16-bit plane (GSE head, FP16, BF16), 2 head + tail1, 3 all three.
__host__ __device__ constexpr int planes_of(int fmt) {
  return fmt == kCsr64 ? 0 : (fmt >= kFp16 ? 1 : fmt);
}
__host__ __device__ constexpr bool is_gse(int fmt) { return fmt >= 1 && fmt <= 3; }

// Epilogue of an SpMV launch.
enum Epi : int {
  kEpiPlain = 0,  // y = A x
  kEpiDot = 1,    // y = A x, and the dot x.y over the launch
  kEpiResid = 2,  // y = b - A x, and y.y
};

// ---------------------------------------------------------------- helpers --
// Workgroup id -> tile id so that every XCD (8 per MI355X, workgroups handed
// out round-robin) works on one contiguous range of tiles: neighbouring tiles
// share x entries, which then stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int wg, int n_wg) {
  const int per = n_wg >> 3, rem = n_wg & 7;
  const int xcd = wg & 7, local = wg >> 3;
  return (xcd < rem) ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum (fixed tree) over a workgroup of NT threads;
// every thread gets the result.
template <int NT = kWG>
__device__ __forceinline__ double block_sum(double v, double* red /* [NT / 64] */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Sum of partials[0..n) by one workgroup in a fixed order (every thread
// gets the result).  The partials come from an earlier kernel on the same
// stream, so the launch boundary has made them visible.
__device__ __forceinline__ double sum_partials(const double* partials, int n, double* red) {
  // Thread t adds entries t, t + kWG, t + 2 kWG, ... in that order, then
  // the block sum.  Eight strides are loaded before any is added (indices
  // past n clamped to a valid entry, their additions masked): a plain loop
  // waits for each load before issuing the next.
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 8 * kWG) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = i + k * kWG;
      v[k] = partials[e < n ? e : i];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) s = (i + k * kWG < n) ? s + v[k] : s;
  }
  return block_sum(s, red);
}

__device__ __forceinline__ double bits_to_double(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ uint64_t double_to_bits(double d) { return (uint64_t)__double_as_longlong(d); }

// ------------------------------------------------------- column words --
// With k shared exponents the slot index takes the top b = ceil(log2 k) bits
// of the 32-bit column word (b = 0: the word is the bare column).
__host__ __device__ inline int index_bits(int num_exp) {
  int b = 0;
  while ((1 << b) < num_exp) ++b;
  return b;
}

// Where a non-zero's column and slot are: column = word & col_mask; slot =
// ((word >> shift) & slot_mask) | ((head >> hshift) & hmask) -- one of the
// two masks is zero: the slot is in the top of the column word (shift
// 32 - b), or in the head below the sign (hshift 15 - b, Algorithm 1's
// EI_bit).  mag_mask keeps the head's magnitude bits (15 - ei of them) and
// ei shortens W_s.  b = 0: no index at all; the FP64 CSR operand's words
// are bare columns.
struct ColSplit {
  uint32_t shift;
  uint32_t slot_mask;
  uint32_t col_mask;
  uint32_t hshift;
  uint32_t hmask;
  uint32_t mag_mask;
  int32_t ei;
};

__host__ __device__ inline ColSplit col_split(int idx_bits, bool in_value = false) {
  ColSplit c;
  if (in_value) {
    c.shift = 0u;
    c.slot_mask = 0u;
    c.col_mask = 0xFFFFFFFFu;
    c.hshift = 15u - (uint32_t)idx_bits;
    c.hmask = (1u << idx_bits) - 1u;
    c.mag_mask = 0x7FFFu >> idx_bits;
    c.ei = idx_bits;
  } else {
    c.shift = idx_bits > 0 ? 32u - (uint32_t)idx_bits : 0u;
    c.slot_mask = (1u << idx_bits) - 1u;
    c.col_mask = 0xFFFFFFFFu >> idx_bits;
    c.hshift = 0u;
    c.hmask = 0u;
    c.mag_mask = 0x7FFFu;
    c.ei = 0;
  }
  return c;
}

// Scale table entries: one per slot.
constexpr int kScaleEntries = GSE_MAX_EXP;

// Per-row-block tables: the row-vector workgroup stages the tables of every
// block its rows touch.  A workgroup holds at most 2048 rows (one lane per
// row) and a block at least GSE_MIN_BLOCK_ROWS, so it touches at most
// (2048 - 1) / GSE_MIN_BLOCK_ROWS + 2 blocks of up to 64 entries each.
constexpr int kRvMaxRows = 64 * kRvBatch * kWaves;
constexpr int kBlockTabEntries = ((kRvMaxRows - 1) / GSE_MIN_BLOCK_ROWS + 2) * GSE_MAX_EXP;

// ------------------------------------------------------------- launchers --
struct SpmvOperand {
  // GSE planes (fmt 1..3) or CSR values (fmt 0)
  const int32_t* row_ptr;
  const int32_t* tile_row;
  const uint32_t* col;       // col | slot << (32 - b) (GSE) or plain column (CSR)
  const uint16_t* head;
  const uint16_t* tail1;
  const uint32_t* tail2;
  const double* val;
  int32_t n_rows;
  int32_t n_tiles;
  int32_t tile_nnz;
  int32_t nnz;
  int32_t rv_lanes;          // > 0: row-vector schedule with this many lanes per row
  int32_t max_row;           // longest row (<= kShortRow selects the short-row tiles)
  ColSplit split;            // column / slot fields of the column words
  int16_t sem[GSE_MAX_EXP];
  // per-row-block tables (null: the one table `sem`): row r reads
  // block_sem[(r / block_rows) * block_stride + slot]; row-vector schedule only
  const int16_t* block_sem;
  int32_t block_rows;
  int32_t block_stride;
};

struct SpmvEpilogue {
  int epi;                 // Epi
  const double* aux;       // kEpiDot: vector dotted with y (x itself for CG); kEpiResid: b
  double* partials;        // [grid] per-workgroup partial dots (kEpiDot / kEpiResid)
  const int* gate;         // if non-null and *gate != 0 the launch does nothing
  int* grid_out;           // host: receives the number of workgroups (= partials written)
};

hipError_t launch_spmv(int fmt, const SpmvOperand& A, const double* x, double* y,
                       const SpmvEpilogue& ep, hipStream_t st);

// One operand of a grouped row-tile launch (a device array the host fills):
// operand, vectors, epilogue (grid_out unused) and the launch's workgroups
// [wg0, wg0 + wgs) that run the operand's plain-launch grid.
struct RowGroup {
  SpmvOperand A;
  const double* x;
  double* y;
  SpmvEpilogue ep;
  int32_t wg0, wgs;
};

// The row-tile ring instance that launch_spmv(fmt, A, ...) runs -- row bound
// B, index layout IB (3: the 3-bit column-word split fixed at compile time,
// -1: read from the operand) -- and its grid.  False when A takes another
// schedule (rows past 8 non-zeros, another tile size, lanes per row, block
// tables, fewer than 1024 non-zeros).
struct RowClass {
  int fmt, B, IB, grid;
};
bool rows_class(int fmt, const SpmvOperand& A, RowClass* out);
// One dispatch over n_groups operands of class c whose ranges ascend and
// cover [0, total) workgroups.
hipError_t launch_rows_grouped(const RowClass& c, const RowGroup* groups, int n_groups, int total,
                               hipStream_t st);
hipError_t launch_plan(const int32_t* row_ptr, int32_t n_rows, int32_t nnz, int32_t tile_nnz,
                       int32_t n_tiles, int32_t* tile_row, hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
hipError_t launch_stream_reduce8(const double* src, double* dst, size_t n_out, hipStream_t st);
hipError_t launch_rowmax(const int32_t* row_ptr, int32_t n_rows, int* out, hipStream_t st);

// Device record of gse_encode (lives at the start of the encode workspace).
struct EncodeScratch {
  uint32_t hist[2048];
  int8_t slot_of[2048];  // slot of the smallest shared exponent above each field; -1: none
  int32_t nonfinite;
  int32_t range_err;
  int32_t used;
  int32_t max_field;  // pooled-sample encode: the matrix's largest finite exponent field
  int16_t sem[GSE_MAX_EXP];
  unsigned long long covered;
  unsigned long long norm_bits[4];  // max row sums |a|, |a - a_1|, |a - a_2|, |a - a_3| (as bits)
};

hipError_t launch_encode(const int32_t* row_ptr, const int32_t* col, const double* val,
                         int32_t n_rows, int32_t nnz, int32_t num_exp, const int16_t* sem_in,
                         gse_matrix* A, EncodeScratch* sc, hipStream_t st);
// Per-row-block tables: one workgroup per block chooses its table (from the
// block's values, or from sample_rows[b] when given), encodes the block, then
// the perturbations with every row's own table.
hipError_t launch_encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                                int32_t n_rows, int32_t nnz, int32_t num_exp,
                                const int32_t* sample_rows, gse_matrix* A, EncodeScratch* sc,
                                hipStream_t st);

// One table for the matrix from the pooled exponents of one drawn row per
// block of block_rows rows (sample_rows[b] in block b), the matrix's largest
// exponent added when missed; then the planes and perturbations of the
// global encoder.
hipError_t launch_encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                                 int32_t n_rows, int32_t nnz, int32_t num_exp, int32_t block_rows,
                                 const int32_t* sample_rows, gse_matrix* A, EncodeScratch* sc,
                                 hipStream_t st);

int32_t n_tiles_for(int64_t nnz, int32_t tile_nnz);

// api.hip: gse_encode on a scratch record `ws` of ws_bytes (validation,
// launches, table read-back, default plan).
gse_status encode_matrix(const int32_t* row_ptr, const int32_t* col, const double* val,
                         int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                         const int16_t* sem_in, gse_matrix* A, void* ws, size_t ws_bytes,
                         hipStream_t st);
gse_status fail(gse_status code, const char* fmt, ...);
gse_status check_spmv_vectors(int32_t n_rows, int32_t n_cols, const double* x, const double* y);
gse_status hip_fail(hipError_t e, const char* where);

// autotune.hip: time the schedules, plan the fastest (tile_row rewritten)
gse_status autotune(int fmt, int segs, SpmvOperand op, const int32_t* row_ptr, int32_t* tile_row,
                    int32_t tile_cap, int32_t max_row, const double* x, double* y, int32_t reps,
                    hipStream_t st, int32_t* out_tile, int32_t* out_rv, int32_t* out_tiles);

// lowprec.hip: the FP16 / BF16 operand
SpmvOperand operand_of(const gse_lp_matrix* M);
int lp_launch_format(const gse_lp_matrix* M);
gse_status check_lp(const gse_lp_matrix* M);

// solvers.hip
size_t solver_workspace_bytes(int32_t method, int32_t n_rows, int64_t nnz, int32_t restart,
                              int32_t max_iter);
gse_status cg_gse(const gse_matrix* A, const SpmvOperand& op, const double* b, double* x,
                  const gse_params* p, gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st);
gse_status cg_csr(const SpmvOperand& op, const double* b, double* x, const gse_params* p,
                  gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st);
gse_status cg_lp(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                 gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st);
gse_status gmres_lp(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                    gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st);
gse_status gmres_gse(const gse_matrix* A, const SpmvOperand& op, const double* b, double* x,
                     const gse_params* p, gse_report* rep, void* ws, size_t ws_bytes,
                     hipStream_t st);
gse_status gmres_csr(const SpmvOperand& op, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st);
gse_status solve_history(const void* ws, int32_t cap, double* hist, int32_t* seg, hipStream_t st);

}  // namespace gse

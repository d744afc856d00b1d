// lowprec.hip -- the FP16 / BF16 comparators of Section IV-C: every value
// of an FP64 CSR matrix stored as one IEEE binary16 or bfloat16 word next to
// its plain column (the same 6 bytes per non-zero as the head-only GSE-SEM
// operator), widened to FP64 in the SpMV and multiplied / accumulated in
// FP64; CG and GMRES run on that fixed operator (Section IV-D.3).
//
//   k_lp_convert  per value: round to nearest, ties to even, from the FP64
//                 bits (integer arithmetic: guard bit and sticky bits of the
//                 53-bit significand); a magnitude that rounds past the
//                 largest finite value becomes an infinity and is counted.
//   k_lp_eta      per row: sums of |a| and |a - a_h|; the row maxima give
//                 eta_h = ||A - A_h||_inf / ||A||_inf.
#include <string.h>

#include "decode.h"
#include "gse_internal.h"

namespace gse {

gse_status fail(gse_status code, const char* fmt, ...);
gse_status hip_fail(hipError_t e, const char* where);
gse_status plan_common(const int32_t* row_ptr, int32_t n_rows, int64_t nnz, int32_t* tile_row,
                       int32_t tile_cap, int32_t tile_nnz, int32_t rv_lanes, hipStream_t st,
                       int32_t* out_tiles, int32_t* out_rv, int32_t* out_maxrow);
bool aligned16(const void* p);

namespace {

// FP64 bits -> a binary format with EB exponent and MB fraction bits,
// rounded to nearest with ties to even.  Returns the 16-bit word (sign in
// bit 15); *inf is set when a finite value overflowed.
template <int EB, int MB>
__device__ __forceinline__ uint32_t round_bits(uint64_t u, bool* inf) {
  constexpr int BIAS = (1 << (EB - 1)) - 1;
  constexpr uint32_t EMAXF = (1u << EB) - 1u;  // all-ones exponent field
  const uint32_t sign = (uint32_t)(u >> 63) << (EB + MB);
  const int E = (int)((u >> 52) & 0x7FF);
  *inf = false;
  if (E == 0) return sign;  // FP64 zero or subnormal: far below either format's range
  const uint64_t sig = (u & ((uint64_t(1) << 52) - 1)) | (uint64_t(1) << 52);
  const int te = E - 1023 + BIAS;  // biased exponent in the target
  // right shift that leaves the kept bits: MB fraction bits (+ the hidden
  // one) for normals, fewer below the target's normal range
  const int sh = (52 - MB) + (te >= 1 ? 0 : 1 - te);
  if (sh > 62) return sign;  // below half the smallest subnormal: rounds to zero
  uint64_t q = sig >> sh;
  const uint64_t rem = sig & ((uint64_t(1) << sh) - 1);
  const uint64_t half = uint64_t(1) << (sh - 1);
  if (rem > half || (rem == half && (q & 1))) ++q;
  uint32_t mag;
  if (te >= 1) {
    int e = te;
    if (q == (uint64_t(1) << (MB + 1))) {  // rounded up to the next binade
      q >>= 1;
      ++e;
    }
    if (e >= (int)EMAXF) {
      *inf = true;
      mag = EMAXF << MB;
    } else {
      mag = ((uint32_t)e << MB) | ((uint32_t)q & ((1u << MB) - 1u));
    }
  } else {
    mag = (uint32_t)q;  // subnormal; q == 2^MB is the smallest normal's encoding
  }
  return sign | mag;
}

// Groups of 8 values per thread: 16-byte stores of the value and column planes
// (the planes are padded, so the tail group writes zeros past nnz).
template <int FMT>
__global__ __launch_bounds__(256) void k_lp_convert(const double* __restrict__ val,
                                                    const int32_t* __restrict__ col, int nnz,
                                                    uint16_t* __restrict__ out_val,
                                                    int32_t* __restrict__ out_col,
                                                    unsigned long long* __restrict__ overflow) {
  const int n_groups = (nnz + 7) >> 3;
  const int stride = gridDim.x * blockDim.x;
  unsigned cnt = 0;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups; g += stride) {
    uint64_t uv[8];
    int cv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = g * 8 + k;
      uv[k] = j < nnz ? double_to_bits(val[j]) : 0u;
      cv[k] = j < nnz ? col[j] : 0;
    }
    uint32_t hw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      bool inf;
      const uint32_t h = (FMT == kFp16) ? round_bits<5, 10>(uv[k], &inf)
                                        : round_bits<8, 7>(uv[k], &inf);
      cnt += inf ? 1u : 0u;
      hw[k >> 1] |= h << ((k & 1) * 16);
    }
    *reinterpret_cast<uint4*>(out_val + g * 8) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    int4* cp = reinterpret_cast<int4*>(out_col + g * 8);
    cp[0] = make_int4(cv[0], cv[1], cv[2], cv[3]);
    cp[1] = make_int4(cv[4], cv[5], cv[6], cv[7]);
  }
  if (cnt) atomicAdd(overflow, (unsigned long long)cnt);
}

// One row per eight lanes: |a| and |a - a_h| summed per row, their maxima
// over the grid merged into norm_bits[0..1] (bit patterns of non-negative
// doubles order like the values).  An overflowed value gives an infinite
// difference, so eta_h = inf.
template <int FMT>
__global__ __launch_bounds__(256) void k_lp_eta(const int32_t* __restrict__ row_ptr, int n_rows,
                                                const double* __restrict__ val,
                                                const uint16_t* __restrict__ h16,
                                                unsigned long long* norm_bits) {
  __shared__ double red[2][kWaves];
  const int sub = threadIdx.x & 7;
  const int grp = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int ngrp = (gridDim.x * blockDim.x) >> 3;
  const DecodeCtx none{nullptr, col_split(0)};
  double m0 = 0.0, m1 = 0.0;
  for (int r = grp; r < n_rows; r += ngrp) {
    double a = 0.0, d = 0.0;
    for (int j = row_ptr[r] + sub; j < row_ptr[r + 1]; j += 8) {
      int c;
      const double w = decode<FMT>(0u, h16[j], 0u, 0u, 0.0, none, c);
      a += fabs(val[j]);
      d += fabs(val[j] - w);
    }
#pragma unroll
    for (int off = 4; off >= 1; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      d += __shfl_xor(d, off, 64);
    }
    m0 = fmax(m0, a);
    m1 = fmax(m1, d);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    m0 = fmax(m0, __shfl_xor(m0, off, 64));
    m1 = fmax(m1, __shfl_xor(m1, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = m0;
    red[1][threadIdx.x >> 6] = m1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, red[threadIdx.x][w]);
    atomicMax(&norm_bits[threadIdx.x], (unsigned long long)double_to_bits(t));
  }
}

__global__ void k_lp_zero(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Record of one conversion: the two row-sum maxima and the overflow count.
struct LpScratch {
  unsigned long long norm_bits[2];
  unsigned long long overflow;
  unsigned long long pad;
};

template <int FMT>
hipError_t launch_lp(const int32_t* row_ptr, const int32_t* col, const double* val, int32_t n_rows,
                     int32_t nnz, gse_lp_matrix* M, LpScratch* sc, hipStream_t st) {
  hipLaunchKernelGGL(k_lp_zero, dim3(1), dim3(64), 0, st,
                     reinterpret_cast<unsigned long long*>(sc), 4);
  const int groups = (nnz + 7) / 8;
  int eb = (groups + 255) / 256;
  eb = eb < 1 ? 1 : (eb > 16384 ? 16384 : eb);
  hipLaunchKernelGGL(k_lp_convert<FMT>, dim3(eb), dim3(256), 0, st, val, col, nnz, M->val, M->col,
                     &sc->overflow);
  int rb = (n_rows + 31) / 32;
  rb = rb < 1 ? 1 : (rb > 4096 ? 4096 : rb);
  hipLaunchKernelGGL(k_lp_eta<FMT>, dim3(rb), dim3(256), 0, st, row_ptr, n_rows, val, M->val,
                     sc->norm_bits);
  return hipGetLastError();
}

}  // namespace

SpmvOperand operand_of(const gse_lp_matrix* M) {
  SpmvOperand o{};
  o.row_ptr = M->row_ptr;
  o.tile_row = M->tile_row;
  o.col = reinterpret_cast<const uint32_t*>(M->col);
  o.head = M->val;
  o.tail1 = nullptr;
  o.tail2 = nullptr;
  o.val = nullptr;
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

int lp_launch_format(const gse_lp_matrix* M) { return M->fmt == GSE_LP_FP16 ? kFp16 : kBf16; }

gse_status check_lp(const gse_lp_matrix* M) {
  if (!M) return fail(GSE_ERR_ARG, "matrix is NULL");
  if (M->fmt != GSE_LP_FP16 && M->fmt != GSE_LP_BF16) return fail(GSE_ERR_ARG, "unknown 16-bit format");
  if (!M->row_ptr || !M->col || !M->val || !M->tile_row)
    return fail(GSE_ERR_ARG, "matrix has a NULL device buffer");
  if (M->n_rows < 0 || M->n_cols < 0 || M->nnz < 0) return fail(GSE_ERR_ARG, "negative size");
  if (M->nnz > kMaxNnz) return fail(GSE_ERR_RANGE, "nnz exceeds the limit");
  if (M->n_tiles != n_tiles_for(M->nnz, M->tile_nnz) || M->tile_cap < M->n_tiles + 2)
    return fail(GSE_ERR_ARG, "matrix has no valid SpMV schedule (call gse_lp_convert / gse_lp_plan)");
  return GSE_OK;
}

}  // namespace gse

using namespace gse;

extern "C" {

gse_status gse_lp_workspace(size_t* ws_bytes) {
  if (!ws_bytes) return fail(GSE_ERR_ARG, "ws_bytes is NULL");
  *ws_bytes = 256;
  return GSE_OK;
}

gse_status gse_lp_convert(const int32_t* row_ptr, const int32_t* col, const double* val,
                          int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t fmt,
                          gse_lp_matrix* M, void* ws, size_t ws_bytes, void* stream) {
  if (!M) return fail(GSE_ERR_ARG, "matrix is NULL");
  if (fmt != GSE_LP_FP16 && fmt != GSE_LP_BF16) return fail(GSE_ERR_ARG, "fmt must be GSE_LP_FP16 or GSE_LP_BF16");
  if (!row_ptr || (nnz > 0 && (!col || !val))) return fail(GSE_ERR_ARG, "NULL CSR array");
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(GSE_ERR_ARG, "negative size");
  if (nnz > kMaxNnz) return fail(GSE_ERR_RANGE, "nnz %lld exceeds the limit", (long long)nnz);
  if (!M->col || !M->val || !M->tile_row) return fail(GSE_ERR_ARG, "planes / tile_row not set");
  if (!aligned16(M->col) || !aligned16(M->val)) return fail(GSE_ERR_ARG, "planes must be 16-byte aligned");
  if (M->tile_cap < gse_tile_entries(nnz))
    return fail(GSE_ERR_NOMEM, "tile_row holds %d < %d entries", M->tile_cap, gse_tile_entries(nnz));
  if (!ws || ws_bytes < sizeof(LpScratch) || (reinterpret_cast<uintptr_t>(ws) & 255u))
    return fail(GSE_ERR_NOMEM, "workspace of gse_lp_workspace() bytes, 256-byte aligned, is required");
  hipStream_t st = (hipStream_t)stream;
  M->n_rows = n_rows;
  M->n_cols = n_cols;
  M->nnz = nnz;
  M->fmt = fmt;
  M->row_ptr = row_ptr;
  LpScratch* sc = reinterpret_cast<LpScratch*>(ws);
  hipError_t e = fmt == GSE_LP_FP16
                     ? launch_lp<kFp16>(row_ptr, col, val, n_rows, (int32_t)nnz, M, sc, st)
                     : launch_lp<kBf16>(row_ptr, col, val, n_rows, (int32_t)nnz, M, sc, st);
  if (e != hipSuccess) return hip_fail(e, "gse_lp_convert launch");
  LpScratch h;
  e = hipMemcpyAsync(&h, sc, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_lp_convert");
  int32_t nt, rv, mr;
  gse_status ps = plan_common(row_ptr, n_rows, nnz, M->tile_row, M->tile_cap, kDefaultTile, -1, st,
                              &nt, &rv, &mr);
  if (ps != GSE_OK) return ps;
  M->tile_nnz = kDefaultTile;
  M->n_tiles = nt;
  M->rv_lanes = rv;
  M->max_row_nnz = mr;
  M->overflow = (int64_t)h.overflow;
  double a, d;
  memcpy(&a, &h.norm_bits[0], sizeof a);
  memcpy(&d, &h.norm_bits[1], sizeof d);
  M->eta = a > 0.0 ? d / a : 0.0;
  return GSE_OK;
}

gse_status gse_lp_plan(gse_lp_matrix* M, int32_t tile_nnz, int32_t rv_lanes, void* stream) {
  if (!M || !M->row_ptr || !M->tile_row) return fail(GSE_ERR_ARG, "bad matrix");
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

gse_status gse_lp_spmv(const gse_lp_matrix* M, const double* x, double* y, void* stream) {
  gse_status s = check_lp(M);
  if (s != GSE_OK) return s;
  s = check_spmv_vectors(M->n_rows, M->n_cols, x, y);
  if (s != GSE_OK) return s;
  if (M->n_rows == 0) return GSE_OK;
  SpmvEpilogue ep{};
  ep.epi = kEpiPlain;
  hipError_t e = launch_spmv(lp_launch_format(M), operand_of(M), x, y, ep, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "gse_lp_spmv");
  return GSE_OK;
}

}  // extern "C"

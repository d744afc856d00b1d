// spmv.hip -- SpMV over GSE-SEM planes (1, 2 or 3 segments) and plain FP64
// CSR, for gfx950.
//
// Operators: Algorithm 2 (head only) and the head+tail1, head+tail1+tail2
// variants of Section III-C.2; values are widened to FP64 and multiplied and
// accumulated in FP64.  The decode is exact and needs no leading-one search:
// the magnitude field F (15, 31 or 63 bits) converts exactly to FP64 and is
// scaled by the signed power of two +-2^(SEM - 1023 - W) held in LDS.
//
// Schedule (the same for every format, so the FP64 baseline and the GSE
// operators differ only in what they load):
//   * tile t owns the non-zero range [t*T, (t+1)*T), T = 256*E; the rows it
//     writes are those whose first non-zero lies in that range
//     (tile_row[t] .. tile_row[t+1]-1, from gse_plan);
//   * phase 1: every lane loads E consecutive non-zeros with 16-byte vector
//     loads from each plane (fully coalesced), decodes, gathers x and stores
//     the FP64 products in LDS; up to kExtra non-zeros past the tile are
//     staged too when the tile's last row runs over its end;
//   * phase 2: rows of up to kShortRow non-zeros are summed by one thread in
//     row order (the order of the sequential definition);
//   * phase 3: longer rows staged in LDS are summed by one wave each;
//   * phase 4: a row that runs more than kExtra past the tile is summed by the
//     whole workgroup, reading the rest from memory.
// Every sum has a fixed order, so results are bit-reproducible and identical
// whether a matrix runs alone or next to others.
#include "gse_internal.h"

namespace gse {
namespace {

template <int N>
struct Words {
  uint32_t w[N];
};

// Load N 32-bit words from a 16-byte aligned (N % 4 == 0) or 8-byte aligned
// (N == 2) address.
template <int N>
__device__ __forceinline__ Words<N> load_words(const void* p) {
  Words<N> r;
  if constexpr (N % 4 == 0) {
    const uint4* q = reinterpret_cast<const uint4*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const uint4 v = q[i];
      r.w[4 * i + 0] = v.x;
      r.w[4 * i + 1] = v.y;
      r.w[4 * i + 2] = v.z;
      r.w[4 * i + 3] = v.w;
    }
  } else {
    static_assert(N == 2, "unsupported vector width");
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    r.w[0] = v.x;
    r.w[1] = v.y;
  }
  return r;
}

template <int N>
__device__ __forceinline__ uint32_t u16_of(const Words<N>& w, int k) {
  return (w.w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
}

// Signed scale table for s segments: entry (slot | sign << 3) holds
// +-2^(SEM[slot] - 1023 - W_s).  Built as IEEE bits: biased exponent
// SEM - W_s, zero fraction (SEM >= 64 keeps it normal).
template <int FMT>
__device__ __forceinline__ void build_scale(const SpmvOperand& A, double* scale) {
  if constexpr (FMT != kCsr64) {
    constexpr int W = (FMT == 1) ? 15 : (FMT == 2) ? 31 : 63;
    const int i = threadIdx.x;
    if (i < 16) {
      const int S = A.sem[i & 7];
      uint64_t u = 0;
      if (S > W) u = (uint64_t)(S - W) << 52;
      u |= (uint64_t)(i >> 3) << 63;
      scale[i] = bits_to_double(u);
    }
  }
}

// Decode one non-zero: returns the FP64 value and its column.
template <int FMT>
__device__ __forceinline__ double decode(uint32_t c, uint32_t h, uint32_t t1, uint32_t t2, double v,
                                         const double* scale, int& column) {
  if constexpr (FMT == kCsr64) {
    column = (int)c;
    return v;
  } else {
    column = (int)(c & 0x1FFFFFFFu);
    const int ti = (int)(c >> 29) | (int)((h >> 12) & 8u);
    const double sc = scale[ti];
    if constexpr (FMT == 1) {
      return (double)(h & 0x7FFFu) * sc;
    } else if constexpr (FMT == 2) {
      return (double)(((h & 0x7FFFu) << 16) | t1) * sc;
    } else {
      // F = hi * 2^32 + lo with hi = 31 bits, lo = 32 bits; F has at most 53
      // significant bits, so the fused sum below is exact.
      const double sc_hi = bits_to_double(double_to_bits(sc) + (uint64_t(32) << 52));
      const double hi = (double)(((h & 0x7FFFu) << 16) | t1);
      return __builtin_fma(hi, sc_hi, (double)t2 * sc);
    }
  }
}

// Products of the E non-zeros [base, base+E) that fall in [lo, hi); the
// others are left untouched.  base is a multiple of E.
template <int FMT, int E>
__device__ __forceinline__ void stage_products(const SpmvOperand& A, const double* __restrict__ x,
                                               const double* scale, int base, int lo, int hi,
                                               int j0, double* prod) {
  Words<E> cw = load_words<E>(A.col + base);
  Words<(E / 2 > 1 ? E / 2 : 2)> hw{}, t1w{};
  Words<E> t2w{};
  double vv[E];
  if constexpr (FMT != kCsr64) {
    hw = load_words<(E / 2 > 1 ? E / 2 : 2)>(A.head + base);
    if constexpr (FMT >= 2) t1w = load_words<(E / 2 > 1 ? E / 2 : 2)>(A.tail1 + base);
    if constexpr (FMT >= 3) t2w = load_words<E>(A.tail2 + base);
  } else {
    const double2* q = reinterpret_cast<const double2*>(A.val + base);
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
      const double2 d = q[i];
      vv[2 * i] = d.x;
      vv[2 * i + 1] = d.y;
    }
  }
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int j = base + k;
    if (j >= lo && j < hi) {
      int column;
      const uint32_t h = (FMT != kCsr64) ? u16_of(hw, k) : 0u;
      const uint32_t t1 = (FMT >= 2) ? u16_of(t1w, k) : 0u;
      const uint32_t t2 = (FMT >= 3) ? t2w.w[k] : 0u;
      const double v = decode<FMT>(cw.w[k], h, t1, t2, (FMT == kCsr64) ? vv[k] : 0.0, scale, column);
      const int li = j - j0;
      prod[li + li / E] = v * x[column];
    }
  }
}

// One product read straight from memory (phase 4).
template <int FMT>
__device__ __forceinline__ double product_at(const SpmvOperand& A, const double* __restrict__ x,
                                             const double* scale, int j) {
  const uint32_t c = A.col[j];
  uint32_t h = 0, t1 = 0, t2 = 0;
  double v = 0.0;
  if constexpr (FMT != kCsr64) {
    h = A.head[j];
    if constexpr (FMT >= 2) t1 = A.tail1[j];
    if constexpr (FMT >= 3) t2 = A.tail2[j];
  } else {
    v = A.val[j];
  }
  int column;
  const double d = decode<FMT>(c, h, t1, t2, v, scale, column);
  return d * x[column];
}

template <int E>
struct TileLds {
  static constexpr int T = kWG * E;
  static constexpr int NPROD = (T + kExtra) + (T + kExtra) / E;
  static constexpr int NDEF = (T + kExtra) / (kShortRow + 1) + 2;
};

template <int FMT, int E>
__global__ __launch_bounds__(kWG) void k_spmv(SpmvOperand A, const double* __restrict__ x,
                                              double* __restrict__ y, SpmvEpilogue ep) {
  using L = TileLds<E>;
  constexpr int T = L::T;
  __shared__ double prod[L::NPROD];
  __shared__ double scale[16];
  __shared__ int deferred[L::NDEF];
  __shared__ int wave_cnt[kWaves];
  __shared__ double red[kWaves];
  __shared__ bool last_flag;

  if (ep.gate && *ep.gate) return;
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int j0 = tile * T;
  const int j1 = min(j0 + T, A.nnz);
  const int ra = A.tile_row[tile];
  const int rb = A.tile_row[tile + 1];
  double acc = 0.0;  // this thread's share of the epilogue dot

  auto finish_row = [&](int r, double sum) {
    if (ep.epi == kEpiPlain) {
      y[r] = sum;
    } else if (ep.epi == kEpiDot) {
      y[r] = sum;
      acc += ep.aux[r] * sum;
    } else {
      const double v = ep.aux[r] - sum;
      y[r] = v;
      acc += v * v;
    }
  };

  if (ra < rb) {
    build_scale<FMT>(A, scale);
    const int js = A.row_ptr[ra];      // first non-zero this tile needs
    const int je = A.row_ptr[rb];      // end of its last row
    const bool tail_in_lds = (je - j1) <= kExtra;
    const int jl = tail_in_lds ? je : j1;  // [js, jl) staged in LDS
    __syncthreads();  // scale table ready

    // ---- phase 1: coalesced vector loads, decode, gather, products -> LDS
    {
      const int base = j0 + tid * E;
      if (base + E > js && base < jl) stage_products<FMT, E>(A, x, scale, base, js, jl, j0, prod);
      constexpr int extra_lanes = kExtra / E;
      if (tid < extra_lanes) {
        const int b2 = j1 + tid * E;
        if (b2 < jl) stage_products<FMT, E>(A, x, scale, b2, js, jl, j0, prod);
      }
    }
    __syncthreads();

    // ---- phase 2: short rows, one thread each, summed in row order
    const int lane = tid & 63, wave = tid >> 6;
    int ndef = 0;
    const bool long_tail = !tail_in_lds;  // row rb-1 continues past the LDS copy
    for (int cbase = ra; cbase < rb; cbase += kWG) {
      const int r = cbase + tid;
      bool defer = false;
      if (r < rb && !(long_tail && r == rb - 1)) {
        const int s0 = A.row_ptr[r];
        const int s1 = A.row_ptr[r + 1];
        if (s1 - s0 <= kShortRow) {
          double sum = 0.0;
          for (int j = s0; j < s1; ++j) {
            const int li = j - j0;
            sum += prod[li + li / E];
          }
          finish_row(r, sum);
        } else {
          defer = true;
        }
      }
      // deterministic compaction of the deferred rows (ordered by row)
      const unsigned long long m = __ballot(defer);
      if (lane == 0) wave_cnt[wave] = __popcll(m);
      __syncthreads();
      int off = ndef;
      for (int w = 0; w < wave; ++w) off += wave_cnt[w];
      if (defer) deferred[off + __popcll(m & ((1ull << lane) - 1ull))] = r;
      int tot = 0;
      for (int w = 0; w < kWaves; ++w) tot += wave_cnt[w];
      ndef += tot;
      __syncthreads();
    }

    // ---- phase 3: long rows inside LDS, one wave each
    for (int d = wave; d < ndef; d += kWaves) {
      const int r = deferred[d];
      const int s0 = A.row_ptr[r];
      const int s1 = A.row_ptr[r + 1];
      double part = 0.0;
      for (int j = s0 + lane; j < s1; j += 64) {
        const int li = j - j0;
        part += prod[li + li / E];
      }
      part = wave_sum(part);
      if (lane == 0) finish_row(r, part);
    }

    // ---- phase 4: the row running far past the tile, whole workgroup
    if (long_tail) {
      const int r = rb - 1;
      const int s0 = A.row_ptr[r];
      double part = 0.0;
      for (int j = s0 + tid; j < j1; j += kWG) {
        const int li = j - j0;
        part += prod[li + li / E];
      }
      int j = j1 + tid;
      for (; j + 3 * kWG < je; j += 4 * kWG) {
        const double p0 = product_at<FMT>(A, x, scale, j);
        const double p1 = product_at<FMT>(A, x, scale, j + kWG);
        const double p2 = product_at<FMT>(A, x, scale, j + 2 * kWG);
        const double p3 = product_at<FMT>(A, x, scale, j + 3 * kWG);
        part += p0;
        part += p1;
        part += p2;
        part += p3;
      }
      for (; j < je; j += kWG) part += product_at<FMT>(A, x, scale, j);
      const double tot = block_sum(part, red);
      if (tid == 0) finish_row(r, tot);
    }
  }

  // ---- epilogue dot: per-workgroup partial, last workgroup finishes it
  if (ep.epi != kEpiPlain) {
    const double bs = block_sum(acc, red);
    if (tid == 0) ep.partials[blockIdx.x] = bs;
    if (last_block_arrive(ep.counter, &last_flag)) {
      const double tot = sum_partials(ep.partials, gridDim.x, red);
      if (tid == 0) {
        *ep.result = tot;
        *ep.counter = 0u;
      }
    }
  }
}

template <int FMT, int E>
hipError_t launch_fe(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_spmv<FMT, E>), dim3(A.n_tiles), dim3(kWG), 0, st, A, x, y, ep);
  return hipGetLastError();
}

template <int FMT>
hipError_t launch_f(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                    hipStream_t st) {
  switch (A.tile_nnz) {
    case kWG * 4: return launch_fe<FMT, 4>(A, x, y, ep, st);
    case kWG * 8: return launch_fe<FMT, 8>(A, x, y, ep, st);
    case kWG * 16: return launch_fe<FMT, 16>(A, x, y, ep, st);
    default: return hipErrorInvalidValue;
  }
}

// tile_row[t] = first row whose first non-zero is at or after t*T (lower
// bound over row_ptr[0..n_rows)), tile_row[n_tiles] = n_rows.
__global__ void k_plan(const int32_t* __restrict__ row_ptr, int32_t n_rows, int32_t tile_nnz,
                       int32_t n_tiles, int32_t* __restrict__ tile_row) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_tiles) return;
  if (t == n_tiles) {
    tile_row[t] = n_rows;
    return;
  }
  const int target = t * tile_nnz;
  int lo = 0, hi = n_rows;  // first r in [0, n_rows) with row_ptr[r] >= target, else n_rows
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (row_ptr[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  tile_row[t] = lo;
}

__global__ void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

int32_t n_tiles_for(int64_t nnz, int32_t tile_nnz) {
  const int64_t t = (nnz + tile_nnz - 1) / tile_nnz;
  return (int32_t)(t < 1 ? 1 : t);
}

hipError_t launch_spmv(int fmt, const SpmvOperand& A, const double* x, double* y,
                       const SpmvEpilogue& ep, hipStream_t st) {
  switch (fmt) {
    case 0: return launch_f<0>(A, x, y, ep, st);
    case 1: return launch_f<1>(A, x, y, ep, st);
    case 2: return launch_f<2>(A, x, y, ep, st);
    case 3: return launch_f<3>(A, x, y, ep, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_plan(const int32_t* row_ptr, int32_t n_rows, int32_t nnz, int32_t tile_nnz,
                       int32_t n_tiles, int32_t* tile_row, hipStream_t st) {
  (void)nnz;
  const int threads = 256;
  const int blocks = (n_tiles + 1 + threads - 1) / threads;
  hipLaunchKernelGGL(k_plan, dim3(blocks), dim3(threads), 0, st, row_ptr, n_rows, tile_nnz, n_tiles,
                     tile_row);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                     reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n);
  return hipGetLastError();
}

}  // namespace gse

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
//     loads from each plane (fully coalesced; issued before the row lookup),
//     decodes them and stores value and column in LDS; up to kExtra
//     non-zeros past the tile are staged too when the tile's last row runs
//     over its end;
//   * phase 2: rows of up to kShortRow non-zeros are handled by one thread,
//     neighbouring lanes on neighbouring rows (so the x gathers of banded
//     matrices coalesce), summed in row order (the order of the sequential
//     definition);
//   * phase 3: longer rows staged in LDS are summed by one wave each;
//   * phase 4: a row that runs more than kExtra past the tile is summed by the
//     whole workgroup, reading the rest from memory.
// Matrices whose rows all hold at most kShortRow non-zeros (stencils) use a
// lean variant without the row machinery of phases 3-4 (k_spmv_short) and,
// in 1024-non-zero tiles, a ring schedule in which one producer wave streams
// the planes into LDS for three consumer waves (k_spmv_ring; k_spmv_rows
// when no row holds more than eight non-zeros: 192-row tiles, one row per
// consumer lane).  Every sum has
// a fixed order, so results are bit-reproducible and identical whether a
// matrix runs alone or next to others.
#include <atomic>

#include "decode.h"
#include "gse_internal.h"

#ifndef GSE_NT_LOADS
#define GSE_NT_LOADS 1
#endif

namespace gse {
namespace {

template <int N>
struct Words {
  uint32_t w[N];
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename V>
__device__ __forceinline__ V stream_load(const V* p) {
#if GSE_NT_LOADS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Load N 32-bit words from a 16-byte aligned (N % 4 == 0) or 8-byte aligned
// (N == 2) address.  The planes are streamed once per SpMV, so the loads are
// marked non-temporal to leave L2 to the gathered x.
template <int N>
__device__ __forceinline__ Words<N> load_words(const void* p) {
  Words<N> r;
  if constexpr (N % 4 == 0) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
#pragma unroll
    for (int i = 0; i < N / 4; ++i) {
      const u32x4 v = stream_load(q + i);
      r.w[4 * i + 0] = v.x;
      r.w[4 * i + 1] = v.y;
      r.w[4 * i + 2] = v.z;
      r.w[4 * i + 3] = v.w;
    }
  } else {
    static_assert(N == 2, "unsupported vector width");
    const u32x2 v = stream_load(reinterpret_cast<const u32x2*>(p));
    r.w[0] = v.x;
    r.w[1] = v.y;
  }
  return r;
}

template <int N>
__device__ __forceinline__ uint32_t u16_of(const Words<N>& w, int k) {
  return (w.w[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu;
}

// Raw plane data of E consecutive non-zeros [base, base+E), base % E == 0.
template <int FMT, int E>
struct Group {
  static constexpr int HW = (E / 2 > 1) ? E / 2 : 2;
  Words<E> cw;
  Words<HW> hw;
  Words<HW> t1w;
  Words<E> t2w;
  double vv[E];

  __device__ __forceinline__ void load(const SpmvOperand& A, int base) {
    cw = load_words<E>(A.col + base);
    if constexpr (FMT != kCsr64) {
      hw = load_words<HW>(A.head + base);
      if constexpr (planes_of(FMT) >= 2) t1w = load_words<HW>(A.tail1 + base);
      if constexpr (planes_of(FMT) >= 3) t2w = load_words<E>(A.tail2 + base);
    } else {
      const f64x2* q = reinterpret_cast<const f64x2*>(A.val + base);
#pragma unroll
      for (int i = 0; i < E / 2; ++i) {
        const f64x2 d = stream_load(q + i);
        vv[2 * i] = d.x;
        vv[2 * i + 1] = d.y;
      }
    }
  }

  // Decoded values and columns of all E non-zeros into LDS slots off..off+E-1
  // (16-byte stores; no range test: slots outside the staged range are
  // never read).
  __device__ __forceinline__ void stage_all(const DecodeCtx& scale, int off, double* vals,
                                            int* cols) const {
    double d[E];
    int column[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const uint32_t h = (FMT != kCsr64) ? u16_of(hw, k) : 0u;
      const uint32_t t1 = (planes_of(FMT) >= 2) ? u16_of(t1w, k) : 0u;
      const uint32_t t2 = (planes_of(FMT) >= 3) ? t2w.w[k] : 0u;
      d[k] = decode<FMT>(cw.w[k], h, t1, t2, (FMT == kCsr64) ? vv[k] : 0.0, scale, column[k]);
    }
    double2* v2 = reinterpret_cast<double2*>(vals + off);
#pragma unroll
    for (int k = 0; k < E / 2; ++k) v2[k] = make_double2(d[2 * k], d[2 * k + 1]);
    int4* c4 = reinterpret_cast<int4*>(cols + off);
#pragma unroll
    for (int k = 0; k < E / 4; ++k)
      c4[k] = make_int4(column[4 * k], column[4 * k + 1], column[4 * k + 2], column[4 * k + 3]);
  }

  // Decoded values and columns of the non-zeros in [lo, hi) into the LDS
  // slots of the tile starting at j0 (one padding slot per 8 spreads the
  // lanes of a wave over the banks).
  __device__ __forceinline__ void stage(const DecodeCtx& scale, int base, int lo, int hi, int j0,
                                        double* vals, int* cols) const {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int j = base + k;
      if (j >= lo && j < hi) {
        int column;
        const uint32_t h = (FMT != kCsr64) ? u16_of(hw, k) : 0u;
        const uint32_t t1 = (planes_of(FMT) >= 2) ? u16_of(t1w, k) : 0u;
        const uint32_t t2 = (planes_of(FMT) >= 3) ? t2w.w[k] : 0u;
        const double v = decode<FMT>(cw.w[k], h, t1, t2, (FMT == kCsr64) ? vv[k] : 0.0, scale,
                                     column);
        const int li = j - j0;
        vals[li + (li >> 3)] = v;
        cols[li + (li >> 3)] = column;
      }
    }
  }
};

// Plane data of one non-zero (look-ahead past the tile end).
template <int FMT>
struct Elem {
  uint32_t c = 0, h = 0, t1 = 0, t2 = 0;
  double v = 0.0;
  __device__ __forceinline__ void load(const SpmvOperand& A, int j) {
    c = A.col[j];
    if constexpr (FMT != kCsr64) {
      h = A.head[j];
      if constexpr (planes_of(FMT) >= 2) t1 = A.tail1[j];
      if constexpr (planes_of(FMT) >= 3) t2 = A.tail2[j];
    } else {
      v = A.val[j];
    }
  }
  __device__ __forceinline__ double product(const double* __restrict__ x, const DecodeCtx& scale) const {
    int column;
    const double d = decode<FMT>(c, h, t1, t2, v, scale, column);
    return d * x[column];
  }
  __device__ __forceinline__ void stage(const DecodeCtx& scale, int li, double* vals, int* cols) const {
    int column;
    const double d = decode<FMT>(c, h, t1, t2, v, scale, column);
    vals[li + (li >> 3)] = d;
    cols[li + (li >> 3)] = column;
  }
};

// One product read straight from memory (phase 4).
template <int FMT>
__device__ __forceinline__ double product_at(const SpmvOperand& A, const double* __restrict__ x,
                                             const DecodeCtx& scale, int j) {
  Elem<FMT> e;
  e.load(A, j);
  return e.product(x, scale);
}

template <int E>
struct TileLds {
  static constexpr int T = kWG * E;
  static constexpr int NPROD = (T + kExtra) + (T + kExtra) / 8;
  static constexpr int NDEF = (T + kExtra) / (kShortRow + 1) + 2;
};

__device__ __forceinline__ int pslot(int li) { return li + (li >> 3); }

// Position of a tile in the persistent schedule: the tiles are split into
// eight contiguous ranges, one per XCD (workgroups are handed to the XCDs
// round-robin), and the workgroups of an XCD interleave over its range, so
// the tiles in flight on an XCD are neighbours and share x in its L2.
struct TileWalk {
  int t, end, step;
  __device__ __forceinline__ TileWalk(int n_tiles) : TileWalk(n_tiles, blockIdx.x, gridDim.x) {}
  // workgroup wg of the g (a multiple of 8 when g > 8) that share the tiles
  __device__ __forceinline__ TileWalk(int n_tiles, int wg, int g) {
    const int xcd = wg & 7, local = wg >> 3;
    const int nx = (g >> 3) + (((g & 7) > xcd) ? 1 : 0);
    const int tb = (int)(((long long)n_tiles * xcd) >> 3);
    end = (int)(((long long)n_tiles * (xcd + 1)) >> 3);
    t = tb + local;
    step = nx;
  }
};

// Row bookkeeping of one tile (scalars, uniform over the workgroup).
struct TileInfo {
  int t, j0, j1, ra, rb;
};

// Persistent SpMV: every workgroup walks its tiles with a one-tile software
// pipeline -- the plane data and row pointers of tile i+1 are in flight
// while tile i is decoded, multiplied and reduced.
template <int FMT, int E>
__global__ __launch_bounds__(kWG) void k_spmv(SpmvOperand A, const double* __restrict__ x,
                                              double* __restrict__ y, SpmvEpilogue ep) {
  using L = TileLds<E>;
  constexpr int T = L::T;
  constexpr int NPF = 2;  // row pointers prefetched per thread (2 * 256 rows)
  __shared__ double vals[L::NPROD];
  __shared__ int cols[L::NPROD];
  __shared__ uint32_t scale_tab[kScaleEntries];
  __shared__ int rps[NPF * kWG + 1];
  __shared__ int deferred[L::NDEF];
  __shared__ int wave_cnt[kWaves];
  __shared__ double red[kWaves];

  if (ep.gate && *ep.gate) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  build_scale<FMT>(A.sem, scale_tab, A.split.ei);
  const DecodeCtx scale{scale_tab, A.split};
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

  TileWalk walk(A.n_tiles);
  // prefetch state of the next tile
  Group<FMT, E> g_cur, g_nxt;
  Elem<FMT> e_cur, e_nxt;
  int rpv_cur[NPF], rpv_nxt[NPF];
  TileInfo cur{}, nxt{};

  auto issue_planes = [&](int t, TileInfo& ti, Group<FMT, E>& g, Elem<FMT>& e) {
    ti.t = t;
    ti.j0 = t * T;
    ti.j1 = min(ti.j0 + T, A.nnz);
    const int base = ti.j0 + tid * E;
    if (base < A.nnz) g.load(A, base);
    if (tid < kSpec && ti.j1 + tid < A.nnz) e.load(A, ti.j1 + tid);
    ti.ra = A.tile_row[t];
    ti.rb = A.tile_row[t + 1];
  };
  auto issue_rows = [&](const TileInfo& ti, int* rpv) {
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int i = k * kWG + tid;
      rpv[k] = (i <= ti.rb - ti.ra) ? A.row_ptr[ti.ra + i] : 0;
    }
  };

  bool have = walk.t < walk.end;
  if (have) {
    issue_planes(walk.t, cur, g_cur, e_cur);
    issue_rows(cur, rpv_cur);
  }
  while (have) {
    const int tn = walk.t + walk.step;
    const bool have_n = tn < walk.end;
    if (have_n) issue_planes(tn, nxt, g_nxt, e_nxt);

    const int j0 = cur.j0, j1 = cur.j1, ra = cur.ra, rb = cur.rb;
    if (ra < rb) {
      const int nr = rb - ra;
      const int nstage = min(nr, NPF * kWG - 1);  // rps[0..nstage] = row_ptr[ra..ra+nstage]
      __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int i = k * kWG + tid;
        if (i <= nstage) rps[i] = rpv_cur[k];
      }
      __syncthreads();  // rps ready
      const int js = rps[0];
      const int je = (nr <= nstage) ? rps[nr] : A.row_ptr[rb];
      const bool tail_in_lds = (je - j1) <= kExtra;
      const int jl = tail_in_lds ? je : j1;  // [js, jl) staged in LDS

      // ---- phase 1: decode the staged non-zeros into LDS (value, column)
      const int base = j0 + tid * E;
      if (base < jl && base + E > js) g_cur.stage(scale, base, js, jl, j0, vals, cols);
      if (tid < kSpec && j1 + tid < jl) e_cur.stage(scale, j1 + tid - j0, vals, cols);
      if (jl > j1 + kSpec) {  // longer look-ahead for the last row: second round
        for (int j = j1 + kSpec + tid; j < jl; j += kWG) {
          Elem<FMT> e;
          e.load(A, j);
          e.stage(scale, j - j0, vals, cols);
        }
      }
      if (have_n) issue_rows(nxt, rpv_nxt);
      __syncthreads();

      auto rp_at = [&](int r) { return (r - ra <= nstage) ? rps[r - ra] : A.row_ptr[r]; };

      // ---- phase 2: short rows, one thread each, summed in row order
      int ndef = 0;
      const bool long_tail = !tail_in_lds;  // row rb-1 continues past the LDS copy
      for (int cbase = ra; cbase < rb; cbase += kWG) {
        const int r = cbase + tid;
        bool defer = false;
        if (r < rb && !(long_tail && r == rb - 1)) {
          const int s0 = rp_at(r);
          const int s1 = rp_at(r + 1);
          if (s1 - s0 <= kShortRow) {
            // neighbouring lanes hold neighbouring rows: the gathers of a
            // banded matrix fall in few cache lines; eight are issued at
            // once; the row is summed in order, multiply and add rounded
            // separately like the sequential definition
            double sum = 0.0;
            for (int jb = s0; jb < s1; jb += 8) {
              double v[8], xv[8];
              int c[8];
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const int q = pslot(min(jb + k, s1 - 1) - j0);
                v[k] = vals[q];
                c[k] = (jb + k < s1) ? cols[q] : 0;
              }
#pragma unroll
              for (int k = 0; k < 8; ++k) xv[k] = x[c[k]];
#pragma unroll
              for (int k = 0; k < 8; ++k) {
                const double p = __dmul_rn(v[k], xv[k]);
                sum = (jb + k < s1) ? __dadd_rn(sum, p) : sum;
              }
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
        const int s0 = rp_at(r);
        const int s1 = rp_at(r + 1);
        double part = 0.0;
        for (int j = s0 + lane; j < s1; j += 64) {
          const int q = pslot(j - j0);
          part += vals[q] * x[cols[q]];
        }
        part = wave_sum(part);
        if (lane == 0) finish_row(r, part);
      }

      // ---- phase 4: the row running far past the tile, whole workgroup
      if (long_tail) {
        const int r = rb - 1;
        const int s0 = rp_at(r);
        double part = 0.0;
        for (int j = s0 + tid; j < j1; j += kWG) {
          const int q = pslot(j - j0);
          part += vals[q] * x[cols[q]];
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
    } else if (have_n) {
      issue_rows(nxt, rpv_nxt);
    }
    walk.t = tn;
    have = have_n;
    cur = nxt;
    g_cur = g_nxt;
    e_cur = e_nxt;
#pragma unroll
    for (int k = 0; k < NPF; ++k) rpv_cur[k] = rpv_nxt[k];
  }

  // ---- epilogue dot: one partial per workgroup (finished by the caller's
  // next kernel, after the launch boundary has made them visible)
  if (ep.epi != kEpiPlain) {
    const double bs = block_sum(acc, red);
    if (tid == 0) ep.partials[blockIdx.x] = bs;
  }
}

// Short-row tile schedule, for matrices whose rows all have at most
// kShortRow non-zeros (stencils): a row running over the tile end needs at
// most kShortRow-1 look-ahead non-zeros, which are loaded with the tile, so
// there are no deferred rows and no long tails.  Per element: one decode in
// phase 1 (16-byte loads, unpredicated, 16-byte LDS stores) and, in phase 2,
// two LDS reads, one gather (neighbouring lanes on neighbouring rows, eight
// gathers in flight per lane) and a multiply-add in row order.  Two barriers
// per tile; the same persistent one-tile software pipeline as k_spmv.
constexpr int kLook = 32;  // look-ahead non-zeros (>= kShortRow - 1)

template <int FMT, int E>
__global__ __launch_bounds__(kWG) void k_spmv_short(SpmvOperand A, const double* __restrict__ x,
                                                    double* __restrict__ y, SpmvEpilogue ep) {
  constexpr int T = kWG * E;
  constexpr int NS = T + kLook + 8;
  constexpr int LOOK_LANES = kLook / E;
  constexpr int NPF = 2;
  static_assert(kLook >= kShortRow, "look-ahead must cover the longest row");
  __shared__ __attribute__((aligned(16))) double vals[NS];
  __shared__ __attribute__((aligned(16))) int cols[NS];
  __shared__ uint32_t scale_tab[kScaleEntries];
  __shared__ int rps[NPF * kWG + 1];
  __shared__ double red[kWaves];

  if (ep.gate && *ep.gate) return;
  const int tid = threadIdx.x;
  build_scale<FMT>(A.sem, scale_tab, A.split.ei);
  const DecodeCtx scale{scale_tab, A.split};
  double acc = 0.0;

  TileWalk walk(A.n_tiles);
  Group<FMT, E> g_cur, g_nxt, l_cur, l_nxt;
  int rpv_cur[NPF], rpv_nxt[NPF];
  TileInfo cur{}, nxt{};

  auto issue_planes = [&](int t, TileInfo& ti, Group<FMT, E>& g, Group<FMT, E>& l) {
    ti.t = t;
    ti.j0 = t * T;
    ti.j1 = min(ti.j0 + T, A.nnz);
    const int base = ti.j0 + tid * E;
    if (base < A.nnz) g.load(A, base);
    const int lb = ti.j1 + tid * E;
    if (tid < LOOK_LANES && lb < A.nnz) l.load(A, lb);
    ti.ra = A.tile_row[t];
    ti.rb = A.tile_row[t + 1];
  };
  auto issue_rows = [&](const TileInfo& ti, int* rpv) {
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int i = k * kWG + tid;
      rpv[k] = (i <= ti.rb - ti.ra) ? A.row_ptr[ti.ra + i] : 0;
    }
  };

  bool have = walk.t < walk.end;
  if (have) {
    issue_planes(walk.t, cur, g_cur, l_cur);
    issue_rows(cur, rpv_cur);
  }
  while (have) {
    const int tn = walk.t + walk.step;
    const bool have_n = tn < walk.end;
    if (have_n) issue_planes(tn, nxt, g_nxt, l_nxt);
    const int j0 = cur.j0, ra = cur.ra, rb = cur.rb;
    if (ra < rb) {
      const int nr = rb - ra;
      const int nstage = min(nr, NPF * kWG - 1);
      __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int i = k * kWG + tid;
        if (i <= nstage) rps[i] = rpv_cur[k];
      }
      g_cur.stage_all(scale, tid * E, vals, cols);
      if (tid < LOOK_LANES) l_cur.stage_all(scale, T + tid * E, vals, cols);
      if (have_n) issue_rows(nxt, rpv_nxt);
      __syncthreads();
      for (int r = ra + tid; r < rb; r += kWG) {
        const int s0 = (r - ra <= nstage) ? rps[r - ra] : A.row_ptr[r];
        const int s1 = (r + 1 - ra <= nstage) ? rps[r + 1 - ra] : A.row_ptr[r + 1];
        const int o = s0 - j0;
        const int len = s1 - s0;
        double sum = 0.0;
        for (int kb = 0; kb < len; kb += 8) {
          double v[8], xv[8];
          int c[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            v[k] = vals[o + kb + k];
            c[k] = (kb + k < len) ? cols[o + kb + k] : 0;
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) xv[k] = x[c[k]];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const double p = __dmul_rn(v[k], xv[k]);
            sum = (kb + k < len) ? __dadd_rn(sum, p) : sum;
          }
        }
        if (ep.epi == kEpiPlain) {
          y[r] = sum;
        } else if (ep.epi == kEpiDot) {
          y[r] = sum;
          acc += ep.aux[r] * sum;
        } else {
          const double vres = ep.aux[r] - sum;
          y[r] = vres;
          acc += vres * vres;
        }
      }
    } else if (have_n) {
      issue_rows(nxt, rpv_nxt);
    }
    walk.t = tn;
    have = have_n;
    cur = nxt;
    g_cur = g_nxt;
    l_cur = l_nxt;
#pragma unroll
    for (int k = 0; k < NPF; ++k) rpv_cur[k] = rpv_nxt[k];
  }
  if (ep.epi != kEpiPlain) {
    const double bs = block_sum(acc, red);
    if (tid == 0) ep.partials[blockIdx.x] = bs;
  }
}

// ---------------------------------------------------------------------------
// Ring schedule for short rows (no row longer than kShortRow), 1024-non-zero
// tiles.  A workgroup is one producer wave and three consumer waves.  The
// producer copies the plane bytes of the coming tiles (with the look-ahead)
// and their row pointers straight into an LDS ring of D stages with
// global_load_lds -- no registers, no decode -- and keeps D-1 tiles in
// flight.  The consumers decode each non-zero from the ring, gather x and
// sum their row in row order.  Vector-memory loads complete in issue order
// within a wave, so a wave that both prefetches planes and gathers x must
// wait for its prefetch whenever it waits for a gather; here the producer
// issues nothing but ring loads (the tile table is read through scalar
// loads) and its waits count exactly its own stages, while the consumers'
// gathers never queue behind plane loads.  Two barriers per tile: A (the
// stage has landed) and B (the stage has been consumed); the producer
// refills the stage consumed in the previous tile between A and B.
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kRingTile = 1024;          // non-zeros per tile (the plan's tile_nnz)
constexpr int kRingConsumers = 3 * 64;   // consumer threads
constexpr int kRingThreads = kRingConsumers + 64;

// LDS ring geometry: D stages, each holding the planes of TL staged
// non-zeros (column words first, then the value or the segment planes) and
// RP row pointers.
template <int FMT, int TL_, int D_>
struct RingGeom {
  static constexpr int TL = TL_;            // staged non-zeros per stage
  static constexpr int RP = 256;            // row pointers staged per stage
  static constexpr int D = D_;
  static constexpr int OFF_COL = 0;
  static constexpr int OFF_HEAD = TL * 4;
  static constexpr int OFF_T1 = OFF_HEAD + TL * 2;
  static constexpr int OFF_T2 = OFF_T1 + TL * 2;
  static constexpr int OFF_VAL = TL * 4;
  static constexpr int END = (FMT == kCsr64) ? OFF_VAL + TL * 8
                             : (planes_of(FMT) == 1)    ? OFF_HEAD + TL * 2
                             : (planes_of(FMT) == 2)    ? OFF_T1 + TL * 2
                                             : OFF_T2 + TL * 4;
  static constexpr int OFF_RPS = END;
  static constexpr int STAGE = (OFF_RPS + RP * 4 + 15) / 16 * 16;
  // load instructions the producer issues per stage (64 lanes x 16 bytes,
  // 64 x 4 bytes for row pointers)
  static constexpr int NCOL = (TL * 4 / 16 + 63) / 64;
  static constexpr int NHALF = (TL * 2 / 16 + 63) / 64;
  static constexpr int NVAL = (TL * 8 / 16 + 63) / 64;
  static constexpr int NRPS = RP / 64;
  static constexpr int NI = NCOL + NRPS + ((FMT == kCsr64) ? NVAL
                                           : (planes_of(FMT) == 1)    ? NHALF
                                           : (planes_of(FMT) == 2)    ? 2 * NHALF
                                                           : 2 * NHALF + NCOL);
  // bytes the last load of a region writes past its end (into the next one)
  static constexpr int SPILL_COL = NCOL * 1024 - TL * 4;
  static constexpr int SPILL_HALF = NHALF * 1024 - TL * 2;
  static constexpr int SPILL_VAL = NVAL * 1024 - TL * 8;
  static_assert(TL % 16 == 0 && RP % 64 == 0, "chunking");
  static_assert(SPILL_COL <= TL * 2 && SPILL_COL <= RP * 4 && SPILL_HALF <= RP * 4 &&
                    SPILL_HALF <= TL * 2 && SPILL_VAL <= RP * 4,
                "a region's spill must stay inside the region loaded after it");
  static_assert((D - 1) * NI < 64, "the vector-memory counter holds at most 63");
};

// Non-zero tiles of kRingTile entries plus the look-ahead.  Three stages for
// every format: 22-42 KiB per workgroup, so six or seven workgroups share a
// CU (four stages of 320 row pointers fitted five for s = 1: same time on
// 128^3, 4-9 % slower on the 1024^2 operator, whose shorter runs per
// workgroup gain from the wider grid).
template <int FMT>
struct RingLayout : RingGeom<FMT, kRingTile + kLook, 3> {
  static constexpr int T = kRingTile;
};

// s_waitcnt vmcnt(N), leaving the other counters alone (gfx9 encoding).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | 0x70 | 0xF00);
}

// The producer's stage k has landed once at most `later` stages issued
// after it are still outstanding.
template <class L>
__device__ __forceinline__ void ring_wait(int later) {
  constexpr int NI = L::NI;
  switch (later) {
    case 0: wait_vmcnt<0>(); break;
    case 1: wait_vmcnt<NI>(); break;
    default: wait_vmcnt<2 * NI>(); break;
  }
}

// Barrier of the producer: its own LDS writes (stage headers) are complete,
// its ring loads stay in flight (a workgroup fence here would wait for them).
__device__ __forceinline__ void producer_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Barrier of the consumers: LDS accesses ordered, nothing else waited for.
__device__ __forceinline__ void consumer_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Producer: planes of tile t (non-zeros t*T .. t*T+TL-1) and row pointers
// ra .. ra+RP-1 into `stage`.  Lane l of load i moves 16-byte chunk 64i+l
// to region + 1024i + 16l.  Every lane of every load takes part (no branch
// around a load: the LDS address of a load is one per wave, so loads must
// not sit in divergent code); the chunks past a region's end land at the
// start of the next region, which is loaded later by the same wave and so
// overwritten (loads of one wave complete in issue order), and the row
// pointers, loaded last, fill their region exactly.  Chunk addresses are
// clamped to the last chunk before jlim (a multiple of 16, at most pad and
// at least j0 + 16: every chunk is either inside the planes' padding or a
// repeat of the last one needed) and row indices to rlim (<= n_rows); a
// repeated address costs no extra memory traffic, and clamped data lands in
// slots that are never read.
template <int FMT, class L>
__device__ __forceinline__ void ring_issue(const SpmvOperand& A, lds_char* stage, int j0, int ra,
                                           int jlim, int rlim, int lane) {
#pragma unroll
  for (int i = 0; i < L::NCOL; ++i) {
    const int e = min(j0 + 4 * (i * 64 + lane), jlim - 4);
    __builtin_amdgcn_global_load_lds(A.col + e, (lds_void*)(stage + L::OFF_COL + i * 1024), 16, 0, 0);
  }
  if constexpr (FMT == kCsr64) {
#pragma unroll
    for (int i = 0; i < L::NVAL; ++i) {
      const int e = min(j0 + 2 * (i * 64 + lane), jlim - 2);
      __builtin_amdgcn_global_load_lds(A.val + e, (lds_void*)(stage + L::OFF_VAL + i * 1024), 16, 0, 0);
    }
  } else {
#pragma unroll
    for (int i = 0; i < L::NHALF; ++i) {
      const int e = min(j0 + 8 * (i * 64 + lane), jlim - 8);
      __builtin_amdgcn_global_load_lds(A.head + e, (lds_void*)(stage + L::OFF_HEAD + i * 1024), 16, 0, 0);
    }
    if constexpr (planes_of(FMT) >= 2) {
#pragma unroll
      for (int i = 0; i < L::NHALF; ++i) {
        const int e = min(j0 + 8 * (i * 64 + lane), jlim - 8);
        __builtin_amdgcn_global_load_lds(A.tail1 + e, (lds_void*)(stage + L::OFF_T1 + i * 1024), 16, 0, 0);
      }
    }
    if constexpr (planes_of(FMT) == 3) {
#pragma unroll
      for (int i = 0; i < L::NCOL; ++i) {
        const int e = min(j0 + 4 * (i * 64 + lane), jlim - 4);
        __builtin_amdgcn_global_load_lds(A.tail2 + e, (lds_void*)(stage + L::OFF_T2 + i * 1024), 16, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < L::NRPS; ++i) {
    const int r = min(ra + i * 64 + lane, rlim);
    __builtin_amdgcn_global_load_lds(A.row_ptr + r, (lds_void*)(stage + L::OFF_RPS + i * 256), 4, 0, 0);
  }
}

// The exclusive chunk limit of a staged window [j0, jend): jend rounded up
// to 16, at least j0 + 16, at most pad (pad >= 16 here: these schedules
// run on 1024 non-zeros or more).
__device__ __forceinline__ int window_limit(int j0, int jend, int pad) {
  return min(max((jend + 15) & ~15, j0 + 16), pad);
}

// Consumer: the decoded value and column of staged non-zero `pos`.
template <int FMT, class L>
__device__ __forceinline__ double ring_value(const lds_char* stage, int pos, const DecodeCtx& scale,
                                             int& column) {
  typedef const __attribute__((address_space(3))) uint32_t* u32p;
  typedef const __attribute__((address_space(3))) uint16_t* u16p;
  const uint32_t c = *reinterpret_cast<u32p>(stage + L::OFF_COL + 4 * pos);
  uint32_t h = 0, t1 = 0, t2 = 0;
  double v = 0.0;
  if constexpr (FMT == kCsr64) {
    v = *reinterpret_cast<const __attribute__((address_space(3))) double*>(stage + L::OFF_VAL + 8 * pos);
  } else {
    h = *reinterpret_cast<u16p>(stage + L::OFF_HEAD + 2 * pos);
    if constexpr (planes_of(FMT) >= 2) t1 = *reinterpret_cast<u16p>(stage + L::OFF_T1 + 2 * pos);
    if constexpr (planes_of(FMT) == 3) t2 = *reinterpret_cast<u32p>(stage + L::OFF_T2 + 4 * pos);
  }
  return decode<FMT>(c, h, t1, t2, v, scale, column);
}

template <int FMT>
__global__ __launch_bounds__(kRingThreads) void k_spmv_ring(SpmvOperand A,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ y, SpmvEpilogue ep) {
  using L = RingLayout<FMT>;
  constexpr int PRODUCER = kRingConsumers / 64;  // wave index of the producer
  __shared__ __attribute__((aligned(16))) char ring_raw[L::D * L::STAGE];
  __shared__ int hdr[L::D][4];  // per stage: first row, row end, first non-zero
  __shared__ uint32_t scale_tab[kScaleEntries];
  __shared__ double red[kRingThreads / 64];
  lds_char* ring = (lds_char*)ring_raw;

  if (ep.gate && *ep.gate) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  build_scale<FMT>(A.sem, scale_tab, A.split.ei);
  const DecodeCtx scale{scale_tab, A.split};
  const int pad = (A.nnz + 15) & ~15;
  TileWalk walk(A.n_tiles);
  const int count = walk.t < walk.end ? (walk.end - walk.t + walk.step - 1) / walk.step : 0;
  double acc = 0.0;
  __syncthreads();
  if (wave == PRODUCER) {
    // scalar loads of the tile table (constant address space): the wave's
    // vector-memory counter holds ring loads only
    const __attribute__((address_space(4))) int32_t* trow =
        (const __attribute__((address_space(4))) int32_t*)(A.tile_row);
    auto issue = [&](int k) {
      const int t = walk.t + k * walk.step;
      const int ra = trow[t];
      const int rb = trow[t + 1];
      const int st = k % L::D;
      ring_issue<FMT, L>(A, ring + st * L::STAGE, t * L::T, ra,
                         window_limit(t * L::T, t * L::T + L::TL, pad), A.n_rows, lane);
      if (lane == 0) {
        hdr[st][0] = ra;
        hdr[st][1] = rb;
        hdr[st][2] = t * L::T;
      }
    };
    for (int k = 0; k < L::D - 1 && k < count; ++k) issue(k);
    for (int k = 0; k < count; ++k) {
      ring_wait<L>(min(L::D - 2, count - 1 - k));
      producer_barrier();  // A
      if (k + L::D - 1 < count) issue(k + L::D - 1);  // the stage consumed in tile k-1
      producer_barrier();  // B
    }
  } else {
    for (int k = 0; k < count; ++k) {
      consumer_barrier();  // A
      const int st = k % L::D;
      const lds_char* stage = ring + st * L::STAGE;
      const int ra = hdr[st][0], rb = hdr[st][1], j0 = hdr[st][2];
      const int nst = min(rb - ra, L::RP - 1);
      const __attribute__((address_space(3))) int* rps =
          reinterpret_cast<const __attribute__((address_space(3))) int*>(stage + L::OFF_RPS);
      for (int r = ra + tid; r < rb; r += kRingConsumers) {
        const int s0 = (r - ra <= nst) ? rps[r - ra] : A.row_ptr[r];
        const int s1 = (r + 1 - ra <= nst) ? rps[r + 1 - ra] : A.row_ptr[r + 1];
        const int o = s0 - j0;
        const int len = s1 - s0;
        double sum = 0.0;
        for (int kb = 0; kb < len; kb += 8) {
          double v[8], xv[8];
          int c[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            int col;
            v[q] = ring_value<FMT, L>(stage, o + kb + q, scale, col);
            c[q] = (kb + q < len) ? col : 0;
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) xv[q] = x[c[q]];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double p = __dmul_rn(v[q], xv[q]);
            sum = (kb + q < len) ? __dadd_rn(sum, p) : sum;
          }
        }
        if (ep.epi == kEpiPlain) {
          y[r] = sum;
        } else if (ep.epi == kEpiDot) {
          y[r] = sum;
          acc += ep.aux[r] * sum;
        } else {
          const double vres = ep.aux[r] - sum;
          y[r] = vres;
          acc += vres * vres;
        }
      }
      consumer_barrier();  // B
    }
  }
  if (ep.epi != kEpiPlain) {
    const double w = wave_sum(acc);
    __syncthreads();
    if (lane == 0) red[wave] = w;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < kRingThreads / 64; ++i) t += red[i];
      ep.partials[blockIdx.x] = t;
    }
  }
}

// Row-tile ring for operators whose rows all hold at most B <= 8 non-zeros
// (stencils): tile t is rows 192t .. 192t+191, one row per consumer lane, so
// every lane of the three consumer waves has a row and each row is one batch
// of B.  The producer reads the tile's first row pointer through a scalar
// load and stages the window that starts there, rounded down to 16
// non-zeros (chunk alignment), with 192 B + 16 entries: the tile's rows hold
// at most 192 B non-zeros, so the window covers them and every unconditional
// B-wide read of a row.  No tile table: the schedule follows from n_rows.
// Two stages: 18-35 KiB per workgroup, eight workgroups per CU at s = 1
// (three stages, five per CU, were 2-6 % slower on 128^3 and up to 9 % on
// the 1024^2 operator).
constexpr int kRowTile = kRingConsumers;

template <int FMT, int B>
using RowRing = RingGeom<FMT, kRowTile * B + 16, 2>;

// BLK: per-row-block tables.  A tile of 192 rows touches at most
// kRowTabEntries / 64 blocks (blocks of GSE_MIN_BLOCK_ROWS rows or more);
// their tables are staged by the consumers, one entry per thread, into one
// of two halves of scale_tab: tile k reads half k & 1 while the consumers
// fill the other half for tile k + 1 (the barrier at the end of tile k
// publishes it).  A row reads its block's table at (r / R - ra / R) * stride.
constexpr int kRowTabEntries = ((kRowTile - 1) / GSE_MIN_BLOCK_ROWS + 2) * GSE_MAX_EXP;
static_assert(kRowTabEntries <= kRingConsumers, "one table entry per consumer thread");

template <int FMT>
__device__ __forceinline__ void stage_tile_tables(const SpmvOperand& A, int t, uint32_t* tab,
                                                  int tid) {
  const int ra = t * kRowTile;
  const int rb = min(ra + kRowTile, A.n_rows);
  const int b0 = ra / A.block_rows;
  const int n = ((rb - 1) / A.block_rows - b0 + 1) * A.block_stride;
  if (tid < n) {
    const int W = ((FMT == 1) ? 15 : (FMT == 2) ? 31 : 63) - A.split.ei;
    const int S = A.block_sem[(size_t)b0 * A.block_stride + tid];
    tab[tid] = S > W ? (uint32_t)(S - W) << 20 : 0u;
  }
}

// IB >= 0: the operand has one table and its slot index in the top IB bits
// of the column word, fixed at compile time (IB = 3 for tables of five to
// eight shared exponents, the default k = 8): the field split folds into
// immediate shifts and masks and only 2^IB scale entries are built.  The
// general instance (IB = -1) reads the split from the operand.
//
// The body runs for one operand on workgroup wg of the g that share its
// tiles: the whole grid of a plain launch, or one operand's range of a
// grouped launch.
template <int FMT, int B, bool BLK>
struct RowsLds {
  using L = RowRing<FMT, B>;
  __attribute__((aligned(16))) char ring_raw[L::D * L::STAGE];
  int hdr[L::D][4];  // per stage: first row, row end, first staged non-zero
  uint32_t scale_tab[BLK ? 2 * kRowTabEntries : kScaleEntries];
  double red[kRingThreads / 64];
};

template <int FMT, int B, bool BLK, int IB>
__device__ __forceinline__ void rows_body(const SpmvOperand& A, const double* __restrict__ x,
                                          double* __restrict__ y, const SpmvEpilogue& ep, int wg,
                                          int g, RowsLds<FMT, B, BLK>& lds) {
  using L = RowRing<FMT, B>;
  constexpr int PRODUCER = kRingConsumers / 64;
  auto& hdr = lds.hdr;
  uint32_t* scale_tab = lds.scale_tab;
  double* red = lds.red;
  lds_char* ring = (lds_char*)lds.ring_raw;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int pad = (A.nnz + 15) & ~15;
  const int n_rt = (A.n_rows + kRowTile - 1) / kRowTile;
  TileWalk walk(n_rt, wg, g);
  const int count = walk.t < walk.end ? (walk.end - walk.t + walk.step - 1) / walk.step : 0;
  if constexpr (BLK) {
    if (count > 0 && tid < kRingConsumers) stage_tile_tables<FMT>(A, walk.t, scale_tab, tid);
  } else {
    build_scale_n<FMT>(A.sem, IB >= 0 ? (1 << IB) : kScaleEntries, scale_tab,
                       IB >= 0 ? 0 : A.split.ei);
  }
  const DecodeCtx scale{scale_tab, IB >= 0 ? col_split(IB, false) : A.split};
  double acc = 0.0;
  __syncthreads();
  if (wave == PRODUCER) {
    const __attribute__((address_space(4))) int32_t* rp =
        (const __attribute__((address_space(4))) int32_t*)(A.row_ptr);
    auto issue = [&](int k) {
      const int t = walk.t + k * walk.step;
      const int ra = t * kRowTile;
      const int rb = min(ra + kRowTile, A.n_rows);
      const int ja = rp[ra] & ~15;
      const int st = k % L::D;
      // exactly the tile's non-zeros [rp[ra], rp[rb]) (in 16-entry chunks)
      // and its rb - ra + 1 row pointers
      ring_issue<FMT, L>(A, ring + st * L::STAGE, ja, ra, window_limit(ja, rp[rb], pad), rb, lane);
      if (lane == 0) {
        hdr[st][0] = ra;
        hdr[st][1] = rb;
        hdr[st][2] = ja;
      }
    };
    for (int k = 0; k < L::D - 1 && k < count; ++k) issue(k);
    for (int k = 0; k < count; ++k) {
      ring_wait<L>(min(L::D - 2, count - 1 - k));
      producer_barrier();  // A
      if (k + L::D - 1 < count) issue(k + L::D - 1);  // the stage consumed in tile k-1
      producer_barrier();  // B
    }
  } else {
    for (int k = 0; k < count; ++k) {
      consumer_barrier();  // A
      if constexpr (BLK) {
        if (k + 1 < count)
          stage_tile_tables<FMT>(A, walk.t + (k + 1) * walk.step,
                                 scale_tab + ((k + 1) & 1) * kRowTabEntries, tid);
      }
      const int st = k % L::D;
      const lds_char* stage = ring + st * L::STAGE;
      const int ra = hdr[st][0], rb = hdr[st][1], ja = hdr[st][2];
      const __attribute__((address_space(3))) int* rps =
          reinterpret_cast<const __attribute__((address_space(3))) int*>(stage + L::OFF_RPS);
      const int r = ra + tid;
      if (r < rb) {
        const int s0 = rps[tid], s1 = rps[tid + 1];
        const int o = s0 - ja;
        const int len = s1 - s0;
        DecodeCtx own = scale;
        if constexpr (BLK)
          own.tab = scale_tab + (k & 1) * kRowTabEntries +
                    (r / A.block_rows - ra / A.block_rows) * A.block_stride;
        double v[B], xv[B];
        int c[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
          int col;
          v[q] = ring_value<FMT, L>(stage, o + q, own, col);
          c[q] = (q < len) ? col : 0;
        }
#pragma unroll
        for (int q = 0; q < B; ++q) xv[q] = x[c[q]];
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < B; ++q) {
          const double p = __dmul_rn(v[q], xv[q]);
          sum = (q < len) ? __dadd_rn(sum, p) : sum;
        }
        if (ep.epi == kEpiPlain) {
          y[r] = sum;
        } else if (ep.epi == kEpiDot) {
          y[r] = sum;
          acc += ep.aux[r] * sum;
        } else {
          const double vres = ep.aux[r] - sum;
          y[r] = vres;
          acc += vres * vres;
        }
      }
      consumer_barrier();  // B
    }
  }
  if (ep.epi != kEpiPlain) {
    const double w = wave_sum(acc);
    __syncthreads();
    if (lane == 0) red[wave] = w;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < kRingThreads / 64; ++i) t += red[i];
      ep.partials[wg] = t;
    }
  }
}

template <int FMT, int B, bool BLK = false, int IB = -1>
__global__ __launch_bounds__(kRingThreads) void k_spmv_rows(SpmvOperand A,
                                                            const double* __restrict__ x,
                                                            double* __restrict__ y, SpmvEpilogue ep) {
  __shared__ RowsLds<FMT, B, BLK> lds;
  if (ep.gate && *ep.gate) return;
  rows_body<FMT, B, BLK, IB>(A, x, y, ep, blockIdx.x, gridDim.x, lds);
}

// Grouped launch: the products of several operands of one format, row bound
// and index layout in one dispatch.  Operand i runs on workgroups
// [wg0_i, wg0_i + g_i) with g_i its own plain launch's grid (a multiple of
// 8, so every workgroup sits on the XCD it has in that launch) and writes
// its partials to its own ep.partials[0, g_i): each product and its
// partials equal those of the operand's plain launch bit for bit.
template <int FMT, int B, int IB>
__global__ __launch_bounds__(kRingThreads) void k_spmv_rows_grouped(const RowGroup* __restrict__ groups,
                                                                    int n_groups) {
  const int wg = blockIdx.x;
  int lo = 0, hi = n_groups - 1;  // the last range that starts at or before wg
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].wg0 <= wg) lo = mid;
    else hi = mid - 1;
  }
  const RowGroup& G = groups[lo];
  __shared__ RowsLds<FMT, B, false> lds;
  if (G.ep.gate && *G.ep.gate) return;
  rows_body<FMT, B, false, IB>(G.A, G.x, G.y, G.ep, wg - G.wg0, G.wgs, lds);
}

// Resident workgroups of one kernel instance on this device (occupancy x
// compute units), cached per instance.  Threads that race on the first call
// compute and store the same value.
enum Kind : int { kGeneralTiles = 0, kShortTiles = 1, kRingTiles = 2, kRowTiles = 3 };

template <int FMT, int E, int KIND, int B = 8, bool BLK = false, int IB = -1>
int resident_groups() {
  static std::atomic<int> cache{0};
  int cached = cache.load(std::memory_order_relaxed);
  if (cached == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    hipError_t e;
    if constexpr (KIND == kRowTiles)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmv_rows<FMT, B, BLK, IB>,
                                                       kRingThreads, 0);
    else if constexpr (KIND == kRingTiles)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmv_ring<FMT>, kRingThreads, 0);
    else if constexpr (KIND == kShortTiles)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmv_short<FMT, E>, kWG, 0);
    else
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmv<FMT, E>, kWG, 0);
    if (e != hipSuccess) return 0;
    cached = cus * (per_cu > 0 ? per_cu : 1);
    cache.store(cached, std::memory_order_relaxed);
  }
  return cached;
}

// Resident workgroups of the chosen kernel, at most what the tiles need and
// at least one per XCD range.  Every format runs at its own best occupancy,
// so launches that leave per-workgroup partial sums group them per format:
// results are bit-reproducible for a given format and matrix, and two
// formats that decode to the same values agree to rounding.
template <int FMT, int E, int KIND, int B = 8>
int grid_for(const SpmvOperand& A) {
  int g = resident_groups<FMT, E, KIND, B>();
  if (g <= 0) return 0;
  const int need = (A.n_tiles + 7) / 8 * 8;
  if (g > need) g = need;
  if (g < 8) g = 8;
  return g;
}

template <int FMT>
hipError_t launch_ring(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                       hipStream_t st) {
  const int g = grid_for<FMT, 4, kRingTiles>(A);
  if (g <= 0) return hipErrorInvalidDevice;
  if (ep.grid_out) *ep.grid_out = g;
  hipLaunchKernelGGL((k_spmv_ring<FMT>), dim3(g), dim3(kRingThreads), 0, st, A, x, y, ep);
  return hipGetLastError();
}

// Grid of a plain row-tile launch: the instance's resident workgroups, at
// most the row tiles rounded up to 8, at least 8.
template <int FMT, int B, bool BLK, int IB>
int rows_grid(const SpmvOperand& A) {
  int g = resident_groups<FMT, 4, kRowTiles, B, BLK, IB>();
  if (g <= 0) return 0;
  const int n_rt = (A.n_rows + kRowTile - 1) / kRowTile;
  const int need = (n_rt + 7) / 8 * 8;
  if (g > need) g = need;
  if (g < 8) g = 8;
  return g;
}

template <int FMT, int B, bool BLK = false, int IB = -1>
hipError_t launch_rows(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                       hipStream_t st) {
  if constexpr (!BLK && IB < 0 && is_gse(FMT)) {
    // a 3-bit index in the column word: the instance with the split folded in
    const ColSplit c3 = col_split(3, false);
    if (A.split.shift == c3.shift && A.split.slot_mask == c3.slot_mask &&
        A.split.col_mask == c3.col_mask && A.split.hmask == c3.hmask && A.split.ei == c3.ei)
      return launch_rows<FMT, B, false, 3>(A, x, y, ep, st);
  }
  if constexpr (BLK) {
    // the staged tables fit kRowTabEntries only for blocks this tall
    if (A.n_rows < 1 || !A.block_sem || A.block_rows < GSE_MIN_BLOCK_ROWS ||
        A.block_stride < 1 || A.block_stride > GSE_MAX_EXP)
      return hipErrorInvalidValue;
  }
  const int g = rows_grid<FMT, B, BLK, IB>(A);
  if (g <= 0) return hipErrorInvalidDevice;
  if (ep.grid_out) *ep.grid_out = g;
  hipLaunchKernelGGL((k_spmv_rows<FMT, B, BLK, IB>), dim3(g), dim3(kRingThreads), 0, st, A, x, y, ep);
  return hipGetLastError();
}

// Class and grid of the row-tile ring for operand A (the choices launch_f
// and launch_rows make).
template <int FMT>
bool rows_class_f(const SpmvOperand& A, RowClass* out) {
  const int B = A.max_row <= 3 ? 3 : A.max_row <= 5 ? 5 : A.max_row <= 7 ? 7 : 8;
  bool ib3 = false;
  if constexpr (is_gse(FMT)) {
    const ColSplit c3 = col_split(3, false);
    ib3 = A.split.shift == c3.shift && A.split.slot_mask == c3.slot_mask &&
          A.split.col_mask == c3.col_mask && A.split.hmask == c3.hmask && A.split.ei == c3.ei;
  }
  int g = 0;
  switch (B) {
    case 3: g = ib3 ? rows_grid<FMT, 3, false, 3>(A) : rows_grid<FMT, 3, false, -1>(A); break;
    case 5: g = ib3 ? rows_grid<FMT, 5, false, 3>(A) : rows_grid<FMT, 5, false, -1>(A); break;
    case 7: g = ib3 ? rows_grid<FMT, 7, false, 3>(A) : rows_grid<FMT, 7, false, -1>(A); break;
    default: g = ib3 ? rows_grid<FMT, 8, false, 3>(A) : rows_grid<FMT, 8, false, -1>(A); break;
  }
  if (g <= 0) return false;
  *out = RowClass{FMT, B, ib3 ? 3 : -1, g};
  return true;
}

template <int FMT, int B, int IB>
hipError_t launch_grouped_i(const RowGroup* groups, int n_groups, int total, hipStream_t st) {
  hipLaunchKernelGGL((k_spmv_rows_grouped<FMT, B, IB>), dim3(total), dim3(kRingThreads), 0, st,
                     groups, n_groups);
  return hipGetLastError();
}

template <int FMT, int B>
hipError_t launch_grouped_b(int IB, const RowGroup* groups, int n_groups, int total, hipStream_t st) {
  if constexpr (is_gse(FMT)) {
    if (IB == 3) return launch_grouped_i<FMT, B, 3>(groups, n_groups, total, st);
  }
  if (IB != -1) return hipErrorInvalidValue;
  return launch_grouped_i<FMT, B, -1>(groups, n_groups, total, st);
}

template <int FMT>
hipError_t launch_grouped_f(const RowClass& c, const RowGroup* groups, int n_groups, int total,
                            hipStream_t st) {
  switch (c.B) {
    case 3: return launch_grouped_b<FMT, 3>(c.IB, groups, n_groups, total, st);
    case 5: return launch_grouped_b<FMT, 5>(c.IB, groups, n_groups, total, st);
    case 7: return launch_grouped_b<FMT, 7>(c.IB, groups, n_groups, total, st);
    case 8: return launch_grouped_b<FMT, 8>(c.IB, groups, n_groups, total, st);
    default: return hipErrorInvalidValue;
  }
}


// Schedule for one tile size.  With the default 1024-non-zero tiles: the
// row-tile ring when no row holds more than eight non-zeros, the non-zero
// ring for rows of up to kShortRow; otherwise (or in smaller matrices) the
// lean short-row tiles, else the general tiles.
template <int FMT, int E>
hipError_t launch_fe(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                     hipStream_t st) {
  const bool short_rows = A.max_row <= kShortRow;
  int g = 0;
  if constexpr (E * kWG == kRingTile) {
    if (short_rows && A.nnz >= kRingTile) {
      if (A.max_row <= 3) return launch_rows<FMT, 3>(A, x, y, ep, st);
      if (A.max_row <= 5) return launch_rows<FMT, 5>(A, x, y, ep, st);
      if (A.max_row <= 7) return launch_rows<FMT, 7>(A, x, y, ep, st);
      if (A.max_row <= 8) return launch_rows<FMT, 8>(A, x, y, ep, st);
      return launch_ring<FMT>(A, x, y, ep, st);
    }
  }
  if (short_rows) {
    g = grid_for<FMT, E, kShortTiles>(A);
    if (g <= 0) return hipErrorInvalidDevice;
    if (ep.grid_out) *ep.grid_out = g;
    hipLaunchKernelGGL((k_spmv_short<FMT, E>), dim3(g), dim3(kWG), 0, st, A, x, y, ep);
  } else {
    g = grid_for<FMT, E, kGeneralTiles>(A);
    if (g <= 0) return hipErrorInvalidDevice;
    if (ep.grid_out) *ep.grid_out = g;
    hipLaunchKernelGGL((k_spmv<FMT, E>), dim3(g), dim3(kWG), 0, st, A, x, y, ep);
  }
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

// Row-vector schedule for matrices whose rows are short and of similar
// length (stencils): L lanes per row, 64/L rows per wave at a time and U
// rows per lane group in flight.  Lane `sub` of a group reads the row's
// non-zeros sub, sub+L, ... -- so a wave's loads cover consecutive
// non-zeros (coalesced) -- decodes them, gathers x and accumulates; the
// group then combines its L partial sums with a fixed butterfly.  No LDS
// staging and no barriers: every wave is independent, which keeps many
// loads in flight per compute unit.
//
// BLK: per-row-block tables.  The workgroup's rows [wr0, wr1) touch the
// blocks wr0 / R .. (wr1 - 1) / R; their tables are staged back to back in
// LDS and a row reads its own at offset (r / R - first block) * stride.
template <int FMT, int L, bool BLK = false>
__global__ __launch_bounds__(kWG) void k_spmv_rv(SpmvOperand A, const double* __restrict__ x,
                                                 double* __restrict__ y, SpmvEpilogue ep) {
  constexpr int G = 64 / L;
  constexpr int U = kRvBatch;
  constexpr int RB = G * U;  // rows per wave
  __shared__ uint32_t scale_tab[BLK ? kBlockTabEntries : kScaleEntries];
  __shared__ double red[kWaves];

  if (ep.gate && *ep.gate) return;
  const int wtile = xcd_tile(blockIdx.x, gridDim.x);
  int b0 = 0;
  if constexpr (BLK) {
    const int wr0 = wtile * (kWaves * RB);
    const int wr1 = min(wr0 + kWaves * RB, A.n_rows);
    b0 = wr0 / A.block_rows;
    const int n = wr1 > wr0 ? ((wr1 - 1) / A.block_rows - b0 + 1) * A.block_stride : 0;
    build_scale_n<FMT>(A.block_sem + (size_t)b0 * A.block_stride, n, scale_tab, A.split.ei);
  } else {
    build_scale<FMT>(A.sem, scale_tab, A.split.ei);
  }
  const DecodeCtx scale{scale_tab, A.split};
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane / L, sub = lane % L;
  const int wblk = wtile * kWaves + wave;
  const int r0 = wblk * RB;
  double acc = 0.0;
  int toff[U];  // BLK: offset of each row's table in scale_tab
#pragma unroll
  for (int u = 0; u < U; ++u) {
    toff[u] = 0;
    if constexpr (BLK) {
      const int rr = min(r0 + u * G + g, A.n_rows - 1);
      toff[u] = (rr / A.block_rows - b0) * A.block_stride;
    }
  }

  int s0[U], s1[U];
  int mylen = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {  // all 2U row-pointer loads issued before any use
    const int r = r0 + u * G + g;
    const int rr = r < A.n_rows ? r : 0;
    s0[u] = A.row_ptr[rr];
    s1[u] = A.row_ptr[rr + 1];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (r0 + u * G + g >= A.n_rows) s1[u] = s0[u];
    mylen = max(mylen, s1[u] - s0[u]);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mylen = max(mylen, __shfl_xor(mylen, off, 64));
  const int maxlen = mylen;  // uniform over the wave

  double sum[U];
#pragma unroll
  for (int u = 0; u < U; ++u) sum[u] = 0.0;
  for (int kb = 0; kb < maxlen; kb += L) {
    Elem<FMT> e[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = s0[u] + kb + sub;
      ok[u] = j < s1[u];
      e[u].load(A, ok[u] ? j : 0);  // unconditional: all U loads in flight together
    }
    double d[U], xv[U];
    int column[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (BLK) {
        const DecodeCtx own{scale_tab + toff[u], A.split};
        d[u] = decode<FMT>(e[u].c, e[u].h, e[u].t1, e[u].t2, e[u].v, own, column[u]);
      } else {
        d[u] = decode<FMT>(e[u].c, e[u].h, e[u].t1, e[u].t2, e[u].v, scale, column[u]);
      }
      if (!ok[u]) column[u] = 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[column[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double p = __dmul_rn(d[u], xv[u]);
      sum[u] = ok[u] ? __dadd_rn(sum[u], p) : sum[u];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int off = L / 2; off >= 1; off >>= 1) sum[u] += __shfl_xor(sum[u], off, 64);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = r0 + u * G + g;
    if (sub == 0 && r < A.n_rows) {
      if (ep.epi == kEpiPlain) {
        y[r] = sum[u];
      } else if (ep.epi == kEpiDot) {
        y[r] = sum[u];
        acc += ep.aux[r] * sum[u];
      } else {
        const double v = ep.aux[r] - sum[u];
        y[r] = v;
        acc += v * v;
      }
    }
  }

  if (ep.epi != kEpiPlain) {
    const double bs = block_sum(acc, red);
    if (tid == 0) ep.partials[blockIdx.x] = bs;
  }
}

template <int FMT, int L, bool BLK = false>
hipError_t launch_rv(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                     hipStream_t st) {
  constexpr int rows_per_wg = (64 / L) * kRvBatch * kWaves;
  static_assert(rows_per_wg <= kRvMaxRows, "staged block tables sized for kRvMaxRows rows");
  if constexpr (BLK) {
    // the staged tables fit kBlockTabEntries only for blocks this tall
    if (A.n_rows < 1 || !A.block_sem || A.block_rows < GSE_MIN_BLOCK_ROWS ||
        A.block_stride < 1 || A.block_stride > GSE_MAX_EXP)
      return hipErrorInvalidValue;
  }
  int g = (A.n_rows + rows_per_wg - 1) / rows_per_wg;
  if (g < 1) g = 1;
  if (ep.grid_out) *ep.grid_out = g;
  hipLaunchKernelGGL((k_spmv_rv<FMT, L, BLK>), dim3(g), dim3(kWG), 0, st, A, x, y, ep);
  return hipGetLastError();
}

template <int FMT, bool BLK = false>
hipError_t launch_rv_f(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                       hipStream_t st) {
  switch (A.rv_lanes) {
    case 1: return launch_rv<FMT, 1, BLK>(A, x, y, ep, st);
    case 2: return launch_rv<FMT, 2, BLK>(A, x, y, ep, st);
    case 4: return launch_rv<FMT, 4, BLK>(A, x, y, ep, st);
    case 8: return launch_rv<FMT, 8, BLK>(A, x, y, ep, st);
    case 16: return launch_rv<FMT, 16, BLK>(A, x, y, ep, st);
    case 32: return launch_rv<FMT, 32, BLK>(A, x, y, ep, st);
    case 64: return launch_rv<FMT, 64, BLK>(A, x, y, ep, st);
    default: return hipErrorInvalidValue;
  }
}

// Per-row-block tables: the row-tile ring when a 1024-non-zero tile plan was
// asked for and no row holds more than eight non-zeros, else the row-vector
// schedule (its lanes from the plan, or from the mean row length).
template <int FMT>
hipError_t launch_blocks(const SpmvOperand& A, const double* x, double* y, const SpmvEpilogue& ep,
                         hipStream_t st) {
  if (A.rv_lanes == 0 && A.tile_nnz == kRingTile && A.nnz >= kRingTile && A.max_row <= 8) {
    if (A.max_row <= 3) return launch_rows<FMT, 3, true>(A, x, y, ep, st);
    if (A.max_row <= 5) return launch_rows<FMT, 5, true>(A, x, y, ep, st);
    if (A.max_row <= 7) return launch_rows<FMT, 7, true>(A, x, y, ep, st);
    return launch_rows<FMT, 8, true>(A, x, y, ep, st);
  }
  if (A.rv_lanes > 0) return launch_rv_f<FMT, true>(A, x, y, ep, st);
  SpmvOperand o = A;
  const int64_t half = A.n_rows > 0 ? ((int64_t)A.nnz + 2 * (int64_t)A.n_rows - 1) /
                                          (2 * (int64_t)A.n_rows)
                                    : 1;
  o.rv_lanes = 1;
  while (o.rv_lanes < 64 && o.rv_lanes < half) o.rv_lanes *= 2;
  return launch_rv_f<FMT, true>(o, x, y, ep, st);
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

// Longest row: grid-stride, workgroup maximum, one atomic per workgroup.
__global__ __launch_bounds__(256) void k_rowmax(const int32_t* __restrict__ row_ptr, int n_rows,
                                                int* __restrict__ out) {
  __shared__ int red[kWaves];
  int m = 0;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n_rows; r += gridDim.x * blockDim.x)
    m = max(m, row_ptr[r + 1] - row_ptr[r]);
  for (int off = 32; off >= 1; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) m = max(m, red[w]);
    atomicMax(out, m);
  }
}



}  // namespace

int32_t n_tiles_for(int64_t nnz, int32_t tile_nnz) {
  const int64_t t = (nnz + tile_nnz - 1) / tile_nnz;
  return (int32_t)(t < 1 ? 1 : t);
}

hipError_t launch_spmv(int fmt, const SpmvOperand& A, const double* x, double* y,
                       const SpmvEpilogue& ep, hipStream_t st) {
  if (A.block_sem) {  // per-row-block tables
    switch (fmt) {
      case 1: return launch_blocks<1>(A, x, y, ep, st);
      case 2: return launch_blocks<2>(A, x, y, ep, st);
      case 3: return launch_blocks<3>(A, x, y, ep, st);
      default: return hipErrorInvalidValue;
    }
  }
  if (A.rv_lanes > 0) {
    switch (fmt) {
      case 0: return launch_rv_f<0>(A, x, y, ep, st);
      case 1: return launch_rv_f<1>(A, x, y, ep, st);
      case 2: return launch_rv_f<2>(A, x, y, ep, st);
      case 3: return launch_rv_f<3>(A, x, y, ep, st);
      case kFp16: return launch_rv_f<kFp16>(A, x, y, ep, st);
      case kBf16: return launch_rv_f<kBf16>(A, x, y, ep, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (fmt) {
    case 0: return launch_f<0>(A, x, y, ep, st);
    case 1: return launch_f<1>(A, x, y, ep, st);
    case 2: return launch_f<2>(A, x, y, ep, st);
    case 3: return launch_f<3>(A, x, y, ep, st);
    case kFp16: return launch_f<kFp16>(A, x, y, ep, st);
    case kBf16: return launch_f<kBf16>(A, x, y, ep, st);
    default: return hipErrorInvalidValue;
  }
}

bool rows_class(int fmt, const SpmvOperand& A, RowClass* out) {
  if (A.block_sem || A.rv_lanes > 0 || A.tile_nnz != kRingTile || A.nnz < kRingTile || A.max_row > 8 ||
      A.n_rows < 1)
    return false;
  switch (fmt) {
    case 0: return rows_class_f<0>(A, out);
    case 1: return rows_class_f<1>(A, out);
    case 2: return rows_class_f<2>(A, out);
    case 3: return rows_class_f<3>(A, out);
    default: return false;
  }
}

hipError_t launch_rows_grouped(const RowClass& c, const RowGroup* groups, int n_groups, int total,
                               hipStream_t st) {
  if (n_groups < 1 || total < 1) return hipErrorInvalidValue;
  switch (c.fmt) {
    case 0: return launch_grouped_f<0>(c, groups, n_groups, total, st);
    case 1: return launch_grouped_f<1>(c, groups, n_groups, total, st);
    case 2: return launch_grouped_f<2>(c, groups, n_groups, total, st);
    case 3: return launch_grouped_f<3>(c, groups, n_groups, total, st);
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

hipError_t launch_rowmax(const int32_t* row_ptr, int32_t n_rows, int* out, hipStream_t st) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(int), st);
  if (e != hipSuccess) return e;
  int blocks = (n_rows + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_rowmax, dim3(blocks), dim3(256), 0, st, row_ptr, n_rows, out);
  return hipGetLastError();
}

}  // namespace gse

// batch.hip -- batched stepped CG on gfx950: many independent systems of
// uneven size advanced by ONE set of kernel launches per iteration.
//
// Each system keeps its own operator (GSE-SEM planes at its own segment
// count, or FP64 CSR), vectors, state record and stepped controller
// (Section III-D: Algorithm 3, Eqs. 3-6, Conditions 1-3, applied per
// system).  The work of an iteration is flattened into lists -- SpMV tiles
// and row chunks of every live system -- that persistent workgroups walk;
// per-system scalars (alpha, beta, the controller) are finished by one
// workgroup per system.  Kernel boundaries are the only barriers, so no
// workgroup ever waits on another and there are no cross-XCD fences.
//
// A system of at least kRingRows rows of short rows leaves the product
// list: its product runs on the single-system row-tile ring.  All such
// systems that run one ring instance (segment count, row bound, index
// layout) share one grouped launch per iteration, placed between the
// batched product and the r step; in it each system runs its own plain
// launch's grid on a range of workgroups of its own (gated on its stop
// flag on the device) and writes its p.q partials to slots reserved for
// it.  Its vector steps stay in the batched kernels.
//
// The kernels read the list lengths from device memory, so the iteration
// epoch (16 iterations) is captured into a HIP graph once per engine and
// replayed whatever the batch holds (epochs with ring systems, whose
// descriptors are uploaded per epoch, run directly); between epochs the host reads the
// state records back, runs the actions a switch or a convergence candidate
// needs (residual replacement, the all-segment residual check) for the
// systems concerned, and rebuilds the lists when systems finish or arrive.
//
// Every partial sum of a system goes to a slot fixed by that system's own
// tile / chunk index and is summed in a fixed order, so a system's iterates
// are bit-identical whether it is solved alone or among others.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>

#include "batch.h"
#include "decode.h"

namespace gse {

gse_status fail(gse_status code, const char* fmt, ...);
gse_status hip_fail(hipError_t e, const char* where);

namespace {

constexpr int kNS = 2048;       // non-zeros of one tile staged in LDS
constexpr int kLongRow = 64;    // unstaged tiles: longer rows take the whole workgroup
constexpr int kEpochIters = 16;

enum Phase : int {
  kPhFree = 0,
  kPhInit,
  kPhRun,
  kPhCheck,    // the recursive residual met the tolerance: check with all segments
  kPhReplace,  // residual replacement after a switch or a failed check
  kPhFinal,    // stopped: final all-segment residual for the report
  kPhZero,     // b = 0: x = 0
  kPhResetP,   // p = r after a replacement that moved ||r|| by more than 2x
  kPhDone,
};
enum Origin : int { kFromSwitch = 0, kFromCheck = 1 };

// Persistent walk over [0, n): workgroup w works in the range of its XCD
// (workgroups are dispatched to the eight XCDs round-robin), so tiles in
// flight on one XCD are neighbours and share x in its L2.  The grid is a
// multiple of 8; the eight ranges partition [0, n).
struct Walk {
  int i, end, step;
};
__device__ __forceinline__ Walk walk_of(int n) {
  const int nx = (int)(gridDim.x >> 3);
  const int xcd = (int)(blockIdx.x & 7), local = (int)(blockIdx.x >> 3);
  const int b = (int)(((long long)n * xcd) >> 3);
  const int e = (int)(((long long)n * (xcd + 1)) >> 3);
  return Walk{b + local, e, nx};
}

template <int FMT>
__device__ __forceinline__ double load_decode(const BatchSlot& B, int j, const DecodeCtx& scale,
                                              int& col) {
  const uint32_t c = B.col[j];
  uint32_t h = 0, t1 = 0, t2 = 0;
  double v = 0.0;
  if constexpr (FMT == kCsr64) {
    v = B.val[j];
  } else {
    h = B.head[j];
    if constexpr (FMT >= 2) t1 = B.tail1[j];
    if constexpr (FMT == 3) t2 = B.tail2[j];
  }
  return decode<FMT>(c, h, t1, t2, v, scale, col);
}

// Row sums of a staged tile, one thread per row, BW non-zeros per batch: the
// gathers of a batch are issued before any is used; slots past the row's
// end gather x[0] and are left out of the sum.
template <int BW, class Emit>
__device__ __forceinline__ void sum_staged(const BatchSlot& B, int ra, int rb, int j0,
                                           const double* vals, const int* cols,
                                           const double* __restrict__ xin, Emit& emit) {
  for (int r = ra + (int)threadIdx.x; r < rb; r += kWG) {
    const int s0 = B.row_ptr[r], s1 = B.row_ptr[r + 1];
    const int o = s0 - j0, len = s1 - s0;
    double sum = 0.0;
    for (int kb = 0; kb < len; kb += BW) {
      double v[BW], xv[BW];
      int c[BW];
#pragma unroll
      for (int k = 0; k < BW; ++k) {
        v[k] = vals[o + kb + k];
        c[k] = (kb + k < len) ? cols[o + kb + k] : 0;
      }
#pragma unroll
      for (int k = 0; k < BW; ++k) xv[k] = xin[c[k]];
#pragma unroll
      for (int k = 0; k < BW; ++k) {
        const double pr = __dmul_rn(v[k], xv[k]);
        sum = (kb + k < len) ? __dadd_rn(sum, pr) : sum;
      }
    }
    emit(r, sum);
  }
}

// Rows of tile t (those whose first non-zero lies in the tile's range, from
// the matrix's own tile table).  The non-zeros of these rows are decoded
// into LDS when they fit, then each row is summed by one thread in row
// order.  Otherwise (a row running far past the tile) short rows are summed
// from memory by one thread and long ones by the whole workgroup.  Returns
// this thread's share of the epilogue dot.
template <int FMT>
__device__ double tile_rows(const BatchSlot& B, int t, const double* __restrict__ xin,
                            double* __restrict__ yout, const double* __restrict__ aux, int epi,
                            double* vals, int* cols, uint32_t* scale_tab, double* red) {
  const int tid = threadIdx.x;
  const int ra = B.tile_row[t], rb = B.tile_row[t + 1];
  const int j0 = B.row_ptr[ra], j1 = B.row_ptr[rb];
  const int ext = j1 - j0;
  __syncthreads();  // the previous tile is done with LDS
  build_scale<FMT>(B.sem, scale_tab, B.split.ei);
  __syncthreads();
  const DecodeCtx scale{scale_tab, B.split};
  double acc = 0.0;
  auto emit = [&](int r, double sum) {
    if (epi == kEpiDot) {
      yout[r] = sum;
      acc += aux[r] * sum;
    } else {
      const double v = aux[r] - sum;
      yout[r] = v;
      acc += v * v;
    }
  };
  if (ext <= kNS) {
    for (int i = tid; i < ext; i += kWG) {
      int c;
      vals[i] = load_decode<FMT>(B, j0 + i, scale, c);
      cols[i] = c;
    }
    __syncthreads();
    // batches as wide as the longest row when that is at most seven (no
    // gathers for padding slots), else eight; the same row-order sums
    if (B.max_row <= 5)
      sum_staged<5>(B, ra, rb, j0, vals, cols, xin, emit);
    else if (B.max_row <= 7)
      sum_staged<7>(B, ra, rb, j0, vals, cols, xin, emit);
    else
      sum_staged<8>(B, ra, rb, j0, vals, cols, xin, emit);
  } else {
    for (int r = ra + tid; r < rb; r += kWG) {
      const int s0 = B.row_ptr[r], s1 = B.row_ptr[r + 1];
      if (s1 - s0 > kLongRow) continue;
      double sum = 0.0;
      for (int j = s0; j < s1; ++j) {
        int c;
        const double v = load_decode<FMT>(B, j, scale, c);
        sum = __dadd_rn(sum, __dmul_rn(v, xin[c]));
      }
      emit(r, sum);
    }
    for (int r = ra; r < rb; ++r) {  // uniform over the workgroup
      const int s0 = B.row_ptr[r], s1 = B.row_ptr[r + 1];
      if (s1 - s0 <= kLongRow) continue;
      double part = 0.0;
      for (int j = s0 + tid; j < s1; j += kWG) {
        int c;
        const double v = load_decode<FMT>(B, j, scale, c);
        part = __dadd_rn(part, __dmul_rn(v, xin[c]));
      }
      const double sum = block_sum(part, red);
      if (tid == 0) emit(r, sum);
    }
  }
  return acc;
}

// mode 0 (iteration): q = A_s p and the partials of p.q, for systems still
// running.  mode 1 (actions): r = b - A_s x (init / replacement) or
// w = b - A_3 x (check) and the partials of their squared norms.
__global__ __launch_bounds__(kWG) void k_b_spmv(BatchView v, int mode) {
  __shared__ __attribute__((aligned(16))) double vals[kNS + 8];
  __shared__ __attribute__((aligned(16))) int cols[kNS + 8];
  __shared__ uint32_t scale[kScaleEntries];
  __shared__ double red[kWaves];
  const int n = v.list.counts[0];
  for (Walk w = walk_of(n); w.i < w.end; w.i += w.step) {
    const WorkItem it = v.list.tiles[w.i];
    const BatchSlot& B = v.slot[it.slot];
    const SolverState* S = v.S + it.slot;
    int f;
    const double* xin;
    double* yout;
    const double* aux;
    int epi;
    if (mode == 0) {
      if (S->stop) continue;
      f = B.fmt ? S->s : kCsr64;
      xin = B.p;
      yout = B.q;
      aux = B.p;
      epi = kEpiDot;
    } else {
      const int a = v.act[it.slot];
      if (a == kActCheck) {
        f = B.fmt ? 3 : kCsr64;
        yout = B.w;
      } else if (a == kActInit || a == kActReplace || a == kActReplaceP) {
        f = B.fmt ? S->s : kCsr64;
        yout = B.r;
      } else {
        continue;
      }
      xin = B.x;
      aux = B.b;
      epi = kEpiResid;
    }
    double acc;
    switch (f) {
      case 1: acc = tile_rows<1>(B, it.idx, xin, yout, aux, epi, vals, cols, scale, red); break;
      case 2: acc = tile_rows<2>(B, it.idx, xin, yout, aux, epi, vals, cols, scale, red); break;
      case 3: acc = tile_rows<3>(B, it.idx, xin, yout, aux, epi, vals, cols, scale, red); break;
      default: acc = tile_rows<kCsr64>(B, it.idx, xin, yout, aux, epi, vals, cols, scale, red);
    }
    const double bs = block_sum(acc, red);
    if (threadIdx.x == 0) v.part[it.part] = bs;
  }
}

// The scalar steps of an iteration run inside the vector kernels, as in the
// single-system solver: every workgroup that works on a system sums that
// system's partials (a few per system) in a fixed order, and the workgroup
// on the system's chunk 0 publishes the scalars.  Fields a kernel reads are
// never written by another workgroup of that kernel (rho alternates between
// two slots by iteration parity).  A chunk item carries its system's first
// tile partial in `pad` and its own chunk partial in `part` (a system's
// chunk partials are consecutive, so they start at part - idx).

// alpha = rho / p.q; r -= alpha q and the partials of r.r, per row chunk.
__global__ __launch_bounds__(kWG) void k_b_rstep(BatchView v) {
  __shared__ double red[kWaves];
  const int n = v.list.counts[1];
  for (Walk w = walk_of(n); w.i < w.end; w.i += w.step) {
    const WorkItem it = v.list.chunks[w.i];
    SolverState* S = v.S + it.slot;
    const int stop = S->stop;
    if (it.idx == 0 && threadIdx.x == 0) S->go = 0;
    if (stop) continue;
    const BatchSlot& B = v.slot[it.slot];
    const int j = S->it;
    const double rho = S->rho_p[j & 1];
    const double pq = sum_partials(v.part + it.pad, B.n_prod, red);
    const bool broke = !(pq > 0.0) || !isfinite(pq);
    const double alpha = rho / pq;
    // a breakdown (p.q not positive) leaves go at 0 and becomes a stop in
    // the x step: stop is not written here, where other workgroups read it
    // (a stop seen by some waves of a workgroup and not by others would
    // split its barriers); every workgroup reaches the same verdict from pq
    if (it.idx == 0 && threadIdx.x == 0) {
      S->pq = pq;
      if (!broke) {
        S->alpha = alpha;
        S->go = 1;
        S->it_next = j + 1;
      }
    }
    if (broke) continue;
    const int lo = it.idx * kChunk;
    const int hi = min(B.n_rows, lo + kChunk);
    double* __restrict__ r = B.r;
    const double* __restrict__ q = B.q;
    double acc = 0.0;
    if (hi - lo == kChunk) {
      // a whole chunk: the same elements per thread, every load issued first
      constexpr int K = kChunk / kWG;
      double rv[K], qv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        rv[k] = r[lo + threadIdx.x + k * kWG];
        qv[k] = q[lo + threadIdx.x + k * kWG];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double t = rv[k] - alpha * qv[k];
        r[lo + threadIdx.x + k * kWG] = t;
        acc += t * t;
      }
    } else {
      for (int i = lo + threadIdx.x; i < hi; i += kWG) {
        const double rv = r[i] - alpha * q[i];
        r[i] = rv;
        acc += rv * rv;
      }
    }
    const double bs = block_sum(acc, red);
    if (threadIdx.x == 0) v.part2[it.part] = bs;
  }
}

// beta = rho' / rho; x += alpha p, p = r + beta p per row chunk; on chunk 0
// the history, the iteration count and the controller.
__global__ __launch_bounds__(kWG) void k_b_xstep(BatchView v) {
  __shared__ double red[kWaves];
  __shared__ double bc_rel;
  const int n = v.list.counts[1];
  for (Walk w = walk_of(n); w.i < w.end; w.i += w.step) {
    const WorkItem it = v.list.chunks[w.i];
    SolverState* S = v.S + it.slot;
    if (!S->go) {
      // the r step found no positive p.q for a running system: stop it
      if (it.idx == 0 && threadIdx.x == 0 && S->stop == kRun) {
        const double pq = S->pq;
        if (!(pq > 0.0) || !isfinite(pq)) S->stop = kBreak;
      }
      continue;
    }
    const BatchSlot& B = v.slot[it.slot];
    const int j = S->it_next;
    const double rho_old = S->rho_p[(j - 1) & 1];
    const double alpha = S->alpha;
    const double rho_new = sum_partials(v.part2 + (it.part - it.idx), B.n_chunks, red);
    const double beta = rho_new / rho_old;
    const int lo = it.idx * kChunk;
    const int hi = min(B.n_rows, lo + kChunk);
    double* __restrict__ x = B.x;
    double* __restrict__ p = B.p;
    const double* __restrict__ r = B.r;
    if (hi - lo == kChunk) {
      // a whole chunk: the same elements per thread, every load issued first
      constexpr int K = kChunk / kWG;
      double xv[K], pv[K], rv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = lo + threadIdx.x + k * kWG;
        xv[k] = x[i];
        pv[k] = p[i];
        rv[k] = r[i];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = lo + threadIdx.x + k * kWG;
        x[i] = xv[k] + alpha * pv[k];
        p[i] = rv[k] + beta * pv[k];
      }
    } else {
      for (int i = lo + threadIdx.x; i < hi; i += kWG) {
        const double pv = p[i];
        x[i] += alpha * pv;
        p[i] = r[i] + beta * pv;
      }
    }
    if (it.idx != 0) continue;
    const int s = S->s;
    if (threadIdx.x == 0) {
      const double rel = sqrt(rho_new) / S->nb;
      S->beta = beta;
      S->rho_p[j & 1] = rho_new;
      S->rho = rho_new;
      S->it = j;
      S->relres = rel;
      B.hist[j] = rel;
      B.seg_hist[j] = s;
      bc_rel = rel;
    }
    __syncthreads();
    controller(S, B.hist, red, j, bc_rel, s);
    __syncthreads();
  }
}

// Actions: partials of b.b for systems being initialised.
__global__ __launch_bounds__(kWG) void k_b_bdot(BatchView v) {
  __shared__ double red[kWaves];
  const int n = v.list.counts[1];
  for (Walk w = walk_of(n); w.i < w.end; w.i += w.step) {
    const WorkItem it = v.list.chunks[w.i];
    if (v.act[it.slot] != kActInit) continue;
    const BatchSlot& B = v.slot[it.slot];
    const int lo = it.idx * kChunk;
    const int hi = min(B.n_rows, lo + kChunk);
    double acc = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += kWG) acc += B.b[i] * B.b[i];
    const double bs = block_sum(acc, red);
    if (threadIdx.x == 0) v.part2[it.part] = bs;
  }
}

// Actions: finish the sums of k_b_bdot / k_b_spmv(mode 1) per system.
__global__ __launch_bounds__(kWG) void k_b_act_finish(BatchView v) {
  __shared__ double red[kWaves];
  const int n = v.list.counts[2];
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const SlotItem si = v.list.slots[k];
    const int a = v.act[si.slot];
    SolverState* S = v.S + si.slot;
    const BatchSlot& B = v.slot[si.slot];
    if (a == kActInit) {
      const double nb2 = sum_partials(v.part2 + si.vpart, B.n_chunks, red);
      const double rho = sum_partials(v.part + si.part, B.n_tiles, red);
      if (threadIdx.x == 0) {
        const double nb = sqrt(nb2);
        const double rel = nb > 0.0 ? sqrt(rho) / nb : 0.0;
        S->nb2 = nb2;
        S->nb = nb;
        S->rho = rho;
        S->rho_p[S->it & 1] = rho;
        S->relres = rel;
        B.hist[0] = rel;
        B.seg_hist[0] = S->s;
      }
    } else if (a == kActReplace || a == kActReplaceP) {
      const double rho = sum_partials(v.part + si.part, B.n_tiles, red);
      if (threadIdx.x == 0) {
        S->rho = rho;
        S->rho_p[S->it & 1] = rho;
      }
    } else if (a == kActCheck) {
      const double ww = sum_partials(v.part + si.part, B.n_tiles, red);
      if (threadIdx.x == 0) S->scratch[0] = ww;
    }
    __syncthreads();
  }
}

// Actions: p = r (init, replacement with restart, reset after a large
// replacement), x = 0 (b = 0).
__global__ __launch_bounds__(kWG) void k_b_copy(BatchView v) {
  const int n = v.list.counts[1];
  for (Walk w = walk_of(n); w.i < w.end; w.i += w.step) {
    const WorkItem it = v.list.chunks[w.i];
    const int a = v.act[it.slot];
    if (a != kActInit && a != kActReplaceP && a != kActZeroX && a != kActResetP) continue;
    const BatchSlot& B = v.slot[it.slot];
    const int lo = it.idx * kChunk;
    const int hi = min(B.n_rows, lo + kChunk);
    if (a == kActZeroX) {
      for (int i = lo + threadIdx.x; i < hi; i += kWG) B.x[i] = 0.0;
    } else {
      for (int i = lo + threadIdx.x; i < hi; i += kWG) B.p[i] = B.r[i];
    }
  }
}

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

constexpr int64_t kMagic = 0x4253454742415443LL;

template <typename K>
int grid_for(K kernel, int64_t items) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWG, 0) != hipSuccess) return 0;
  int64_t g = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  const int64_t need = (items + 7) / 8 * 8;
  if (g > need) g = need;
  g = g / 8 * 8;
  return g < 8 ? 8 : (int)g;
}

}  // namespace

// ---------------------------------------------------------------- engine --
size_t BatchEngine::region_bytes(int cap_slots, int64_t cap_tiles, int64_t cap_chunks) {
  size_t b = align_up(sizeof(RegionHeader));
  for (int l = 0; l < 2; ++l) {
    b += align_up(4 * sizeof(int32_t));
    b += align_up((size_t)cap_tiles * sizeof(WorkItem));
    b += align_up((size_t)cap_chunks * sizeof(WorkItem));
    b += align_up((size_t)cap_slots * sizeof(SlotItem));
  }
  b += align_up((size_t)cap_slots * sizeof(BatchSlot));
  b += align_up((size_t)cap_slots * sizeof(SolverState));
  b += align_up((size_t)cap_slots * sizeof(int32_t));
  b += align_up((size_t)cap_tiles * sizeof(double));
  b += align_up((size_t)cap_chunks * sizeof(double));
  b += align_up((size_t)cap_slots * sizeof(RowGroup));
  return b;
}

gse_status BatchEngine::init(void* region, size_t bytes, int cap_slots, int64_t cap_tiles,
                             int64_t cap_chunks, hipStream_t st, bool graphs) {
  if (cap_slots < 1 || cap_tiles < 1 || cap_chunks < 1 || cap_tiles > INT32_MAX ||
      cap_chunks > INT32_MAX)
    return fail(GSE_ERR_ARG, "batch capacities out of range");
  if (region_bytes(cap_slots, cap_tiles, cap_chunks) > bytes)
    return fail(GSE_ERR_NOMEM, "batch tables need %zu bytes",
                region_bytes(cap_slots, cap_tiles, cap_chunks));
  cap_slots_ = cap_slots;
  cap_tiles_ = cap_tiles;
  cap_chunks_ = cap_chunks;
  st_ = st;
  graphs_ = graphs;
  char* p = reinterpret_cast<char*>(region);
  size_t off = 0;
  auto take = [&](size_t n) {
    char* q = p + off;
    off += align_up(n);
    return q;
  };
  RegionHeader* hdr = reinterpret_cast<RegionHeader*>(take(sizeof(RegionHeader)));
  for (int l = 0; l < 2; ++l) {
    counts_[l] = reinterpret_cast<int32_t*>(take(4 * sizeof(int32_t)));
    tiles_[l] = reinterpret_cast<WorkItem*>(take((size_t)cap_tiles * sizeof(WorkItem)));
    chunks_[l] = reinterpret_cast<WorkItem*>(take((size_t)cap_chunks * sizeof(WorkItem)));
    slot_items_[l] = reinterpret_cast<SlotItem*>(take((size_t)cap_slots * sizeof(SlotItem)));
  }
  slots_ = reinterpret_cast<BatchSlot*>(take((size_t)cap_slots * sizeof(BatchSlot)));
  S_ = reinterpret_cast<SolverState*>(take((size_t)cap_slots * sizeof(SolverState)));
  act_ = reinterpret_cast<int32_t*>(take((size_t)cap_slots * sizeof(int32_t)));
  part_ = reinterpret_cast<double*>(take((size_t)cap_tiles * sizeof(double)));
  part2_ = reinterpret_cast<double*>(take((size_t)cap_chunks * sizeof(double)));
  groups_ = reinterpret_cast<RowGroup*>(take((size_t)cap_slots * sizeof(RowGroup)));

  hslot_.assign((size_t)cap_slots, BatchSlot{});
  hS_.assign((size_t)cap_slots, SolverState{});
  hact_.assign((size_t)cap_slots, 0);
  meta_.assign((size_t)cap_slots, SlotHost{});
  used_.assign((size_t)cap_slots, 0);
  prod_off_.assign((size_t)cap_slots, 0);
  ring_ids_.clear();
  for (int l = 0; l < 2; ++l) {
    hcounts_[l][0] = hcounts_[l][1] = hcounts_[l][2] = hcounts_[l][3] = 0;
  }
  hhdr_ = RegionHeader{kMagic, cap_slots, 0, (int64_t)((char*)slots_ - p),
                       (int64_t)((char*)S_ - p)};
  grid_spmv_ = grid_for(k_b_spmv, cap_tiles);
  grid_vec_ = grid_for(k_b_rstep, cap_chunks);
  grid_slot_ = cap_slots < 1024 ? cap_slots : 1024;
  if (grid_spmv_ <= 0 || grid_vec_ <= 0) return fail(GSE_ERR_HIP, "batch: device query failed");
  hipError_t e = hipMemcpyAsync(hdr, &hhdr_, sizeof hhdr_, hipMemcpyHostToDevice, st_);
  if (e == hipSuccess)
    e = hipMemcpyAsync(counts_[0], hcounts_[0], sizeof hcounts_[0], hipMemcpyHostToDevice, st_);
  if (e == hipSuccess)
    e = hipMemcpyAsync(counts_[1], hcounts_[1], sizeof hcounts_[1], hipMemcpyHostToDevice, st_);
  if (e == hipSuccess)
    e = hipMemcpyAsync(act_, hact_.data(), hact_.size() * sizeof(int32_t), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return hip_fail(e, "batch init");
  return GSE_OK;
}

BatchEngine::~BatchEngine() {
  if (graph_) (void)hipGraphExecDestroy(graph_);
}

int BatchEngine::add(const BatchSlot& d, const gse_params* p, const double* eta) {
  int id = -1;
  for (int i = 0; i < cap_slots_; ++i)
    if (!used_[i]) {
      id = i;
      break;
    }
  if (id < 0) return fail(GSE_ERR_NOMEM, "no free batch slot");
  BatchSlot dd = d;
  RowClass rc{};
  dd.ring = (d.n_rows >= kRingRows && rows_class(d.fmt ? 1 : kCsr64, ring_operand(d), &rc)) ? 1 : 0;
  // the ring's grid is at most the row tiles rounded up to 8, and at least 8
  const int32_t rt = (int32_t)(((int64_t)d.n_rows + 191) / 192);
  const int32_t rt8 = (rt + 7) / 8 * 8;
  dd.parts = dd.ring ? std::max(d.n_tiles, std::max(rt8, 8)) : d.n_tiles;
  dd.n_prod = d.n_tiles;
  int64_t tiles = dd.parts, chunks = d.n_chunks;
  for (int i = 0; i < cap_slots_; ++i)
    if (used_[i] && meta_[i].phase != kPhDone) {
      tiles += hslot_[i].parts;
      chunks += hslot_[i].n_chunks;
    }
  if (tiles > cap_tiles_ || chunks > cap_chunks_)
    return fail(GSE_ERR_NOMEM, "batch lists full (%lld tiles, %lld chunks)", (long long)tiles,
                (long long)chunks);
  hslot_[id] = dd;
  SolverState& S = hS_[id];
  memset(&S, 0, sizeof S);
  const bool gse = d.fmt != 0;
  const bool stepped = gse && p->fixed_segments == 0;
  S.tol = p->tol;
  for (int i = 0; i < 3; ++i) S.eta[i] = (gse && eta) ? eta[i] : 0.0;
  S.floor_c = p->floor_c;
  S.rsd_limit = p->rsd_limit;
  S.reldec_limit = p->reldec_limit;
  S.s = gse ? (stepped ? p->start_segments : p->fixed_segments) : 0;
  S.max_iter = p->max_iter;
  S.stepped = stepped ? 1 : 0;
  S.fixed = gse ? p->fixed_segments : -1;
  S.l = p->l;
  S.t = p->t;
  S.m = p->m;
  S.ndec_limit = p->ndec_limit;
  S.ndec_rule = p->ndec_rule;
  S.hist_cap = p->max_iter + 2;
  SlotHost& m = meta_[id];
  m = SlotHost{};
  m.phase = kPhInit;
  m.stepped = stepped;
  m.s_final = gse ? 3 : 0;
  m.tol = p->tol;
  m.max_iter = p->max_iter;
  m.switch_mode = p->switch_mode;
  m.rep.switch_iter[0] = m.rep.switch_iter[1] = -1;
  m.t0 = std::chrono::steady_clock::now();
  used_[id] = 1;
  hact_[id] = kActNone;
  ++n_live_;
  hipError_t e = hipMemcpyAsync(slots_ + id, &hslot_[id], sizeof(BatchSlot), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  if (e != hipSuccess) return hip_fail(e, "batch add");
  return id;
}

void BatchEngine::release(int slot) {
  if (slot < 0 || slot >= cap_slots_ || !used_[slot]) return;
  if (meta_[slot].phase != kPhDone) {
    --n_live_;
    run_dirty_ = true;
  }
  used_[slot] = 0;
  meta_[slot].phase = kPhFree;
}

gse_status BatchEngine::upload_list(int l, const std::vector<int>& ids) {
  std::vector<WorkItem>& wt = wt_[l];
  std::vector<WorkItem>& wc = wc_[l];
  std::vector<SlotItem>& wsl = ws_[l];
  wt.clear();
  wc.clear();
  wsl.clear();
  int64_t pt = 0, pc = 0;
  if (l == 0) ring_ids_.clear();
  for (int id : ids) {
    const BatchSlot& B = hslot_[id];
    wsl.push_back(SlotItem{id, (int32_t)pt, (int32_t)pc, 0});
    // in the iteration list a ring system's product is its own launch
    if (l == 0 && B.ring) {
      ring_ids_.push_back(id);
    } else {
      for (int t = 0; t < B.n_tiles; ++t) wt.push_back(WorkItem{id, t, (int32_t)(pt + t), 0});
    }
    for (int c = 0; c < B.n_chunks; ++c) wc.push_back(WorkItem{id, c, (int32_t)(pc + c), (int32_t)pt});
    if (l == 0) prod_off_[id] = (int32_t)pt;
    pt += B.parts;
    pc += B.n_chunks;
  }
  if (pt > cap_tiles_ || pc > cap_chunks_ || (int64_t)ids.size() > cap_slots_)
    return fail(GSE_ERR_NOMEM, "batch lists overflow");
  hcounts_[l][0] = (int32_t)wt.size();
  hcounts_[l][1] = (int32_t)wc.size();
  hcounts_[l][2] = (int32_t)wsl.size();
  hcounts_[l][3] = 0;
  hipError_t e = hipSuccess;
  if (!wt.empty())
    e = hipMemcpyAsync(tiles_[l], wt.data(), wt.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess && !wc.empty())
    e = hipMemcpyAsync(chunks_[l], wc.data(), wc.size() * sizeof(WorkItem), hipMemcpyHostToDevice, st_);
  if (e == hipSuccess && !wsl.empty())
    e = hipMemcpyAsync(slot_items_[l], wsl.data(), wsl.size() * sizeof(SlotItem), hipMemcpyHostToDevice,
                       st_);
  if (e == hipSuccess)
    e = hipMemcpyAsync(counts_[l], hcounts_[l], sizeof hcounts_[l], hipMemcpyHostToDevice, st_);
  if (e != hipSuccess) return hip_fail(e, "batch lists");
  return GSE_OK;
}

BatchView BatchEngine::view(int l) const {
  BatchView v{};
  v.list.counts = counts_[l];
  v.list.tiles = tiles_[l];
  v.list.chunks = chunks_[l];
  v.list.slots = slot_items_[l];
  v.slot = slots_;
  v.S = S_;
  v.act = act_;
  v.part = part_;
  v.part2 = part2_;
  return v;
}

hipError_t BatchEngine::launch_epoch_kernels(int iters) {
  const BatchView v = view(0);
  // the ring systems' products at this epoch's segment counts, grouped by
  // kernel instance: each system keeps the grid and partials of its own
  // plain launch, so its product does not depend on the batch around it
  ring_launches_.clear();
  hgroups_.clear();
  if (!ring_ids_.empty()) {
    std::vector<std::pair<RowClass, int>> cls;
    for (int id : ring_ids_) {
      const BatchSlot& B = hslot_[id];
      RowClass c{};
      if (!rows_class(B.fmt ? hS_[id].s : kCsr64, ring_operand(B), &c) || c.grid > B.parts)
        return hipErrorInvalidValue;
      cls.push_back({c, id});
    }
    auto key = [](const RowClass& c) { return (c.fmt * 16 + c.B) * 8 + (c.IB + 1); };
    std::stable_sort(cls.begin(), cls.end(),
                     [&](const std::pair<RowClass, int>& a, const std::pair<RowClass, int>& b) {
                       return key(a.first) < key(b.first);
                     });
    for (size_t i = 0; i < cls.size(); ++i) {
      const RowClass& c = cls[i].first;
      const int id = cls[i].second;
      if (i == 0 || key(c) != key(cls[i - 1].first))
        ring_launches_.push_back(RingLaunch{c, (int)hgroups_.size(), 0, 0});
      RingLaunch& L = ring_launches_.back();
      BatchSlot& B = hslot_[id];
      SpmvEpilogue ep{};
      ep.epi = kEpiDot;
      ep.aux = B.p;
      ep.partials = part_ + prod_off_[id];
      ep.gate = &S_[id].stop;
      hgroups_.push_back(RowGroup{ring_operand(B), B.p, B.q, ep, L.total, c.grid});
      L.total += c.grid;
      ++L.n;
      if (c.grid != B.n_prod) {  // ordered before the r step that sums them
        B.n_prod = c.grid;
        const hipError_t e = hipMemcpyAsync(&slots_[id].n_prod, &B.n_prod, sizeof(int32_t),
                                            hipMemcpyHostToDevice, st_);
        if (e != hipSuccess) return e;
      }
    }
    const hipError_t e = hipMemcpyAsync(groups_, hgroups_.data(), hgroups_.size() * sizeof(RowGroup),
                                        hipMemcpyHostToDevice, st_);
    if (e != hipSuccess) return e;
  }
  // a captured epoch keeps the batched product whatever the lists hold; a
  // direct one leaves it out when no system has tiles in it
  const bool tiles = ring_ids_.empty() || hcounts_[0][0] > 0;
  for (int k = 0; k < iters; ++k) {
    if (tiles) hipLaunchKernelGGL(k_b_spmv, dim3(grid_spmv_), dim3(kWG), 0, st_, v, 0);
    for (const RingLaunch& L : ring_launches_) {
      const hipError_t e = launch_rows_grouped(L.c, groups_ + L.first, L.n, L.total, st_);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_b_rstep, dim3(grid_vec_), dim3(kWG), 0, st_, v);
    hipLaunchKernelGGL(k_b_xstep, dim3(grid_vec_), dim3(kWG), 0, st_, v);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

SpmvOperand ring_operand(const BatchSlot& B) {
  SpmvOperand op{};
  op.row_ptr = B.row_ptr;
  op.tile_row = B.tile_row;
  op.col = B.col;
  op.head = B.head;
  op.tail1 = B.tail1;
  op.tail2 = B.tail2;
  op.val = B.val;
  op.n_rows = B.n_rows;
  op.n_tiles = B.n_tiles;
  op.tile_nnz = B.tile_nnz;
  op.nnz = B.nnz;
  op.rv_lanes = B.rv_lanes;
  op.max_row = B.max_row;
  op.split = B.split;
  for (int i = 0; i < GSE_MAX_EXP; ++i) op.sem[i] = B.sem[i];
  op.block_sem = nullptr;
  op.block_rows = 0;
  op.block_stride = 0;
  return op;
}

hipError_t BatchEngine::sync_states_in() {
  hipError_t e = hipMemcpyAsync(hS_.data(), S_, hS_.size() * sizeof(SolverState),
                                hipMemcpyDeviceToHost, st_);
  if (e == hipSuccess) e = hipStreamSynchronize(st_);
  return e;
}

hipError_t BatchEngine::sync_states_out() {
  return hipMemcpyAsync(S_, hS_.data(), hS_.size() * sizeof(SolverState), hipMemcpyHostToDevice, st_);
}

void BatchEngine::resume(int id) {
  SolverState& S = hS_[id];
  S.stop = kRun;
  S.trig = 0;
  S.go = 0;
  meta_[id].phase = kPhRun;
  run_dirty_ = true;
}

void BatchEngine::tol_met(int id) {
  SlotHost& m = meta_[id];
  SolverState& S = hS_[id];
  const bool exact_op = !m.stepped || S.s >= 3 || S.eta[S.s - 1] == 0.0;
  if (exact_op) {
    m.phase = kPhCheck;
    return;
  }
  if (m.nsw < 2) {
    m.rep.switch_iter[m.nsw] = S.it;
    m.rep.switch_trigger[m.nsw] = GSE_TRIG_TOL;
  }
  ++m.nsw;
  S.s += 1;
  m.phase = kPhReplace;
  m.reset_p = m.switch_mode == 0;
  m.rho_before = S.rho_p[S.it & 1];
  m.origin = kFromSwitch;
}

gse_status BatchEngine::finish(int id, int status, std::vector<int>* done) {
  SlotHost& m = meta_[id];
  const SolverState& S = hS_[id];
  m.rep.status = status;
  m.rep.iters = S.it;
  m.rep.relres_recursive = S.relres;
  m.rep.iters_per_seg[0] = m.rep.iters_per_seg[1] = m.rep.iters_per_seg[2] = 0;
  const int cnt = S.it;
  if (cnt > 0) {
    seg_buf_.resize((size_t)cnt + 1);
    hipError_t e = hipMemcpyAsync(seg_buf_.data(), hslot_[id].seg_hist, sizeof(int32_t) * (size_t)(cnt + 1),
                                  hipMemcpyDeviceToHost, st_);
    if (e == hipSuccess) e = hipStreamSynchronize(st_);
    if (e != hipSuccess) return hip_fail(e, "batch report");
    for (int i = 1; i <= cnt; ++i) {
      const int sg = seg_buf_[i] <= 0 ? 3 : seg_buf_[i];
      m.rep.iters_per_seg[sg - 1] += 1;
    }
  }
  m.rep.time_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - m.t0).count();
  m.phase = kPhDone;
  --n_live_;
  run_dirty_ = true;
  if (done) done->push_back(id);
  return GSE_OK;
}

// One round of per-system actions (the host logic of the single-system CG
// driver, applied to every system that stopped).
gse_status BatchEngine::actions(std::vector<int>* done) {
  std::vector<int>& ids = ids_;
  ids.clear();
  for (int i = 0; i < cap_slots_; ++i) {
    if (!used_[i]) continue;
    int a = kActNone;
    switch (meta_[i].phase) {
      case kPhInit: a = kActInit; break;
      case kPhCheck: a = kActCheck; break;
      case kPhFinal: a = kActCheck; break;
      case kPhReplace: a = meta_[i].reset_p ? kActReplaceP : kActReplace; break;
      case kPhResetP: a = kActResetP; break;
      case kPhZero: a = kActZeroX; break;
      default: break;
    }
    hact_[i] = a;
    if (a != kActNone) ids.push_back(i);
  }
  if (ids.empty()) return GSE_OK;
  gse_status s = upload_list(1, ids);
  if (s != GSE_OK) return s;
  hipError_t e = hipMemcpyAsync(act_, hact_.data(), hact_.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st_);
  if (e == hipSuccess) e = sync_states_out();
  if (e == hipSuccess) {
    const BatchView v = view(1);
    hipLaunchKernelGGL(k_b_bdot, dim3(grid_vec_), dim3(kWG), 0, st_, v);
    hipLaunchKernelGGL(k_b_spmv, dim3(grid_spmv_), dim3(kWG), 0, st_, v, 1);
    hipLaunchKernelGGL(k_b_act_finish, dim3(grid_slot_), dim3(kWG), 0, st_, v);
    hipLaunchKernelGGL(k_b_copy, dim3(grid_vec_), dim3(kWG), 0, st_, v);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = sync_states_in();
  if (e != hipSuccess) return hip_fail(e, "batch actions");
  for (int id : ids) {
    SlotHost& m = meta_[id];
    SolverState& S = hS_[id];
    hact_[id] = kActNone;
    switch (m.phase) {
      case kPhInit:
        if (S.nb == 0.0) {
          m.phase = kPhZero;
        } else if (S.relres <= m.tol) {
          tol_met(id);
        } else {
          resume(id);
        }
        break;
      case kPhZero:
        m.rep.relres_true = 0.0;
        S.relres = 0.0;
        s = finish(id, GSE_OK, done);
        break;
      case kPhCheck: {
        const double rt = sqrt(S.scratch[0]) / S.nb;
        if (rt <= m.tol) {
          m.rep.relres_true = rt;
          s = finish(id, GSE_OK, done);
        } else {  // the recursive residual drifted from the true one
          m.phase = kPhReplace;
          m.reset_p = true;
          m.origin = kFromCheck;
        }
        break;
      }
      case kPhFinal:
        m.rep.relres_true = sqrt(S.scratch[0]) / S.nb;
        s = finish(id, m.final_status, done);
        break;
      case kPhReplace:
      case kPhResetP: {
        if (m.phase == kPhReplace && m.origin == kFromSwitch && m.switch_mode == 2 &&
            restart_direction(2, m.rho_before, S.rho)) {
          m.phase = kPhResetP;  // one more round: p = r
          break;
        }
        S.relres = sqrt(S.rho) / S.nb;
        if (m.origin == kFromCheck) {
          if (S.relres <= m.tol || S.it >= m.max_iter) {
            m.final_status = GSE_NOT_CONVERGED;
            m.phase = kPhFinal;
          } else {
            resume(id);
          }
        } else {
          if (S.relres <= m.tol) {
            tol_met(id);
          } else if (S.it >= m.max_iter) {
            m.final_status = GSE_NOT_CONVERGED;
            m.phase = kPhFinal;
          } else {
            resume(id);
          }
        }
        break;
      }
      default: break;
    }
    if (s != GSE_OK) return s;
  }
  return GSE_OK;
}

// One epoch of iterations for every running system, then the stops.
gse_status BatchEngine::epoch() {
  std::vector<int>& ids = ids_;
  ids.clear();
  for (int i = 0; i < cap_slots_; ++i)
    if (used_[i] && meta_[i].phase == kPhRun) ids.push_back(i);
  if (ids.empty()) return GSE_OK;
  gse_status s = GSE_OK;
  if (run_dirty_) {
    s = upload_list(0, ids);
    if (s != GSE_OK) return s;
    run_dirty_ = false;
  }
  hipError_t e = sync_states_out();
  if (e == hipSuccess) {
    // the captured epoch holds the batched kernels only: epochs with ring
    // systems (one product launch each, host-side arguments) run directly
    if (graphs_ && ring_ids_.empty()) {
      if (!graph_) e = capture(st_, &graph_, [&] { return launch_epoch_kernels(kEpochIters); });
      if (e == hipSuccess) e = hipGraphLaunch(graph_, st_);
    } else {
      e = launch_epoch_kernels(kEpochIters);
    }
  }
  if (e == hipSuccess) e = sync_states_in();
  if (e != hipSuccess) return hip_fail(e, "batch epoch");
  for (int id : ids) {
    SlotHost& m = meta_[id];
    SolverState& S = hS_[id];
    if (S.stop == kRun) continue;
    int reason = S.stop, trig = S.trig;
    run_dirty_ = true;
    if (reason == kBreak) {
      if (m.stepped && S.s < 3) {
        reason = kSwitch;
        trig = GSE_TRIG_BREAKDOWN;
      } else {
        m.final_status = GSE_ERR_BREAKDOWN;
        m.phase = kPhFinal;
        continue;
      }
    }
    if (reason == kConv) {
      m.phase = kPhCheck;
    } else if (reason == kSwitch) {
      if (m.nsw < 2) {
        m.rep.switch_iter[m.nsw] = S.it;
        m.rep.switch_trigger[m.nsw] = trig;
      }
      ++m.nsw;
      S.s += 1;
      m.phase = kPhReplace;
      m.reset_p = m.switch_mode == 0;
      m.rho_before = S.rho_p[S.it & 1];
      m.origin = kFromSwitch;
    } else {  // cap
      m.final_status = GSE_NOT_CONVERGED;
      m.phase = kPhFinal;
    }
  }
  return GSE_OK;
}

gse_status BatchEngine::step(std::vector<int>* done) {
  bool pending = false, running = false;
  for (int i = 0; i < cap_slots_; ++i) {
    if (!used_[i]) continue;
    const int ph = meta_[i].phase;
    if (ph == kPhRun) running = true;
    else if (ph != kPhDone && ph != kPhFree) pending = true;
  }
  if (pending) return actions(done);
  if (running) return epoch();
  return GSE_OK;
}

// --------------------------------------------------------- gse_batch_cg --
namespace {

struct BatchLayout {
  size_t engine = 0;  // region at offset 0
  std::vector<size_t> vec_off;  // per system: r, p, q, w, hist, seg
  size_t bytes = 0;
  int64_t tiles = 0, chunks = 0;
};

BatchLayout batch_layout(int32_t n_sys, const BatchSystemDesc* d, int32_t max_iter) {
  BatchLayout L;
  for (int i = 0; i < n_sys; ++i) {
    // room for the ring's partials too (BatchEngine::add reserves the same)
    const int64_t rt8 = ((int64_t)(d[i].n_rows + 191) / 192 + 7) / 8 * 8;
    L.tiles += std::max<int64_t>(d[i].n_tiles, std::max<int64_t>(rt8, 8));
    L.chunks += (d[i].n_rows + kChunk - 1) / kChunk;
  }
  L.engine = BatchEngine::region_bytes(n_sys, L.tiles, L.chunks);
  size_t off = L.engine;
  for (int i = 0; i < n_sys; ++i) {
    L.vec_off.push_back(off);
    const size_t n = (size_t)d[i].n_rows;
    off += 4 * align_up(n * sizeof(double));
    off += align_up((size_t)(max_iter + 2) * sizeof(double));
    off += align_up((size_t)(max_iter + 2) * sizeof(int32_t));
  }
  L.bytes = off;
  return L;
}

}  // namespace

size_t batch_workspace_bytes(int32_t n_sys, const BatchSystemDesc* d, int32_t max_iter) {
  return batch_layout(n_sys, d, max_iter).bytes;
}

gse_status batch_cg(int32_t n_sys, const BatchSystemDesc* d, const gse_params* p, gse_report* rep,
                    void* ws, size_t ws_bytes, hipStream_t caller) {
  const BatchLayout L = batch_layout(n_sys, d, p->max_iter);
  if (L.bytes > ws_bytes) return fail(GSE_ERR_NOMEM, "batch workspace needs %zu bytes", L.bytes);
  SolveStream ss(caller);
  if (ss.err != hipSuccess) return hip_fail(ss.err, "batch stream");
  BatchEngine eng;
  gse_status s = eng.init(ws, L.engine, n_sys, L.tiles, L.chunks, ss.s, p->launch_mode == 0);
  if (s != GSE_OK) return s;
  char* base = reinterpret_cast<char*>(ws);
  for (int i = 0; i < n_sys; ++i) {
    BatchSlot B = d[i].slot;
    const size_t n = (size_t)B.n_rows;
    char* q = base + L.vec_off[i];
    auto take = [&](size_t nbytes) {
      char* r = q;
      q += align_up(nbytes);
      return r;
    };
    B.r = reinterpret_cast<double*>(take(n * sizeof(double)));
    B.p = reinterpret_cast<double*>(take(n * sizeof(double)));
    B.q = reinterpret_cast<double*>(take(n * sizeof(double)));
    B.w = reinterpret_cast<double*>(take(n * sizeof(double)));
    B.hist = reinterpret_cast<double*>(take((size_t)(p->max_iter + 2) * sizeof(double)));
    B.seg_hist = reinterpret_cast<int32_t*>(take((size_t)(p->max_iter + 2) * sizeof(int32_t)));
    B.n_chunks = (B.n_rows + kChunk - 1) / kChunk;
    const int id = eng.add(B, p, d[i].eta);
    if (id < 0) return id;
    if (id != i) return fail(GSE_ERR_ARG, "batch slot order");
  }
  while (!eng.idle()) {
    s = eng.step(nullptr);
    if (s != GSE_OK) return s;
  }
  gse_status worst = GSE_OK;
  for (int i = 0; i < n_sys; ++i) {
    rep[i] = eng.report(i);
    if (rep[i].status != GSE_OK && worst == GSE_OK) worst = rep[i].status;
  }
  return worst == GSE_OK ? GSE_OK : (worst == GSE_NOT_CONVERGED ? GSE_NOT_CONVERGED : worst);
}

gse_status batch_history(const void* ws, int32_t index, int32_t cap, double* hist, int32_t* seg,
                         hipStream_t st) {
  RegionHeader h;
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_batch_history");
  if (h.magic != kMagic) return fail(GSE_ERR_ARG, "no batch solve recorded in this workspace");
  if (index < 0 || index >= h.n_slots) return fail(GSE_ERR_ARG, "system index out of range");
  const char* base = reinterpret_cast<const char*>(ws);
  BatchSlot B;
  SolverState S;
  e = hipMemcpyAsync(&B, base + h.slots_off + (int64_t)index * (int64_t)sizeof(BatchSlot), sizeof B,
                     hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&S, base + h.states_off + (int64_t)index * (int64_t)sizeof(SolverState),
                       sizeof S, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_batch_history");
  int cnt = S.it + 1;
  if (cnt > S.hist_cap) cnt = S.hist_cap;
  if (cnt > cap) cnt = cap;
  e = hipMemcpyAsync(hist, B.hist, sizeof(double) * (size_t)cnt, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(seg, B.seg_hist, sizeof(int32_t) * (size_t)cnt, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_batch_history");
  return GSE_OK;
}

}  // namespace gse

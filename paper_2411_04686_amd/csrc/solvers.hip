// solvers.hip -- stepped mixed-precision CG and GMRES(m) on gfx950.
//
// Only the operator reads reduced segments; dot products, residuals and the
// x / r / p updates are FP64 (Section IV-D.3).  The iteration runs on the
// device: scalars (rho, alpha, beta, the residual history, the segment
// count) live in a state record in the workspace.  Kernels that reduce
// write one partial per workgroup; a one-workgroup kernel launched after
// them sums the partials in a fixed order (so results are reproducible) and
// runs the scalar logic, including the stepped controller of Section III-D
// (Algorithm 3, Eqs. 3-6, Conditions 1-3).  The host replays chunks of
// iterations from HIP graphs and reads the state back between chunks; a stop
// (switch, convergence candidate, breakdown, cap) makes the rest of the
// chunk a no-op.
#include <math.h>
#include <string.h>

#include <chrono>
#include <string>
#include <type_traits>
#include <vector>

#include "decode.h"
#include "gse_internal.h"
#include "solver_state.h"

namespace gse {

gse_status fail(gse_status code, const char* fmt, ...);
gse_status hip_fail(hipError_t e, const char* where);

namespace {

constexpr int kVecBlocks = 2048;

// ------------------------------------------------------------- finisher ---
// out[k] = sum over i < n of partials[k*stride + i], k < nk, each sum in a
// fixed order by one workgroup (workgroup b takes k = b, b + grid, ...; the
// partials were written by the previous kernel).
__global__ __launch_bounds__(kWG) void k_finish(const double* __restrict__ partials, int n,
                                                int stride, int nk, double* __restrict__ out,
                                                const int* gate) {
  __shared__ double red[kWaves];
  if (gate && *gate) return;
  for (int k = blockIdx.x; k < nk; k += gridDim.x) {
    const double t = sum_partials(partials + (size_t)k * stride, n, red);
    if (threadIdx.x == 0) out[k] = t;
  }
}

// ----------------------------------------------------------- CG kernels ---
// One iteration is three kernels: the SpMV q = A_s p (partials of p.q),
// k_cg_rstep and k_cg_xstep.  The scalar steps need no kernel of their own:
// every workgroup sums the partials of the kernel before it in the same
// fixed order (so all of them get the same bits) and workgroup 0 publishes
// the results.  Fields a kernel reads are never written by that kernel's
// workgroup 0, so no workgroup depends on another inside one launch:
//   rstep reads stop, it, rho_p[it & 1];  writes pq, alpha, go, it_next (and
//         stop on a breakdown -- every workgroup reaches the same verdict);
//   xstep reads go, it_next, alpha, rho_p[(it_next - 1) & 1];  writes the
//         history, rho_p[it_next & 1], it, relres, beta and, through the
//         controller, stop.

// r -= alpha q with alpha = rho / p.q; partials of r.r.
__global__ __launch_bounds__(kWG) void k_cg_rstep(SolverState* S, double* __restrict__ r,
                                                  const double* __restrict__ q, int n,
                                                  const double* __restrict__ part_pq, int n_pq,
                                                  double* __restrict__ part_rr) {
  __shared__ double red[kWaves];
  const int stop = S->stop;
  if (blockIdx.x == 0 && threadIdx.x == 0) S->go = 0;
  if (stop) return;
  const int j = S->it;
  const double rho = S->rho_p[j & 1];
  const double pq = sum_partials(part_pq, n_pq, red);
  const bool broke = !(pq > 0.0) || !isfinite(pq);
  const double alpha = rho / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->pq = pq;
    if (broke) {
      S->stop = kBreak;
    } else {
      S->alpha = alpha;
      S->go = 1;
      S->it_next = j + 1;
    }
  }
  if (broke) return;
  double acc = 0.0;
  const int n2 = n >> 1;
  double2* r2 = reinterpret_cast<double2*>(r);
  const double2* q2 = reinterpret_cast<const double2*>(q);
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n2; i += gridDim.x * kWG) {
    double2 rv = r2[i];
    const double2 qv = q2[i];
    rv.x -= alpha * qv.x;
    rv.y -= alpha * qv.y;
    r2[i] = rv;
    acc += rv.x * rv.x;
    acc += rv.y * rv.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double v = r[n - 1] - alpha * q[n - 1];
    r[n - 1] = v;
    acc += v * v;
  }
  const double bs = block_sum(acc, red);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = bs;
}

// x += alpha p; p = r + beta p with beta = rho' / rho (rho' = r.r from the
// partials); workgroup 0 records the history and runs the controller.
__global__ __launch_bounds__(kWG) void k_cg_xstep(SolverState* S, double* __restrict__ x,
                                                  double* __restrict__ p,
                                                  const double* __restrict__ r, int n,
                                                  const double* __restrict__ part_rr, int n_rr,
                                                  double* hist, int* seg_hist) {
  __shared__ double red[kWaves];
  __shared__ double bc_rel;
  if (!S->go) return;
  const int j = S->it_next;
  const double rho_old = S->rho_p[(j - 1) & 1];
  const double alpha = S->alpha;
  const double rho_new = sum_partials(part_rr, n_rr, red);
  const double beta = rho_new / rho_old;
  const int n2 = n >> 1;
  double2* x2 = reinterpret_cast<double2*>(x);
  double2* p2 = reinterpret_cast<double2*>(p);
  const double2* r2 = reinterpret_cast<const double2*>(r);
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n2; i += gridDim.x * kWG) {
    double2 xv = x2[i];
    double2 pv = p2[i];
    const double2 rv = r2[i];
    xv.x += alpha * pv.x;
    xv.y += alpha * pv.y;
    pv.x = rv.x + beta * pv.x;
    pv.y = rv.y + beta * pv.y;
    x2[i] = xv;
    p2[i] = pv;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    x[n - 1] += alpha * p[n - 1];
    p[n - 1] = r[n - 1] + beta * p[n - 1];
  }
  if (blockIdx.x != 0) return;
  const int s = S->s;
  if (threadIdx.x == 0) {
    const double rel = sqrt(rho_new) / S->nb;
    S->beta = beta;
    S->rho_p[j & 1] = rho_new;
    S->rho = rho_new;
    S->it = j;
    S->relres = rel;
    hist[j] = rel;
    seg_hist[j] = s;
    bc_rel = rel;
  }
  __syncthreads();
  controller(S, hist, red, j, bc_rel, s);
}

// ------------------------------------------------------ small systems ---
// A system this small is bound by latency, not bytes: three launches per
// iteration cost ~13 us on a 4096-row Poisson system.  One workgroup of
// 1024 threads then runs every iteration of a segment count in a single
// launch, with workgroup barriers where the large path has launch
// boundaries, until the controller (or a breakdown) stops it.  The loop
// keeps its state on the chip: thread t decodes its rows (t + k*1024, at
// most L = 4, 6 or 8 non-zeros each, L from the longest row) into registers
// once per launch and holds its entries of r there; p (which the product
// gathers) and the solver record live in LDS; x is read early in a pass and
// written late, off the critical path; q lives within a pass.  (Reading
// the planes from L2 in every pass, row per thread, measured 10.7 us per
// iteration: one CU's memory pipeline.)  The arithmetic is that of the
// large path: rows summed in row order with the multiply and add rounded
// separately, the same CG updates, the same controller; only the dot
// products' summation tree differs (one workgroup's).
constexpr int kSmallThreads = 1024;
constexpr int kSmallRpt = 4;                            // rows per thread at most
constexpr int kSmallRows = kSmallThreads * kSmallRpt;   // systems up to this many rows
constexpr int kSmallRow = 8;                            // ... whose rows hold at most 8 non-zeros

// One non-zero decoded without the LDS table: the slot's exponent
// SEM - 1023 - W_s comes from eight registers and the value is
// ldexp(+-F, exponent), exact and bit-identical to F times the table's
// power of two (the product is a normal number or zero for SEM >= 64).
// The compiler may recompute it in every pass rather than hold 32 FP64
// values per thread, so it costs ALU work only.
// The eight slot exponents SEM - 1023 - W_s as 16-bit fields, two per
// word (scalars: an array here would be indexed per lane from scratch).
struct SlotExp {
  uint32_t w01, w23, w45, w67;
  __device__ __forceinline__ int operator()(uint32_t slot) const {
    const uint32_t w = (slot & 4u) ? ((slot & 2u) ? w67 : w45) : ((slot & 2u) ? w23 : w01);
    return (int)(int16_t)(uint16_t)(w >> ((slot & 1u) * 16u));
  }
};

template <int FMT>
__device__ __forceinline__ SlotExp slot_exponents(const int16_t* sem) {
  constexpr int W = (FMT == 1) ? 15 : (FMT == 2) ? 31 : 63;
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    w[i] = (uint32_t)(uint16_t)(int16_t)(sem[2 * i] - 1023 - W) |
           ((uint32_t)(uint16_t)(int16_t)(sem[2 * i + 1] - 1023 - W) << 16);
  return SlotExp{w[0], w[1], w[2], w[3]};
}

template <int FMT>
__device__ __forceinline__ double small_elem(const SpmvOperand& A, int j, const SlotExp& ex,
                                             int& column) {
  const uint32_t c = A.col[j];
  if constexpr (FMT == kCsr64) {
    column = (int)c;
    return A.val[j];
  } else {
    column = (int)(c & A.split.col_mask);
    const int e = ex((c >> A.split.shift) & A.split.slot_mask);
    const uint32_t h = A.head[j];
    double v;
    if constexpr (FMT == 1) {
      v = ldexp((double)(h & 0x7FFFu), e);
    } else if constexpr (FMT == 2) {
      v = ldexp((double)(((h & 0x7FFFu) << 16) | (uint32_t)A.tail1[j]), e);
    } else {
      const double hi = (double)(((h & 0x7FFFu) << 16) | (uint32_t)A.tail1[j]);
      v = ldexp(hi, e + 32) + ldexp((double)A.tail2[j], e);  // at most 53 significant bits: exact
    }
    return (h & 0x8000u) ? -v : v;
  }
}

// f(integral_constant<int, K>) for K = B .. E-1, expanded at compile time
// (a loop over a thread's rows must index its register arrays with
// constants; left as a loop, the arrays go to scratch).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Barrier ordering LDS only: the loop's shared data lives in LDS, and a
// full barrier would also wait for the history stores in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// block_sum with LDS-only barriers (same tree, same bits).
template <int NT>
__device__ __forceinline__ double block_sum_lds(double v, double* red /* [NT / 64] */) {
  v = wave_sum(v);
  lds_barrier();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  lds_barrier();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

template <int FMT, int RPT, int L>
__global__ __launch_bounds__(kSmallThreads) void k_cg_small(SolverState* Sg, SpmvOperand A,
                                                            double* __restrict__ xg,
                                                            double* __restrict__ rg,
                                                            double* __restrict__ pg,
                                                            double* __restrict__ qg, double* hist,
                                                            int* seg_hist) {
  constexpr int NT = kSmallThreads;
  static_assert(L % 2 == 0 && L <= kSmallRow, "row slots");
  __shared__ double red[NT / 64];
  __shared__ double pl[NT * RPT];
  __shared__ SolverState Sl;
  __shared__ double bc_rel;
  const int tid = threadIdx.x;
  const int n = A.n_rows;
  if (tid == 0) Sl = *Sg;
  const SlotExp ex = slot_exponents<FMT>(A.sem);
  double rr[RPT], qr[RPT];  // x stays in memory: loaded early in a pass, stored late
  double av[RPT][L];
  uint32_t ac[RPT][L / 2];  // two 16-bit columns per word (n <= 4096)
  int len[RPT];
  static_for<0, RPT>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const int i = tid + k * NT;
    const bool in = i < n;
    rr[k] = in ? rg[i] : 0.0;
    qr[k] = 0.0;
    if (in) pl[i] = pg[i];
    const int s0 = in ? A.row_ptr[i] : 0;
    const int s1 = in ? A.row_ptr[i + 1] : 0;
    len[k] = s1 - s0;
    int cc[L];
#pragma unroll
    for (int e = 0; e < L; ++e) {
      // clamped into the row, or to entry 0 for an empty row (nnz > 0 then)
      int jj = min(s0 + e, s1 - 1);
      jj = jj < 0 ? 0 : jj;
      int c = 0;
      const double v = A.nnz > 0 ? small_elem<FMT>(A, jj, ex, c) : 0.0;
      const bool use = e < s1 - s0;
      av[k][e] = use ? v : 0.0;
      cc[e] = use ? c : 0;
    }
#pragma unroll
    for (int e = 0; e < L / 2; ++e) ac[k][e] = (uint32_t)cc[2 * e] | ((uint32_t)cc[2 * e + 1] << 16);
  });
  __syncthreads();
  SolverState* S = &Sl;
  for (;;) {
    if (S->stop) break;
    // x of this pass, loaded now and used after both reductions
    double xo[RPT];
    static_for<0, RPT>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      xo[k] = (tid + k * NT < n) ? xg[tid + k * NT] : 0.0;
    });
    // q = A_s p and p.q
    double acc = 0.0;
    static_for<0, RPT>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      double xv[L];
      static_for<0, L>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        xv[e] = pl[(ac[k][e >> 1] >> (16 * (e & 1))) & 0xFFFFu];
      });
      double sum = 0.0;
      static_for<0, L>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        const double pr = __dmul_rn(av[k][e], xv[e]);
        sum = (e < len[k]) ? __dadd_rn(sum, pr) : sum;
      });
      qr[k] = sum;
      if (tid + k * NT < n) acc += pl[tid + k * NT] * sum;
    });
    const double pq = block_sum_lds<NT>(acc, red);  // its barriers end the gathers from pl
    const int j = S->it;
    const double rho = S->rho_p[j & 1];
    if (!(pq > 0.0) || !isfinite(pq)) {  // uniform: every thread holds the same pq
      if (tid == 0) {
        S->pq = pq;
        S->stop = kBreak;
      }
      break;
    }
    const double alpha = rho / pq;
    acc = 0.0;
    static_for<0, RPT>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if (tid + k * NT < n) {
        const double v = rr[k] - alpha * qr[k];
        rr[k] = v;
        acc += v * v;
      }
    });
    const double rho_new = block_sum_lds<NT>(acc, red);
    const double beta = rho_new / rho;
    static_for<0, RPT>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const int i = tid + k * NT;
      if (i < n) {
        const double pv = pl[i];
        xg[i] = xo[k] + alpha * pv;
        pl[i] = rr[k] + beta * pv;
      }
    });
    const int s = S->s;
    const int jn = j + 1;
    if (tid == 0) {
      const double rel = sqrt(rho_new) / S->nb;
      S->pq = pq;
      S->alpha = alpha;
      S->beta = beta;
      S->rho_p[jn & 1] = rho_new;
      S->rho = rho_new;
      S->it = jn;
      S->relres = rel;
      hist[jn] = rel;
      seg_hist[jn] = s;
      bc_rel = rel;
    }
    lds_barrier();
    // Conditions 1-3 read the history from memory: then the history stores
    // must be complete first (a full barrier); otherwise they stay in flight
    if (on_check_grid(S, jn, bc_rel, s)) __syncthreads();
    controller<NT>(S, hist, red, jn, bc_rel, s);
    lds_barrier();  // p and the stop flag for the next pass
  }
  __syncthreads();
  static_for<0, RPT>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    const int i = tid + k * NT;
    if (i < n) {
      rg[i] = rr[k];
      pg[i] = pl[i];
    }
  });
  if (tid == 0) *Sg = Sl;
}

bool cg_small_path(const SpmvOperand& op) {
  // (the eight slot exponents held in scalar words cover index widths <= 3
  // in the column word and one table for the whole matrix)
  return op.n_rows <= kSmallRows && op.max_row <= kSmallRow && op.split.slot_mask <= 7u &&
         op.split.hmask == 0u && op.block_sem == nullptr;
}

template <int RPT, int L>
hipError_t launch_cg_small_rl(const SpmvOperand& op, int s, SolverState* S, double* x, double* r,
                              double* p, double* q, double* hist, int* seg_hist, hipStream_t st) {
  const dim3 g(1), b(kSmallThreads);
#define GSE_SMALL(F) \
  hipLaunchKernelGGL((k_cg_small<F, RPT, L>), g, b, 0, st, S, op, x, r, p, q, hist, seg_hist)
  switch (s) {
    case 0: GSE_SMALL(0); break;
    case 1: GSE_SMALL(1); break;
    case 2: GSE_SMALL(2); break;
    default: GSE_SMALL(3); break;
  }
#undef GSE_SMALL
  return hipGetLastError();
}

template <int L>
hipError_t launch_cg_small_l(const SpmvOperand& op, int s, SolverState* S, double* x, double* r,
                             double* p, double* q, double* hist, int* seg_hist, hipStream_t st) {
  if (op.n_rows <= kSmallThreads)
    return launch_cg_small_rl<1, L>(op, s, S, x, r, p, q, hist, seg_hist, st);
  if (op.n_rows <= 2 * kSmallThreads)
    return launch_cg_small_rl<2, L>(op, s, S, x, r, p, q, hist, seg_hist, st);
  return launch_cg_small_rl<4, L>(op, s, S, x, r, p, q, hist, seg_hist, st);
}

hipError_t launch_cg_small(const SpmvOperand& op, int s, SolverState* S, double* x, double* r,
                           double* p, double* q, double* hist, int* seg_hist, hipStream_t st) {
  if (op.max_row <= 4) return launch_cg_small_l<4>(op, s, S, x, r, p, q, hist, seg_hist, st);
  if (op.max_row <= 6) return launch_cg_small_l<6>(op, s, S, x, r, p, q, hist, seg_hist, st);
  return launch_cg_small_l<8>(op, s, S, x, r, p, q, hist, seg_hist, st);
}

// dst = src (n doubles)
__global__ __launch_bounds__(kWG) void k_copy(double* __restrict__ dst, const double* __restrict__ src,
                                              int n) {
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) dst[i] = src[i];
}

// partials of a.b (grid-stride; one partial per workgroup)
__global__ __launch_bounds__(kWG) void k_dot(const double* __restrict__ a, const double* __restrict__ b,
                                             int n, double* __restrict__ partials) {
  __shared__ double red[kWaves];
  double acc = 0.0;
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) acc += a[i] * b[i];
  const double bs = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = bs;
}

// ---------------------------------------------------------------- layout --
struct Workspace {
  SolverState* S;
  double* partials;    // [np] per-workgroup partial sums
  double* partials2;   // [np] a second set (two reductions in flight)
  double* r;
  double* p;
  double* q;
  double* w;
  double* hist;        // [max_iter + 2]
  int* seg_hist;       // [max_iter + 2]
  double* gm;          // GMRES: V (restart+1) x n, then small arrays
  size_t bytes;
};

size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

int64_t partial_entries(int32_t n_rows, int64_t nnz) {
  int64_t a = (int64_t)n_tiles_for(nnz, kMinTile) + 16;
  int64_t b = (int64_t)n_rows / 32 + 16;
  int64_t c = (int64_t)64 * 1024 + 16;  // GMRES multi-dot partials (k x workgroups)
  int64_t m = a > b ? a : b;
  return m > c ? m : c;
}

// Small per-cycle GMRES arrays: H (m+1) x m, cs, sn, g, y, h scratch.
int64_t gmres_small_entries(int32_t restart) {
  const int64_t m = restart;
  // H, cs, sn, g, h2, h1 and one spare; delayed CGS2: Hu, hp and the sums
  return (m + 1) * m + 4 * (m + 1) + 2 * (m + 1) + (m + 1) * m + (m + 1) + 2 * (m + 1);
}

// Row stride of the GMRES basis in doubles: whole 8 KiB pages plus 4 KiB,
// so that the same element of consecutive basis vectors sits an odd number
// of 4 KiB pages apart and the j+1 streams of a Gram-Schmidt pass spread
// over the HBM channels instead of meeting in the same ones (a power-of-two
// stride, e.g. n = 2^20, put them all in step).
size_t gm_ld(int32_t n_rows) {
  const size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
  const size_t bytes = (n * sizeof(double) + 8191) / 8192 * 8192 + 4096;
  return bytes / sizeof(double);
}

Workspace carve(void* base, int32_t method, int32_t n_rows, int64_t nnz, int32_t restart,
                int32_t max_iter) {
  Workspace w{};
  char* p = reinterpret_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + off : nullptr;
    off += align_up(bytes);
    return q;
  };
  const size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
  w.S = reinterpret_cast<SolverState*>(take(sizeof(SolverState)));
  w.partials = reinterpret_cast<double*>(take((size_t)partial_entries(n_rows, nnz) * sizeof(double)));
  w.partials2 = reinterpret_cast<double*>(take((size_t)partial_entries(n_rows, nnz) * sizeof(double)));
  w.r = reinterpret_cast<double*>(take(n * sizeof(double)));
  w.p = reinterpret_cast<double*>(take(n * sizeof(double)));
  w.q = reinterpret_cast<double*>(take(n * sizeof(double)));
  w.w = reinterpret_cast<double*>(take(n * sizeof(double)));
  w.hist = reinterpret_cast<double*>(take((size_t)(max_iter + 2) * sizeof(double)));
  w.seg_hist = reinterpret_cast<int*>(take((size_t)(max_iter + 2) * sizeof(int)));
  if (method == GSE_GMRES) {
    w.gm = reinterpret_cast<double*>(
        take(((size_t)(restart + 1) * gm_ld(n_rows) + (size_t)gmres_small_entries(restart)) *
             sizeof(double)));
  }
  w.bytes = off;
  return w;
}

int vec_blocks(int n, int cap = kVecBlocks) {
  int b = (n / 2 + kWG - 1) / kWG;
  if (b < 1) b = 1;
  return b > cap ? cap : b;
}

// CG vector kernels: every workgroup sums the partials of the kernel before
// it, so fewer (longer-running) workgroups keep that redundant read small.
constexpr int kCgBlocks = 1024;

// Instantiated graphs of one solve, one per segment count.
// Executable graphs kept across solves of this host thread.  A captured
// graph holds its kernels' arguments by value; they all follow from the key
// (device, method, segment count, operand, workspace, vectors and the sizes
// the workspace is carved by), so a later solve with the same key replays
// the graph instead of capturing it again.  At most kGraphKeep graphs are
// kept; the least recently used one is destroyed first.
constexpr size_t kGraphKeep = 24;

struct GraphKey {
  std::string bytes;
  template <typename T>
  void add(const T& v) {
    bytes.append(reinterpret_cast<const char*>(&v), sizeof v);
  }
  void add_operand(const SpmvOperand& o) {
    add(o.row_ptr), add(o.tile_row), add(o.col), add(o.head), add(o.tail1), add(o.tail2);
    add(o.val), add(o.n_rows), add(o.n_tiles), add(o.tile_nnz), add(o.nnz), add(o.rv_lanes);
    add(o.max_row), add(o.split.shift), add(o.split.slot_mask), add(o.split.col_mask);
    add(o.split.hshift), add(o.split.hmask), add(o.split.mag_mask), add(o.split.ei);
    for (int i = 0; i < GSE_MAX_EXP; ++i) add(o.sem[i]);
    add(o.block_sem), add(o.block_rows), add(o.block_stride);
  }
};

struct GraphCache {
  struct Entry {
    std::string key;
    hipGraphExec_t exec;
    unsigned long long used;
  };
  std::vector<Entry> entries;
  unsigned long long tick = 0;
  ~GraphCache() {
    for (auto& e : entries) (void)hipGraphExecDestroy(e.exec);
  }
  hipGraphExec_t find(const std::string& key) {
    for (auto& e : entries)
      if (e.key == key) {
        e.used = ++tick;
        return e.exec;
      }
    return nullptr;
  }
  void put(const std::string& key, hipGraphExec_t exec) {
    if (entries.size() >= kGraphKeep) {
      size_t old = 0;
      for (size_t i = 1; i < entries.size(); ++i)
        if (entries[i].used < entries[old].used) old = i;
      (void)hipGraphExecDestroy(entries[old].exec);
      entries.erase(entries.begin() + (long)old);
    }
    entries.push_back(Entry{key, exec, ++tick});
  }
};

GraphCache& thread_graphs() {
  thread_local GraphCache cache;
  return cache;
}

// The replayed graph of `key`, captured by `body` on `st` when missing.
template <typename F>
hipError_t cached_graph(const GraphKey& key, hipStream_t st, hipGraphExec_t* out, F&& body) {
  GraphCache& c = thread_graphs();
  *out = c.find(key.bytes);
  if (*out) return hipSuccess;
  hipError_t e = capture(st, out, body);
  if (e == hipSuccess) c.put(key.bytes, *out);
  return e;
}

struct Operator {
  int fmt;  // 1..3 GSE (stepped), 0 a fixed operator (FP64 CSR, FP16 or BF16)
  SpmvOperand op;
  const double* eta;
  int launch_fmt = kCsr64;  // SpMV format of a fixed operator: kCsr64, kFp16 or kBf16
};

// y = A_s x; with kEpiDot the dot aux.y, with kEpiResid y = b - A_s x and
// y.y, are left as per-workgroup partials (their count in *grid) and, if
// `result` is given, summed into *result by a one-workgroup finisher.
hipError_t apply(const Operator& A, int s, const double* x, double* y, int epi, const double* aux,
                 double* result, const Workspace& w, const int* gate, hipStream_t st,
                 int* grid = nullptr) {
  SpmvEpilogue ep{};
  int g = 0;
  ep.epi = epi;
  ep.aux = aux;
  ep.partials = w.partials;
  ep.gate = gate;
  ep.grid_out = &g;
  hipError_t e = launch_spmv(A.fmt == 0 ? A.launch_fmt : s, A.op, x, y, ep, st);
  if (e != hipSuccess) return e;
  if (grid) *grid = g;
  if (result && epi != kEpiPlain) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, st, w.partials, g, 0, 1, result, gate);
    e = hipGetLastError();
  }
  return e;
}

hipError_t read_state(const Workspace& w, SolverState* h, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(h, w.S, sizeof(SolverState), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

hipError_t write_state(const Workspace& w, const SolverState* h, hipStream_t st) {
  return hipMemcpyAsync(w.S, h, sizeof(SolverState), hipMemcpyHostToDevice, st);
}

void init_state(SolverState* S, const gse_params* p, const Operator& A, int s0) {
  memset(S, 0, sizeof *S);
  S->tol = p->tol;
  for (int i = 0; i < 3; ++i) S->eta[i] = A.eta ? A.eta[i] : 0.0;
  S->floor_c = p->floor_c;
  S->rsd_limit = p->rsd_limit;
  S->reldec_limit = p->reldec_limit;
  S->s = s0;
  S->max_iter = p->max_iter;
  S->stepped = (A.fmt != 0 && p->fixed_segments == 0) ? 1 : 0;
  S->fixed = (A.fmt == 0) ? -1 : p->fixed_segments;
  S->l = p->l;
  S->t = p->t;
  S->m = p->m;
  S->ndec_limit = p->ndec_limit;
  S->ndec_rule = p->ndec_rule;
}

// ------------------------------------------------------------------- CG ---
gse_status run_cg(const Operator& A, const double* b, double* x, const gse_params* p,
                  gse_report* rep, void* ws, size_t ws_bytes, hipStream_t caller) {
  auto t0 = std::chrono::steady_clock::now();
  SolveStream ss(caller);
  if (ss.err != hipSuccess) return hip_fail(ss.err, "cg stream");
  hipStream_t st = ss.s;
  const int n = A.op.n_rows;
  Workspace w = carve(ws, GSE_CG, n, A.op.nnz, p->restart, p->max_iter);
  if (w.bytes > ws_bytes) return fail(GSE_ERR_NOMEM, "solver workspace needs %zu bytes", w.bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GSE_ERR_HIP, "cg: no device");
  // what the captured iterations' kernel arguments follow from
  auto graph_key = [&](int s_use) {
    GraphKey k;
    k.add(dev), k.add(GSE_CG), k.add(s_use), k.add(A.fmt), k.add(A.launch_fmt);
    k.add_operand(A.op);
    k.add(ws), k.add(n), k.add(A.op.nnz), k.add(p->restart), k.add(p->max_iter), k.add(x), k.add(b);
    return k;
  };
  memset(rep, 0, sizeof *rep);
  rep->switch_iter[0] = rep->switch_iter[1] = -1;
  const bool stepped = A.fmt != 0 && p->fixed_segments == 0;
  int s = (A.fmt == 0) ? 0 : (stepped ? p->start_segments : p->fixed_segments);
  const int s_final = (A.fmt == 0) ? 0 : 3;
  const int vb = vec_blocks(n, kCgBlocks);
  hipError_t e;
  SolverState h;
  init_state(&h, p, A, s);
  h.hist_off = (long long)((char*)w.hist - (char*)ws);
  h.seg_off = (long long)((char*)w.seg_hist - (char*)ws);
  h.hist_cap = p->max_iter + 2;
  int nsw = 0;
  gse_status status = GSE_NOT_CONVERGED;
  // replacement: r = b - A_s x, rho = r.r (into the slot of h.it), optionally p = r
  auto restart = [&](int s_use, bool reset_p) -> hipError_t {
    hipError_t err =
        apply(A, s_use, x, w.r, kEpiResid, b, &w.S->rho_p[h.it & 1], w, nullptr, st);
    if (err == hipSuccess && reset_p) {
      hipLaunchKernelGGL(k_copy, dim3(vb), dim3(kWG), 0, st, w.p, w.r, n);
      err = hipGetLastError();
    }
    return err;
  };
  auto true_relres = [&](double* out) -> hipError_t {
    hipError_t err = apply(A, s_final, x, w.w, kEpiResid, b, &w.S->scratch[0], w, nullptr, st);
    if (err != hipSuccess) return err;
    SolverState t;
    err = read_state(w, &t, st);
    *out = t.nb > 0.0 ? sqrt(t.scratch[0]) / t.nb : 0.0;
    return err;
  };
  e = write_state(w, &h, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_dot, dim3(vb), dim3(kWG), 0, st, b, b, n, w.partials);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, st, w.partials, vb, 0, 1, &w.S->nb2,
                       nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = restart(s, true);
  if (e == hipSuccess) e = read_state(w, &h, st);
  if (e != hipSuccess) return hip_fail(e, "cg setup");
  h.nb = sqrt(h.nb2);
  if (h.nb == 0.0) {
    e = hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "cg");
    rep->status = GSE_OK;
    return GSE_OK;
  }
  h.rho = h.rho_p[0];
  h.relres = sqrt(h.rho) / h.nb;
  double h0 = h.relres;
  int s0i = s;
  e = hipMemcpyAsync(w.hist, &h0, sizeof h0, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w.seg_hist, &s0i, sizeof s0i, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = write_state(w, &h, st);
  if (e != hipSuccess) return hip_fail(e, "cg setup");

  // K iterations: q = A_s p (partials of p.q) ; alpha, r -= alpha q
  // (partials of r.r) ; beta, x += alpha p, p = r + beta p, history, controller
  auto launch_iters = [&](int K, int s_use) -> hipError_t {
    for (int k = 0; k < K; ++k) {
      int g1 = 0;
      hipError_t err = apply(A, s_use, w.p, w.q, kEpiDot, w.p, nullptr, w, &w.S->stop, st, &g1);
      if (err != hipSuccess) return err;
      hipLaunchKernelGGL(k_cg_rstep, dim3(vb), dim3(kWG), 0, st, w.S, w.r, w.q, n, w.partials, g1,
                         w.partials2);
      hipLaunchKernelGGL(k_cg_xstep, dim3(vb), dim3(kWG), 0, st, w.S, x, w.p, w.r, n, w.partials2,
                         vb, w.hist, w.seg_hist);
      err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  };
  constexpr int kGraphIters = 16;
  int chunk = 4;
  bool done = false;
  bool pending_check = h.relres <= p->tol;  // converged at x0 already
  const bool small = cg_small_path(A.op) && A.launch_fmt == kCsr64;
  while (!done) {
    if (pending_check) {
      // the recursive residual meets the tolerance outside an iteration (at
      // x0, or after a residual replacement): convergence is judged only on
      // an exact operator; an inexact one escalates as the controller does
      const bool exact_op = !stepped || h.s >= 3 || h.eta[h.s - 1] == 0.0;
      h.stop = exact_op ? kConv : kSwitch;
      h.trig = exact_op ? GSE_TRIG_NONE : GSE_TRIG_TOL;
    } else {
      if (small) {
        // every iteration of this segment count in one launch
        e = launch_cg_small(A.op, h.s, w.S, x, w.r, w.p, w.q, w.hist, w.seg_hist, st);
      } else if (p->launch_mode == 1 || chunk < kGraphIters) {
        e = launch_iters(chunk, h.s);
        chunk = chunk < 64 ? chunk * 2 : 64;
      } else {
        const int s_use = h.s;
        hipGraphExec_t ge = nullptr;
        e = cached_graph(graph_key(s_use), st, &ge,
                         [&] { return launch_iters(kGraphIters, s_use); });
        if (e == hipSuccess) e = hipGraphLaunch(ge, st);
      }
      if (e == hipSuccess) e = read_state(w, &h, st);
      if (e != hipSuccess) return hip_fail(e, "cg iterations");
      if (h.stop == kRun) continue;
    }
    pending_check = false;
    int reason = h.stop;
    int trig = h.trig;
    if (reason == kBreak) {
      if (stepped && h.s < 3) {
        reason = kSwitch;
        trig = GSE_TRIG_BREAKDOWN;
      } else {
        status = GSE_ERR_BREAKDOWN;
        break;
      }
    }
    if (reason == kConv) {
      double rt = 0.0;
      e = true_relres(&rt);
      if (e != hipSuccess) return hip_fail(e, "cg check");
      if (rt <= p->tol) {
        status = GSE_OK;
        break;
      }
      // the recursive residual drifted from the true one: replace it
      SolverState t;
      e = restart(h.s, true);
      if (e == hipSuccess) e = read_state(w, &t, st);
      if (e != hipSuccess) return hip_fail(e, "cg replace");
      h.rho_p[h.it & 1] = t.rho_p[h.it & 1];
      h.rho = h.rho_p[h.it & 1];
      h.relres = sqrt(h.rho) / h.nb;
      if (h.relres <= p->tol || h.it >= p->max_iter) break;
    } else if (reason == kSwitch) {
      if (nsw < 2) {
        rep->switch_iter[nsw] = h.it;
        rep->switch_trigger[nsw] = trig;
      }
      ++nsw;
      h.s += 1;
      const double rho_old = h.rho_p[h.it & 1];
      SolverState t;
      e = restart(h.s, p->switch_mode == 0);
      if (e == hipSuccess) e = read_state(w, &t, st);
      if (e != hipSuccess) return hip_fail(e, "cg switch");
      if (p->switch_mode == 2 && restart_direction(2, rho_old, t.rho_p[h.it & 1])) {
        hipLaunchKernelGGL(k_copy, dim3(vb), dim3(kWG), 0, st, w.p, w.r, n);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "cg switch");
      }
      h.rho_p[h.it & 1] = t.rho_p[h.it & 1];
      h.rho = h.rho_p[h.it & 1];
      h.relres = sqrt(h.rho) / h.nb;
      if (h.relres <= p->tol) pending_check = true;
    } else if (reason == kCap) {
      break;
    }
    if (h.it >= p->max_iter && !pending_check) break;
    h.stop = kRun;
    h.trig = 0;
    h.go = 0;
    chunk = 4;
    e = write_state(w, &h, st);
    if (e != hipSuccess) return hip_fail(e, "cg state");
  }
  // final report
  SolverState f;
  e = read_state(w, &f, st);
  if (e != hipSuccess) return hip_fail(e, "cg report");
  double rt = 0.0;
  e = true_relres(&rt);
  if (e != hipSuccess) return hip_fail(e, "cg report");
  rep->status = status;
  rep->iters = f.it;
  rep->relres_recursive = f.relres;
  rep->relres_true = rt;
  {
    // iterations per segment count from the segment history
    const int cnt = f.it;
    int* seg = new int[(size_t)cnt + 1];
    e = hipMemcpyAsync(seg, w.seg_hist, sizeof(int) * (size_t)(cnt + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      delete[] seg;
      return hip_fail(e, "cg report");
    }
    for (int i = 1; i <= cnt; ++i) {
      const int sg = seg[i] <= 0 ? 3 : seg[i];
      rep->iters_per_seg[sg - 1] += 1;
    }
    delete[] seg;
  }
  rep->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return status;
}


// ----------------------------------------------------------- GMRES(m) ---
// Arnoldi with classical Gram-Schmidt applied twice (CGS2); V holds m+1
// basis vectors of n entries; small arrays: H (m+1) x m row-major, cs, sn,
// g (m+1 each), h2 scratch.  Per step j (device, gated on stop):
//   w = A_s v_j                            (SpMV into v_{j+1})
//   h = V^T w                              (k_gm_dots + k_finish)
//   w -= V h ; h2 = V^T w, n1 = ||w||^2    (k_gm_axpy_dots + k_finish)
//   w -= V h2 ; v_{j+1} = w / b with       (k_gm_axpy_scale: every workgroup
//     b^2 = n1 - ||h2||^2 ; H[:,j] = h + h2,  updates and scales its rows,
//     H[j+1,j] = b, Givens, controller        workgroup 0 then runs the rest)
// b^2 = n1 - ||h2||^2 is ||w - V h2||^2 for orthonormal V (the second pass
// removes a component of relative size ~ eps, so the difference loses no
// accuracy), which saves the reduction of a third pass and the separate
// scaling pass.  A b^2 at or below 1e-28 n1 is taken as 0: w lies in the
// span of V (the Krylov space is exhausted).  The finishers stay kernels of
// their own: summing the (j+1) x 512 partials in every workgroup of the
// next pass instead cost more than the launch it saved.
constexpr int kGmBlocks = 512;  // measured best for the 1M-row passes (fewer, longer workgroups)

struct GmSmall {
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* h2;
};

// partials[k * stride + block] = workgroup sum of acc[k] for k < count: the
// same arithmetic as block_sum (wave sums, then the waves in order), with
// one barrier for all k.
template <int NA>
__device__ __forceinline__ void block_sums_out(const double (&acc)[NA], int count,
                                               double* red /* [NA * kWaves] */,
                                               double* __restrict__ partials, int stride) {
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    if (k < count) {
      const double v = wave_sum(acc[k]);
      if ((threadIdx.x & 63) == 0) red[k * kWaves + w] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < count) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[threadIdx.x * kWaves + i];
    partials[(size_t)threadIdx.x * stride + blockIdx.x] = t;
  }
}

// The basis-vector loads of one element are issued unconditionally, all
// before the arithmetic: a load guarded by `k <= j` becomes a branch whose
// body waits for its own load, which serialises the JB loads of a lane.
// Vectors past v_j are read as v_j again (a cache hit) and enter with a zero
// coefficient (axpy) or a discarded accumulator (dots), so the arithmetic on
// the real terms, and its order, is that of the guarded loop.
template <int JB>
__global__ __launch_bounds__(kWG) void k_gm_dots(const SolverState* S, const double* __restrict__ V,
                                                 const double* __restrict__ w, int n, size_t ld,
                                                 int j, double* __restrict__ partials) {
  __shared__ double red[JB * kWaves];
  if (S->stop) return;
  double acc[JB];
#pragma unroll
  for (int k = 0; k < JB; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    double v[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k) v[k] = V[(size_t)(k <= j ? k : j) * ld + i];
    const double wi = w[i];
    __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the arithmetic
#pragma unroll
    for (int k = 0; k < JB; ++k) acc[k] += v[k] * wi;
  }
  block_sums_out(acc, j + 1, red, partials, gridDim.x);
}

// w -= V h (h finished from the previous pass); then partials of V_k . w
// for k <= j (rows 0..j of `partials`) and of w.w (row j + 1).
template <int JB>
__global__ __launch_bounds__(kWG) void k_gm_axpy_dots(const SolverState* S,
                                                      const double* __restrict__ V,
                                                      double* __restrict__ w, int n, size_t ld,
                                                      int j, const double* __restrict__ h,
                                                      double* __restrict__ partials) {
  __shared__ double red[(JB + 1) * kWaves];
  __shared__ double hs[JB];
  if (S->stop) return;
  if (threadIdx.x < JB) hs[threadIdx.x] = (threadIdx.x <= j) ? h[threadIdx.x] : 0.0;
  __syncthreads();
  double acc[JB];
  double nrm = 0.0;
#pragma unroll
  for (int k = 0; k < JB; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    double v[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k) v[k] = V[(size_t)(k <= j ? k : j) * ld + i];
    double wi = w[i];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < JB; ++k) wi -= hs[k] * v[k];
    w[i] = wi;
    nrm += wi * wi;
#pragma unroll
    for (int k = 0; k < JB; ++k) acc[k] += v[k] * wi;
  }
  // the same arithmetic as block_sums_out, with the norm as row j + 1
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < JB; ++k) {
    if (k <= j) {
      const double t = wave_sum(acc[k]);
      if ((threadIdx.x & 63) == 0) red[k * kWaves + wv] = t;
    }
  }
  {
    const double t = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) red[JB * kWaves + wv] = t;
  }
  __syncthreads();
  const int row = (int)threadIdx.x;
  if (row <= j + 1) {
    const int src = row <= j ? row : JB;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[src * kWaves + i];
    partials[(size_t)row * gridDim.x + blockIdx.x] = t;
  }
}

// The second pass and the end of Arnoldi step j.  Every workgroup: b from
// n1 = ||w||^2 (h2[j + 1]) and h2 (the same bits everywhere), then for its
// rows w -= V h2 and v_{j+1} = w / b.  Workgroup 0 afterwards: H[:,j] =
// h1 + h2, H[j+1,j] = b, the rotations, the residual estimate and the
// controller (the column and the earlier rotations are gathered into LDS by
// all its threads, the rotations run in one thread from there, and the
// rotated column is written back by all threads).  Workgroup 0 may set stop
// while the others run; whether they still scale then does not matter,
// because a stopped cycle ends with x += V(:, 0..j) y and never reads
// v_{j+1}.
template <int JB>
__global__ __launch_bounds__(kWG) void k_gm_axpy_scale(SolverState* S, GmSmall sm, int m, int j,
                                                       const double* __restrict__ V,
                                                       double* __restrict__ w, int n, size_t ld,
                                                       const double* __restrict__ h1,
                                                       double* hist, int* seg_hist) {
  __shared__ double red[kWaves];
  __shared__ double hs[JB];
  __shared__ double col[64], c_s[64], s_s[64];
  __shared__ int bc_j, bc_s, bc_go;
  __shared__ double bc_rel;
  if (S->stop) return;
  const double* h2 = sm.h2;
  if (threadIdx.x < JB) hs[threadIdx.x] = (threadIdx.x <= j) ? h2[threadIdx.x] : 0.0;
  __syncthreads();
  const double n1 = h2[j + 1];
  double t2 = 0.0;
  for (int k = 0; k <= j; ++k) t2 += hs[k] * hs[k];
  const double b2 = n1 - t2;
  const double hn = b2 > 1e-28 * n1 ? sqrt(b2) : 0.0;
  const double inv = hn != 0.0 ? 1.0 / hn : 1.0;
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    double v[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k) v[k] = V[(size_t)(k <= j ? k : j) * ld + i];
    double wi = w[i];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < JB; ++k) wi -= hs[k] * v[k];
    w[i] = hn != 0.0 ? wi * inv : wi;
  }
  if (blockIdx.x != 0) return;
  const int t = threadIdx.x;
  if (t <= j) {
    col[t] = h1[t] + h2[t];
    if (t < j) {
      c_s[t] = sm.cs[t];
      s_s[t] = sm.sn[t];
    }
  }
  __syncthreads();
  if (t == 0) {
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = c_s[i] * a + s_s[i] * b;
      col[i + 1] = -s_s[i] * a + c_s[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double rr = sqrt(a * a + b * b);
    const double c = rr == 0.0 ? 1.0 : a / rr;
    const double sv = rr == 0.0 ? 0.0 : b / rr;
    sm.cs[j] = c;
    sm.sn[j] = sv;
    col[j] = c * a + sv * b;
    col[j + 1] = 0.0;
    const double gj = sm.g[j];
    sm.g[j + 1] = -sv * gj;
    sm.g[j] = c * gj;
    const int it = S->it + 1;
    const double rel = fabs(-sv * gj) / S->nb;
    S->it = it;
    S->relres = rel;
    S->scratch[1] = hn;     // norm of the new basis vector
    S->scratch[2] = j + 1;  // columns completed in this cycle
    hist[it] = rel;
    seg_hist[it] = S->s;
    bc_j = it;
    bc_s = S->s;
    bc_rel = rel;
    bc_go = hn != 0.0;
    if (hn == 0.0) S->stop = kConv;  // exact in this space: end the cycle
  }
  __syncthreads();
  if (t <= j + 1) sm.H[(size_t)t * m + j] = col[t];  // row-major (m+1) x m
  if (bc_go) controller(S, hist, red, bc_j, bc_rel, bc_s);
}

// y = H(1:k,1:k) \ g(1:k) (every workgroup solves the small system the same
// way), then x += V(:,1:k) y.  k = columns completed in the cycle (<= JB);
// the loads are issued unconditionally as in the Gram-Schmidt passes, with
// y = 0 past k.
template <int JB>
__global__ __launch_bounds__(kWG) void k_gm_update(const SolverState* S, GmSmall sm, int m,
                                                   const double* __restrict__ V, size_t ld,
                                                   double* __restrict__ x, int n) {
  __shared__ double y[JB];
  __shared__ double Hs[JB * JB];  // the leading k x k block of H, gathered by all threads
  const int k = (int)S->scratch[2];
  if (k <= 0) return;
  for (int e = threadIdx.x; e < k * k; e += kWG) {
    const int i = e / k, q = e - i * k;
    Hs[i * JB + q] = sm.H[(size_t)i * m + q];
  }
  if ((int)threadIdx.x < JB) y[threadIdx.x] = (int)threadIdx.x < k ? sm.g[threadIdx.x] : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double acc = y[i];
      for (int q = i + 1; q < k; ++q) acc -= Hs[i * JB + q] * y[q];
      y[i] = acc / Hs[i * JB + i];
    }
  }
  __syncthreads();
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    double v[JB];
#pragma unroll
    for (int q = 0; q < JB; ++q) v[q] = V[(size_t)(q < k ? q : k - 1) * ld + i];
    double xi = x[i];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < JB; ++q) xi += y[q] * v[q];
    x[i] = xi;
  }
}

// v_0 = r / beta (r already in v_0), g = beta e_1, cycle bookkeeping reset.
__global__ __launch_bounds__(kWG) void k_gm_start(SolverState* S, GmSmall sm, int m,
                                                  double* __restrict__ v0, int n) {
  const double beta = sqrt(S->rho);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) v0[i] *= inv;
  if (blockIdx.x == 0 && threadIdx.x <= m) {
    sm.g[threadIdx.x] = threadIdx.x == 0 ? beta : 0.0;
    if (threadIdx.x == 0) S->scratch[2] = 0.0;
  }
}

// ------------------------------------------------- GMRES, delayed CGS2 ---
// Gram-Schmidt applied twice with the second pass delayed one step, so each
// Arnoldi step needs a single reduction (DCGS2: Swirydowicz et al. 2020,
// Bielich et al. 2022).  V[j] holds u_j, the new direction after its first
// projection only (V[0] = r, not normalised); q_0..q_{j-1} are final.  Step
// j (0 <= j <= m):
//   z = A_s u_j                                   (SpMV into w; not at j = m)
//   a = Q^T u_j, omega = u_j.u_j, c = Q^T z, gamma = u_j.z
//                                                 (k_dg_dots + k_finish)
//   beta = sqrt(omega - |a|^2), t = (gamma - a.c) / beta, and per row
//   q_j = (u_j - Q a) / beta, u_{j+1} = (z - Q c - t q_j) / beta
//                                                 (k_dg_axpy, every workgroup)
// Workgroup 0 of k_dg_axpy then closes Arnoldi column j - 1 (H = hp + a,
// H[j][j-1] = beta, before the rotations in Hu and rotated in H), runs the
// rotations, the residual estimate and the controller, and forms the
// provisional column j, hp = ([c; t] - Hu a) / beta (Hu: the columns closed
// so far; A Q = Q_j Hu is the Arnoldi relation).  Two passes over the basis
// and four launches per step, against three passes and six for CGS2; the
// residual estimate of column j - 1 arrives one product later.

// Longest restart of the delayed CGS2: its dots keep two accumulators per
// basis vector in each thread.
constexpr int kDgMaxRestart = 32;

struct DgSmall {
  double* Hu;    // (m+1) x m, row-major: the Hessenberg matrix before the rotations
  double* hp;    // m+1: provisional (first-projection) column of the open step
  double* sums;  // 2m+2: a (j), omega, c (j), gamma of the current step
};

// Partials of a = Q^T u, omega, c = Q^T z, gamma (rows 0..j-1, j, j+1..2j,
// 2j+1).  z null (j = m): c and gamma are zero.  Vectors past q_{j-1} are
// read as u again (a cache hit) and their accumulators discarded.
template <int JB>
__global__ __launch_bounds__(kWG) void k_dg_dots(const SolverState* S, const double* __restrict__ V,
                                                 size_t ld, int n, int j,
                                                 const double* __restrict__ z,
                                                 double* __restrict__ partials) {
  __shared__ double red[(2 * JB + 2) * kWaves];
  if (S->stop) return;
  const double* u = V + (size_t)j * ld;
  double acc_a[JB], acc_c[JB];
  double om = 0.0, ga = 0.0;
#pragma unroll
  for (int k = 0; k < JB; ++k) acc_a[k] = acc_c[k] = 0.0;
  for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
    double v[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k) v[k] = V[(size_t)(k < j ? k : j) * ld + i];
    const double ui = u[i];
    const double zi = z ? z[i] : 0.0;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < JB; ++k) {
      acc_a[k] += v[k] * ui;
      acc_c[k] += v[k] * zi;
    }
    om += ui * ui;
    ga += ui * zi;
  }
  // the arithmetic of block_sums_out over the 2j + 2 rows
  const int wv = threadIdx.x >> 6;
  const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
  for (int k = 0; k < JB; ++k) {
    if (k < j) {
      const double ta = wave_sum(acc_a[k]);
      const double tc = wave_sum(acc_c[k]);
      if (lead) {
        red[k * kWaves + wv] = ta;
        red[(j + 1 + k) * kWaves + wv] = tc;
      }
    }
  }
  {
    const double to = wave_sum(om);
    const double tg = wave_sum(ga);
    if (lead) {
      red[j * kWaves + wv] = to;
      red[(2 * j + 1) * kWaves + wv] = tg;
    }
  }
  __syncthreads();
  const int row = (int)threadIdx.x;
  if (row <= 2 * j + 1) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += red[row * kWaves + i];
    partials[(size_t)row * gridDim.x + blockIdx.x] = t;
  }
}

// Step j's vector pass and, in workgroup 0, the close of column j - 1.
template <int JB>
__global__ __launch_bounds__(kWG) void k_dg_axpy(SolverState* S, GmSmall sm, DgSmall dg, int m,
                                                 int j, double* __restrict__ V, size_t ld, int n,
                                                 const double* __restrict__ z, double* hist,
                                                 int* seg_hist) {
  __shared__ double red[kWaves];
  __shared__ double as[JB], cs_[JB];
  __shared__ double col[64], c_s[64], s_s[64];
  __shared__ int bc_j, bc_s, bc_go;
  __shared__ double bc_rel;
  if (S->stop) return;
  const double* sums = dg.sums;
  if (threadIdx.x < JB) {
    as[threadIdx.x] = (int)threadIdx.x < j ? sums[threadIdx.x] : 0.0;
    cs_[threadIdx.x] = (int)threadIdx.x < j ? sums[j + 1 + threadIdx.x] : 0.0;
  }
  __syncthreads();
  // the same bits in every workgroup: sums in index order
  const double om = sums[j];
  double aa = 0.0, ac = 0.0;
  for (int k = 0; k < j; ++k) {
    aa += as[k] * as[k];
    ac += as[k] * cs_[k];
  }
  const double b2 = om - aa;
  const double bet = b2 > 1e-28 * om ? sqrt(b2) : 0.0;
  const double inv = bet != 0.0 ? 1.0 / bet : 0.0;
  const double t = (sums[2 * j + 1] - ac) * inv;
  if (j < m && bet != 0.0) {
    double* u = V + (size_t)j * ld;
    double* un = V + (size_t)(j + 1) * ld;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
      double v[JB];
#pragma unroll
      for (int k = 0; k < JB; ++k) v[k] = V[(size_t)(k < j ? k : j) * ld + i];
      double q = u[i];
      double w = z[i];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < JB; ++k) {
        q -= as[k] * v[k];
        w -= cs_[k] * v[k];
      }
      q *= inv;
      w -= t * q;
      u[i] = q;
      un[i] = w * inv;
    }
  }
  if (blockIdx.x != 0) return;
  const int tid = threadIdx.x;
  if (j == 0) {
    if (tid == 0) sm.g[0] = bet;
  } else {
    // close column j - 1
    if (tid < j) {
      const double h = dg.hp[tid] + as[tid];
      dg.Hu[(size_t)tid * m + (j - 1)] = h;
      col[tid] = h;
      if (tid < j - 1) {
        c_s[tid] = sm.cs[tid];
        s_s[tid] = sm.sn[tid];
      }
    }
    if (tid == 0) dg.Hu[(size_t)j * m + (j - 1)] = bet;
    __syncthreads();
    if (tid == 0) {
      const int c = j - 1;
      col[j] = bet;
      for (int i = 0; i < c; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = c_s[i] * a + s_s[i] * b;
        col[i + 1] = -s_s[i] * a + c_s[i] * b;
      }
      const double a = col[c], b = col[c + 1];
      const double rr = sqrt(a * a + b * b);
      const double cg = rr == 0.0 ? 1.0 : a / rr;
      const double sg = rr == 0.0 ? 0.0 : b / rr;
      sm.cs[c] = cg;
      sm.sn[c] = sg;
      col[c] = cg * a + sg * b;
      col[c + 1] = 0.0;
      const double gc = sm.g[c];
      sm.g[c + 1] = -sg * gc;
      sm.g[c] = cg * gc;
      const int it = S->it + 1;
      const double rel = fabs(-sg * gc) / S->nb;
      S->it = it;
      S->relres = rel;
      S->scratch[1] = bet;
      S->scratch[2] = j;  // columns closed in this cycle
      hist[it] = rel;
      seg_hist[it] = S->s;
      bc_j = it;
      bc_s = S->s;
      bc_rel = rel;
      bc_go = bet != 0.0;
      if (bet == 0.0) S->stop = kConv;  // exact in this space: end the cycle
    }
    __syncthreads();
    if (tid <= j) sm.H[(size_t)tid * m + (j - 1)] = col[tid];  // row-major (m+1) x m
    if (bc_go) controller(S, hist, red, bc_j, bc_rel, bc_s);
  }
  // the provisional column j, from the columns closed so far (Hu reads the
  // column just written by this workgroup).  Row i of a Hessenberg matrix is
  // zero left of column i - 1, and those entries of Hu are never written in
  // this cycle: the sum starts at column i - 1.
  __syncthreads();
  if (j < m && bet != 0.0 && tid <= j) {
    double c = tid < j ? cs_[tid] : t;
    for (int k = tid > 0 ? tid - 1 : 0; k < j; ++k) c -= dg.Hu[(size_t)tid * m + k] * as[k];
    dg.hp[tid] = c * inv;
  }
}

// Cycle start for DCGS2: V[0] = r stays unnormalised (step 0 normalises it
// and sets g[0]); g = 0, no column closed yet.
__global__ __launch_bounds__(kWG) void k_dg_start(SolverState* S, GmSmall sm, int m) {
  if ((int)threadIdx.x <= m) sm.g[threadIdx.x] = 0.0;
  if (threadIdx.x == 0) S->scratch[2] = 0.0;
}

gse_status run_gmres(const Operator& A, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, hipStream_t caller) {
  auto t0 = std::chrono::steady_clock::now();
  SolveStream ss(caller);
  if (ss.err != hipSuccess) return hip_fail(ss.err, "gmres stream");
  hipStream_t st = ss.s;
  const int n = A.op.n_rows;
  const int m = p->restart;
  if (m > 60) return fail(GSE_ERR_ARG, "restart must be <= 60");
  if (p->orth < 0 || p->orth > 2) return fail(GSE_ERR_ARG, "orth must be 0, 1 or 2");
  if (p->orth == 2 && m > kDgMaxRestart)
    return fail(GSE_ERR_ARG, "delayed CGS2 takes restart <= %d", kDgMaxRestart);
  // orth 0: the delayed CGS2 wherever its per-thread accumulators fit
  const bool dcgs2 = p->orth == 2 || (p->orth == 0 && m <= kDgMaxRestart);
  Workspace w = carve(ws, GSE_GMRES, n, A.op.nnz, m, p->max_iter);
  if (w.bytes > ws_bytes) return fail(GSE_ERR_NOMEM, "solver workspace needs %zu bytes", w.bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GSE_ERR_HIP, "gmres: no device");
  // what the captured cycle's kernel arguments follow from
  auto graph_key = [&](int s_use) {
    GraphKey k;
    k.add(dev), k.add(GSE_GMRES), k.add(s_use), k.add(A.fmt), k.add(A.launch_fmt);
    k.add_operand(A.op);
    k.add(ws), k.add(n), k.add(A.op.nnz), k.add(m), k.add(p->max_iter), k.add(x), k.add(b);
    k.add(dcgs2);
    return k;
  };
  memset(rep, 0, sizeof *rep);
  rep->switch_iter[0] = rep->switch_iter[1] = -1;
  const bool stepped = A.fmt != 0 && p->fixed_segments == 0;
  const int s_final = (A.fmt == 0) ? 0 : 3;
  const size_t ld = gm_ld(n);
  double* V = w.gm;
  GmSmall sm;
  sm.H = V + (size_t)(m + 1) * ld;
  sm.cs = sm.H + (size_t)(m + 1) * m;
  sm.sn = sm.cs + (m + 1);
  sm.g = sm.sn + (m + 1);
  sm.h2 = sm.g + (m + 1);
  double* h1 = sm.h2 + (m + 1);  // pass-1 dots (m+1), pass-2 dots in sm.h2
  DgSmall dg;
  dg.Hu = h1 + 2 * (m + 1);
  dg.hp = dg.Hu + (size_t)(m + 1) * m;
  dg.sums = dg.hp + (m + 1);
  const int vb = vec_blocks(n);
  const int gb = vb < kGmBlocks ? vb : kGmBlocks;
  hipError_t e;
  SolverState h;
  const int s_start = (A.fmt == 0) ? 0 : (stepped ? p->start_segments : p->fixed_segments);
  init_state(&h, p, A, s_start);
  h.hist_off = (long long)((char*)w.hist - (char*)ws);
  h.seg_off = (long long)((char*)w.seg_hist - (char*)ws);
  h.hist_cap = p->max_iter + 2;
  e = write_state(w, &h, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_dot, dim3(vb), dim3(kWG), 0, st, b, b, n, w.partials);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kWG), 0, st, w.partials, vb, 0, 1, &w.S->nb2,
                       nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = read_state(w, &h, st);
  if (e != hipSuccess) return hip_fail(e, "gmres setup");
  h.nb = sqrt(h.nb2);
  if (h.nb == 0.0) {
    e = hipMemsetAsync(x, 0, sizeof(double) * (size_t)n, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gmres");
    rep->status = GSE_OK;
    return GSE_OK;
  }
  e = write_state(w, &h, st);
  if (e != hipSuccess) return hip_fail(e, "gmres setup");
  int nsw = 0;
  gse_status status = GSE_NOT_CONVERGED;
  bool first = true;
  for (;;) {
    // explicit residual of the current operator into v_0
    SolverState t;
    e = apply(A, h.s, x, V, kEpiResid, b, &w.S->rho, w, nullptr, st);
    if (e == hipSuccess) e = read_state(w, &t, st);
    if (e != hipSuccess) return hip_fail(e, "gmres residual");
    h.rho = t.rho;
    h.relres = sqrt(h.rho) / h.nb;
    if (first) {
      double h0 = h.relres;
      int s0i = h.s;
      e = hipMemcpyAsync(w.hist, &h0, sizeof h0, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(w.seg_hist, &s0i, sizeof s0i, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "gmres setup");
      first = false;
    }
    int trig = GSE_TRIG_NONE;
    if (h.relres <= p->tol) {
      if (A.fmt == 0 || h.s >= 3) {  // the residual just formed is the all-segment one
        status = GSE_OK;
        break;
      }
      if (h.fixed != 0 || h.eta[h.s - 1] == 0.0) {
        // convergence is judged on the all-segment residual; a fixed
        // segment count cannot escalate, so it ends here either way
        SolverState t3;
        e = apply(A, s_final, x, w.w, kEpiResid, b, &w.S->scratch[0], w, nullptr, st);
        if (e == hipSuccess) e = read_state(w, &t3, st);
        if (e != hipSuccess) return hip_fail(e, "gmres check");
        if (sqrt(t3.scratch[0]) / h.nb <= p->tol) {
          status = GSE_OK;
          break;
        }
        if (h.fixed != 0) break;
      }
      trig = GSE_TRIG_TOL;
    }
    if (trig != GSE_TRIG_NONE) {
      if (nsw < 2) {
        rep->switch_iter[nsw] = h.it;
        rep->switch_trigger[nsw] = trig;
      }
      ++nsw;
      h.s += 1;
      continue;
    }
    if (h.it >= p->max_iter) break;
    h.stop = kRun;
    h.trig = 0;
    e = write_state(w, &h, st);
    if (e != hipSuccess) return hip_fail(e, "gmres state");
    // one cycle: v_0 = r/beta, m Arnoldi steps (gated: a stop ends the cycle),
    // x += V y
    // delayed CGS2: steps 0..m, the last one without a product
    auto launch_cycle_dg = [&](int s_use) -> hipError_t {
      hipLaunchKernelGGL(k_dg_start, dim3(1), dim3(kWG), 0, st, w.S, sm, m);
      for (int j = 0; j <= m; ++j) {
        double* uj = V + (size_t)j * ld;
        const double* z = j < m ? w.w : nullptr;
        if (j < m) {
          hipError_t err = apply(A, s_use, uj, w.w, kEpiPlain, nullptr, nullptr, w, &w.S->stop, st);
          if (err != hipSuccess) return err;
        }
        const int* gate = &w.S->stop;
        double* P = w.partials;
#define GSE_DG_STEP(JB)                                                                             \
  hipLaunchKernelGGL((k_dg_dots<JB>), dim3(gb), dim3(kWG), 0, st, w.S, V, ld, n, j, z, P);         \
  hipLaunchKernelGGL(k_finish, dim3(2 * j + 2), dim3(kWG), 0, st, P, gb, gb, 2 * j + 2, dg.sums,   \
                     gate);                                                                        \
  hipLaunchKernelGGL((k_dg_axpy<JB>), dim3(gb), dim3(kWG), 0, st, w.S, sm, dg, m, j, V, ld, n, z, \
                     w.hist, w.seg_hist)
        // final vectors q_0..q_{j-1}, rounded up to a multiple of 4 (m <= 32)
        switch ((j + 3) >> 2) {
          case 0:
          case 1: GSE_DG_STEP(4); break;
          case 2: GSE_DG_STEP(8); break;
          case 3: GSE_DG_STEP(12); break;
          case 4: GSE_DG_STEP(16); break;
          case 5: GSE_DG_STEP(20); break;
          case 6: GSE_DG_STEP(24); break;
          case 7: GSE_DG_STEP(28); break;
          default: GSE_DG_STEP(32); break;
        }
#undef GSE_DG_STEP
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
      }
#define GSE_GM_UPDATE(JB) \
  hipLaunchKernelGGL((k_gm_update<JB>), dim3(gb), dim3(kWG), 0, st, w.S, sm, m, V, ld, x, n)
      if (m <= 8) GSE_GM_UPDATE(8);
      else if (m <= 16) GSE_GM_UPDATE(16);
      else if (m <= 24) GSE_GM_UPDATE(24);
      else GSE_GM_UPDATE(32);
#undef GSE_GM_UPDATE
      return hipGetLastError();
    };
    auto launch_cycle = [&](int s_use) -> hipError_t {
      if (dcgs2) return launch_cycle_dg(s_use);
      hipLaunchKernelGGL(k_gm_start, dim3(vb), dim3(kWG), 0, st, w.S, sm, m, V, n);
      for (int j = 0; j < m; ++j) {
        double* vj = V + (size_t)j * ld;
        double* wv = V + (size_t)(j + 1) * ld;
        hipError_t err = apply(A, s_use, vj, wv, kEpiPlain, nullptr, nullptr, w, &w.S->stop, st);
        if (err != hipSuccess) return err;
        const int* gate = &w.S->stop;
        double* P = w.partials;
#define GSE_GM_PASSES(JB)                                                                         \
  hipLaunchKernelGGL((k_gm_dots<JB>), dim3(gb), dim3(kWG), 0, st, w.S, V, wv, n, ld, j, P);        \
  hipLaunchKernelGGL(k_finish, dim3(j + 1), dim3(kWG), 0, st, P, gb, gb, j + 1, h1, gate);         \
  hipLaunchKernelGGL((k_gm_axpy_dots<JB>), dim3(gb), dim3(kWG), 0, st, w.S, V, wv, n, ld, j, h1, P); \
  hipLaunchKernelGGL(k_finish, dim3(j + 2), dim3(kWG), 0, st, P, gb, gb, j + 2, sm.h2, gate);      \
  hipLaunchKernelGGL((k_gm_axpy_scale<JB>), dim3(gb), dim3(kWG), 0, st, w.S, sm, m, j, V, wv, n, ld, \
                     h1, w.hist, w.seg_hist)
        // vector count rounded up to a multiple of 4 (m <= 60)
        switch ((j + 4) >> 2) {
          case 1: GSE_GM_PASSES(4); break;
          case 2: GSE_GM_PASSES(8); break;
          case 3: GSE_GM_PASSES(12); break;
          case 4: GSE_GM_PASSES(16); break;
          case 5: GSE_GM_PASSES(20); break;
          case 6: GSE_GM_PASSES(24); break;
          case 7: GSE_GM_PASSES(28); break;
          case 8: GSE_GM_PASSES(32); break;
          case 9: GSE_GM_PASSES(36); break;
          case 10: GSE_GM_PASSES(40); break;
          case 11: GSE_GM_PASSES(44); break;
          case 12: GSE_GM_PASSES(48); break;
          case 13: GSE_GM_PASSES(52); break;
          case 14: GSE_GM_PASSES(56); break;
          default: GSE_GM_PASSES(60); break;
        }
#undef GSE_GM_PASSES
        err = hipGetLastError();
        if (err != hipSuccess) return err;
      }
      // k <= m columns: the tier of m bounds the unrolled loads
#define GSE_GM_UPDATE(JB) \
  hipLaunchKernelGGL((k_gm_update<JB>), dim3(gb), dim3(kWG), 0, st, w.S, sm, m, V, ld, x, n)
      if (m <= 8) GSE_GM_UPDATE(8);
      else if (m <= 16) GSE_GM_UPDATE(16);
      else if (m <= 24) GSE_GM_UPDATE(24);
      else if (m <= 32) GSE_GM_UPDATE(32);
      else if (m <= 48) GSE_GM_UPDATE(48);
      else GSE_GM_UPDATE(60);
#undef GSE_GM_UPDATE
      return hipGetLastError();
    };
    if (p->launch_mode == 1) {
      e = launch_cycle(h.s);
    } else {
      const int s_use = h.s;
      hipGraphExec_t ge = nullptr;
      e = cached_graph(graph_key(s_use), st, &ge, [&] { return launch_cycle(s_use); });
      if (e == hipSuccess) e = hipGraphLaunch(ge, st);
    }
    if (e != hipSuccess) return hip_fail(e, "gmres cycle");
    e = hipGetLastError();
    if (e == hipSuccess) e = read_state(w, &t, st);
    if (e != hipSuccess) return hip_fail(e, "gmres update");
    h.it = t.it;
    h.relres = t.relres;
    if (t.stop == kSwitch) {
      if (nsw < 2) {
        rep->switch_iter[nsw] = t.it;
        rep->switch_trigger[nsw] = t.trig;
      }
      ++nsw;
      h.s += 1;
    }
    if (t.stop == kCap && t.it >= p->max_iter) {
      // one more explicit residual for the report, then stop
      break;
    }
  }
  SolverState f;
  e = read_state(w, &f, st);
  if (e != hipSuccess) return hip_fail(e, "gmres report");
  double rt = 0.0;
  {
    e = apply(A, s_final, x, w.w, kEpiResid, b, &w.S->scratch[0], w, nullptr, st);
    SolverState t;
    if (e == hipSuccess) e = read_state(w, &t, st);
    if (e != hipSuccess) return hip_fail(e, "gmres report");
    rt = sqrt(t.scratch[0]) / f.nb;
  }
  rep->status = status;
  rep->iters = f.it;
  rep->relres_recursive = h.relres;
  rep->relres_true = rt;
  {
    const int cnt = f.it;
    int* seg = new int[(size_t)cnt + 1];
    e = hipMemcpyAsync(seg, w.seg_hist, sizeof(int) * (size_t)(cnt + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      delete[] seg;
      return hip_fail(e, "gmres report");
    }
    for (int i = 1; i <= cnt; ++i) {
      const int sg = seg[i] <= 0 ? 3 : seg[i];
      rep->iters_per_seg[sg - 1] += 1;
    }
    delete[] seg;
  }
  rep->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

}  // namespace

gse_status solve_history(const void* ws, int32_t cap, double* hist, int32_t* seg, hipStream_t st) {
  SolverState h;
  hipError_t e = hipMemcpyAsync(&h, ws, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_solve_history");
  if (h.hist_cap <= 0 || h.hist_off <= 0) return fail(GSE_ERR_ARG, "no solve recorded in this workspace");
  int cnt = h.it + 1;
  if (cnt > h.hist_cap) cnt = h.hist_cap;
  if (cnt > cap) cnt = cap;
  const char* base = reinterpret_cast<const char*>(ws);
  e = hipMemcpyAsync(hist, base + h.hist_off, sizeof(double) * (size_t)cnt, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(seg, base + h.seg_off, sizeof(int32_t) * (size_t)cnt, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "gse_solve_history");
  return GSE_OK;
}

size_t solver_workspace_bytes(int32_t method, int32_t n_rows, int64_t nnz, int32_t restart,
                              int32_t max_iter) {
  return carve(nullptr, method, n_rows, nnz, restart, max_iter).bytes;
}

gse_status cg_gse(const gse_matrix* A, const SpmvOperand& op, const double* b, double* x,
                  const gse_params* p, gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st) {
  Operator o{1, op, A->eta};
  return run_cg(o, b, x, p, rep, ws, ws_bytes, st);
}

gse_status cg_csr(const SpmvOperand& op, const double* b, double* x, const gse_params* p,
                  gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st) {
  Operator o{0, op, nullptr};
  return run_cg(o, b, x, p, rep, ws, ws_bytes, st);
}

gse_status gmres_gse(const gse_matrix* A, const SpmvOperand& op, const double* b, double* x,
                     const gse_params* p, gse_report* rep, void* ws, size_t ws_bytes,
                     hipStream_t st) {
  Operator o{1, op, A->eta};
  return run_gmres(o, b, x, p, rep, ws, ws_bytes, st);
}

gse_status gmres_csr(const SpmvOperand& op, const double* b, double* x, const gse_params* p,
                     gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st) {
  Operator o{0, op, nullptr};
  return run_gmres(o, b, x, p, rep, ws, ws_bytes, st);
}

gse_status cg_lp(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                 gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st) {
  Operator o{0, operand_of(M), nullptr, lp_launch_format(M)};
  return run_cg(o, b, x, p, rep, ws, ws_bytes, st);
}

gse_status gmres_lp(const gse_lp_matrix* M, const double* b, double* x, const gse_params* p,
                    gse_report* rep, void* ws, size_t ws_bytes, hipStream_t st) {
  Operator o{0, operand_of(M), nullptr, lp_launch_format(M)};
  return run_gmres(o, b, x, p, rep, ws, ws_bytes, st);
}

}  // namespace gse

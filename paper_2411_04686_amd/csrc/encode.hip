// encode.hip -- FP64 CSR -> GSE-SEM planes on gfx950.
//
//   k_hist   exponent histogram (Section III-B.1: occurrences of each
//            distinct exponent), LDS-privatised, 2048 bins; bin 2047 flags
//            Inf/NaN.
//   k_topk   one workgroup: the k most frequent exponents (count descending,
//            larger exponent first on ties), the maximum exponent forced into
//            the last slot when missing (Section III-B.2), stored +1.
//   k_encode per value: slot of the smallest shared exponent above the value's
//            own (an exact match when SEM = e + 1; looked up per exponent
//            field in a table k_topk fills), magnitude on that slot's 63-bit
//            fixed-point grid (Algorithm 1, denormalised by minDiff,
//            truncated), the slot in the top ceil(log2 k) bits of the column
//            word, written to the four planes with 16-byte stores.
//   k_eta    per row: sums of |a| and |a - a_s| for s = 1, 2, 3; the row
//            maxima give eta_s = ||A - A_s||_inf / ||A||_inf.
// The pooled-sample encoder (Section III-B.1, sampling) replaces k_hist by
//   k_field_scan  the matrix's largest finite exponent field and its count
//                 of Inf/NaN values,
//   k_hist_rows   the histogram of one drawn row per block of rows,
// and k_topk adds the matrix's largest exponent when the pooled choice
// misses it; k_encode then counts the exactly shared values itself
// (k_fold_covered adds up its partial counts).
#include "gse_internal.h"

namespace gse {
namespace {

struct SemIn {
  int16_t sem[GSE_MAX_EXP];
  int32_t have;
};

__global__ __launch_bounds__(256) void k_hist(const double* __restrict__ val, int nnz,
                                              EncodeScratch* sc) {
  __shared__ uint32_t h[2048];
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
    const uint64_t u = double_to_bits(val[i]);
    atomicAdd(&h[(u >> 52) & 0x7FFu], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2048; i += blockDim.x)
    if (h[i]) atomicAdd(&sc->hist[i], h[i]);
}

// Largest exponent field below 2047 over all values (into sc->max_field)
// and the number of Inf/NaN values (into sc->nonfinite): one atomic of each
// per workgroup.
__global__ __launch_bounds__(256) void k_field_scan(const double* __restrict__ val, int nnz,
                                                   EncodeScratch* sc) {
  __shared__ int red_m[kWaves], red_n[kWaves];
  int m = 0, nf = 0;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
    const int e = (int)((double_to_bits(val[i]) >> 52) & 0x7FFu);
    if (e == 2047) ++nf;
    else m = e > m ? e : m;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    m = max(m, __shfl_xor(m, off, 64));
    nf += __shfl_xor(nf, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red_m[threadIdx.x >> 6] = m;
    red_n[threadIdx.x >> 6] = nf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) {
      m = max(m, red_m[w]);
      nf += red_n[w];
    }
    if (m > 0) atomicMax(&sc->max_field, m);
    if (nf) atomicAdd(&sc->nonfinite, nf);
  }
}

// Pooled histogram of the drawn rows: one wave per block of rows, block b
// adds the exponent fields of row sample_rows[b] (bit 4 of range_err when
// that row lies outside block b).  LDS-privatised like k_hist.
__global__ __launch_bounds__(256) void k_hist_rows(const int32_t* __restrict__ row_ptr, int n_rows,
                                                   const double* __restrict__ val, int block_rows,
                                                   const int32_t* __restrict__ sample_rows,
                                                   EncodeScratch* sc) {
  __shared__ uint32_t h[2048];
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const int n_blocks = (int)(((long long)n_rows + block_rows - 1) / block_rows);
  const int lane = threadIdx.x & 63;
  const int wstride = gridDim.x * kWaves;
  bool bad = false;
  for (int b = blockIdx.x * kWaves + (threadIdx.x >> 6); b < n_blocks; b += wstride) {
    const long long r0 = (long long)b * block_rows;
    const long long r1 = min(r0 + block_rows, (long long)n_rows);
    const int sr = sample_rows[b];
    if (sr < r0 || sr >= r1) {
      bad = true;
      continue;
    }
    const int j1 = row_ptr[sr + 1];
    for (int j = row_ptr[sr] + lane; j < j1; j += 64)
      atomicAdd(&h[(double_to_bits(val[j]) >> 52) & 0x7FFu], 1u);
  }
  if (bad && lane == 0) atomicOr(&sc->range_err, 4);
  __syncthreads();
  for (int i = threadIdx.x; i < 2048; i += blockDim.x)
    if (h[i]) atomicAdd(&sc->hist[i], h[i]);
}

__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v,
                                                            unsigned long long* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long m = red[0];
  for (int i = 1; i < kWaves; ++i) m = red[i] > m ? red[i] : m;
  return m;
}

// Slot of the smallest shared exponent above each exponent field (the
// slot search of Algorithm 1, done once per field instead of per value):
// -1 when no shared exponent is above it, and for the Inf/NaN field.
__device__ __forceinline__ void fill_slot_lookup(const int16_t* tab, int8_t* slot_of) {
  for (int e = threadIdx.x; e < 2048; e += blockDim.x) {
    int slot = -1, best = 1 << 30;
    if (e < 2047) {
      for (int q = 0; q < GSE_MAX_EXP; ++q) {
        const int S = tab[q];
        if (S > e && S < best) {
          best = S;
          slot = q;
        }
      }
    }
    slot_of[e] = (int8_t)slot;
  }
}

// pooled: sc->hist holds the drawn rows' counts (k_hist_rows) and
// sc->max_field, sc->nonfinite the whole matrix's (k_field_scan); the
// matrix's largest exponent then takes the next free slot, or the last, when
// the table misses it (as for a block's table, k_blk_encode), and the count
// of exactly shared values is left to k_encode.
__global__ __launch_bounds__(256) void k_topk(EncodeScratch* sc, int num_exp, SemIn in,
                                              int pooled) {
  __shared__ uint32_t h[2048];
  __shared__ unsigned char taken[2048];
  __shared__ unsigned long long red[kWaves];
  __shared__ int chosen[GSE_MAX_EXP];
  __shared__ int16_t tab[GSE_MAX_EXP];
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) {
    h[i] = sc->hist[i];
    taken[i] = 0;
    // pooled: the counts now live in LDS; the global bins become the
    // per-workgroup partial counts of k_encode<true>
    if (pooled) sc->hist[i] = 0u;
  }
  __syncthreads();
  if (in.have) {
    if (threadIdx.x == 0) {
      int used = 0;
      unsigned long long cov = 0;
      for (int i = 0; i < GSE_MAX_EXP; ++i) {
        sc->sem[i] = in.sem[i];
        tab[i] = in.sem[i];
        if (in.sem[i] > 0) {
          ++used;
          cov += h[in.sem[i] - 1];
        }
      }
      sc->used = used;
      sc->covered = cov;
      sc->nonfinite = (int)h[2047];
    }
    __syncthreads();
    fill_slot_lookup(tab, sc->slot_of);
    return;
  }
  int used = 0;
  for (int slot = 0; slot < num_exp; ++slot) {
    unsigned long long best = 0;
    for (int e = 1 + threadIdx.x; e <= 2046; e += blockDim.x) {
      if (!taken[e] && h[e] > 0) {
        const unsigned long long key = ((unsigned long long)h[e] << 11) | (unsigned long long)e;
        best = key > best ? key : best;
      }
    }
    best = block_max_u64(best, red);
    if (best == 0) break;
    const int e = (int)(best & 0x7FFu);
    if (threadIdx.x == 0) {
      taken[e] = 1;
      chosen[used] = e;
    }
    ++used;
    __syncthreads();
  }
  unsigned long long me = 0;
  for (int e = 1 + threadIdx.x; e <= 2046; e += blockDim.x)
    if (h[e] > 0) me = (unsigned long long)e > me ? (unsigned long long)e : me;
  const int max_e = (int)block_max_u64(me, red);
  if (threadIdx.x == 0) {
    if (used == 0) {
      chosen[0] = 1023;
      used = 1;
    } else if (!taken[max_e]) {
      chosen[used - 1] = max_e;
    }
    int range_err = 0;
    for (int i = 0; i < used; ++i)
      if (chosen[i] < 63) range_err = 1;
    const int gmax = pooled ? sc->max_field : 0;
    if (gmax > 0) {
      bool present = false;
      for (int i = 0; i < used; ++i) present = present || chosen[i] == gmax;
      if (!present) {
        if (used < num_exp) ++used;
        chosen[used - 1] = gmax;
        if (gmax < 63) range_err = 1;
      }
    }
    unsigned long long cov = 0;
    for (int i = 0; i < GSE_MAX_EXP; ++i) {
      sc->sem[i] = 0;
      tab[i] = 0;
    }
    for (int i = 0; i < used; ++i) {
      sc->sem[i] = (int16_t)(chosen[i] + 1);
      tab[i] = (int16_t)(chosen[i] + 1);
      cov += h[chosen[i]];
    }
    sc->used = used;
    if (range_err) sc->range_err |= 1;
    if (!pooled) {
      sc->covered = cov;
      sc->nonfinite = (int)h[2047];
    }
  }
  __syncthreads();
  fill_slot_lookup(tab, sc->slot_of);
}

// One value (bits u, column cv) against a table: the slot of the smallest
// shared exponent above the value's exponent field (slot_s, -1: none ->
// *bad), the magnitude on that slot's grid (Algorithm 1: hidden one made
// explicit, shifted right by minDiff, truncated; the field holds 63 - ei
// bits), and the words of the four planes.  *exact: the value's exponent is
// itself shared (SEM = e + 1).
struct Words4 {
  uint32_t c, h16, t1, t2;
};

__device__ __forceinline__ Words4 encode_value(uint64_t u, int cv, const int8_t* slot_s,
                                               const int* sem_s, int idx_bits, int in_value,
                                               int* bad, int* exact) {
  const int ei = in_value ? idx_bits : 0;
  const int e = (int)((u >> 52) & 0x7FFu);
  int slot = slot_s[e];
  uint64_t F = 0;
  if (slot < 0) {
    *bad = 1;
    slot = 0;
  } else {
    const int best = sem_s[slot];
    *exact = best == e + 1;
    const uint64_t frac = u & ((uint64_t(1) << 52) - 1);
    const uint64_t sig = e ? ((uint64_t(1) << 52) | frac) : frac;
    const int sh = 11 - ei - (best - (e ? e : 1));
    F = (sh >= 0) ? (sig << sh) : ((-sh >= 64) ? 0 : (sig >> (-sh)));
  }
  Words4 w;
  if (in_value) {
    w.c = (uint32_t)cv;
    w.h16 = (uint32_t)((u >> 63) << 15) | ((uint32_t)slot << (15 - idx_bits)) |
            (uint32_t)(F >> 48);
  } else {
    w.c = (uint32_t)cv | (idx_bits > 0 ? ((uint32_t)slot << (32 - idx_bits)) : 0u);
    w.h16 = (uint32_t)((u >> 63) << 15) | (uint32_t)(F >> 48);
  }
  w.t1 = (uint32_t)((F >> 32) & 0xFFFFu);
  w.t2 = (uint32_t)(F & 0xFFFFFFFFu);
  return w;
}

// Groups of 8 values per thread; writes 32 + 16 + 16 + 32 bytes per group
// (the planes are padded, so the tail group writes zeros past nnz).
// COUNT: also count the values whose own exponent is shared, one partial
// sum per workgroup added to bin (blockIdx & 2047) of sc->hist: thousands of
// atomics on a single word serialise in its L2 channel and cost more than
// the encode itself.  k_fold_covered adds the bins up.
template <bool COUNT>
__global__ __launch_bounds__(256) void k_encode(const double* __restrict__ val,
                                                const int32_t* __restrict__ col, int nnz,
                                                EncodeScratch* sc, int idx_bits, int in_value,
                                                uint32_t* __restrict__ col_idx,
                                                uint16_t* __restrict__ head,
                                                uint16_t* __restrict__ tail1,
                                                uint32_t* __restrict__ tail2) {
  __shared__ int sem_s[GSE_MAX_EXP];
  __shared__ int8_t slot_s[2048];
  if (threadIdx.x < GSE_MAX_EXP) sem_s[threadIdx.x] = sc->sem[threadIdx.x];
  for (int e = threadIdx.x; e < 2048; e += blockDim.x) slot_s[e] = sc->slot_of[e];
  __syncthreads();
  // the slot goes to the top of the column word, or (in_value) below the
  // sign of the value word, whose magnitude field then loses idx_bits bits
  const int n_groups = (nnz + 7) >> 3;
  const int stride = gridDim.x * blockDim.x;
  int bad = 0;
  unsigned covered = 0;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_groups; g += stride) {
    uint32_t cw[8], t2[8], hh[4], tt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) hh[k] = tt[k] = 0u;
    // All sixteen loads of a group go out before any arithmetic: behind a
    // per-value `j < nnz` branch each load waited for itself.  Only the
    // last, partial group keeps the guard.
    uint64_t uv[8];
    int cv[8];
    if (g * 8 + 8 <= nnz) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        uv[k] = double_to_bits(val[g * 8 + k]);
        cv[k] = col[g * 8 + k];
      }
      __builtin_amdgcn_sched_barrier(0);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int j = g * 8 + k;
        uv[k] = j < nnz ? double_to_bits(val[j]) : 0u;
        cv[k] = j < nnz ? col[j] : 0;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = g * 8 + k;
      uint32_t c = 0, h16 = 0, t116 = 0, t232 = 0;
      if (j < nnz) {
        int exact = 0;
        const Words4 w = encode_value(uv[k], cv[k], slot_s, sem_s, idx_bits, in_value, &bad, &exact);
        if constexpr (COUNT) covered += (unsigned)exact;
        c = w.c;
        h16 = w.h16;
        t116 = w.t1;
        t232 = w.t2;
      }
      cw[k] = c;
      t2[k] = t232;
      hh[k >> 1] |= h16 << ((k & 1) * 16);
      tt[k >> 1] |= t116 << ((k & 1) * 16);
    }
    uint4* cp = reinterpret_cast<uint4*>(col_idx + g * 8);
    cp[0] = make_uint4(cw[0], cw[1], cw[2], cw[3]);
    cp[1] = make_uint4(cw[4], cw[5], cw[6], cw[7]);
    *reinterpret_cast<uint4*>(head + g * 8) = make_uint4(hh[0], hh[1], hh[2], hh[3]);
    *reinterpret_cast<uint4*>(tail1 + g * 8) = make_uint4(tt[0], tt[1], tt[2], tt[3]);
    uint4* tp = reinterpret_cast<uint4*>(tail2 + g * 8);
    tp[0] = make_uint4(t2[0], t2[1], t2[2], t2[3]);
    tp[1] = make_uint4(t2[4], t2[5], t2[6], t2[7]);
  }
  if (bad) atomicOr(&sc->range_err, 2);
  if constexpr (COUNT) {
    __shared__ unsigned red[kWaves];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) covered += __shfl_xor(covered, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = covered;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned t = 0;
      for (int w = 0; w < kWaves; ++w) t += red[w];
      if (t) atomicAdd(&sc->hist[blockIdx.x & 2047], t);
    }
  }
}

// sc->covered = the sum of k_encode<true>'s partial counts (one workgroup).
__global__ __launch_bounds__(256) void k_fold_covered(EncodeScratch* sc) {
  __shared__ unsigned long long red[kWaves];
  unsigned long long t = 0;
  for (int i = threadIdx.x; i < 2048; i += blockDim.x) t += sc->hist[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) t += red[w];
    sc->covered = t;
  }
}

__device__ __forceinline__ int slot_in(uint32_t c, uint32_t h, const ColSplit& cs) {
  return (int)(((c >> cs.shift) & cs.slot_mask) | ((h >> cs.hshift) & cs.hmask));
}

// Value read with s segments (exact; same decode as the SpMV operators);
// sem is the shared exponent of the value's slot.
__device__ __forceinline__ double value_s(uint32_t h, uint32_t t1, uint32_t t2, int sem,
                                          const ColSplit& cs, int s) {
  const int fb = 63 - cs.ei;  // bits of the magnitude field
  const int W = fb - ((s == 1) ? 48 : (s == 2) ? 32 : 0);
  const uint64_t Ff = ((uint64_t)(h & cs.mag_mask) << 48) | ((uint64_t)t1 << 32) | (uint64_t)t2;
  const uint64_t F = Ff >> (fb - W);
  const double sc = bits_to_double((uint64_t)(sem - W) << 52);
  const double mag = (double)F * sc;  // F <= 53 significant bits: exact
  return (h >> 15) ? -mag : mag;
}

// Eight lanes per row, grid-stride over rows; the row maxima of the four
// sums are reduced per workgroup and then merged into norm_bits (the bit
// patterns of non-negative doubles order like the values).  BLK: row r reads
// the table of its block, bsem + (r / block_rows) * stride.
template <bool BLK>
__global__ __launch_bounds__(256) void k_eta(const int32_t* __restrict__ row_ptr, int n_rows,
                                             const double* __restrict__ val,
                                             const uint32_t* __restrict__ col_idx,
                                             const uint16_t* __restrict__ head,
                                             const uint16_t* __restrict__ tail1,
                                             const uint32_t* __restrict__ tail2,
                                             EncodeScratch* sc, ColSplit cs,
                                             const int16_t* __restrict__ bsem, int block_rows,
                                             int stride) {
  __shared__ int sem_s[GSE_MAX_EXP];
  __shared__ double red[4][kWaves];
  if (threadIdx.x < GSE_MAX_EXP) sem_s[threadIdx.x] = sc->sem[threadIdx.x];
  __syncthreads();
  auto table_of = [&](int r) -> const int16_t* {
    return BLK ? bsem + (size_t)(r / block_rows) * stride : nullptr;
  };
  const int sub = threadIdx.x & 7;
  const int grp = (blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int ngrp = (gridDim.x * blockDim.x) >> 3;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  // One row per eight lanes, two rows per pass: the first eight entries of
  // both rows are loaded unconditionally (clamped into the row, masked when
  // past its end) before any arithmetic, so a pass costs one memory round
  // trip after the row pointers; longer rows continue in a loop.  Each
  // lane adds its entries of a row in the order j = start + sub, +8, ...
  struct Ent {
    double v;
    uint32_t c, h, t1, t2;
  };
  auto load_ent = [&](int j) {
    return Ent{val[j], col_idx[j], head[j], tail1[j], tail2[j]};
  };
  // adds the four terms of entry x, or exact zeros when !use (the sums are
  // non-negative, so a + 0.0 == a) -- no branch for the loads to sink into;
  // Sb: the row's block table (BLK)
  auto add_terms = [&](double (&a)[4], const Ent& x, bool use, const int16_t* Sb) {
    const int slot = slot_in(x.c, x.h, cs);
    const int sem = BLK ? (int)Sb[slot] : sem_s[slot];
    const double t0 = fabs(x.v);
    const double t1 = fabs(x.v - value_s(x.h, x.t1, x.t2, sem, cs, 1));
    const double t2 = fabs(x.v - value_s(x.h, x.t1, x.t2, sem, cs, 2));
    const double t3 = fabs(x.v - value_s(x.h, x.t1, x.t2, sem, cs, 3));
    a[0] += use ? t0 : 0.0;
    a[1] += use ? t1 : 0.0;
    a[2] += use ? t2 : 0.0;
    a[3] += use ? t3 : 0.0;
  };
  auto finish = [&](double (&a)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double t = a[q];
      t += __shfl_xor(t, 4, 64);
      t += __shfl_xor(t, 2, 64);
      t += __shfl_xor(t, 1, 64);
      m[q] = fmax(m[q], t);
    }
  };
  const int nnz = row_ptr[n_rows];
  for (int r = grp; r < n_rows; r += 2 * ngrp) {
    const int r2 = r + ngrp;
    const bool has2 = r2 < n_rows;
    const int a0 = row_ptr[r], a1 = row_ptr[r + 1];
    const int b0 = has2 ? row_ptr[r2] : 0, b1 = has2 ? row_ptr[r2 + 1] : 0;
    double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
    if (nnz > 0) {
      const int16_t* Sa = table_of(r);
      const int16_t* Sb = table_of(has2 ? r2 : r);
      const int ja = a0 + sub, jb = b0 + sub;
      const Ent ea = load_ent(max(min(ja, a1 - 1), 0));
      const Ent eb = load_ent(max(min(jb, b1 - 1), 0));
      add_terms(a, ea, ja < a1, Sa);
      add_terms(b, eb, jb < b1, Sb);
      for (int j = ja + 8; j < a1; j += 8) add_terms(a, load_ent(j), true, Sa);
      for (int j = jb + 8; j < b1; j += 8) add_terms(b, load_ent(j), true, Sb);
    }
    finish(a);
    if (has2) finish(b);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double t = m[q];
    for (int off = 32; off >= 1; off >>= 1) t = fmax(t, __shfl_xor(t, off, 64));
    if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, red[threadIdx.x][w]);
    // the four maxima share one cache line, where every atomic serialises:
    // skip it when the value already there (possibly stale, hence only
    // ever smaller) is not below this workgroup's
    const unsigned long long bits = (unsigned long long)double_to_bits(t);
    if (__hip_atomic_load(&sc->norm_bits[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
        bits)
      atomicMax(&sc->norm_bits[threadIdx.x], bits);
  }
}

// Per-row-block tables: workgroup b owns rows [b*R, min((b+1)*R, n_rows)).
// The table comes from the exponent histogram of the sample (row
// sample_rows[b], or the whole block when sample_rows is null) by the rules
// of k_topk; then the block's own largest exponent goes into the next free
// slot, or the last, if the table misses it.  The block's values are encoded
// against that table with one thread per value.  The last workgroup also
// zeroes the planes' padding.
__global__ __launch_bounds__(256) void k_blk_encode(
    const int32_t* __restrict__ row_ptr, int n_rows, const int32_t* __restrict__ col,
    const double* __restrict__ val, int nnz, int pad, int block_rows,
    const int32_t* __restrict__ sample_rows, int num_exp, int idx_bits, int in_value, int stride,
    int16_t* __restrict__ block_sem, EncodeScratch* sc, uint32_t* __restrict__ col_idx,
    uint16_t* __restrict__ head, uint16_t* __restrict__ tail1, uint32_t* __restrict__ tail2) {
  __shared__ uint32_t h[2048];
  __shared__ unsigned char taken[2048];
  __shared__ int8_t slot_s[2048];
  __shared__ unsigned long long red[kWaves];
  __shared__ int chosen[GSE_MAX_EXP];
  __shared__ int sem_s[GSE_MAX_EXP];
  __shared__ int16_t tab[GSE_MAX_EXP];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int r0 = (int)((long long)b * block_rows);
  const int r1 = (int)min((long long)r0 + block_rows, (long long)n_rows);
  const int j0 = row_ptr[r0], j1 = row_ptr[r1];
  for (int i = tid; i < 2048; i += blockDim.x) {
    h[i] = 0u;
    taken[i] = 0;
  }
  __syncthreads();
  int s0 = j0, s1 = j1;
  bool bad_sample = false;
  if (sample_rows) {
    const int sr = sample_rows[b];
    if (sr < r0 || sr >= r1) {
      bad_sample = true;
      s0 = s1 = 0;
    } else {
      s0 = row_ptr[sr];
      s1 = row_ptr[sr + 1];
    }
  }
  for (int j = s0 + tid; j < s1; j += blockDim.x) atomicAdd(&h[(double_to_bits(val[j]) >> 52) & 0x7FFu], 1u);
  unsigned long long me = 0;
  int nonfinite = 0;
  for (int j = j0 + tid; j < j1; j += blockDim.x) {
    const unsigned e = (unsigned)((double_to_bits(val[j]) >> 52) & 0x7FFu);
    if (e == 2047u) ++nonfinite;
    else me = e > me ? e : me;
  }
  if (nonfinite) atomicAdd(&sc->nonfinite, nonfinite);
  if (bad_sample && tid == 0) atomicOr(&sc->range_err, 4);
  const int max_e = (int)block_max_u64(me, red);  // its barriers also end the histogram
  int used = 0;
  for (int slot = 0; slot < num_exp; ++slot) {
    unsigned long long best = 0;
    for (int e = 1 + tid; e <= 2046; e += blockDim.x) {
      if (!taken[e] && h[e] > 0) {
        const unsigned long long key = ((unsigned long long)h[e] << 11) | (unsigned long long)e;
        best = key > best ? key : best;
      }
    }
    best = block_max_u64(best, red);
    if (best == 0) break;
    const int e = (int)(best & 0x7FFu);
    if (tid == 0) {
      taken[e] = 1;
      chosen[used] = e;
    }
    ++used;
    __syncthreads();
  }
  unsigned long long ms = 0;
  for (int e = 1 + tid; e <= 2046; e += blockDim.x)
    if (h[e] > 0) ms = (unsigned long long)e > ms ? (unsigned long long)e : ms;
  const int sample_max = (int)block_max_u64(ms, red);
  if (tid == 0) {
    if (used == 0) {
      chosen[0] = 1023;
      used = 1;
    } else if (!taken[sample_max]) {
      chosen[used - 1] = sample_max;
    }
    int range_err = 0;
    for (int i = 0; i < used; ++i)
      if (chosen[i] < 63) range_err = 1;
    if (max_e > 0) {
      bool present = false;
      for (int i = 0; i < used; ++i) present = present || chosen[i] == max_e;
      if (!present) {
        if (used < num_exp) ++used;
        chosen[used - 1] = max_e;
        if (max_e < 63) range_err = 1;
      }
    }
    for (int i = 0; i < GSE_MAX_EXP; ++i) {
      tab[i] = i < used ? (int16_t)(chosen[i] + 1) : (int16_t)0;
      sem_s[i] = tab[i];
    }
    if (range_err) atomicOr(&sc->range_err, 1);
    atomicMax(&sc->used, used);
  }
  __syncthreads();
  for (int i = tid; i < stride; i += blockDim.x) block_sem[(size_t)b * stride + i] = tab[i];
  fill_slot_lookup(tab, slot_s);
  __syncthreads();
  int bad = 0;
  unsigned long long covered = 0;
  for (int j = j0 + tid; j < j1; j += blockDim.x) {
    int exact = 0;
    const Words4 w = encode_value(double_to_bits(val[j]), col[j], slot_s, sem_s, idx_bits,
                                  in_value, &bad, &exact);
    col_idx[j] = w.c;
    head[j] = (uint16_t)w.h16;
    tail1[j] = (uint16_t)w.t1;
    tail2[j] = w.t2;
    covered += (unsigned long long)exact;
  }
  if (b == (int)gridDim.x - 1) {
    for (int j = nnz + tid; j < pad; j += blockDim.x) {
      col_idx[j] = 0u;
      head[j] = 0;
      tail1[j] = 0;
      tail2[j] = 0u;
    }
  }
  if (covered) atomicAdd(&sc->covered, covered);
  if (bad) atomicOr(&sc->range_err, 2);
}

// Zero `n` 8-byte words with one workgroup.
__global__ void __launch_bounds__(256) k_zero_words(unsigned long long* p, int n) {
  for (int i = threadIdx.x; i < n; i += 256) p[i] = 0ull;
}

}  // namespace

hipError_t launch_encode(const int32_t* row_ptr, const int32_t* col, const double* val,
                         int32_t n_rows, int32_t nnz, int32_t num_exp, const int16_t* sem_in,
                         gse_matrix* A, EncodeScratch* sc, hipStream_t st) {
  // cleared by a kernel rather than a memset node, so that the sequence
  // can also be recorded into a HIP graph
  static_assert(sizeof(EncodeScratch) % 8 == 0, "the scratch record is cleared in 8-byte words");
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(sc),
                     (int)(sizeof(EncodeScratch) / 8));
  SemIn in{};
  in.have = sem_in != nullptr;
  for (int i = 0; i < GSE_MAX_EXP; ++i) in.sem[i] = (sem_in && i < num_exp) ? sem_in[i] : 0;
  int hb = (nnz + 256 * 16 - 1) / (256 * 16);
  hb = hb < 1 ? 1 : (hb > 2048 ? 2048 : hb);
  hipLaunchKernelGGL(k_hist, dim3(hb), dim3(256), 0, st, val, nnz, sc);
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(256), 0, st, sc, num_exp, in, 0);
  const int groups = (nnz + 7) / 8;
  int eb = (groups + 255) / 256;
  eb = eb < 1 ? 1 : (eb > 16384 ? 16384 : eb);
  const bool in_value = A->idx_layout == GSE_IDX_VALUE;
  hipLaunchKernelGGL(k_encode<false>, dim3(eb), dim3(256), 0, st, val, col, nnz, sc, A->idx_bits,
                     in_value ? 1 : 0, A->col_idx, A->head, A->tail1, A->tail2);
  int rbk = (n_rows + 31) / 32;
  rbk = rbk < 1 ? 1 : (rbk > 4096 ? 4096 : rbk);
  hipLaunchKernelGGL(k_eta<false>, dim3(rbk), dim3(256), 0, st, row_ptr, n_rows, val, A->col_idx,
                     A->head, A->tail1, A->tail2, sc, col_split(A->idx_bits, in_value),
                     (const int16_t*)nullptr, 1, 0);
  return hipGetLastError();
}

hipError_t launch_encode_sampled(const int32_t* row_ptr, const int32_t* col, const double* val,
                                 int32_t n_rows, int32_t nnz, int32_t num_exp, int32_t block_rows,
                                 const int32_t* sample_rows, gse_matrix* A, EncodeScratch* sc,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(sc),
                     (int)(sizeof(EncodeScratch) / 8));
  int hb = (nnz + 256 * 16 - 1) / (256 * 16);
  hb = hb < 1 ? 1 : (hb > 2048 ? 2048 : hb);
  hipLaunchKernelGGL(k_field_scan, dim3(hb), dim3(256), 0, st, val, nnz, sc);
  const int64_t n_blocks = ((int64_t)n_rows + block_rows - 1) / block_rows;
  // four drawn rows per workgroup, at most 1024 workgroups (grid-stride)
  int sb = (int)((n_blocks + kWaves - 1) / kWaves);
  sb = sb < 1 ? 1 : (sb > 1024 ? 1024 : sb);
  hipLaunchKernelGGL(k_hist_rows, dim3(sb), dim3(256), 0, st, row_ptr, n_rows, val, block_rows,
                     sample_rows, sc);
  SemIn in{};
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(256), 0, st, sc, num_exp, in, 1);
  const int groups = (nnz + 7) / 8;
  int eb = (groups + 255) / 256;
  eb = eb < 1 ? 1 : (eb > 16384 ? 16384 : eb);
  const bool in_value = A->idx_layout == GSE_IDX_VALUE;
  hipLaunchKernelGGL(k_encode<true>, dim3(eb), dim3(256), 0, st, val, col, nnz, sc, A->idx_bits,
                     in_value ? 1 : 0, A->col_idx, A->head, A->tail1, A->tail2);
  hipLaunchKernelGGL(k_fold_covered, dim3(1), dim3(256), 0, st, sc);
  int rbk = (n_rows + 31) / 32;
  rbk = rbk < 1 ? 1 : (rbk > 4096 ? 4096 : rbk);
  hipLaunchKernelGGL(k_eta<false>, dim3(rbk), dim3(256), 0, st, row_ptr, n_rows, val, A->col_idx,
                     A->head, A->tail1, A->tail2, sc, col_split(A->idx_bits, in_value),
                     (const int16_t*)nullptr, 1, 0);
  return hipGetLastError();
}

hipError_t launch_encode_blocks(const int32_t* row_ptr, const int32_t* col, const double* val,
                                int32_t n_rows, int32_t nnz, int32_t num_exp,
                                const int32_t* sample_rows, gse_matrix* A, EncodeScratch* sc,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(sc),
                     (int)(sizeof(EncodeScratch) / 8));
  if (n_rows < 1) return hipGetLastError();
  const int n_blocks = (int)(((int64_t)n_rows + A->block_rows - 1) / A->block_rows);
  const int pad = (int)((nnz + kPadTo - 1) / kPadTo * kPadTo);
  const bool in_value = A->idx_layout == GSE_IDX_VALUE;
  hipLaunchKernelGGL(k_blk_encode, dim3(n_blocks), dim3(256), 0, st, row_ptr, n_rows, col, val, nnz,
                     pad, A->block_rows, sample_rows, num_exp, A->idx_bits, in_value ? 1 : 0,
                     A->block_stride, A->block_sem, sc, A->col_idx, A->head, A->tail1, A->tail2);
  int rbk = (n_rows + 31) / 32;
  rbk = rbk < 1 ? 1 : (rbk > 4096 ? 4096 : rbk);
  hipLaunchKernelGGL(k_eta<true>, dim3(rbk), dim3(256), 0, st, row_ptr, n_rows, val, A->col_idx,
                     A->head, A->tail1, A->tail2, sc, col_split(A->idx_bits, in_value),
                     (const int16_t*)A->block_sem, A->block_rows, A->block_stride);
  return hipGetLastError();
}

}  // namespace gse

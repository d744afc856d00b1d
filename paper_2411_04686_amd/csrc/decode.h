// decode.h -- exact decode of one GSE-SEM non-zero (Algorithm 2 and its
// two wider variants, Section III-C.2), shared by the SpMV schedules.
#pragma once

#include "gse_internal.h"

namespace gse {

// What the decode needs: the scale table (in LDS) and the split of the
// column words.
struct DecodeCtx {
  const uint32_t* tab;
  ColSplit split;
};

// Scale table for s segments: entry `slot` holds the high word of
// 2^(SEM[slot] - 1023 - W_s) as IEEE bits -- biased exponent SEM - W_s, zero
// fraction (SEM >= 64 keeps it normal); the low word is zero, and the value's
// sign goes into bit 31 of the high word.  W_s = 15, 31, 63 less ei, the
// index bits the value word gives up in the index-in-value layout.  Every
// thread of the workgroup takes part; build_scale_n fills n entries from n
// consecutive shared exponents (several blocks' tables back to back).
template <int FMT>
__device__ __forceinline__ void build_scale_n(const int16_t* sem, int n, uint32_t* tab, int ei) {
  if constexpr (is_gse(FMT)) {
    const int W = ((FMT == 1) ? 15 : (FMT == 2) ? 31 : 63) - ei;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int S = sem[i];
      tab[i] = S > W ? (uint32_t)(S - W) << 20 : 0u;
    }
  }
}

template <int FMT>
__device__ __forceinline__ void build_scale(const int16_t* sem, uint32_t* tab, int ei = 0) {
  build_scale_n<FMT>(sem, kScaleEntries, tab, ei);
}

// Decode one non-zero: returns the FP64 value and its column.
template <int FMT>
__device__ __forceinline__ double decode(uint32_t c, uint32_t h, uint32_t t1, uint32_t t2, double v,
                                         const DecodeCtx& dc, int& column) {
  if constexpr (FMT == kCsr64) {
    column = (int)c;
    return v;
  } else if constexpr (FMT == kFp16) {
    // binary16 -> binary32 -> binary64: both widenings are exact
    column = (int)c;
    return (double)(float)__builtin_bit_cast(_Float16, (unsigned short)h);
  } else if constexpr (FMT == kBf16) {
    // bfloat16 is the top half of a binary32
    column = (int)c;
    return (double)__uint_as_float(h << 16);
  } else {
    const ColSplit& cs = dc.split;
    column = (int)(c & cs.col_mask);
    const uint32_t slot = ((c >> cs.shift) & cs.slot_mask) | ((h >> cs.hshift) & cs.hmask);
    const uint32_t hi = dc.tab[slot] | ((h & 0x8000u) << 16);
    const double sc = __hiloint2double((int)hi, 0);
    const uint32_t hm = h & cs.mag_mask;
    if constexpr (FMT == 1) {
      return (double)hm * sc;
    } else if constexpr (FMT == 2) {
      return (double)((hm << 16) | t1) * sc;
    } else {
      // F = hi31 * 2^32 + lo32; F has at most 53 significant bits, so the
      // fused sum below is exact (2^32 * sc: 32 added to the exponent field).
      const double sc_hi = __hiloint2double((int)(hi + (32u << 20)), 0);
      const double fhi = (double)((hm << 16) | t1);
      return __builtin_fma(fhi, sc_hi, (double)t2 * sc);
    }
  }
}

}  // namespace gse

// decode.h -- exact decode of one GSE-SEM non-zero (Algorithm 2 and its
// two wider variants, Section III-C.2), shared by the SpMV schedules.
#pragma once

#include "gse_internal.h"

namespace gse {

// Signed scale table for s segments: entry (slot | sign << 3) holds
// +-2^(SEM[slot] - 1023 - W_s).  Built as IEEE bits: biased exponent
// SEM - W_s, zero fraction (SEM >= 64 keeps it normal).
template <int FMT>
__device__ __forceinline__ void build_scale(const int16_t* sem, double* scale) {
  if constexpr (FMT != kCsr64) {
    constexpr int W = (FMT == 1) ? 15 : (FMT == 2) ? 31 : 63;
    const int i = threadIdx.x;
    if (i < 16) {
      const int S = sem[i & 7];
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

}  // namespace gse

// diag.hip -- streaming kernels that measure what the memory system gives a
// launch of a given size: the practical ceilings the SpMV is compared with,
// and the reference for scaling the HBM traffic counters.
//
//   k_stream_copy     dst = src in 16-byte chunks (half the bytes read).
//   k_stream_reduce8  dst[i] = src[8i] + ... + src[8i+7] (eight of every
//                     nine bytes read, the read share of the SpMV): each
//                     lane loads one 16-byte chunk, four consecutive lanes
//                     add their pairs through two shuffles and the first
//                     writes the sum.  Loads are non-temporal (streamed
//                     once); a grid of eight workgroups per CU strides over
//                     the chunks.
#include "gse_internal.h"

namespace gse {
namespace {

typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = src[i];
}

// n_out outputs, 4 n_out chunks.  blockDim and the grid stride are
// multiples of 4, so the four lanes of an output are in or out together.
__global__ __launch_bounds__(256) void k_stream_reduce8(const f64x2* __restrict__ src,
                                                        double* __restrict__ dst, size_t n_out) {
  const size_t n_ch = 4 * n_out;
  size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; c < n_ch; c += stride) {
    const f64x2 v = __builtin_nontemporal_load(src + c);
    double s = v.x + v.y;
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if ((c & 3) == 0) dst[c >> 2] = s;
  }
}

}  // namespace

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                     reinterpret_cast<const uint4*>(src), reinterpret_cast<uint4*>(dst), n);
  return hipGetLastError();
}

hipError_t launch_stream_reduce8(const double* src, double* dst, size_t n_out, hipStream_t st) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  size_t blocks = (4 * n_out + 255) / 256;
  const size_t cap = 8 * (size_t)(cus > 0 ? cus : 1);
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_stream_reduce8, dim3((unsigned)blocks), dim3(256), 0, st,
                     reinterpret_cast<const f64x2*>(src), dst, n_out);
  return hipGetLastError();
}

}  // namespace gse

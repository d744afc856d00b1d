// noalloc.hip -- gse_encode_static: the encoder without a caller workspace,
// for callers that cannot allocate device memory.  The encoder's scratch
// record (exponent histogram, error counters, selected table, coverage count
// and the four row-sum maxima behind eta) lives in a file-scope device array
// that every GPU holds for the life of the process.
#include <mutex>

#include "gse_internal.h"

namespace gse {
namespace {

// Bytes of the static scratch array (per GPU).  The encoder's record needs
// sizeof(EncodeScratch) whatever the matrix; the rest is headroom.
constexpr size_t kStaticScratchBytes = 16384;
static_assert(sizeof(EncodeScratch) <= kStaticScratchBytes,
              "the encoder's scratch record must fit the static array");

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (the host-side name is not a device address).
gse_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "gse_encode_static: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(GSE_ERR_ARG, "gse_encode_static: device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "gse_encode_static: hipGetSymbolAddress");
    if (!p) return fail(GSE_ERR_HIP, "gse_encode_static: no device address for the scratch array");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return GSE_OK;
}

}  // namespace
}  // namespace gse

using namespace gse;

extern "C" {

size_t gse_encode_static_scratch_bytes(void) { return kStaticScratchBytes; }

gse_status gse_encode_static(const int32_t* row_ptr, const int32_t* col, const double* val,
                             int32_t n_rows, int32_t n_cols, int64_t nnz, int32_t num_exp,
                             const int16_t* sem_in, gse_matrix* A, void* stream) {
  size_t need = 0;
  gse_status s = gse_encode_workspace(nnz, n_rows, &need);
  if (s != GSE_OK) return s;
  if (need > kStaticScratchBytes)
    return fail(GSE_ERR_NOMEM, "gse_encode_static: scratch needs %zu bytes, the static array holds %zu",
                need, kStaticScratchBytes);
  void* ws = nullptr;
  s = scratch_ptr(&ws);
  if (s != GSE_OK) return s;
  return encode_matrix(row_ptr, col, val, n_rows, n_cols, nnz, num_exp, sem_in, A, ws,
                       kStaticScratchBytes, (hipStream_t)stream);
}

}  // extern "C"

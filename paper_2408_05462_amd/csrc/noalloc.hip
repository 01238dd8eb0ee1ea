// noalloc.hip -- reconstruction that allocates nothing: for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The compact grids of the coarser levels, which chr_reconstruct keeps in a
// caller workspace, live here in one file-scope device array.  Each GPU the
// library runs on holds its own copy of the array until the process ends.
// Host code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and that
// address is what the reconstruction kernels receive.
//
// The reconstruction writes every grid point before reading it, so nothing
// in the array has to start at zero; the array keeps the last call's
// contents.  Calls that overlap on one GPU (two streams, two threads) share
// the array and race.
#include <mutex>
#include <string>

#include "capi_internal.h"

namespace chr {

constexpr size_t kScratchBytes = CHR_STATIC_SCRATCH_BYTES;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

}  // namespace chr

namespace {

using chr::kScratchBytes;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device).
int scratch_ptr(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return chr::api_fail(CHR_E_HIP, "chr_reconstruct_static: no current device");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(chr::scratch));
    if (e != hipSuccess || !p)
      return chr::api_fail(CHR_E_HIP, std::string("chr_reconstruct_static: hipGetSymbolAddress: ") +
                                          hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return CHR_OK;
}

}  // namespace

extern "C" {

int chr_reconstruct_static(const chr_info *info, const void *d_stream, size_t stream_bytes, int level,
                           double error_bound, float *d_out, int32_t *d_status, void *stream) {
  if (!info) return chr::api_fail(CHR_E_INVAL, "NULL argument");
  const size_t need = chr::reconstruct_need(info, level);
  if (need > kScratchBytes)
    return chr::api_fail(CHR_E_NOMEM, "chr_reconstruct_static: this level needs " + std::to_string(need) +
                                          " bytes of coarser-level grids; the static array holds " +
                                          std::to_string(kScratchBytes));
  void *ptr = nullptr;
  const int rc = scratch_ptr(&ptr);
  if (rc) return rc;
  return chr::reconstruct_impl(info, d_stream, stream_bytes, level, error_bound, nullptr, d_out, d_status, ptr,
                               kScratchBytes, stream);
}

}  // extern "C"

// gbs_mps_sample_noalloc: photon-number sampling without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The sampling sweep's buffers (left vectors, their norms, parities, running
// sums and shot partitions) live in one file-scope device array instead of
// stream-ordered allocations.  Each GPU the library runs on holds its own copy
// of the array for the life of the process.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): its
// device address is looked up once per device with hipGetSymbolAddress and
// that pointer is what the kernels receive.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "gbs_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)GBS_SAMPLE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device, with that device current).
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return gbs_fail(GBS_E_DEVICE, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
  }
  if (dev < 0 || dev >= kMaxDevices) return gbs_fail(GBS_E_DEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return gbs_fail(GBS_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return GBS_OK;
}

}  // namespace

extern "C" {

int gbs_mps_sample_noalloc(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, void* stream) {
  // argument errors first: they need no device
  if (!h || shots < 0 || (shots > 0 && !out)) return gbs_sample_in_region(h, shots, seed, out, nullptr, nullptr, 0);
  if (shots == 0) return GBS_OK;
  void* ws = nullptr;
  if (int rc = scratch_ptr(&ws)) return rc;
  return gbs_sample_in_region(h, shots, seed, out, (hipStream_t)stream, ws, kScratchBytes);
}

}  // extern "C"

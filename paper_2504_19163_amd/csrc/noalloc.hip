// bbc_query_irradiance_noalloc: the staged query (include/bbc.h) for callers
// that cannot allocate device memory.  Its work space is `scratch`, a
// file-scope device array of kScratchBytes that every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): the device
// address is looked up once per device with hipGetSymbolAddress and kept.
#include <mutex>
#include <string>

#include "internal.hpp"

namespace bbc {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on device `dev`, resolved with that device
// current on the first call that runs there.
static bbc_status scratch_ptr(int dev, void** out) {
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the no-allocation query's table");
    return BBC_EINVAL;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return BBC_OK;
}

}  // namespace bbc

using namespace bbc;

extern "C" bbc_status bbc_query_irradiance_noalloc(const bbc_bounds* h, const float* points_dev, int64_t n,
                                                   int32_t spp, uint64_t seed, int64_t point_index_base, int32_t mode,
                                                   float* out_E_dev, float* stats_dev, void* stream) {
  if (!h) {
    set_error("null bounds handle");
    return BBC_EINVAL;
  }
  if (n < 0 || n > (int64_t(1) << 31)) {
    set_error("n must be in [0, 2^31]");
    return BBC_EINVAL;
  }
  if (n > 0 && (!points_dev || !out_E_dev)) {
    set_error("null points or output");
    return BBC_EINVAL;
  }
  if (spp < 1) {
    set_error("spp must be >= 1");
    return BBC_EINVAL;
  }
  if (point_index_base < 0) {
    set_error("point_index_base must be >= 0");
    return BBC_EINVAL;
  }
  if ((mode & 15) != BBC_QUERY_STAGED || (mode & ~(15 | BBC_QUERY_EXHAUSTIVE | BBC_QUERY_SAMPLERS)) ||
      ((mode & BBC_QUERY_SAMPLERS) && (mode & BBC_QUERY_EXHAUSTIVE))) {
    set_error("the no-allocation query takes BBC_QUERY_STAGED, optionally with EXHAUSTIVE or one sampler");
    return BBC_EINVAL;
  }
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  int dev = 0;
  BBC_HIP(hipGetDevice(&dev));
  if (dev != b->device) {
    set_error("current device differs from the handle's device");
    return BBC_EINVAL;
  }
  if (n == 0) return BBC_OK;
  void* work = nullptr;
  bbc_status e = scratch_ptr(dev, &work);
  if (e) return e;
  return launch_query_staged_in(b, points_dev, n, spp, seed, point_index_base, mode, out_E_dev, stats_dev, work,
                                kScratchBytes, static_cast<hipStream_t>(stream));
}

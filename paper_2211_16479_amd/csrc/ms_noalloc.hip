// ms_sort_noalloc: the plain sort of ms_sort with its scratch in a fixed
// device array of this library instead of memory the library allocates, for
// callers that cannot allocate (code under graph capture, serving loops).
//
// The array `scratch` is a file-scope __device__ variable: every GPU that the
// library runs on holds its own copy from module load until the process
// ends.  Its name in host code is only a host-side stand-in, so the device
// address is looked up once per device with hipGetSymbolAddress (on the first
// call on that device, with that device current) and only that address is
// passed to kernels.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "ms_internal.hpp"
#include "ms_plan.hpp"

namespace ms {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(MS_NOALLOC_SCRATCH_BYTES);

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> device address of `scratch`

// Device address of `scratch` on the current device (looked up once).
ms_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress (no-alloc scratch)");
    if (p == nullptr) {
      set_error("hipGetSymbolAddress returned NULL for the no-alloc scratch");
      return MS_ERR_HIP;
    }
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return MS_OK;
}

template <class K>
ms_status noalloc_sort(void* d_keys, size_t n, hipStream_t s) {
  const size_t need = plain_temp_bytes<K, NoVal>(n);
  if (need > NOALLOC_SCRATCH_BYTES) {
    set_error("ms_sort_noalloc: n = " + std::to_string(n) + " needs " + std::to_string(need) +
              " bytes of scratch, above the fixed " + std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte array");
    return MS_ERR_INVALID_ARG;
  }
  void* ws = nullptr;
  ms_status st = scratch_address(&ws);
  if (st != MS_OK) return st;
  // the event profiler would create HIP events: keep it out of this call
  ProfSuppress quiet;
  return plain_sort<K, NoVal>(static_cast<K*>(d_keys), nullptr, n, DevCtl{nullptr, nullptr, nullptr}, s, ws);
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" ms_status ms_sort_noalloc(void* d_keys, size_t n, ms_key_type kt, void* stream) {
  if (n > 0 && d_keys == nullptr) {
    set_error("d_keys is NULL with n > 0");
    return MS_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  try {
    switch (kt) {
      case MS_KEY_U32: return n ? noalloc_sort<uint32_t>(d_keys, n, s) : MS_OK;
      case MS_KEY_I32: return n ? noalloc_sort<int32_t>(d_keys, n, s) : MS_OK;
      case MS_KEY_U64: return n ? noalloc_sort<uint64_t>(d_keys, n, s) : MS_OK;
      case MS_KEY_I64: return n ? noalloc_sort<int64_t>(d_keys, n, s) : MS_OK;
    }
    set_error("unknown key type");
    return MS_ERR_UNSUPPORTED;
  } catch (...) {
    set_error("unexpected exception");
    return MS_ERR_INTERNAL;
  }
}

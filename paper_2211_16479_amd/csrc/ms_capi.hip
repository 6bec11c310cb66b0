// C ABI of the library: argument checks, key/value type dispatch, scratch
// management, error reporting and the event profiler.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ms_internal.hpp"
#include "ms_plan.hpp"

namespace ms {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

ms_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? MS_ERR_OUT_OF_MEMORY : MS_ERR_HIP;
}

// --------------------------------------------------------------- workspace
namespace {
struct Buf {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Buf> g_ws;
}  // namespace

ms_status get_workspace(hipStream_t s, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return MS_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  Buf& b = g_ws[{dev, s}];
  if (b.bytes < bytes) {
    if (b.ptr) {
      e = hipFreeAsync(b.ptr, s);
      b.ptr = nullptr;
      b.bytes = 0;
      if (e != hipSuccess) return hip_fail(e, "hipFreeAsync (workspace)");
    }
    const size_t want = align_up(bytes + bytes / 8, size_t(1) << 20);  // a little headroom
    e = hipMallocAsync(&b.ptr, want, s);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return hip_fail(e, "hipMallocAsync (workspace)");
    }
    b.bytes = want;
  }
  *out = b.ptr;
  return MS_OK;
}

// ---------------------------------------------------------------- profiler
namespace {
struct ProfRec {
  int kernel;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pool;
size_t g_prof_used = 0;
}  // namespace

ProfScope::ProfScope(int k, hipStream_t s) : kernel(k), stream(s), slot(-1) {
  if (!g_prof_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_prof_used == g_prof_pool.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    g_prof_pool.push_back({a, b});
  }
  slot = int(g_prof_used++);
  (void)hipEventRecord(g_prof_pool[slot].first, s);
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  (void)hipEventRecord(g_prof_pool[slot].second, stream);
  g_prof_recs.push_back({kernel, g_prof_pool[slot].first, g_prof_pool[slot].second});
}

// ---------------------------------------------------------------- dispatch
static size_t key_bytes(ms_key_type kt) {
  switch (kt) {
    case MS_KEY_U32: case MS_KEY_I32: return 4;
    case MS_KEY_U64: case MS_KEY_I64: return 8;
  }
  return 0;
}

template <class F>
static ms_status with_key_type(ms_key_type kt, F&& f) {
  switch (kt) {
    case MS_KEY_U32: return f(uint32_t{});
    case MS_KEY_I32: return f(int32_t{});
    case MS_KEY_U64: return f(uint64_t{});
    case MS_KEY_I64: return f(int64_t{});
  }
  set_error("unknown key type");
  return MS_ERR_UNSUPPORTED;
}

template <class F>
static ms_status with_val_type(size_t vb, F&& f) {
  switch (vb) {
    case 0: return f(NoVal{});
    case 4: return f(uint32_t{});
    case 8: return f(uint64_t{});
  }
  set_error("value width must be 4 or 8 bytes");
  return MS_ERR_UNSUPPORTED;
}

static ms_status check_common(const void* d_keys, size_t n, ms_key_type kt) {
  if (key_bytes(kt) == 0) {
    set_error("unknown key type");
    return MS_ERR_UNSUPPORTED;
  }
  if (n > 0 && d_keys == nullptr) {
    set_error("d_keys is NULL with n > 0");
    return MS_ERR_INVALID_ARG;
  }
  if (n > (uint64_t(1) << 40)) {
    set_error("n too large");
    return MS_ERR_INVALID_ARG;
  }
  return MS_OK;
}

static ms_status sort_impl(void* d_keys, void* d_vals, size_t n, ms_key_type kt, size_t vb, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  return with_key_type(kt, [&](auto kz) -> ms_status {
    using K = decltype(kz);
    return with_val_type(vb, [&](auto vz) -> ms_status {
      using V = decltype(vz);
      void* ws = nullptr;
      ms_status st = get_workspace(s, plain_temp_bytes<K, V>(n), &ws);
      if (st != MS_OK) return st;
      return plain_sort<K, V>(static_cast<K*>(d_keys), static_cast<V*>(d_vals), n, DevCtl{nullptr, nullptr}, s,
                              ws);
    });
  });
}

}  // namespace ms

using namespace ms;

extern "C" {

int ms_version(void) { return 100; }

const char* ms_status_string(ms_status s) {
  switch (s) {
    case MS_OK: return "ok";
    case MS_ERR_INVALID_ARG: return "invalid argument";
    case MS_ERR_UNSUPPORTED: return "unsupported key type or value width";
    case MS_ERR_OUT_OF_MEMORY: return "out of device memory";
    case MS_ERR_HIP: return "HIP runtime error";
    case MS_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* ms_last_error(void) { return g_last_error.c_str(); }

ms_status ms_sort(void* d_keys, size_t n, ms_key_type kt, void* stream) {
  ms_status st = check_common(d_keys, n, kt);
  if (st != MS_OK || n == 0) return st;
  try {
    return sort_impl(d_keys, nullptr, n, kt, 0, stream);
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return MS_ERR_INTERNAL;
  } catch (...) {
    set_error("unexpected exception");
    return MS_ERR_INTERNAL;
  }
}

ms_status ms_sort_pairs(void* d_keys, void* d_vals, size_t n, ms_key_type kt, size_t val_bytes, void* stream) {
  ms_status st = check_common(d_keys, n, kt);
  if (st != MS_OK) return st;
  if (val_bytes != 4 && val_bytes != 8) {
    set_error("value width must be 4 or 8 bytes");
    return MS_ERR_UNSUPPORTED;
  }
  if (n == 0) return MS_OK;
  if (d_vals == nullptr) {
    set_error("d_vals is NULL with n > 0");
    return MS_ERR_INVALID_ARG;
  }
  if (d_vals == d_keys) {
    set_error("key and value buffers overlap");
    return MS_ERR_INVALID_ARG;
  }
  try {
    return sort_impl(d_keys, d_vals, n, kt, val_bytes, stream);
  } catch (...) {
    set_error("unexpected exception");
    return MS_ERR_INTERNAL;
  }
}

size_t ms_temp_bytes(size_t n, ms_key_type kt, size_t val_bytes) {
  size_t out = 0;
  ms_status st = with_key_type(kt, [&](auto kz) -> ms_status {
    using K = decltype(kz);
    return with_val_type(val_bytes, [&](auto vz) -> ms_status {
      using V = decltype(vz);
      out = plain_temp_bytes<K, V>(n);
      return MS_OK;
    });
  });
  return st == MS_OK ? out : 0;
}

ms_status ms_plan_query(size_t n, ms_key_type kt, size_t val_bytes, int* tile, int* merge_tile, int* passes,
                        int* in_place) {
  int t = 0, mt = 0;
  ms_status st = with_key_type(kt, [&](auto kz) -> ms_status {
    using K = decltype(kz);
    return with_val_type(val_bytes, [&](auto vz) -> ms_status {
      using V = decltype(vz);
      plain_geometry<K, V>(&t, &mt);
      return MS_OK;
    });
  });
  if (st != MS_OK) return st;
  const int p = plan_passes(n, uint64_t(t));
  if (tile) *tile = t;
  if (merge_tile) *merge_tile = mt;
  if (passes) *passes = p;
  if (in_place) *in_place = tile_sort_in_place(p) ? 1 : 0;
  return MS_OK;
}

ms_status ms_release_workspace(void) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto it = g_ws.begin(); it != g_ws.end();) {
    if (it->first.first == dev) {
      if (it->second.ptr) {
        e = hipFree(it->second.ptr);
        if (e != hipSuccess) return hip_fail(e, "hipFree (workspace)");
      }
      it = g_ws.erase(it);
    } else {
      ++it;
    }
  }
  return MS_OK;
}

ms_status ms_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return MS_OK;
}

ms_status ms_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_recs) (void)hipEventSynchronize(r.b);
  g_prof_recs.clear();
  g_prof_used = 0;
  return MS_OK;
}

ms_status ms_profile_read(int kernel, uint64_t* launches, double* total_ms) {
  if (kernel < 0 || kernel >= PK_COUNT) {
    set_error("unknown kernel class");
    return MS_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  uint64_t cnt = 0;
  double tot = 0.0;
  for (auto& r : g_prof_recs) {
    if (r.kernel != kernel) continue;
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms_ = 0.f;
    e = hipEventElapsedTime(&ms_, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    ++cnt;
    tot += ms_;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = tot;
  return MS_OK;
}

}  // extern "C"

// C ABI of the library: argument checks, key/value type dispatch, scratch
// management, error reporting and the event profiler.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "ms_internal.hpp"
#include "ms_plan.hpp"
#include "ms_segmented.hpp"
#include "ms_tuning.hpp"

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

// ------------------------------------------------------------- device info
int device_cu_count() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  cache[dev] = cus;
  return cus;
}

// --------------------------------------------------------- tuning table
namespace {
std::mutex g_tune_mu;
int g_tune[4][3][SEG_MAX_CLASSES] = {};
uint64_t g_tune_gen = 1;
}  // namespace

int* seg_tuning_row(ms_key_type kt, size_t vb) {
  const int k = int(kt);
  const int v = vb == 0 ? 0 : vb == 4 ? 1 : vb == 8 ? 2 : -1;
  if (k < 0 || k > 3 || v < 0) return nullptr;
  return g_tune[k][v];
}
uint64_t seg_tuning_generation() { return g_tune_gen; }
void seg_tuning_bump() { ++g_tune_gen; }

// ---------------------------------------------------------------- profiler
namespace {
struct ProfRec {
  int kernel;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
uint32_t g_prof_mask = ~0u;  // kernel classes that are timed
std::vector<ProfRec> g_prof_recs;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pool;
size_t g_prof_used = 0;
thread_local int g_prof_suppress = 0;
}  // namespace

ProfSuppress::ProfSuppress() { ++g_prof_suppress; }
ProfSuppress::~ProfSuppress() { --g_prof_suppress; }

ProfScope::ProfScope(int k, hipStream_t s) : kernel(k), stream(s), slot(-1) {
  if (!g_prof_on || g_prof_suppress || ((g_prof_mask >> k) & 1u) == 0) return;
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

// Small keys-only sorts are latency-bound (a tile sort and a few dependent
// merge launches over few workgroups).  From the second call with the same
// key type and size on a stream, they replay a cached graph (the caller's
// buffer bound per launch), which saves the per-launch host and queue
// overhead; a size seen once runs directly, so a stream of distinct sizes
// captures nothing.
constexpr uint64_t SMALL_GRAPH_MAX_N = uint64_t(1) << 22;

static bool small_graph_repeat(ms_key_type kt, uint64_t n, hipStream_t s) {
  static std::mutex mu;
  static std::map<std::tuple<int, uint64_t, int, uint64_t>, int> seen;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(mu);
  if (seen.size() > 256) seen.clear();
  int& c = seen[std::make_tuple(dev, reinterpret_cast<uint64_t>(s), int(kt), n)];
  return ++c >= 2;
}

static ms_status sort_impl(void* d_keys, void* d_vals, size_t n, ms_key_type kt, size_t vb, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  return with_key_type(kt, [&](auto kz) -> ms_status {
    using K = decltype(kz);
    if (vb == 0 && n > uint64_t(PlainCfg<K, NoVal>::TILE) && n <= SMALL_GRAPH_MAX_N && small_graph_repeat(kt, n, s)) {
      K* keys = static_cast<K*>(d_keys);
      return cached_graph_launch(
          {5, uint64_t(kt), n}, plain_temp_bytes<K, NoVal>(n), {d_keys},
          [&](void* ws, void* const* io, hipStream_t cs, SegFork) {
            return plain_sort<K, NoVal>(keys, nullptr, n, DevCtl{nullptr, nullptr, nullptr, Rebind{keys, &io[0]}}, cs,
                                        ws);
          },
          s);
    }
    return with_val_type(vb, [&](auto vz) -> ms_status {
      using V = decltype(vz);
      void* ws = nullptr;
      ms_status st = get_workspace(s, plain_temp_bytes<K, V>(n), &ws);
      if (st != MS_OK) return st;
      return plain_sort<K, V>(static_cast<K*>(d_keys), static_cast<V*>(d_vals), n, DevCtl{nullptr, nullptr, nullptr}, s,
                              ws);
    });
  });
}

ms_status plain_sort_capped(void* d_keys, size_t n, ms_key_type kt, uint64_t max_grid, hipStream_t s) {
  return with_key_type(kt, [&](auto kz) -> ms_status {
    using K = decltype(kz);
    void* ws = nullptr;
    ms_status st = get_workspace(s, plain_temp_bytes<K, NoVal>(n), &ws);
    if (st != MS_OK) return st;
    return plain_sort<K, NoVal>(static_cast<K*>(d_keys), nullptr, n, DevCtl{nullptr, nullptr, nullptr}, s, ws,
                                max_grid);
  });
}

template <class F>
static ms_status with_types(ms_key_type kt, size_t vb, F&& f) {
  return with_key_type(kt, [&](auto kz) -> ms_status {
    return with_val_type(vb, [&](auto vz) -> ms_status { return f(kz, vz); });
  });
}

// ------------------------------------------------------------ graph cache
// Pipelines whose launch sequence is fixed on the host are captured once into
// a hipGraph per (device, stream, sizes, options) and replayed with one
// hipGraphLaunch.  A graph owns its scratch; its first 256 bytes are the
// binding block: before every replay a one-thread kernel writes the call's
// buffer pointers there, and the graph's kernels read the caller's buffers
// from it, so new buffers of the same sizes replay the same graph (no
// capture, instantiation or allocation).  An entry is evicted (least
// recently used, at most 8) only after its last launch has completed, by
// waiting on an event recorded after that launch.
namespace {
constexpr size_t BIND_BYTES = 256;
constexpr int BIND_SLOTS = 4;

struct BindArgs {
  void* p[BIND_SLOTS];
};

__global__ void ms_bind_kernel(void** io, BindArgs a) {
  if (threadIdx.x < BIND_SLOTS) io[threadIdx.x] = a.p[threadIdx.x];
}

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  void* ws = nullptr;
  hipEvent_t done = nullptr;  // recorded after the entry's latest launch
  uint64_t last_use = 0;
};
std::mutex g_graph_mu;
std::map<std::vector<uint64_t>, GraphEntry> g_graphs;
struct CaptureStreams {
  hipStream_t main = nullptr, side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};
std::map<int, CaptureStreams> g_capture_streams;
uint64_t g_graph_clock = 0;
uint64_t g_graph_captures = 0;
constexpr size_t GRAPH_CACHE_MAX = 8;

// Destroys an entry whose launches have completed (or never ran).
void drop_graph(GraphEntry& e) {
  if (e.done) (void)hipEventSynchronize(e.done);
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.ws) (void)hipFree(e.ws);
  if (e.done) (void)hipEventDestroy(e.done);
  e.exec = nullptr;
  e.ws = nullptr;
  e.done = nullptr;
}
}  // namespace

size_t graph_bind_bytes() { return BIND_BYTES; }

uint64_t graph_capture_count() {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  return g_graph_captures;
}

ms_status cached_graph_launch(std::vector<uint64_t> key, size_t ws_bytes, const std::vector<void*>& bind,
                              const std::function<ms_status(void* ws, void* const* io, hipStream_t cs, SegFork fork)>&
                                  enqueue,
                              hipStream_t s) {
  if (bind.size() > size_t(BIND_SLOTS)) {
    set_error("too many bound buffers");
    return MS_ERR_INTERNAL;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  key.push_back(uint64_t(dev));
  key.push_back(reinterpret_cast<uint64_t>(s));
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    if (g_graphs.size() >= GRAPH_CACHE_MAX) {
      auto lru = g_graphs.begin();
      for (auto jt = g_graphs.begin(); jt != g_graphs.end(); ++jt)
        if (jt->second.last_use < lru->second.last_use) lru = jt;
      drop_graph(lru->second);  // waits for that entry's last launch only
      g_graphs.erase(lru);
    }
    GraphEntry ent;
    e = hipMalloc(&ent.ws, BIND_BYTES + (ws_bytes ? ws_bytes : 256));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (graph scratch)");
    e = hipEventCreateWithFlags(&ent.done, hipEventDisableTiming);
    if (e != hipSuccess) { drop_graph(ent); return hip_fail(e, "hipEventCreate"); }
    CaptureStreams& cap = g_capture_streams[dev];
    if (!cap.main) {
      e = hipStreamCreateWithFlags(&cap.main, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap.side, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&cap.ev_fork, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&cap.ev_join, hipEventDisableTiming);
      if (e != hipSuccess) { drop_graph(ent); return hip_fail(e, "capture streams"); }
    }
    e = hipStreamBeginCapture(cap.main, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) { drop_graph(ent); return hip_fail(e, "hipStreamBeginCapture"); }
    void* const* io = static_cast<void* const*>(ent.ws);
    ms_status st = enqueue(static_cast<char*>(ent.ws) + BIND_BYTES, io, cap.main,
                           SegFork{cap.side, cap.ev_fork, cap.ev_join});
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap.main, &graph);
    if (st != MS_OK || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      drop_graph(ent);
      return st != MS_OK ? st : hip_fail(e2, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&ent.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) { drop_graph(ent); return hip_fail(e, "hipGraphInstantiate"); }
    ++g_graph_captures;
    it = g_graphs.emplace(key, ent).first;
  }
  GraphEntry& ent = it->second;
  ent.last_use = ++g_graph_clock;
  BindArgs a{};
  for (size_t i = 0; i < bind.size(); ++i) a.p[i] = bind[i];
  ms_bind_kernel<<<1, 64, 0, s>>>(static_cast<void**>(ent.ws), a);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "binding launch");
  e = hipGraphLaunch(ent.exec, s);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  e = hipEventRecord(ent.done, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  return MS_OK;
}

static ms_status seg_run(void* d_keys, void* d_vals, const int64_t* d_off, uint64_t nseg, uint64_t n_total,
                         uint64_t max_len, ms_key_type kt, size_t vb, hipStream_t s) {
  size_t bytes = 0;
  ms_status st = with_types(kt, vb, [&](auto kz, auto vz) -> ms_status {
    bytes = seg_temp_bytes<decltype(kz), decltype(vz)>(nseg, n_total);
    return MS_OK;
  });
  if (st != MS_OK) return st;
  // buffers are bound per launch: the graph depends only on the sizes
  std::vector<uint64_t> key = {1, uint64_t(kt), vb, nseg, n_total, max_len, seg_tuning_generation()};
  const int* tune = seg_tuning_row(kt, vb);
  return cached_graph_launch(
      key, bytes, {d_keys, d_vals, const_cast<int64_t*>(d_off)},
      [&](void* ws, void* const* io, hipStream_t cs, SegFork fork) -> ms_status {
        return with_types(kt, vb, [&](auto kz, auto vz) -> ms_status {
          using K = decltype(kz);
          using V = decltype(vz);
          return seg_enqueue<K, V>(static_cast<K*>(d_keys), static_cast<V*>(d_vals), d_off, nseg, n_total, max_len,
                                   ws, cs, tune, fork, nullptr, io);
        });
      },
      s);
}

static void release_graphs(int dev) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto it = g_graphs.begin(); it != g_graphs.end();) {
    if (it->first[it->first.size() - 2] == uint64_t(dev)) {
      drop_graph(it->second);
      it = g_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace ms

using namespace ms;

extern "C" {

int ms_version(void) { return 101; }

uint64_t ms_graph_captures(void) { return graph_capture_count(); }

ms_status ms_device_errors(uint32_t* flags) {
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  const uint32_t v = dev_errors_plain() | dev_errors_seg32() | dev_errors_seg64();
  if (flags) *flags = v & 0x7FFFFFFFu;
  if (v & 0x80000000u) {
    set_error("reading the device error words failed");
    return MS_ERR_HIP;
  }
  return MS_OK;
}

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

size_t ms_temp_bytes_segmented(size_t num_segments, size_t n_total, ms_key_type kt, size_t val_bytes) {
  size_t out = 0;
  ms_status st = with_types(kt, val_bytes, [&](auto kz, auto vz) -> ms_status {
    out = graph_bind_bytes() + seg_temp_bytes<decltype(kz), decltype(vz)>(num_segments, n_total);
    return MS_OK;
  });
  return st == MS_OK ? out : 0;
}

ms_status ms_plan_query(size_t n, ms_key_type kt, size_t val_bytes, int* tile, int* merge_tile, int* passes,
                        int* in_place, int* hbm_passes, int* merge4_tile) {
  int t = 0, mt = 0, mt4 = 0, fused = 0;
  ms_status st = with_key_type(kt, [&](auto kz) -> ms_status {
    using K = decltype(kz);
    return with_val_type(val_bytes, [&](auto vz) -> ms_status {
      using V = decltype(vz);
      plain_geometry<K, V>(&t, &mt, &mt4, &fused);
      return MS_OK;
    });
  });
  if (st != MS_OK) return st;
  const int p = plan_passes(n, uint64_t(t));
  const int h = plan_hbm_passes(p, fused != 0);
  if (tile) *tile = t;
  if (merge_tile) *merge_tile = mt;
  if (passes) *passes = p;
  if (in_place) *in_place = tile_sort_in_place(h) ? 1 : 0;
  if (hbm_passes) *hbm_passes = h;
  if (merge4_tile) *merge4_tile = fused ? mt4 : 0;
  return MS_OK;
}

ms_status ms_release_workspace(void) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  release_graphs(dev);
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

ms_status ms_segmented_sort(void* d_keys, void* d_vals, const int64_t* d_offsets, size_t num_segments,
                            size_t n_total, size_t max_segment_len, ms_key_type kt, size_t val_bytes,
                            void* stream) {
  ms_status st = check_common(d_keys, n_total, kt);
  if (st != MS_OK) return st;
  if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) {
    set_error("value width must be 0 (keys only), 4 or 8 bytes");
    return MS_ERR_UNSUPPORTED;
  }
  if (num_segments == 0 || n_total == 0) return MS_OK;
  if (d_offsets == nullptr) {
    set_error("d_offsets is NULL with num_segments > 0");
    return MS_ERR_INVALID_ARG;
  }
  if (val_bytes != 0 && d_vals == nullptr) {
    set_error("d_vals is NULL with val_bytes > 0");
    return MS_ERR_INVALID_ARG;
  }
  if (val_bytes != 0 && d_vals == d_keys) {
    set_error("key and value buffers overlap");
    return MS_ERR_INVALID_ARG;
  }
  if (num_segments >= (size_t(1) << 26) || n_total >= (size_t(1) << 32)) {
    set_error("segmented sort supports fewer than 2^26 segments and 2^32 keys per call");
    return MS_ERR_UNSUPPORTED;
  }
  const uint64_t max_len = (max_segment_len == 0 || max_segment_len > n_total) ? n_total : max_segment_len;
  try {
    return seg_run(d_keys, val_bytes ? d_vals : nullptr, d_offsets, num_segments, n_total, max_len, kt, val_bytes,
                   static_cast<hipStream_t>(stream));
  } catch (...) {
    set_error("unexpected exception");
    return MS_ERR_INTERNAL;
  }
}

ms_status ms_seg_num_classes(ms_key_type kt, size_t val_bytes, int* num_classes) {
  int nc = 0;
  ms_status st = with_types(kt, val_bytes, [&](auto kz, auto vz) -> ms_status {
    nc = seg_num_classes<decltype(kz), decltype(vz)>();
    return MS_OK;
  });
  if (st == MS_OK && num_classes) *num_classes = nc;
  return st;
}

ms_status ms_seg_class_info(ms_key_type kt, size_t val_bytes, int cls, uint32_t* max_len, int* num_candidates) {
  int nc = 0;
  ms_status st = ms_seg_num_classes(kt, val_bytes, &nc);
  if (st != MS_OK) return st;
  if (cls < 0 || cls >= nc) {
    set_error("size class out of range");
    return MS_ERR_INVALID_ARG;
  }
  uint32_t b = 0;
  int c = 0;
  with_types(kt, val_bytes, [&](auto kz, auto vz) -> ms_status {
    seg_class_info<decltype(kz), decltype(vz)>(cls, &b, &c);
    return MS_OK;
  });
  if (max_len) *max_len = b;
  if (num_candidates) *num_candidates = c;
  return MS_OK;
}

ms_status ms_seg_candidate(ms_key_type kt, size_t val_bytes, int cls, int idx, int* wg, int* ipt) {
  int nc = 0;
  ms_status st = ms_seg_class_info(kt, val_bytes, cls, nullptr, &nc);
  if (st != MS_OK) return st;
  if (idx < 0 || idx >= nc) {
    set_error("candidate index out of range");
    return MS_ERR_INVALID_ARG;
  }
  int w = 0, p = 0;
  with_types(kt, val_bytes, [&](auto kz, auto vz) -> ms_status {
    seg_candidate<decltype(kz), decltype(vz)>(cls, idx, &w, &p);
    return MS_OK;
  });
  if (wg) *wg = w;
  if (ipt) *ipt = p;
  return MS_OK;
}

ms_status ms_tuning_set(ms_key_type kt, size_t val_bytes, int cls, int wg, int ipt) {
  int nc = 0;
  ms_status st = ms_seg_class_info(kt, val_bytes, cls, nullptr, &nc);
  if (st != MS_OK) return st;
  for (int i = 0; i < nc; ++i) {
    int w = 0, p = 0;
    ms_seg_candidate(kt, val_bytes, cls, i, &w, &p);
    if (w == wg && p == ipt) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      seg_tuning_row(kt, val_bytes)[cls] = i;
      seg_tuning_bump();
      return MS_OK;
    }
  }
  set_error("no compiled variant with that workgroup size and items per thread");
  return MS_ERR_UNSUPPORTED;
}

ms_status ms_tuning_get(ms_key_type kt, size_t val_bytes, int cls, int* wg, int* ipt) {
  int nc = 0;
  ms_status st = ms_seg_class_info(kt, val_bytes, cls, nullptr, &nc);
  if (st != MS_OK) return st;
  int idx = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    idx = seg_tuning_row(kt, val_bytes)[cls];
  }
  return ms_seg_candidate(kt, val_bytes, cls, idx, wg, ipt);
}

ms_status ms_tuning_load(const char* path, const char* arch, int* applied) {
  if (applied) *applied = 0;
  if (!path) {
    set_error("path is NULL");
    return MS_ERR_INVALID_ARG;
  }
  std::string want;
  if (arch) {
    want = arch;
  } else {
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device properties");
    want = prop.gcnArchName;
    want = want.substr(0, want.find(':'));
  }
  FILE* f = std::fopen(path, "r");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return MS_ERR_INVALID_ARG;
  }
  char line[512];
  int n = 0;
  int lineno = 0;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    char a[64], k[16];
    size_t vb = 0;
    int cls = 0, wg = 0, ipt = 0;
    if (line[0] == '#' || line[0] == '\n') continue;
    if (std::sscanf(line, "%63s %15s %zu %d %d %d", a, k, &vb, &cls, &wg, &ipt) != 6) {
      std::fclose(f);
      set_error("malformed tuning line " + std::to_string(lineno));
      return MS_ERR_INVALID_ARG;
    }
    if (want != a) continue;
    ms_key_type kt;
    if (!std::strcmp(k, "u32")) kt = MS_KEY_U32;
    else if (!std::strcmp(k, "i32")) kt = MS_KEY_I32;
    else if (!std::strcmp(k, "u64")) kt = MS_KEY_U64;
    else if (!std::strcmp(k, "i64")) kt = MS_KEY_I64;
    else {
      std::fclose(f);
      set_error("unknown key type on tuning line " + std::to_string(lineno));
      return MS_ERR_INVALID_ARG;
    }
    ms_status st = ms_tuning_set(kt, vb, cls, wg, ipt);
    if (st != MS_OK) {
      std::fclose(f);
      return st;
    }
    ++n;
  }
  std::fclose(f);
  if (applied) *applied = n;
  return MS_OK;
}

ms_status ms_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return MS_OK;
}

ms_status ms_profile_select(uint32_t class_mask) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_mask = class_mask;
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

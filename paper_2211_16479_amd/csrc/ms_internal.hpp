// Library-internal declarations shared by the C-ABI and the launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/msort.h"
#include "ms_common.hpp"

namespace ms {

// Kernel classes timed by the event profiler.
enum ProfKernel {
  PK_BLOCK_SORT = 0,
  PK_PARTITION = 1,
  PK_MERGE = 2,
  PK_SEG_CLASSIFY = 3,
  PK_SEG_SMALL = 4,
  PK_SEG_LARGE = 5,
  PK_LEARN_TRAIN = 6,
  PK_LEARN_HIST = 7,
  PK_LEARN_SCATTER = 8,
  PK_LEARN_BUCKET = 9,
  PK_LEARN_OTHER = 10,
  PK_PARTITION4 = 11,
  PK_MERGE4 = 12,
  PK_LEARN_HIST2 = 13,
  PK_LEARN_SCATTER2 = 14,
  PK_PARTITION_SAMPLES = 15,
  PK_LEARN_EST = 16,
  PK_COUNT = 17
};

// Records a start/stop event pair around a launch when profiling is on.
struct ProfScope {
  ProfScope(int kernel, hipStream_t s);
  ~ProfScope();
  int kernel;
  hipStream_t stream;
  int slot;
};

// While one of these lives on a thread, ProfScope records nothing there
// (entry points that must not create HIP objects).
struct ProfSuppress {
  ProfSuppress();
  ~ProfSuppress();
};

void set_error(const std::string& msg);
ms_status hip_fail(hipError_t e, const char* what);

// Scratch memory owned by the library, one buffer per (device, stream),
// grown on demand in stream order.
ms_status get_workspace(hipStream_t s, size_t bytes, void** out);

// Plain merge sort of n keys (and values) already resident on the device.
// ctl may carry a device-side count (n is then an upper bound) and a gate.
// max_grid > 0 caps every launch's grid (workgroups then loop over tiles);
// gated uses pass a small cap so that skipped stages cost little.
template <class K, class V>
ms_status plain_sort(K* keys, V* vals, uint64_t n, DevCtl ctl, hipStream_t s, void* ws, uint64_t max_grid = 0);
template <class K, class V>
size_t plain_temp_bytes(uint64_t n);
// Keys-only plain sort with every launch's grid capped at max_grid (0: none),
// scratch from the per-stream workspace.
ms_status plain_sort_capped(void* d_keys, size_t n, ms_key_type kt, uint64_t max_grid, hipStream_t s);
template <class K, class V>
void plain_geometry(int* tile, int* merge_tile, int* merge4_tile, int* fused);
// One merge of src[0, split) with src[split, n) into dst (split on the device),
// as the plain sort's partition + merge kernels; part needs ceil(n/merge tile).
template <class K, class V>
ms_status merge_two_runs(const K* src, K* dst, uint64_t n, DevCtl ctl, int64_t* part, hipStream_t s,
                         uint64_t max_grid = 0);

// Segmented sort (ms_seg_launch.hpp): enqueue the whole pipeline on s.  If
// fork.side is set, the small classes go to that stream between a fork and a
// join event (used while capturing, so the graph gets two branches).
struct SegFork {
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
};
// keys_sel: if non-null the small classes sort *keys_sel (chosen on the
// device); io: if non-null the caller's buffers are read from io[0..2]
// (keys, values, offsets) at run time (graph replays on new buffers).
template <class K, class V>
ms_status seg_enqueue(K* keys, V* vals, const int64_t* off, uint64_t nseg, uint64_t n_total, uint64_t max_len,
                      void* ws, hipStream_t s, const int* tune, SegFork fork, void* const* keys_sel = nullptr,
                      void* const* io = nullptr);
template <class K, class V>
size_t seg_temp_bytes(uint64_t nseg, uint64_t n_total);
template <class K, class V>
int seg_num_classes();
template <class K, class V>
void seg_class_info(int cls, uint32_t* bound, int* ncand);
template <class K, class V>
void seg_candidate(int cls, int idx, int* wg, int* ipt);

int device_cu_count();

// Capture `enqueue` once per key into a hipGraph that owns ws_bytes of
// scratch, then launch it on s (cache of 8 graphs, least recently used out).
// `bind` (at most 4 pointers) is written to the graph's binding block io
// before every launch; enqueue must make the graph read the caller's
// buffers from io, not from the pointers it was captured with.
ms_status cached_graph_launch(std::vector<uint64_t> key, size_t ws_bytes, const std::vector<void*>& bind,
                              const std::function<ms_status(void* ws, void* const* io, hipStream_t cs, SegFork fork)>&
                                  enqueue,
                              hipStream_t s);
// Read and clear the device error words of the translation units whose
// kernels can raise them (see g_dev_errors).
unsigned int dev_errors_plain();
unsigned int dev_errors_seg32();
unsigned int dev_errors_seg64();

// Graphs captured so far in this process (all devices).
uint64_t graph_capture_count();
// Bytes of a cached graph's scratch taken by its binding block.
size_t graph_bind_bytes();

}  // namespace ms

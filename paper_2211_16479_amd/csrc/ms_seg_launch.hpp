// Host side of the segmented sort: scratch layout, per-class variant choice
// (autotuned), the launch sequence, and its capture into one hipGraph.
#pragma once
#include <algorithm>

#include "ms_internal.hpp"
#include "ms_plan.hpp"
#include "ms_segmented.hpp"
#include "ms_tuning.hpp"

namespace ms {

template <class F>
static hipError_t seg_allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(bytes));
}

int device_cu_count();

template <class K, class V, int WG, int IPT>
static hipError_t launch_small(K* keys, V* vals, const int64_t* off, SegState st, int cls, uint64_t nseg,
                               hipStream_t s) {
  constexpr int PAD = PlainCfg<K, V>::SEG_PAD;
  using TS = TileSort<K, V, WG, IPT, PAD>;
  static const hipError_t ok = seg_allow_lds(&seg_small_kernel<K, V, WG, IPT, PAD>, TS::LDS_BYTES);
  if (ok != hipSuccess) return ok;
  const uint64_t per_cu = std::max(1, 2048 / WG);
  const uint64_t slots = uint64_t(device_cu_count()) * per_cu;
  // segments per work grab: enough that every resident workgroup gets a few
  // grabs when the whole batch sits in this class
  const uint32_t chunk = uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(64, nseg / (slots * 4))));
  const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(nseg, chunk), slots));
  seg_small_kernel<K, V, WG, IPT, PAD><<<dim3(unsigned(grid)), dim3(WG), TS::LDS_BYTES, s>>>(keys, vals, off, st, cls,
                                                                                            nseg, chunk);
  return hipGetLastError();
}

// Candidate (WG, IPT) shapes per class bound; index 0 is the default.
// Keys-only families and 32-bit keys with values get every candidate;
// 64-bit keys with values the default only, to bound compile time.
template <class K, class V>
struct SegCands {
  static constexpr bool FULL = !HasVal<V>::value || sizeof(K) == 4;
  static constexpr int MAXC = 3;
  // {wg, ipt} per class bound, default first
  static int table(uint32_t bound, int (*t)[2]) {
    switch (bound) {
      case 256: t[0][0] = 64; t[0][1] = 4; t[1][0] = 128; t[1][1] = 2; return 2;
      case 512: t[0][0] = 64; t[0][1] = 8; t[1][0] = 128; t[1][1] = 4; return 2;
      case 1024: t[0][0] = 128; t[0][1] = 8; t[1][0] = 64; t[1][1] = 16; t[2][0] = 256; t[2][1] = 4; return 3;
      case 2048: t[0][0] = 256; t[0][1] = 8; t[1][0] = 128; t[1][1] = 16; return 2;
      case 4096: t[0][0] = 256; t[0][1] = 16; t[1][0] = 512; t[1][1] = 8; t[2][0] = 1024; t[2][1] = 4; return 3;
      case 8192: t[0][0] = 512; t[0][1] = 16; t[1][0] = 1024; t[1][1] = 8; return 2;
      case 16384: t[0][0] = 1024; t[0][1] = 16; t[1][0] = 512; t[1][1] = 32; return 2;
    }
    return 0;
  }
  static int count(uint32_t bound) {
    int t[MAXC][2];
    const int c = table(bound, t);
    return FULL ? c : (c ? 1 : 0);
  }
  static void shape(uint32_t bound, int idx, int* wg, int* ipt) {
    int t[MAXC][2];
    table(bound, t);
    *wg = t[idx][0];
    *ipt = t[idx][1];
  }
  static hipError_t launch(uint32_t bound, int idx, K* keys, V* vals, const int64_t* off, SegState st, int cls,
                           uint64_t nseg, hipStream_t s) {
    switch (bound) {
      case 256:
        if constexpr (FULL) if (idx == 1) return launch_small<K, V, 128, 2>(keys, vals, off, st, cls, nseg, s);
        return launch_small<K, V, 64, 4>(keys, vals, off, st, cls, nseg, s);
      case 512:
        if constexpr (FULL) if (idx == 1) return launch_small<K, V, 128, 4>(keys, vals, off, st, cls, nseg, s);
        return launch_small<K, V, 64, 8>(keys, vals, off, st, cls, nseg, s);
      case 1024:
        if constexpr (FULL) {
          if (idx == 1) return launch_small<K, V, 64, 16>(keys, vals, off, st, cls, nseg, s);
          if (idx == 2) return launch_small<K, V, 256, 4>(keys, vals, off, st, cls, nseg, s);
        }
        return launch_small<K, V, 128, 8>(keys, vals, off, st, cls, nseg, s);
      case 2048:
        if constexpr (FULL) if (idx == 1) return launch_small<K, V, 128, 16>(keys, vals, off, st, cls, nseg, s);
        return launch_small<K, V, 256, 8>(keys, vals, off, st, cls, nseg, s);
      case 4096:
        if constexpr (FULL) {
          if (idx == 1) return launch_small<K, V, 512, 8>(keys, vals, off, st, cls, nseg, s);
          if (idx == 2) return launch_small<K, V, 1024, 4>(keys, vals, off, st, cls, nseg, s);
        }
        return launch_small<K, V, 256, 16>(keys, vals, off, st, cls, nseg, s);
      case 8192:
        if constexpr (sizeof(K) == 4 && !HasVal<V>::value) {
          if (idx == 1) return launch_small<K, V, 1024, 8>(keys, vals, off, st, cls, nseg, s);
          return launch_small<K, V, 512, 16>(keys, vals, off, st, cls, nseg, s);
        }
        break;
      case 16384:
        if constexpr (sizeof(K) == 4 && !HasVal<V>::value) {
          if (idx == 1) return launch_small<K, V, 512, 32>(keys, vals, off, st, cls, nseg, s);
          return launch_small<K, V, 1024, 16>(keys, vals, off, st, cls, nseg, s);
        }
        break;
    }
    return hipErrorInvalidValue;
  }
};

struct SegLayout {
  size_t cls_count, cls_work, large_ctr, max_steps, queues, large_seg, large_mbase, desc, part, part4, head, tail, tk, tv,
      bytes;
  uint64_t mt_cap;
};

template <class K, class V>
SegLayout seg_layout(uint64_t nseg, uint64_t n_total) {
  using S = SegCfg<K, V>;
  const size_t vb = HasVal<V>::value ? sizeof(typename std::conditional<HasVal<V>::value, V, int>::type) : 0;
  SegLayout L{};
  L.mt_cap = (n_total / S::TILE + nseg + 1) * S::C;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes, 256); return at; };
  L.cls_count = take(sizeof(uint32_t) * SEG_MAX_CLASSES);
  L.cls_work = take(sizeof(uint32_t) * SEG_MAX_CLASSES);
  L.large_ctr = take(sizeof(unsigned long long));
  L.max_steps = take(sizeof(uint32_t));
  L.queues = take(sizeof(int32_t) * SEG_MAX_CLASSES * nseg);
  L.large_seg = take(sizeof(int32_t) * nseg);
  L.large_mbase = take(sizeof(int64_t) * nseg);
  L.desc = take(sizeof(int4) * L.mt_cap);
  L.part = take(sizeof(int64_t) * L.mt_cap);
  L.part4 = take(sizeof(int64_t) * 4 * L.mt_cap);
  L.head = take(sizeof(K) * L.mt_cap);
  L.tail = take(sizeof(K) * L.mt_cap);
  L.tk = take(sizeof(K) * n_total);
  L.tv = take(vb * n_total);
  L.bytes = o;
  return L;
}

// Enqueue the whole segmented pipeline on stream s (possibly capturing).
// max_len is the caller's bound on segment lengths: merge steps up to that
// bound are launched over every reserved merge tile; the steps that longer
// segments (up to n_total) would need are launched too, with a small grid,
// and return at once unless classify found such a segment, so a bound that
// is too small costs time, never correctness.
template <class K, class V>
ms_status seg_enqueue(K* keys, V* vals, const int64_t* off, uint64_t nseg, uint64_t n_total, uint64_t max_len,
                      void* ws, hipStream_t s, const int* tune, SegFork fork, void* const* keys_sel,
                      void* const* io) {
  using S = SegCfg<K, V>;
  using P = PlainCfg<K, V>;
  const SegLayout L = seg_layout<K, V>(nseg, n_total);
  char* w = static_cast<char*>(ws);
  SegState st;
  st.cls_count = reinterpret_cast<uint32_t*>(w + L.cls_count);
  st.cls_work = reinterpret_cast<uint32_t*>(w + L.cls_work);
  st.large_ctr = reinterpret_cast<unsigned long long*>(w + L.large_ctr);
  st.queues = reinterpret_cast<int32_t*>(w + L.queues);
  st.large_seg = reinterpret_cast<int32_t*>(w + L.large_seg);
  st.large_mbase = reinterpret_cast<int64_t*>(w + L.large_mbase);
  st.desc = reinterpret_cast<int4*>(w + L.desc);
  st.part = reinterpret_cast<int64_t*>(w + L.part);
  st.part4 = reinterpret_cast<int64_t*>(w + L.part4);
  st.head = w + L.head;
  st.tail = w + L.tail;
  st.keys_sel = keys_sel;
  st.io = io;
  st.max_steps = reinterpret_cast<uint32_t*>(w + L.max_steps);
  K* tk = reinterpret_cast<K*>(w + L.tk);
  V* tv = reinterpret_cast<V*>(w + L.tv);
  const uint64_t cus = uint64_t(device_cu_count());

  seg_init_kernel<<<1, 64, 0, s>>>(st);
  seg_classify_kernel<K, V><<<dim3(unsigned(ceil_div(nseg, 256 * SEG_CLASSIFY_PER))), dim3(256), 0, s>>>(off, nseg,
                                                                                                        st);
  seg_owner_kernel<K, V><<<dim3(unsigned(std::min<uint64_t>(nseg, cus * 4))), dim3(256), 0, s>>>(off, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "segment classification launch");
  // small classes run on a side branch (fork/join through events) so that
  // they overlap the large-segment passes
  hipStream_t side = fork.side ? fork.side : s;
  if (fork.side) {
    e = hipEventRecord(fork.ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork.ev_fork, 0);
    if (e != hipSuccess) return hip_fail(e, "graph fork");
  }
  for (int c = 0; c < S::NCLS; ++c) {
    e = SegCands<K, V>::launch(S::cls_max(c), tune[c], keys, vals, off, st, c, nseg, side);
    if (e != hipSuccess) return hip_fail(e, "small-segment sort launch");
  }
  // segments longer than the last small class take the large path (a tile
  // sort, then merge passes when they span several tiles)
  if (n_total > uint64_t(S::cls_max(S::NCLS - 1))) {
    using TS = TileSort<K, V, S::LWG, S::LIPT, P::SEG_LPAD>;
    using MT = MergeTile<K, V, P::MG_WG, P::MG_IPT, P::MG_PAD>;
    using M4 = Merge4Tile<K, V, P::MG_WG, P::MG_IPT, P::M4_PAD, P::M4_REUSE>;
    static const hipError_t lds_ok = [] {
      hipError_t a = seg_allow_lds(&seg_large_tile_kernel<K, V, S::LWG, S::LIPT, P::SEG_LPAD>, TS::LDS_BYTES);
      hipError_t b = seg_allow_lds(&seg_merge_kernel<K, V, P::MG_WG, P::MG_IPT, P::MG_PAD>, MT::LDS_BYTES);
      hipError_t c = seg_allow_lds(&seg_merge4_kernel<K, V, P::MG_WG, P::MG_IPT, P::M4_PAD, P::M4_REUSE>,
                                   M4::LDS_BYTES);
      return a != hipSuccess ? a : (b != hipSuccess ? b : c);
    }();
    if (lds_ok != hipSuccess) return hip_fail(lds_ok, "LDS size attribute");
    // one workgroup per reserved (merge) tile up to the host-side bound
    const uint64_t tiles_cap = L.mt_cap / S::C;
    seg_large_tile_kernel<K, V, S::LWG, S::LIPT, P::SEG_LPAD>
        <<<dim3(unsigned(tiles_cap)), dim3(S::LWG), TS::LDS_BYTES, s>>>(keys, vals, tk, tv, st);
    const int steps_hint = max_len > uint64_t(S::cls_max(S::NCLS - 1))
                               ? plan_hbm_passes(plan_passes(max_len, S::TILE), true) : 0;
    const int steps_all = plan_hbm_passes(plan_passes(n_total, S::TILE), true);
    const uint64_t small_grid = cus * 2;
    for (int j = 0; j < steps_all; ++j) {
      const bool full = j < steps_hint;
      const uint64_t gm = full ? L.mt_cap : std::min<uint64_t>(L.mt_cap, small_grid);
      const uint64_t gp = full ? ceil_div(L.mt_cap, 256) : std::min<uint64_t>(ceil_div(L.mt_cap, 256), small_grid);
      seg_partition_kernel<K, V><<<dim3(unsigned(gp)), dim3(256), 0, s>>>(keys, tk, st, j);
      seg_partition4_kernel<K, V><<<dim3(unsigned(gp)), dim3(256), 0, s>>>(keys, tk, st, j);
      if (j == 0)  // two-run steps occur only first
        seg_merge_kernel<K, V, P::MG_WG, P::MG_IPT, P::MG_PAD>
            <<<dim3(unsigned(gm)), dim3(P::MG_WG), MT::LDS_BYTES, s>>>(keys, vals, tk, tv, st, j);
      seg_merge4_kernel<K, V, P::MG_WG, P::MG_IPT, P::M4_PAD, P::M4_REUSE>
          <<<dim3(unsigned(gm)), dim3(P::MG_WG), M4::LDS_BYTES, s>>>(keys, vals, tk, tv, st, j);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "large-segment launch");
  }
  if (fork.side) {
    e = hipEventRecord(fork.ev_join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, fork.ev_join, 0);
    if (e != hipSuccess) return hip_fail(e, "graph join");
  }
  return MS_OK;
}

template <class K, class V>
size_t seg_temp_bytes(uint64_t nseg, uint64_t n_total) {
  return seg_layout<K, V>(nseg, n_total).bytes;
}

template <class K, class V>
int seg_num_classes() {
  return SegCfg<K, V>::NCLS;
}

template <class K, class V>
void seg_class_info(int cls, uint32_t* bound, int* ncand) {
  using S = SegCfg<K, V>;
  *bound = S::cls_max(cls);
  *ncand = SegCands<K, V>::count(*bound);
}

template <class K, class V>
void seg_candidate(int cls, int idx, int* wg, int* ipt) {
  SegCands<K, V>::shape(SegCfg<K, V>::cls_max(cls), idx, wg, ipt);
}

#define MS_SEG_INSTANTIATE(K, V)                                                                              \
  template ms_status seg_enqueue<K, V>(K*, V*, const int64_t*, uint64_t, uint64_t, uint64_t, void*, hipStream_t, \
                                       const int*, SegFork, void* const*, void* const*);                      \
  template size_t seg_temp_bytes<K, V>(uint64_t, uint64_t);                                                   \
  template int seg_num_classes<K, V>();                                                                       \
  template void seg_class_info<K, V>(int, uint32_t*, int*);                                                   \
  template void seg_candidate<K, V>(int, int, int*, int*);

}  // namespace ms

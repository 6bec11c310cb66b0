// Plain merge sort launcher: tile sort, then merge-path passes with
// ping-pong buffers (see ms_plan.hpp for the pass count and parity); pairs
// of tree levels run as one fused pass.
#include <algorithm>
#include <type_traits>

#include "ms_adaptive.hpp"
#include "ms_block_sort.hpp"
#include "ms_internal.hpp"
#include "ms_merge.hpp"
#include "ms_plan.hpp"
#include "ms_plain_cfg.hpp"

namespace ms {

// Lets a kernel take more than the default dynamic LDS (once per kernel).
template <class F>
static hipError_t allow_lds(F* kernel, size_t bytes) {
  if (bytes <= 48 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(bytes));
}

template <class K, class V>
void plain_geometry(int* tile, int* merge_tile, int* merge4_tile, int* fused) {
  *tile = PlainCfg<K, V>::TILE;
  *merge_tile = PlainCfg<K, V>::MTILE;
  *merge4_tile = PlainCfg<K, V>::M4TILE;
  *fused = PlainCfg<K, V>::FUSED ? 1 : 0;
}

// Lanes per partition search.  With few searches, groups of G lanes fill the
// chip and each search takes fewer dependent rounds; with many, one lane
// each, since a group multiplies the scattered line fetches that bound the
// kernels there.  Measured best on MI355X: the largest G of 1, 4, 16, 64
// that keeps a launch at or below 2^16 lanes (2^20 u32 keys: four-way
// partition 60 -> 15 us; 2^27: one lane).
static int search_group(uint64_t searches) {
  const uint64_t lanes = uint64_t(1) << 16;
  return searches * 64 <= lanes ? 64 : searches * 16 <= lanes ? 16 : searches * 4 <= lanes ? 4 : 1;
}
template <class F>
static void with_search_group(int g, F&& f) {
  switch (g) {
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

template <class K, class V>
size_t plain_temp_bytes(uint64_t n) {
  using C = PlainCfg<K, V>;
  const int P = plan_passes(n, C::TILE);
  const size_t vb = C::PAIRS ? sizeof(typename std::conditional<C::PAIRS, V, int>::type) : 0;
  return plain_layout(n, sizeof(K), vb, C::TILE, C::MTILE, C::M4TILE, P, C::FUSED).bytes;
}

template <class K, class V>
ms_status plain_sort(K* keys, V* vals, uint64_t n, DevCtl ctl, hipStream_t s, void* ws, uint64_t max_grid) {
  using C = PlainCfg<K, V>;
  using BS = TileSort<K, V, C::BS_WG, C::BS_IPT, C::BS_PAD>;
  using MT = MergeTile<K, V, C::MG_WG, C::MG_IPT, C::MG_PAD>;
  using M4 = Merge4Tile<K, V, C::M4_WG, C::M4_IPT, C::M4_PAD, C::M4_REUSE>;
  if (n == 0) return MS_OK;
  const int P = plan_passes(n, C::TILE);
  const int H = plan_hbm_passes(P, C::FUSED);
  const size_t vb = C::PAIRS ? sizeof(typename std::conditional<C::PAIRS, V, int>::type) : 0;
  const PlainLayout L = plain_layout(n, sizeof(K), vb, C::TILE, C::MTILE, C::M4TILE, P, C::FUSED);
  char* w = static_cast<char*>(ws);
  K* tk = P ? reinterpret_cast<K*>(w + L.keys_off) : nullptr;
  V* tv = (P && C::PAIRS) ? reinterpret_cast<V*>(w + L.vals_off) : nullptr;
  int64_t* part = P ? reinterpret_cast<int64_t*>(w + L.part_off) : nullptr;
  int64_t* part4 = P ? reinterpret_cast<int64_t*>(w + L.part4_off) : nullptr;
  K* head = P ? reinterpret_cast<K*>(w + L.head_off) : nullptr;
  K* tail = P ? reinterpret_cast<K*>(w + L.tail_off) : nullptr;
  int* ctlw = P ? reinterpret_cast<int*>(w + L.ctl_off) : nullptr;
  // run-adaptive pass skipping (ms_adaptive.hpp) for plain calls; sorts that
  // are already gated or sized on the device keep every pass
  const bool adaptive = P > 0 && !ctl.gate && !ctl.n_dev && !ctl.split_dev && !ctl.keys.cur;

  K* cur_k = tile_sort_in_place(H) ? keys : tk;
  V* cur_v = tile_sort_in_place(H) ? vals : tv;
  const uint64_t tiles = ceil_div(n, C::TILE);
  static const hipError_t lds_ok = [] {
    hipError_t a = allow_lds(&block_sort_kernel<K, V, C::BS_WG, C::BS_IPT, C::BS_PAD>, BS::LDS_BYTES);
    hipError_t b = allow_lds(&merge_kernel<K, V, C::MG_WG, C::MG_IPT, C::MG_PAD>, MT::LDS_BYTES);
    hipError_t c = allow_lds(&merge4_kernel<K, V, C::M4_WG, C::M4_IPT, C::M4_PAD, C::M4_REUSE>, M4::LDS_BYTES);
    return a != hipSuccess ? a : (b != hipSuccess ? b : c);
  }();
  if (lds_ok != hipSuccess) return hip_fail(lds_ok, "LDS size attribute");
  const uint64_t cap = max_grid ? max_grid : ~uint64_t(0);
  {
    ProfScope ps(PK_BLOCK_SORT, s);
    block_sort_kernel<K, V, C::BS_WG, C::BS_IPT, C::BS_PAD>
        <<<dim3(unsigned(std::min(tiles, cap))), dim3(C::BS_WG), BS::LDS_BYTES, s>>>(keys, vals, cur_k, cur_v, n,
                                                                                     ctl);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "tile sort launch");
  if (adaptive) {
    const PassPlan pp = plan_pass_levels(P, C::FUSED);
    const uint64_t groups = ceil_div(ceil_div(n, C::TILE), RUN_GROUP);
    K* runs = reinterpret_cast<K*>(w + L.runs_off);
    uint32_t* gmask = reinterpret_cast<uint32_t*>(runs + 4 * groups);
    run_bounds_kernel<K><<<dim3(unsigned(groups)), dim3(RUN_GROUP), 0, s>>>(
        keys, tk, n, uint32_t(C::TILE), P, pp.start_in_caller, runs, runs + groups, gmask);
    run_decide_kernel<K><<<1, 1024, 0, s>>>(groups, pp, runs, runs + groups, runs + 2 * groups, runs + 3 * groups,
                                            gmask, ctlw);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "run check launch");
  }
  // splits at every Tm outputs of each pair; with_keys: the keys around them too
  auto partition = [&](const DevCtl& pc, uint64_t W, uint32_t Tm, bool with_keys) {
    const uint64_t nt = ceil_div(n, Tm);
    ProfScope ps(with_keys ? PK_PARTITION_SAMPLES : PK_PARTITION, s);
    with_search_group(search_group(nt), [&](auto gc) {
      constexpr int G = decltype(gc)::value;
      partition_kernel<K, G><<<dim3(unsigned(std::min(ceil_div(nt * G, 256), cap))), dim3(256), 0, s>>>(
          cur_k, n, pc, W, Tm, nt, part, with_keys ? head : nullptr, with_keys ? tail : nullptr);
    });
  };
  // levels p (width W = T * 2^p): an odd level count starts with one two-run
  // pass, then every fused pass takes two levels
  int p = 0, h = 0;
  while (p < P) {
    const uint64_t W = uint64_t(C::TILE) << p;
    K* nxt_k = (cur_k == keys) ? tk : keys;
    V* nxt_v = (cur_k == keys) ? tv : vals;
    const bool fuse = C::FUSED && (P - p) % 2 == 0;
    DevCtl pc = ctl;  // this pass's controls: with run-adaptive skipping, a run flag and a swap flag
    if (adaptive) {
      pc.gate = ctlw + ctl_run(h);
      pc.swap_bit = 1;
      pc.other = nxt_k;
    }
    if (fuse) {
      const uint64_t mt4 = ceil_div(n, C::M4TILE);
      partition(pc, W, C::M4TILE, true);
      {
        ProfScope ps(PK_PARTITION4, s);
        with_search_group(search_group(mt4), [&](auto gc) {
          constexpr int G = decltype(gc)::value;
          partition4_kernel<K, G><<<dim3(unsigned(std::min(ceil_div(mt4 * G, 256), cap))), dim3(256), 0, s>>>(
              cur_k, n, pc, W, C::M4TILE, mt4, part, head, tail, part4);
        });
      }
      {
        ProfScope ps(PK_MERGE4, s);
        merge4_kernel<K, V, C::M4_WG, C::M4_IPT, C::M4_PAD, C::M4_REUSE>
            <<<dim3(unsigned(std::min(mt4, cap))), dim3(C::M4_WG), M4::LDS_BYTES, s>>>(cur_k, cur_v, nxt_k, nxt_v, n,
                                                                                     pc, W, part4);
      }
      p += 2;
    } else {
      const uint64_t mtiles = ceil_div(n, C::MTILE);
      partition(pc, W, C::MTILE, false);
      {
        ProfScope ps(PK_MERGE, s);
        merge_kernel<K, V, C::MG_WG, C::MG_IPT, C::MG_PAD>
            <<<dim3(unsigned(std::min(mtiles, cap))), dim3(C::MG_WG), MT::LDS_BYTES, s>>>(cur_k, cur_v, nxt_k, nxt_v,
                                                                                       n, pc, W, part);
      }
      p += 1;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "merge pass launch");
    cur_k = nxt_k;
    cur_v = nxt_v;
    ++h;
  }
  if (adaptive) {
    copy_back_kernel<K, V><<<dim3(unsigned(std::min<uint64_t>(ceil_div(n, 256), uint64_t(device_cu_count()) * 8))),
                             dim3(256), 0, s>>>(tk, tv, keys, vals, n, ctlw);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "final copy launch");
  }
  return MS_OK;
}

template <class K, class V>
ms_status merge_two_runs(const K* src, K* dst, uint64_t n, DevCtl ctl, int64_t* part, hipStream_t s,
                         uint64_t max_grid) {
  using C = PlainCfg<K, V>;
  using MT = MergeTile<K, V, C::MG_WG, C::MG_IPT, C::MG_PAD>;
  static_assert(!C::PAIRS, "keys only");
  // the run boundary comes from the device (pass widths are powers of two
  // everywhere else, and the kernels' pass geometry relies on that)
  if (!ctl.split_dev) {
    set_error("two-run merge needs a device-side split");
    return MS_ERR_INVALID_ARG;
  }
  if (n == 0) return MS_OK;
  const uint64_t mtiles = ceil_div(n, C::MTILE);
  const uint64_t cap = max_grid ? max_grid : ~uint64_t(0);
  with_search_group(search_group(mtiles), [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    partition_kernel<K, G><<<dim3(unsigned(std::min(ceil_div(mtiles * G, 256), cap))), dim3(256), 0, s>>>(
        src, n, ctl, n, C::MTILE, mtiles, part);
  });
  merge_kernel<K, V, C::MG_WG, C::MG_IPT, C::MG_PAD>
      <<<dim3(unsigned(std::min(mtiles, cap))), dim3(C::MG_WG), MT::LDS_BYTES, s>>>(src, nullptr, dst, nullptr, n,
                                                                                  ctl, n, part);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "two-run merge launch");
}
MS_DEFINE_DEV_ERRORS(dev_errors_plain)

#define MS_MERGE2_INSTANTIATE(K) \
  template ms_status merge_two_runs<K, NoVal>(const K*, K*, uint64_t, DevCtl, int64_t*, hipStream_t, uint64_t);
MS_MERGE2_INSTANTIATE(uint32_t)
MS_MERGE2_INSTANTIATE(int32_t)
MS_MERGE2_INSTANTIATE(uint64_t)
MS_MERGE2_INSTANTIATE(int64_t)

#define MS_INSTANTIATE(K, V)                                                                  \
  template ms_status plain_sort<K, V>(K*, V*, uint64_t, DevCtl, hipStream_t, void*, uint64_t); \
  template size_t plain_temp_bytes<K, V>(uint64_t);                                           \
  template void plain_geometry<K, V>(int*, int*, int*, int*);

MS_INSTANTIATE(uint32_t, NoVal)
MS_INSTANTIATE(int32_t, NoVal)
MS_INSTANTIATE(uint64_t, NoVal)
MS_INSTANTIATE(int64_t, NoVal)
MS_INSTANTIATE(uint32_t, uint32_t)
MS_INSTANTIATE(int32_t, uint32_t)
MS_INSTANTIATE(uint64_t, uint32_t)
MS_INSTANTIATE(int64_t, uint32_t)
MS_INSTANTIATE(uint32_t, uint64_t)
MS_INSTANTIATE(int32_t, uint64_t)
MS_INSTANTIATE(uint64_t, uint64_t)
MS_INSTANTIATE(int64_t, uint64_t)

}  // namespace ms

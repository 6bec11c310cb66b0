// Host-side planning arithmetic of the plain merge sort (no HIP calls, so it
// is exercised by CPU tests through ms_plan_query()).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace ms {

// Merge passes after the tile sort: runs of width T double each pass until
// one run covers n, i.e. ceil(log2(ceil(n / T))) passes (0 when n <= T).
inline int plan_passes(uint64_t n, uint64_t T) {
  if (n <= T) return 0;
  const uint64_t runs = (n + T - 1) / T;
  int p = 0;
  while ((uint64_t(1) << p) < runs) ++p;
  return p;
}

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// HBM round trips of the merge phase: pairs of tree levels are fused into
// one pass (four runs in, one run out); an odd level count leaves one
// two-run pass.
inline int plan_hbm_passes(int levels, bool fused) { return fused ? levels / 2 + levels % 2 : levels; }

// Buffer parity: the tile sort writes the caller's buffer when the number of
// HBM passes is even, the scratch buffer when it is odd, so that the last
// pass lands in the caller's buffer without a copy.
inline bool tile_sort_in_place(int hbm_passes) { return hbm_passes % 2 == 0; }

// The HBM passes of a plan with `levels` merge levels: pass h merges
// levels first_level[h] .. first_level[h] + levels_in[h] - 1 (an odd level
// count starts with one two-run pass, then fused passes take two levels).
constexpr int MAX_HBM_PASSES = 40;
struct PassPlan {
  int hbm;                               // number of HBM passes
  int start_in_caller;                   // the tile sort writes the caller's buffer
  uint8_t first_level[MAX_HBM_PASSES];
  uint8_t levels_in[MAX_HBM_PASSES];
};

inline PassPlan plan_pass_levels(int levels, bool fused) {
  PassPlan pp{};
  const int H = plan_hbm_passes(levels, fused);
  pp.hbm = H;
  pp.start_in_caller = tile_sort_in_place(H) ? 1 : 0;
  int p = 0, h = 0;
  while (p < levels && h < MAX_HBM_PASSES) {
    const int take = (fused && (levels - p) % 2 == 0) ? 2 : 1;
    pp.first_level[h] = uint8_t(p);
    pp.levels_in[h] = uint8_t(take);
    p += take;
    ++h;
  }
  return pp;
}

// Scratch layout of one plain sort:
// [keys n*kb | values n*vb | partitions | fused-pass tile offsets |
//  fused-pass sample head keys | sample tail keys |
//  run-adaptive control words | run boundary keys and level masks per group of tiles].
struct PlainLayout {
  size_t keys_off, vals_off, part_off, part4_off, head_off, tail_off, ctl_off, runs_off, bytes;
};

inline PlainLayout plain_layout(uint64_t n, size_t kb, size_t vb, uint64_t tile, uint64_t merge_tile,
                                uint64_t merge4_tile, int levels, bool fused) {
  PlainLayout L{};
  if (levels == 0) return L;
  const uint64_t tmin = merge_tile < merge4_tile ? merge_tile : merge4_tile;
  const bool f = fused && levels >= 2;
  const uint64_t t4 = ceil_div(n, merge4_tile) + 1;
  L.keys_off = 0;
  L.vals_off = align_up(n * kb, 256);
  L.part_off = align_up(L.vals_off + n * vb, 256);
  L.part4_off = align_up(L.part_off + (ceil_div(n, tmin) + 1) * sizeof(int64_t), 256);
  // four start offsets per fused-pass output tile, and two keys per sample
  L.head_off = align_up(L.part4_off + (f ? t4 * 4 * sizeof(int64_t) : 0), 256);
  L.tail_off = align_up(L.head_off + (f ? t4 * kb : 0), 256);
  L.ctl_off = align_up(L.tail_off + (f ? t4 * kb : 0), 256);
  // control words: final-copy flag, then a gate word (run, swap) per pass
  L.runs_off = align_up(L.ctl_off + (1 + MAX_HBM_PASSES) * sizeof(int32_t), 256);
  // four arrays of one key per group of 256 tiles, one mask word per group
  const uint64_t groups = ceil_div(ceil_div(n, tile), 256);
  L.bytes = align_up(L.runs_off + 4 * groups * kb + groups * sizeof(uint32_t), 256);
  return L;
}

}  // namespace ms

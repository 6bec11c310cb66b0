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

// Scratch layout of one plain sort:
// [keys n*kb | values n*vb | partitions | fused-pass tile offsets |
//  fused-pass sample head keys | sample tail keys].
struct PlainLayout {
  size_t keys_off, vals_off, part_off, part4_off, head_off, tail_off, bytes;
};

inline PlainLayout plain_layout(uint64_t n, size_t kb, size_t vb, uint64_t merge_tile, uint64_t merge4_tile,
                                int levels, bool fused) {
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
  L.bytes = align_up(L.tail_off + (f ? t4 * kb : 0), 256);
  return L;
}

}  // namespace ms

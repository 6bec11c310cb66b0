// Tile shapes of the plain merge sort.
#pragma once
#include <type_traits>

#include "ms_common.hpp"

namespace ms {

// Tile and merge-tile geometry per (key width, value width): workgroup size,
// items per thread and LDS pad shift of the tile sort (BS_*) and of the
// merge pass (MG_*).  Compile-time knobs, so that shapes can be swept by
// building with -D overrides; the defaults are the fastest shapes measured
// on MI355X.  Suffixes: K = 32-bit keys only, P = 32-bit keys with values,
// W = 64-bit keys.
#ifndef MS_BS_WG_K
#define MS_BS_WG_K 1024
#endif
#ifndef MS_BS_IPT_K
#define MS_BS_IPT_K 32
#endif
#ifndef MS_BS_PAD_K
#define MS_BS_PAD_K 5
#endif
// LDS pad of the batched segmented sort's tile sorts for 32-bit keys only
// (small-segment classes, then the large-segment tile), tuned apart from the
// plain sort's 1024 x 32 tile
#ifndef MS_SEG_PAD_K
#define MS_SEG_PAD_K 0
#endif
#ifndef MS_SEG_LPAD_K
#define MS_SEG_LPAD_K 0
#endif
#ifndef MS_MG_WG_K
#define MS_MG_WG_K 256
#endif
#ifndef MS_MG_IPT_K
#define MS_MG_IPT_K 8
#endif
#ifndef MS_MG_PAD_K
#define MS_MG_PAD_K 0
#endif
#ifndef MS_BS_WG_P
#define MS_BS_WG_P 256
#endif
#ifndef MS_BS_IPT_P
#define MS_BS_IPT_P 16
#endif
#ifndef MS_BS_PAD_P
#define MS_BS_PAD_P 5
#endif
#ifndef MS_MG_WG_P
#define MS_MG_WG_P 512
#endif
#ifndef MS_MG_IPT_P
#define MS_MG_IPT_P 8
#endif
#ifndef MS_MG_PAD_P
#define MS_MG_PAD_P 5
#endif
#ifndef MS_BS_WG_W
#define MS_BS_WG_W 256
#endif
#ifndef MS_BS_IPT_W
#define MS_BS_IPT_W 16
#endif
#ifndef MS_MG_WG_W
#define MS_MG_WG_W 256
#endif
#ifndef MS_MG_IPT_W
#define MS_MG_IPT_W 8
#endif
#ifndef MS_PAD_W
#define MS_PAD_W 5
#endif
// Fused two-level merge passes (four runs in, one out) and their shapes.
// MS_FUSED = 0 keeps one HBM pass per tree level.
#ifndef MS_FUSED
#define MS_FUSED 1
#endif
#ifndef MS_M4_WG_K
#define MS_M4_WG_K 512
#endif
#ifndef MS_M4_IPT_K
#define MS_M4_IPT_K 8
#endif
#ifndef MS_M4_PAD_K
#define MS_M4_PAD_K 0
#endif
#ifndef MS_M4_WG_P
#define MS_M4_WG_P 256
#endif
#ifndef MS_M4_IPT_P
#define MS_M4_IPT_P 8
#endif
#ifndef MS_M4_PAD_P
#define MS_M4_PAD_P 0
#endif
#ifndef MS_M4_WG_W
#define MS_M4_WG_W 512
#endif
// fused merge: 1 = stage-1 results overwrite the staged keys (less LDS,
// one more barrier); faster where LDS limits occupancy
#ifndef MS_M4_REUSE_K
#define MS_M4_REUSE_K 0
#endif
#ifndef MS_M4_REUSE_P
#define MS_M4_REUSE_P 1
#endif
#ifndef MS_M4_REUSE_W
#define MS_M4_REUSE_W 1
#endif
#ifndef MS_M4_IPT_W
#define MS_M4_IPT_W 8
#endif
template <class K, class V>
struct PlainCfg {
  static constexpr bool PAIRS = HasVal<V>::value;
  static constexpr bool WIDE = sizeof(K) == 8;
  static constexpr int BS_WG = WIDE ? MS_BS_WG_W : (PAIRS ? MS_BS_WG_P : MS_BS_WG_K);
  static constexpr int BS_IPT = WIDE ? (PAIRS ? 8 : MS_BS_IPT_W) : (PAIRS ? MS_BS_IPT_P : MS_BS_IPT_K);
  static constexpr int BS_PAD = WIDE ? MS_PAD_W : (PAIRS ? MS_BS_PAD_P : MS_BS_PAD_K);
  static constexpr int SEG_PAD = WIDE ? MS_PAD_W : (PAIRS ? MS_BS_PAD_P : MS_SEG_PAD_K);
  static constexpr int SEG_LPAD = WIDE ? MS_PAD_W : (PAIRS ? MS_BS_PAD_P : MS_SEG_LPAD_K);
  static constexpr int MG_WG = WIDE ? MS_MG_WG_W : (PAIRS ? MS_MG_WG_P : MS_MG_WG_K);
  static constexpr int MG_IPT = WIDE ? MS_MG_IPT_W : (PAIRS ? MS_MG_IPT_P : MS_MG_IPT_K);
  static constexpr int MG_PAD = WIDE ? MS_PAD_W : (PAIRS ? MS_MG_PAD_P : MS_MG_PAD_K);
  static constexpr int M4_WG = WIDE ? MS_M4_WG_W : (PAIRS ? MS_M4_WG_P : MS_M4_WG_K);
  static constexpr int M4_IPT = WIDE ? MS_M4_IPT_W : (PAIRS ? MS_M4_IPT_P : MS_M4_IPT_K);
  static constexpr int M4_PAD = WIDE ? MS_PAD_W : (PAIRS ? MS_M4_PAD_P : MS_M4_PAD_K);
  static constexpr int M4_REUSE = WIDE ? MS_M4_REUSE_W : (PAIRS ? MS_M4_REUSE_P : MS_M4_REUSE_K);
  static constexpr bool FUSED = MS_FUSED != 0;
  static constexpr int TILE = BS_WG * BS_IPT;
  static constexpr int MTILE = MG_WG * MG_IPT;
  static constexpr int M4TILE = M4_WG * M4_IPT;
  static_assert((2 * TILE) % MTILE == 0, "a merge tile must never straddle two run pairs");
  static_assert((2 * TILE) % M4TILE == 0, "second-pair samples must sit on merge-tile starts");
};

}  // namespace ms

// Segmented sort: many independent arrays, one call, one graph launch.
//
// Every segment [off[s], off[s+1]) is sorted on its own (stable, in place).
// The pipeline is shape-independent on the host -- the split of segments into
// size classes happens on the device -- so it can be captured once into a
// hipGraph and replayed:
//   1. init      : clear the class counters (a fill kernel, no memset nodes);
//   2. classify  : one thread per segment bins it by length into a small class
//                  queue, or reserves merge tiles for it in the large list;
//   3. owner     : writes, for every reserved merge tile, a descriptor (segment
//                  start, length, tile index) so that the large-segment kernels
//                  need one dependent load before touching keys;
//   4. per small class c, a persistent kernel whose workgroups take segments
//      from the class queue through an atomic work counter and sort each one
//      entirely in LDS (the tile sort of ms_block_sort.hpp with the class's
//      workgroup size and items per thread, picked by the autotuner);
//   5. large segments: the tile sort on each tile, then merge passes bounded
//      to the segment (runs never cross a segment end): an odd level count
//      starts with one two-run pass, the other levels go two at a time as
//      fused four-run passes.  Segments finish after different numbers of
//      passes, so each one picks its own buffer parity so that its last pass
//      lands in the caller's buffer.
#pragma once
#include "ms_block_sort.hpp"
#include "ms_merge.hpp"
#include "ms_plain_cfg.hpp"

namespace ms {

constexpr int SEG_MAX_CLASSES = 8;
constexpr int SEG_MAX_CANDIDATES = 3;

// Device-side state of one segmented sort (all in library scratch).
struct SegState {
  uint32_t* cls_count;   // [SEG_MAX_CLASSES] segments per small class
  uint32_t* cls_work;    // [SEG_MAX_CLASSES] atomic work counters
  unsigned long long* large_ctr;  // (large segment count << 40) | reserved merge tiles
  int32_t* queues;       // [SEG_MAX_CLASSES][nseg] segment ids per small class
  int32_t* large_seg;    // [nseg] segment id per large slot
  int64_t* large_mbase;  // [nseg] first reserved merge tile per large slot
  int4* desc;            // [mt_cap] per reserved merge tile: segment base (lo, hi), length, tile index
  int64_t* part;         // [mt_cap] merge-path splits of the current pass
  int64_t* part4;        // [4 * mt_cap] fused passes: four start offsets per merge tile
  void* head;            // [mt_cap] keys (K) at the splits (fused passes)
  void* tail;            // [mt_cap] keys (K) just before the splits (fused passes)
  void* const* keys_sel; // if non-null, small classes sort the key array *keys_sel (chosen on the device)
  void* const* io;       // if non-null, this launch's caller buffers: io[0] keys, io[1] values,
                         // io[2] offsets (written before each replay of a cached graph)
  uint32_t* max_steps;   // [1] HBM merge steps of the longest large segment (set by classify)
};

// The caller's buffer in slot i of this launch (graph replays rebind them).
template <class T>
__device__ __forceinline__ T* seg_io(const SegState& st, int i, T* p) {
  return st.io ? global_ptr<T>(&st.io[i]) : p;
}
__device__ __forceinline__ const int64_t* seg_bind_off(const SegState& st, const int64_t* off) {
  return st.io ? global_ptr<const int64_t>(&st.io[2]) : off;
}

// A reserved merge tile of a large segment, unpacked from its descriptor.
struct SegTile {
  int64_t base;  // segment start in the key array
  uint64_t L;    // segment length
  uint64_t lt;   // merge-tile index inside the segment
};

__device__ __forceinline__ SegTile seg_tile(const int4* desc, uint64_t g) {
  const int4 d = desc[g];
  SegTile t;
  t.base = int64_t(uint64_t(uint32_t(d.x)) | (uint64_t(uint32_t(d.y)) << 32));
  t.L = uint32_t(d.z);
  t.lt = uint32_t(d.w);
  return t;
}

// The same for a tile index that is one per workgroup (g the same in every
// lane): the fields go to scalar registers.
__device__ __forceinline__ SegTile seg_tile_wg(const int4* desc, uint64_t g) {
  SegTile t = seg_tile(desc, g);
  t.base = int64_t(wave_uniform(uint64_t(t.base)));
  t.L = wave_uniform(t.L);
  t.lt = wave_uniform(t.lt);
  return t;
}

constexpr unsigned long long SEG_SLOT_SHIFT = 40;
constexpr unsigned long long SEG_TILE_MASK = (1ull << SEG_SLOT_SHIFT) - 1;

__device__ __forceinline__ int seg_passes(uint64_t L, uint64_t T) {
  if (L <= T) return 0;
  const uint64_t runs = (L + T - 1) / T;
  return 64 - __builtin_clzll(runs - 1);
}

// HBM passes of a segment with P merge levels: an odd level first as a
// two-run pass, then the levels two at a time as fused four-run passes.
// Step j of a segment is two-run when j < P % 2, else fused over levels
// lv = P % 2 + 2 (j - P % 2) and lv + 1.
__device__ __forceinline__ int seg_steps(int P) { return P / 2 + P % 2; }

// Size classes of one (key, value) family: small classes have the
// power-of-two upper bounds 256, 512, ... up to the large-segment tile
// (at most 16384), so a segment pads its tile sort by less than 2x; longer
// segments go through the tile sort + merge passes.
template <class K, class V>
struct SegCfg {
  using P = PlainCfg<K, V>;
  // large segments: the plain sort's tile-sort shape, at most 16384 items per
  // tile (longer segments merge; a bigger tile pays off only for long arrays)
  static constexpr int LWG = P::BS_WG;
  static constexpr int LIPT = P::TILE > 16384 ? P::BS_IPT / (P::TILE / 16384) : P::BS_IPT;
  static constexpr int TILE = LWG * LIPT;  // large segments: tile-sort tile
  static constexpr int MTILE = P::MTILE;  // large segments: merge tile
  static constexpr int C = TILE / MTILE;  // merge tiles per tile
  static constexpr int log2c(int x) { return x <= 1 ? 0 : 1 + log2c(x / 2); }
  static constexpr int NCLS = log2c(TILE) - 7;  // classes 256 .. TILE
  static __host__ __device__ constexpr uint32_t cls_max(int c) { return 256u << c; }
  static_assert(TILE % MTILE == 0, "tile must be a whole number of merge tiles");
  static_assert((TILE & (TILE - 1)) == 0 && TILE >= 512 && NCLS <= SEG_MAX_CLASSES, "class bounds");
};

template <class K, class V>
__device__ __forceinline__ int seg_class(uint64_t L) {
  using S = SegCfg<K, V>;
#pragma unroll
  for (int c = 0; c < S::NCLS; ++c)
    if (L <= S::cls_max(c)) return c;
  return S::NCLS;  // large
}

static __global__ void seg_init_kernel(SegState st) {
  const int t = threadIdx.x;
  if (t < SEG_MAX_CLASSES) {
    st.cls_count[t] = 0;
    st.cls_work[t] = 0;
  }
  if (t == 0) {
    *st.large_ctr = 0;
    *st.max_steps = 0;
  }
}

// SEG_CLASSIFY_PER segments per thread (segment base + p * blockDim.x +
// thread, coalesced).  Slots are reserved in two steps so that a batch of
// many small segments does not serialise on one global counter: threads
// first count into workgroup-local LDS counters, then one thread per class
// adds the workgroup's total to the global counter, and every segment's
// slot is the global base plus its local offset.  (Order inside a class
// queue is arbitrary; each segment is sorted independently, so results do
// not depend on it.)  The large class uses one packed counter (segments <<
// 40 | merge tiles) so that slot order and merge-tile order agree.
constexpr int SEG_CLASSIFY_PER = 8;
template <class K, class V>
__global__ __launch_bounds__(256) void seg_classify_kernel(const int64_t* __restrict__ off, uint64_t nseg,
                                                           SegState st) {
  using S = SegCfg<K, V>;
  constexpr int PER = SEG_CLASSIFY_PER;
  __shared__ uint32_t l_cnt[SEG_MAX_CLASSES];
  __shared__ uint32_t g_base[SEG_MAX_CLASSES];
  __shared__ unsigned long long l_large, g_large;
  off = seg_bind_off(st, off);
  const uint64_t s0 = uint64_t(blockIdx.x) * blockDim.x * PER + threadIdx.x;
  if (threadIdx.x < SEG_MAX_CLASSES) l_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) l_large = 0;
  __syncthreads();
  int c[PER];
  uint32_t local[PER];
  unsigned long long llocal[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const uint64_t s = s0 + uint64_t(p) * blockDim.x;
    c[p] = -1;
    local[p] = 0;
    llocal[p] = 0;
    if (s < nseg) {
      const int64_t b = off[s], e = off[s + 1];
      if (e - b > 1) {
        const uint64_t L = uint64_t(e - b);
        c[p] = seg_class<K, V>(L);
        if (c[p] < S::NCLS) {
          local[p] = atomicAdd(&l_cnt[c[p]], 1u);
        } else {
          const unsigned long long mt = ((L + S::TILE - 1) / S::TILE) * S::C;
          llocal[p] = atomicAdd(&l_large, (1ull << SEG_SLOT_SHIFT) | mt);
          atomicMax(st.max_steps, uint32_t(seg_steps(seg_passes(L, S::TILE))));
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < S::NCLS && l_cnt[threadIdx.x] != 0)
    g_base[threadIdx.x] = atomicAdd(&st.cls_count[threadIdx.x], l_cnt[threadIdx.x]);
  if (threadIdx.x == 0 && l_large != 0) g_large = atomicAdd(st.large_ctr, l_large);
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const uint64_t s = s0 + uint64_t(p) * blockDim.x;
    if (c[p] < 0) continue;
    if (c[p] < S::NCLS) {
      st.queues[uint64_t(c[p]) * nseg + g_base[c[p]] + local[p]] = int32_t(s);
    } else {
      const unsigned long long at = g_large + llocal[p];
      const uint64_t slot = at >> SEG_SLOT_SHIFT;
      st.large_seg[slot] = int32_t(s);
      st.large_mbase[slot] = int64_t(at & SEG_TILE_MASK);
    }
  }
}

// Writes the descriptor of every reserved merge tile of every large segment.
template <class K, class V>
__global__ __launch_bounds__(256) void seg_owner_kernel(const int64_t* __restrict__ off, SegState st) {
  using S = SegCfg<K, V>;
  off = seg_bind_off(st, off);
  const uint64_t nlarge = (*st.large_ctr) >> SEG_SLOT_SHIFT;
  for (uint64_t slot = blockIdx.x; slot < nlarge; slot += gridDim.x) {
    const int32_t s = st.large_seg[slot];
    const int64_t b = off[s];
    const uint64_t L = uint64_t(off[s + 1] - b);
    const uint64_t mt = ((L + S::TILE - 1) / S::TILE) * S::C;
    const int64_t mb = st.large_mbase[slot];
    for (uint64_t t = threadIdx.x; t < mt; t += blockDim.x)
      st.desc[mb + t] = make_int4(int(uint32_t(uint64_t(b))), int(uint32_t(uint64_t(b) >> 32)), int(uint32_t(L)),
                                  int(uint32_t(t)));
  }
}

// Small class: workgroup b first takes queue chunk b (static), then grabs
// further chunks of `chunk` consecutive queue entries from the class's atomic
// work counter (which starts at gridDim.x chunks) until the queue is
// drained.  Chunks cut the number of atomics on the one counter, which
// otherwise serialises classes with hundreds of thousands of tiny segments.
// Each segment is sorted in place in LDS.
template <class K, class V, int WG, int IPT, int PAD>
__global__ __launch_bounds__(WG) void seg_small_kernel(K* __restrict__ keys, V* __restrict__ vals,
                                                       const int64_t* __restrict__ off, SegState st, int cls,
                                                       uint64_t nseg, uint32_t chunk) {
  using TS = TileSort<K, V, WG, IPT, PAD>;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t cur;
  const uint32_t count = st.cls_count[cls];
  const int32_t* q = st.queues + uint64_t(cls) * nseg;
  keys = seg_io(st, 0, keys);
  vals = seg_io(st, 1, vals);
  off = seg_bind_off(st, off);
  if (st.keys_sel) keys = global_ptr<K>(st.keys_sel);
  uint32_t c0 = blockIdx.x * chunk;
  while (c0 < count) {
    const uint32_t c1 = c0 + chunk < count ? c0 + chunk : count;
    for (uint32_t i = c0; i < c1; ++i) {
      const int32_t s = q[i];
      const int64_t b = off[s];
      const uint32_t L = uint32_t(off[s + 1] - b);
      if constexpr (TS::PAIRS) {
        TS::run(keys + b, vals + b, keys + b, vals + b, L, smem);
      } else {
        TS::template run<int>(keys + b, nullptr, keys + b, nullptr, L, smem);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) cur = (gridDim.x + atomicAdd(&st.cls_work[cls], 1u)) * chunk;
    __syncthreads();
    c0 = cur;
    __syncthreads();
  }
}

// Large segments, step 1: one workgroup per reserved tile (the grid covers
// the host-side bound; workgroups past the device-side count return).
template <class K, class V, int WG, int IPT, int PAD>
__global__ __launch_bounds__(WG) void seg_large_tile_kernel(K* __restrict__ keys, V* __restrict__ vals,
                                                            K* __restrict__ tk, V* __restrict__ tv, SegState st) {
  using S = SegCfg<K, V>;
  using TS = TileSort<K, V, WG, IPT, PAD>;
  static_assert(TS::TILE == S::TILE, "large-segment tile");
  extern __shared__ __align__(16) unsigned char smem[];
  const uint64_t t = blockIdx.x;
  if (t >= ((*st.large_ctr) & SEG_TILE_MASK) / S::C) return;
  keys = seg_io(st, 0, keys);
  vals = seg_io(st, 1, vals);
  const SegTile d = seg_tile(st.desc, t * S::C);
  const uint64_t j = d.lt / S::C;
  if (j * S::TILE >= d.L) return;  // reserved but past the segment end
  const uint64_t rem = d.L - j * S::TILE;
  const uint32_t len = rem < uint64_t(S::TILE) ? uint32_t(rem) : uint32_t(S::TILE);
  const bool to_caller = (seg_steps(seg_passes(d.L, S::TILE)) & 1) == 0;
  const uint64_t o = uint64_t(d.base) + j * S::TILE;
  if constexpr (TS::PAIRS) {
    TS::run(keys + o, vals + o, (to_caller ? keys : tk) + o, (to_caller ? vals : tv) + o, len, smem);
  } else {
    TS::template run<int>(keys + o, nullptr, (to_caller ? keys : tk) + o, nullptr, len, smem);
  }
}

// The merge steps below are launched for every step the host plans; a step
// past the longest segment's (counted on the device by classify) returns at
// once.  Each kernel loops over the reserved merge tiles with a grid stride,
// so the host may launch the steps beyond its length bound with a small grid.

// Large segments, step j: partition (one thread per reserved merge tile):
// the two-run split of a two-run step, or the samples (split, head and tail
// keys) of a fused step.  Each segment's arrays start at its first reserved
// merge tile.
template <class K, class V>
__global__ __launch_bounds__(256) void seg_partition_kernel(const K* __restrict__ keys, const K* __restrict__ tk,
                                                            SegState st, int j) {
  using S = SegCfg<K, V>;
  if (j >= int(*st.max_steps)) return;
  keys = seg_io(st, 0, keys);
  const uint64_t reserved = (*st.large_ctr) & SEG_TILE_MASK;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < reserved; g += stride) {
    const SegTile d = seg_tile(st.desc, g);
    const int P = seg_passes(d.L, S::TILE), H = seg_steps(P), first = P & 1;
    if (j >= H) continue;
    const uint64_t g0 = d.lt * S::MTILE;
    if (g0 >= d.L) continue;
    const K* src = (((H - j) & 1) == 0 ? keys : tk) + d.base;
    const uint64_t mb = g - d.lt;
    if (j < first) {
      const uint64_t W = uint64_t(S::TILE);
      const PassGeom q = pass_geom(g0, d.L, W);
      st.part[g] = int64_t(q.pb + merge_path_split(src + q.pb, q.a_end - q.pb, src + q.a_end, q.b_end - q.a_end,
                                                    g0 - q.pb));
    } else {
      const uint64_t W = uint64_t(S::TILE) << (first + 2 * (j - first));
      partition_group<K, 1>(src, d.L, W, uint32_t(S::MTILE), d.lt, DevCtl{nullptr, nullptr, nullptr}, 0u, 0u,
                            st.part + mb, static_cast<K*>(st.head) + mb, static_cast<K*>(st.tail) + mb);
    }
  }
}

// Large segments, fused step j: the four-way partition of each output tile,
// one lane per tile.
template <class K, class V>
__global__ __launch_bounds__(256) void seg_partition4_kernel(const K* __restrict__ keys, const K* __restrict__ tk,
                                                             SegState st, int j) {
  using S = SegCfg<K, V>;
  if (j >= int(*st.max_steps)) return;
  keys = seg_io(st, 0, keys);
  const uint64_t reserved = (*st.large_ctr) & SEG_TILE_MASK;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < reserved; g += stride) {
    const SegTile d = seg_tile(st.desc, g);
    const int P = seg_passes(d.L, S::TILE), H = seg_steps(P), first = P & 1;
    if (j >= H || j < first) continue;
    if (d.lt * S::MTILE >= d.L) continue;
    const K* src = (((H - j) & 1) == 0 ? keys : tk) + d.base;
    const uint64_t mb = g - d.lt;
    const uint64_t W = uint64_t(S::TILE) << (first + 2 * (j - first));
    // a group of one lane: the lane is its own group's first lane
    partition4_group<K, 1>(src, d.L, W, uint32_t(S::MTILE), d.lt, 0u, __lane_id(), st.part + mb,
                           static_cast<const K*>(st.head) + mb, static_cast<const K*>(st.tail) + mb,
                           st.part4 + 4 * mb);
  }
}

// Large segments, two-run step p (p = 0 of an odd level count): the merge of
// reserved merge tile g by the whole workgroup.
template <class K, class V, int WG, int IPT, int PAD>
__device__ __forceinline__ void seg_merge_tile(K* __restrict__ keys, V* __restrict__ vals, K* __restrict__ tk,
                                               V* __restrict__ tv, const SegState& st, int p, uint64_t g,
                                               unsigned char* smem) {
  using S = SegCfg<K, V>;
  using MT = MergeTile<K, V, WG, IPT, PAD>;
  static_assert(MT::TM == S::MTILE, "large-segment merge tile");
  // the splits are loaded together with the descriptor (both indices are
  // inside the scratch arrays: g + 1 < reserved tiles + C <= mt_cap); values
  // that turn out not to be needed are ignored
  const int64_t part0 = st.part[g], part1 = st.part[g + 1];
  const SegTile d = seg_tile_wg(st.desc, g);
  const int P = seg_passes(d.L, S::TILE), H = seg_steps(P);
  if (p >= (P & 1)) return;  // two-run steps only (the first step of an odd level count)
  const uint64_t g0 = d.lt * S::MTILE;
  if (g0 >= d.L) return;
  const bool from_caller = ((H - p) & 1) == 0;
  K* sk = (from_caller ? keys : tk) + d.base;
  K* dk = (from_caller ? tk : keys) + d.base;
  const uint64_t g1 = g0 + S::MTILE < d.L ? g0 + S::MTILE : d.L;
  const uint64_t W = uint64_t(S::TILE);
  const PassGeom q = pass_geom(g0, d.L, W);
  const uint64_t i0 = wave_uniform(uint64_t(part0));
  const uint64_t j0 = q.a_end + (g0 - q.pb) - (i0 - q.pb);
  uint64_t i1, j1;
  if (g1 == q.b_end) {
    i1 = q.a_end;
    j1 = q.b_end;
  } else {
    i1 = wave_uniform(uint64_t(part1));
    j1 = q.a_end + (g1 - q.pb) - (i1 - q.pb);
  }
  if constexpr (MT::PAIRS) {
    V* sv = (from_caller ? vals : tv) + d.base;
    V* dv = (from_caller ? tv : vals) + d.base;
    MT::run(sk, sv, dk, dv, i0, uint32_t(i1 - i0), j0, uint32_t(j1 - j0), g0, smem);
  } else {
    MT::template run<int>(sk, nullptr, dk, nullptr, i0, uint32_t(i1 - i0), j0, uint32_t(j1 - j0), g0, smem);
  }
}

template <class K, class V, int WG, int IPT, int PAD>
__global__ __launch_bounds__(WG) void seg_merge_kernel(K* __restrict__ keys, V* __restrict__ vals,
                                                       K* __restrict__ tk, V* __restrict__ tv, SegState st, int p) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (p >= int(*st.max_steps)) return;
  keys = seg_io(st, 0, keys);
  vals = seg_io(st, 1, vals);
  const uint64_t reserved = (*st.large_ctr) & SEG_TILE_MASK;
  for (uint64_t g = blockIdx.x; g < reserved; g += gridDim.x) {
    seg_merge_tile<K, V, WG, IPT, PAD>(keys, vals, tk, tv, st, p, g, smem);
    __syncthreads();
  }
}

// Large segments, fused step j: reserved merge tile g by the whole workgroup.
template <class K, class V, int WG, int IPT, int PAD, int REUSE>
__device__ __forceinline__ void seg_merge4_tile(K* __restrict__ keys, V* __restrict__ vals, K* __restrict__ tk,
                                                V* __restrict__ tv, const SegState& st, int j, uint64_t g,
                                                unsigned char* smem) {
  using S = SegCfg<K, V>;
  using MT = Merge4Tile<K, V, WG, IPT, PAD, REUSE>;
  using VV = typename MT::VV;
  static_assert(MT::TM == S::MTILE, "large-segment fused merge tile");
  const SegTile d = seg_tile_wg(st.desc, g);
  const int P = seg_passes(d.L, S::TILE), H = seg_steps(P), first = P & 1;
  if (j >= H || j < first) return;  // workgroup-uniform
  if (d.lt * S::MTILE >= d.L) return;
  const bool from_caller = ((H - j) & 1) == 0;
  const uint64_t mb = g - d.lt;
  const uint64_t W = uint64_t(S::TILE) << (first + 2 * (j - first));
  K* sk = (from_caller ? keys : tk) + d.base;
  K* dk = (from_caller ? tk : keys) + d.base;
  if constexpr (MT::PAIRS) {
    V* sv = (from_caller ? vals : tv) + d.base;
    V* dv = (from_caller ? tv : vals) + d.base;
    merge4_tile<MT>(sk, sv, dk, dv, d.L, W, d.lt, st.part4 + 4 * mb, smem);
  } else {
    merge4_tile<MT>(sk, static_cast<const VV*>(nullptr), dk, static_cast<VV*>(nullptr), d.L, W, d.lt,
                    st.part4 + 4 * mb, smem);
  }
}

template <class K, class V, int WG, int IPT, int PAD, int REUSE>
__global__ __launch_bounds__(WG) void seg_merge4_kernel(K* __restrict__ keys, V* __restrict__ vals,
                                                        K* __restrict__ tk, V* __restrict__ tv, SegState st, int j) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (j >= int(*st.max_steps)) return;
  keys = seg_io(st, 0, keys);
  vals = seg_io(st, 1, vals);
  const uint64_t reserved = (*st.large_ctr) & SEG_TILE_MASK;
  for (uint64_t g = blockIdx.x; g < reserved; g += gridDim.x) {
    seg_merge4_tile<K, V, WG, IPT, PAD, REUSE>(keys, vals, tk, tv, st, j, g, smem);
    __syncthreads();
  }
}

}  // namespace ms

// Tile sort: sorts one tile of up to WG*IPT elements inside one workgroup.
//
// This is the GPU form of the paper's chunk-parallel step (section
// "Multiprocessing Merge Sort": the array is cut into equal chunks that are
// sorted independently) with the hybrid variant's leaf cutoff (the
// sequential_mergesort figure) becoming the tile size.  Within a tile:
//   1. blocked load: thread t holds tile positions [t*IPT, t*IPT + IPT);
//      slots past the tile's end are padded with an item that sorts last;
//   2. each thread sorts its IPT items with a bitonic network in registers;
//   3. wavefront merges: runs of IPT, 2*IPT, ..., 32*IPT items are merged in
//      pairs by bitonic merge stages whose partners sit in other lanes, with
//      the xor lane moves (DPP / ds_swizzle / ds_bpermute) of ms_common.hpp;
//   4. LDS merge-path levels merge the wave runs up to the whole tile; each
//      thread finds its output diagonal by binary search and merges IPT
//      outputs serially, left run first on ties;
//   5. store (and, for pairs, fetch each value by its input position).
// Bitonic stages compare (key, input position) items for pairs, a strict
// total order, so they produce exactly the stable order.
#pragma once
#include <type_traits>

#include "ms_common.hpp"

// Lanes spanned by the runs that the bitonic wavefront merges build before
// LDS merge-path levels take over: 32-bit keys alone stay on lane exchanges
// up to the whole wavefront; pairs and 64-bit keys (wider items, costlier
// exchanges) switch to LDS after 16 lanes.  Measured on MI355X: 32-bit keys
// 1.00 ms (64) vs 1.11 ms (4) per 2^27; Zipf pairs 1.59 (64) vs 1.42 ms (4)
// with a min-and-max exchange, and with the compare-and-select exchange
// 1.16 (4), 1.12 (8, 16), 1.17 (32), 2.14 ms (64); 2^28 int64 2.46 (64)
// vs 1.87 ms (4), then 1.84 (4), 1.78 (16) ms.
#ifndef MS_TS_LANES_K
#define MS_TS_LANES_K 64
#endif
#ifndef MS_TS_LANES_PW
#define MS_TS_LANES_PW 16
#endif

namespace ms {

template <class IT, class T>
__device__ __forceinline__ void cmpswap(T& a, T& b) {
  T lo = IT::vmin(a, b), hi = IT::vmax(a, b);
  a = lo;
  b = hi;
}

// Bitonic sort of N register items ("flip" form: every stage ascending).
template <class IT, int N, class T>
__device__ __forceinline__ void register_sort(T (&v)[N]) {
#pragma unroll
  for (int size = 2; size <= N; size *= 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int j = i ^ (size - 1);
      if (j > i) cmpswap<IT>(v[i], v[j]);
    }
#pragma unroll
    for (int s = size / 4; s >= 1; s /= 2) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int j = i ^ s;
        if (j > i) cmpswap<IT>(v[i], v[j]);
      }
    }
  }
}

// Half-cleaner stage between lanes lane and lane^SL (same register index).
template <class IT, int SL, int N, class T>
__device__ __forceinline__ void lane_half_clean(T (&v)[N], int lane) {
  const bool lower = (lane & SL) == 0;
  if constexpr (IT::MED3) {
    const T sd = IT::side(lower);
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = IT::keep(v[r], xor_lane<SL>(v[r]), sd);
  } else if constexpr (std::is_integral<T>::value) {
    // the lower lane keeps the smaller, the upper one the larger: take the
    // partner's item when it is smaller, for the lower lane, or else when
    // it is not (equal items are interchangeable)
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const T p = xor_lane<SL>(v[r]);
      v[r] = (IT::less(p, v[r]) == lower) ? p : v[r];
    }
  } else {  // (key, position) records: this form keeps them in registers
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const T p = xor_lane<SL>(v[r]);
      v[r] = lower ? IT::vmin(v[r], p) : IT::vmax(v[r], p);
    }
  }
  if constexpr (SL > 1) lane_half_clean<IT, SL / 2>(v, lane);
}

// Merge sorted runs spanning L2/2 lanes each into runs spanning L2 lanes.
template <class IT, int L2, int N, class T>
__device__ __forceinline__ void wave_merge_level(T (&v)[N], int lane) {
  // flip stage: flat index f pairs with f ^ (L2*N - 1), i.e. lane ^ (L2-1),
  // register N-1-r; the lower half of each block keeps the minimum.
  {
    const bool lower = (lane & (L2 / 2)) == 0;
    [[maybe_unused]] T sd{};
    if constexpr (IT::MED3) sd = IT::side(lower);
    auto keep = [&](const T& own, const T& p) -> T {
      if constexpr (IT::MED3) return IT::keep(own, p, sd);
      else if constexpr (std::is_integral<T>::value) return (IT::less(p, own) == lower) ? p : own;
      else return lower ? IT::vmin(own, p) : IT::vmax(own, p);
    };
    if constexpr (IT::WITH_POS) {
      // registers r and N-1-r updated together from each other's partner
      // items: two temporaries live instead of N (keeps pair tiles from
      // spilling)
#pragma unroll
      for (int r = 0; r < N / 2; ++r) {
        const T pr = xor_lane<L2 - 1>(v[N - 1 - r]);  // partner's item for register r
        const T pq = xor_lane<L2 - 1>(v[r]);          // and for register N-1-r
        v[r] = keep(v[r], pr);
        v[N - 1 - r] = keep(v[N - 1 - r], pq);
      }
    } else {
      T p[N];
#pragma unroll
      for (int r = 0; r < N; ++r) p[r] = xor_lane<L2 - 1>(v[N - 1 - r]);
#pragma unroll
      for (int r = 0; r < N; ++r) v[r] = keep(v[r], p[r]);
    }
  }
  if constexpr (L2 >= 4) lane_half_clean<IT, L2 / 4>(v, lane);
  // remaining half cleaners inside each lane's registers
#pragma unroll
  for (int s = N / 2; s >= 1; s /= 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int j = i ^ s;
      if (j > i) cmpswap<IT>(v[i], v[j]);
    }
  }
}

// Wavefront merge levels from runs spanning L2/2 lanes up to runs spanning
// LMAX lanes.
template <class IT, int L2, int LMAX, int N, class T>
__device__ __forceinline__ void wave_merges(T (&v)[N], int lane) {
  if constexpr (L2 <= LMAX) {
    wave_merge_level<IT, L2>(v, lane);
    wave_merges<IT, L2 * 2, LMAX>(v, lane);
  }
}

// Orders LDS accesses among the lanes of one wavefront (merge levels whose
// runs never leave the wavefront's own part of LDS need nothing wider).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One LDS merge-path level: sorted runs of R items (blocked in registers
// across the workgroup) become runs of 2R.  lds must hold WG*N items.
// WAVE: 2R <= 64*N, so every pair of runs lies in the part of LDS that one
// wavefront writes and reads, and a wavefront-wide sync suffices.
// A merged block that lies wholly past the tile's length holds only padding
// items, which are already in order (pad(e) at position e), so it is
// skipped.
// Gap slots after each run in the padded-run form below: at least N + 1,
// a multiple of 16 bytes.
template <int N, class T>
constexpr uint32_t lds_run_gap() { return uint32_t(((N + 1) * sizeof(T) + 15) / 16 * 16 / sizeof(T)); }
// The padded-run form's shapes: 32-bit keys alone with at most 16 items per
// thread (with more, or with 64-bit keys, the tile sorts are at their
// register limit and the form's extra registers spill: 32768-key u32 tiles
// 0.87 -> 1.15 ms).
template <class IT, int N, class T>
constexpr bool lds_padded_runs() { return !IT::WITH_POS && sizeof(T) == 4 && N <= 16; }

template <class IT, int WG, int PAD, bool WAVE = false, int N, class T>
__device__ __forceinline__ void lds_merge_level(T (&v)[N], T* lds, int R, uint32_t len) {
  const int tid = threadIdx.x;
  if constexpr (lds_padded_runs<IT, N, T>() && !WAVE) {
    // Keys only, workgroup-wide levels: each run of R items is followed in
    // LDS by G slots of the type's largest key (run k at k (R + G)), so a
    // merge step is one compare: a used-up run's next "item" is that key,
    // which loses to every smaller key, and against an equal key either
    // choice writes the same value.  Reads stay within N + 1 slots past a
    // run's end.
    constexpr uint32_t G = lds_run_gap<N, T>();
    const uint32_t RG = uint32_t(R) + G;
    const uint32_t x0 = uint32_t(tid) * N;  // this thread's items lie in run x0 / R
#pragma unroll
    for (int r = 0; r < N; ++r) lds[lds_pad<PAD>(x0 + (x0 / uint32_t(R)) * G + r)] = v[r];
    const uint32_t nruns = uint32_t(WG * N) / uint32_t(R);
    for (uint32_t g = uint32_t(tid); g < nruns * G; g += WG) {
      const uint32_t k = g / G;
      lds[lds_pad<PAD>(k * RG + uint32_t(R) + (g - k * G))] = IT::pad(0);
    }
    __syncthreads();
    const int per_blk = (2 * R) / N;  // threads per merged run
    const int blk = tid / per_blk;
    const uint32_t d = uint32_t(tid - blk * per_blk) * N;
    if (uint32_t(blk) * 2 * uint32_t(R) >= len) {
#pragma unroll
      for (int r = 0; r < N; ++r) v[r] = IT::pad(0);
    } else {
      const uint32_t a0 = uint32_t(blk) * 2 * RG, b0 = a0 + RG;  // runs A and B
      uint32_t lo = d > uint32_t(R) ? d - uint32_t(R) : 0, hi = d < uint32_t(R) ? d : uint32_t(R);
      while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (IT::less(lds[lds_pad<PAD>(b0 + d - 1 - m)], lds[lds_pad<PAD>(a0 + m)])) hi = m; else lo = m + 1;
      }
      uint32_t ia = a0 + lo, jb = b0 + (d - lo);
      T a = lds[lds_pad<PAD>(ia)], b = lds[lds_pad<PAD>(jb)];
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const bool tb = IT::less(b, a);
        v[r] = tb ? b : a;
        const uint32_t nx = (tb ? jb : ia) + 1u;
        const T x = lds[lds_pad<PAD>(nx)];
        ia = tb ? ia : nx;
        jb = tb ? nx : jb;
        a = tb ? a : x;
        b = tb ? x : b;
      }
    }
    __syncthreads();
    return;
  }
#pragma unroll
  for (int r = 0; r < N; ++r) lds[lds_pad<PAD>(tid * N + r)] = v[r];
  if constexpr (WAVE) wave_lds_sync(); else __syncthreads();
  const int per_blk = (2 * R) / N;  // threads per merged run
  const int blk = tid / per_blk;
  const int d = (tid - blk * per_blk) * N;
  const uint32_t a0 = blk * 2 * R, b0 = a0 + R;  // runs A and B (through lds_pad)
  // the barrier below is reached by every thread whichever branch it takes
  if (a0 >= len) {
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = IT::pad(a0 + d + r);
  } else {
    int lo = d > R ? d - R : 0, hi = d < R ? d : R;
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (IT::less(lds[lds_pad<PAD>(b0 + d - 1 - m)], lds[lds_pad<PAD>(a0 + m)])) hi = m; else lo = m + 1;
    }
    int i = lo, j = d - lo;
    // i, j <= R throughout (a thread emits at most 2R - d items), so a read
    // one past a run lands in the next run or in the spare slot after the
    // tile; such a value is never taken (that run is exhausted)
    T a = lds[lds_pad<PAD>(a0 + i)], b = lds[lds_pad<PAD>(b0 + j)];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const bool take_b = (j < R) && (i >= R || IT::less(b, a));
      v[r] = take_b ? b : a;
      i += take_b ? 0 : 1;
      j += take_b ? 1 : 0;
      const uint32_t nx = take_b ? b0 + j : a0 + i;
      const T x = lds[lds_pad<PAD>(nx)];
      a = take_b ? a : x;
      b = take_b ? x : b;
    }
  }
  if constexpr (WAVE) wave_lds_sync(); else __syncthreads();
}

template <class K, class V, int WG, int IPT, int PAD>
struct TileSort {
  static constexpr bool PAIRS = HasVal<V>::value;
  using IT = Item<K, PAIRS>;
  using T = typename IT::T;
  static constexpr int TILE = WG * IPT;
  static constexpr int NW = WG / 64;
  static_assert(WG % 64 == 0 && (WG & (WG - 1)) == 0 && WG <= 1024, "WG");
  static_assert((IPT & (IPT - 1)) == 0 && IPT >= 2 && IPT <= 32, "IPT");
  // lane-exchange (bitonic) merges build runs spanning LANES lanes; LDS
  // merge-path levels take them from there to the whole tile
  // (64-bit keys with values, (key, position) records, keep 4 lanes)
  static constexpr int LANES =
      (PAIRS && sizeof(K) == 8) ? 4 : ((PAIRS || sizeof(K) == 8) ? MS_TS_LANES_PW : MS_TS_LANES_K);
  static_assert(LANES >= 1 && LANES <= 64 && (LANES & (LANES - 1)) == 0, "LANES");
  static constexpr bool USE_LDS = NW > 1 || LANES < 64;
  // one spare slot past the tile (reads one past the last run); keys only,
  // the workgroup-wide levels' gaps (one per run of the first such level)
  static constexpr uint32_t GAP_SLOTS =
      (lds_padded_runs<IT, IPT, T>() && NW > 1) ? uint32_t(NW) * lds_run_gap<IPT, T>() : 0u;
  static constexpr size_t LDS_ITEMS =
      USE_LDS ? (sizeof(T) * (lds_padded_size<PAD>(TILE + GAP_SLOTS) + 1) + 15) / 16 * 16 : 0;
  static constexpr size_t LDS_VALS = PAIRS ? sizeof(typename std::conditional<PAIRS, V, int>::type) * TILE : 0;
  static constexpr size_t LDS_BYTES = LDS_ITEMS + LDS_VALS;

  // Sort in_k[0, len) (len <= TILE) into out_k[0, len); values likewise.
  // in and out may alias (the whole tile is read before anything is written).
  template <class VV>
  static __device__ __forceinline__ void run(const K* in_k, const VV* in_v, K* out_k, VV* out_v,
                                             uint32_t len, unsigned char* smem) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    T* lds = reinterpret_cast<T*>(smem);
    VV* lds_v = reinterpret_cast<VV*>(smem + LDS_ITEMS);
    if constexpr (PAIRS) {
      VV vv[IPT];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = uint32_t(tid) + uint32_t(r) * WG;
        if (e < len) vv[r] = in_v[e];
      }
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = uint32_t(tid) + uint32_t(r) * WG;
        if (e < len) lds_v[e] = vv[r];
      }
    }
    T v[IPT];
    const uint32_t e0 = uint32_t(tid) * IPT;
    const bool full = e0 + IPT <= len &&
                      ((reinterpret_cast<uintptr_t>(in_k + e0) & 15) == 0);
    if (full) {
      K kk[IPT];
      load_run<K, IPT>(in_k + e0, kk);
#pragma unroll
      for (int r = 0; r < IPT; ++r) v[r] = IT::make(kk[r], e0 + r);
    } else {
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = e0 + r;
        v[r] = e < len ? IT::make(in_k[e], e) : IT::pad(e);
      }
    }
    // a wavefront whose items are all padding holds them in order already
    // and skips its wavefront-local levels (short segments, partial tiles)
    const bool pad_wave = uint32_t(tid & ~63) * IPT >= len;
    if (!pad_wave) {
      register_sort<IT>(v);
      wave_merges<IT, 2, LANES>(v, lane);
      if constexpr (USE_LDS) {
#pragma unroll
        for (int R = LANES * IPT; R < 64 * IPT && R < TILE; R *= 2)
          lds_merge_level<IT, WG, PAD, true>(v, lds, R, len);
      }
    }
    if constexpr (USE_LDS && NW > 1) {
      // keys only: the workgroup-wide levels lay runs out with gaps, which
      // overlap what the wavefront-local levels above may still be reading
      if constexpr (lds_padded_runs<IT, IPT, T>() && LANES < 64) __syncthreads();
      // all loads of this tile are done before the first barrier, so the
      // output may overwrite the input in place
#pragma unroll
      for (int R = 64 * IPT; R < TILE; R *= 2) lds_merge_level<IT, WG, PAD>(v, lds, R, len);
    }
    // staged values are read across the workgroup below (a multi-wavefront
    // tile already ended its last level with a workgroup barrier)
    if constexpr (NW == 1) __syncthreads();
    // store
    K ko[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) ko[r] = IT::key(v[r]);
    const bool full_out = e0 + IPT <= len &&
                          ((reinterpret_cast<uintptr_t>(out_k + e0) & 15) == 0);
    if (full_out) {
      store_run<K, IPT>(out_k + e0, ko);
    } else {
#pragma unroll
      for (int r = 0; r < IPT; ++r)
        if (e0 + r < len) out_k[e0 + r] = ko[r];
    }
    if constexpr (PAIRS) {
      VV vo[IPT];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t p = IT::pos(v[r]);
        vo[r] = lds_v[p < len ? p : 0];
      }
      const bool fv = e0 + IPT <= len && ((reinterpret_cast<uintptr_t>(out_v + e0) & 15) == 0);
      if (fv) {
        store_run<VV, IPT>(out_v + e0, vo);
      } else {
#pragma unroll
        for (int r = 0; r < IPT; ++r)
          if (e0 + r < len) out_v[e0 + r] = vo[r];
      }
    }
  }
};

// Waves per SIMD the tile sort is compiled for.  32-bit keys with values
// would otherwise take 196 VGPRs (2 waves per SIMD); capped at 168 they run
// 3 waves with a few spilled registers, which measured faster.  The other
// shapes already fit 4 (u32 keys: 1024-thread tiles) or 3 waves.
#ifndef MS_BS_WAVES_P
#define MS_BS_WAVES_P 3
#endif
template <class K, class V>
constexpr int bs_waves_per_eu() {
  return (HasVal<V>::value && sizeof(K) == 4) ? MS_BS_WAVES_P : (HasVal<V>::value ? 3 : 4);
}

// Tiles [t*TILE, min(n, (t+1)*TILE)); workgroup b takes tiles b, b + grid, ...
// (one tile each when the grid covers them all).
template <class K, class V, int WG, int IPT, int PAD>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(bs_waves_per_eu<K, V>())))
void block_sort_kernel(const K* in_k, const V* in_v, K* out_k, V* out_v, uint64_t n_host, DevCtl ctl) {
  using TS = TileSort<K, V, WG, IPT, PAD>;
  extern __shared__ __align__(16) unsigned char smem[];
  if (gated_off(ctl)) return;
  in_k = rebind(in_k, ctl.keys);
  out_k = rebind(out_k, ctl.keys);
  const uint64_t n = live_n(ctl, n_host);
  for (uint64_t base = uint64_t(blockIdx.x) * TS::TILE; base < n; base += uint64_t(gridDim.x) * TS::TILE) {
    const uint64_t rem = n - base;
    const uint32_t len = rem < uint64_t(TS::TILE) ? uint32_t(rem) : uint32_t(TS::TILE);
    if constexpr (TS::PAIRS) {
      TS::run(in_k + base, in_v + base, out_k + base, out_v + base, len, smem);
    } else {
      TS::template run<int>(in_k + base, nullptr, out_k + base, nullptr, len, smem);
    }
    __syncthreads();
  }
}

}  // namespace ms

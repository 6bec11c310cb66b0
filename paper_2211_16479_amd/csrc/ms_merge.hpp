// Global merge passes.
//
// After the tile sort the array holds sorted runs of width T.  Pass p merges
// runs 2j and 2j+1 of width W = T * 2^p into one run of width 2W; the last
// run of an odd count, and a short last run, simply take part with an empty
// or short partner.  Each pass is one level of the paper's merge tree
// (section "Merging the subarrays", where each loop iteration halves the
// number of sorted pieces), run for all pairs at once; pairing is between
// adjacent runs, which keeps the sort stable (the paper's rank tree pairs r
// with r + split, which would not be).
//
// A pass is two kernels:
//   partition: for every merge tile k (outputs [k*Tm, (k+1)*Tm) of its pair)
//     a binary search on the merge-path diagonal d = k*Tm - pair_base finds
//     i(d) = how many of the first d outputs come from run A, under the
//     left-wins-ties rule (A[m] goes first when A[m] <= B[d-1-m]);
//   merge: workgroup k stages A[i(d_k), i(d_k+1)) and B[d_k - i(d_k), ...)
//     in LDS with coalesced loads, each thread finds its own sub-diagonal by
//     the same search and merges IPT outputs serially, then stores them.
#pragma once
#include "ms_common.hpp"

namespace ms {

struct PassGeom {
  uint64_t pb, a_end, b_end;  // pair base, end of run A, end of run B
};

__device__ __forceinline__ PassGeom pass_geom(uint64_t g, uint64_t n, uint64_t W) {
  PassGeom q;
  q.pb = (g / (2 * W)) * (2 * W);
  q.a_end = q.pb + W < n ? q.pb + W : n;
  q.b_end = q.pb + 2 * W < n ? q.pb + 2 * W : n;
  return q;
}

// Pass geometry under a DevCtl: a device-side split point means a single
// merge of [0, split) with [split, n).
__device__ __forceinline__ PassGeom pass_geom(uint64_t g, uint64_t n, uint64_t W, const DevCtl& c) {
  if (c.split_dev) {
    const uint64_t sp = *c.split_dev;
    return PassGeom{0, sp < n ? sp : n, n};
  }
  return pass_geom(g, n, W);
}

// Number of outputs among the first d of merge(A, B) that come from A.
template <class K>
__device__ __forceinline__ uint64_t merge_path_split(const K* A, uint64_t la, const K* B, uint64_t lb,
                                                     uint64_t d) {
  uint64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint64_t m = (lo + hi) >> 1;
    if (B[d - 1 - m] < A[m]) hi = m; else lo = m + 1;
  }
  return lo;
}

// One search per merge tile.  G = 1: one thread runs the binary search.
// G > 1: G lanes cooperate on one diagonal; each round they probe G evenly
// spaced positions of the remaining interval [lo, hi) and a ballot picks the
// sub-interval holding the split, so the interval shrinks by G + 1 per round
// (fewer dependent global loads).  Both use the same predicate:
// split <= m  iff  B[d-1-m] < A[m].
template <class K, int G>
__global__ __launch_bounds__(256) void partition_kernel(const K* __restrict__ src, uint64_t n_host, DevCtl ctl,
                                                        uint64_t W, uint32_t Tm, uint64_t num_tiles,
                                                        int64_t* __restrict__ part) {
  static_assert(G >= 1 && G <= 64 && (64 % G) == 0, "group size");
  if (gated_off(ctl)) return;
  const uint64_t n = live_n(ctl, n_host);
  const uint64_t gid = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t k = gid / G;
  if constexpr (G == 1) {
    for (uint64_t kk = gid; kk < num_tiles; kk += uint64_t(gridDim.x) * blockDim.x) {
      const uint64_t g = kk * Tm;
      if (g >= n) return;
      const PassGeom q = pass_geom(g, n, W, ctl);
      const uint64_t i = merge_path_split(src + q.pb, q.a_end - q.pb, src + q.a_end, q.b_end - q.a_end, g - q.pb);
      part[kk] = int64_t(q.pb + i);
    }
  } else {
    const uint32_t q = uint32_t(gid % G);
    const uint32_t gshift = (__lane_id() / G) * G;
    const bool valid = k < num_tiles && k * Tm < n;
    uint64_t lo = 0, hi = 0, d = 0;
    const K* A = src;
    const K* B = src;
    PassGeom geo{0, 0, 0};
    if (valid) {
      geo = pass_geom(k * Tm, n, W, ctl);
      const uint64_t la = geo.a_end - geo.pb, lb = geo.b_end - geo.a_end;
      d = k * Tm - geo.pb;
      A = src + geo.pb;
      B = src + geo.a_end;
      lo = d > lb ? d - lb : 0;
      hi = d < la ? d : la;
    }
    while (true) {
      const bool active = valid && lo < hi;
      if (!__any(active)) break;
      const uint64_t len = hi - lo;
      const bool small = len <= G;
      const uint64_t m = small ? lo + q : lo + ((q + 1) * len) / (G + 1);
      const bool probe = active && (!small || q < len);
      const bool pred = probe && (B[d - 1 - m] < A[m]);
      const uint32_t gm = uint32_t((__ballot(pred) >> gshift) & ((G == 64) ? ~0ull : ((1ull << G) - 1)));
      if (active) {
        if (small) {
          lo = hi = lo + (gm ? uint64_t(__builtin_ctz(gm)) : len);
        } else if (gm == 0) {
          lo = lo + (uint64_t(G) * len) / (G + 1) + 1;
        } else {
          const uint32_t f = __builtin_ctz(gm);
          hi = lo + ((f + 1) * len) / (G + 1);
          lo = f ? lo + (uint64_t(f) * len) / (G + 1) + 1 : lo;
        }
      }
    }
    if (valid && q == 0) part[k] = int64_t(geo.pb + lo);
  }
}

template <class K, class V, int WG, int IPT, int PAD>
struct MergeTile {
  static constexpr bool PAIRS = HasVal<V>::value;
  static constexpr int TM = WG * IPT;
  static constexpr size_t LDS_KEYS = (sizeof(K) * lds_padded_size<PAD>(TM) + 15) / 16 * 16;
  static constexpr size_t LDS_BYTES =
      LDS_KEYS + (PAIRS ? sizeof(typename std::conditional<PAIRS, V, int>::type) * lds_padded_size<PAD>(TM) : 0);

  // Merge A = src[a0, a0+la) and B = src[b0, b0+lb) (la + lb <= TM) into
  // dst[o0, o0+la+lb); A's elements win ties.
  template <class VV>
  static __device__ __forceinline__ void run(const K* __restrict__ src_k, const VV* __restrict__ src_v,
                                             K* __restrict__ dst_k, VV* __restrict__ dst_v,
                                             uint64_t a0, uint32_t la, uint64_t b0, uint32_t lb, uint64_t o0,
                                             unsigned char* smem) {
    const int tid = threadIdx.x;
    K* sk = reinterpret_cast<K*>(smem);
    VV* sv = reinterpret_cast<VV*>(smem + LDS_KEYS);
    const uint32_t total = la + lb;
    // coalesced staging of both pieces, A then B: all IPT loads of a thread
    // are issued before any of them is waited on
    if (total == uint32_t(TM)) {  // full tile (workgroup-uniform): no predicates
      K kv[IPT];
      VV vv[PAIRS ? IPT : 1];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = uint32_t(tid) + uint32_t(r) * WG;
        const uint64_t g = e < la ? a0 + e : b0 + (e - la);
        kv[r] = src_k[g];
        if constexpr (PAIRS) vv[r] = src_v[g];
      }
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = uint32_t(tid) + uint32_t(r) * WG;
        sk[lds_pad<PAD>(e)] = kv[r];
        if constexpr (PAIRS) sv[lds_pad<PAD>(e)] = vv[r];
      }
    } else {
      K kv[IPT];
      VV vv[PAIRS ? IPT : 1];
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = uint32_t(tid) + uint32_t(r) * WG;
        if (e < total) {
          const uint64_t g = e < la ? a0 + e : b0 + (e - la);
          kv[r] = src_k[g];
          if constexpr (PAIRS) vv[r] = src_v[g];
        }
      }
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        const uint32_t e = uint32_t(tid) + uint32_t(r) * WG;
        if (e < total) {
          sk[lds_pad<PAD>(e)] = kv[r];
          if constexpr (PAIRS) sv[lds_pad<PAD>(e)] = vv[r];
        }
      }
    }
    __syncthreads();
    const uint32_t d = uint32_t(tid) * IPT;
    if (d >= total) return;
    // A is sk[0, la), B is sk[la, total), both through lds_pad
    uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
    while (lo < hi) {
      const uint32_t m = (lo + hi) >> 1;
      if (sk[lds_pad<PAD>(la + d - 1 - m)] < sk[lds_pad<PAD>(m)]) hi = m; else lo = m + 1;
    }
    uint32_t i = lo, j = d - lo;
    const uint32_t last = total - 1;
    K a = sk[lds_pad<PAD>(i < last ? i : last)];
    K b = sk[lds_pad<PAD>(la + j < last ? la + j : last)];
    K ko[IPT];
    uint32_t src_idx[IPT];
    // branch-free serial merge: one LDS read per output, at the index of the
    // side that was just consumed
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const bool take_b = (j < lb) && (i >= la || b < a);
      ko[r] = take_b ? b : a;
      src_idx[r] = take_b ? la + j : i;
      i += take_b ? 0u : 1u;
      j += take_b ? 1u : 0u;
      const uint32_t nx = take_b ? la + j : i;
      const K x = sk[lds_pad<PAD>(nx < last ? nx : last)];
      a = take_b ? a : x;
      b = take_b ? x : b;
    }
    const uint32_t cnt = total - d < uint32_t(IPT) ? total - d : uint32_t(IPT);
    K* out = dst_k + o0 + d;
    if (cnt == IPT && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
      store_run<K, IPT>(out, ko);
    } else {
#pragma unroll
      for (int r = 0; r < IPT; ++r)
        if (uint32_t(r) < cnt) out[r] = ko[r];
    }
    if constexpr (PAIRS) {
      VV vo[IPT];
#pragma unroll
      for (int r = 0; r < IPT; ++r) vo[r] = sv[lds_pad<PAD>(src_idx[r] < last ? src_idx[r] : last)];
      VV* ov = dst_v + o0 + d;
      if (cnt == IPT && (reinterpret_cast<uintptr_t>(ov) & 15) == 0) {
        store_run<VV, IPT>(ov, vo);
      } else {
#pragma unroll
        for (int r = 0; r < IPT; ++r)
          if (uint32_t(r) < cnt) ov[r] = vo[r];
      }
    }
  }
};

template <class K, class V, int WG, int IPT, int PAD>
__global__ __launch_bounds__(WG) void merge_kernel(const K* __restrict__ src_k, const V* __restrict__ src_v,
                                                   K* __restrict__ dst_k, V* __restrict__ dst_v,
                                                   uint64_t n_host, DevCtl ctl, uint64_t W,
                                                   const int64_t* __restrict__ part) {
  using MT = MergeTile<K, V, WG, IPT, PAD>;
  extern __shared__ __align__(16) unsigned char smem[];
  if (gated_off(ctl)) return;
  const uint64_t n = live_n(ctl, n_host);
  // workgroup b merges tiles b, b + grid, ... (one each when the grid covers them)
  for (uint64_t k = blockIdx.x; k * MT::TM < n; k += gridDim.x) {
    const uint64_t g0 = k * MT::TM;
    const uint64_t g1 = g0 + MT::TM < n ? g0 + MT::TM : n;
    const PassGeom q = pass_geom(g0, n, W, ctl);
    const uint64_t i0 = uint64_t(part[k]);
    const uint64_t j0 = q.a_end + (g0 - q.pb) - (i0 - q.pb);
    uint64_t i1, j1;
    if (g1 == q.b_end) {
      i1 = q.a_end;
      j1 = q.b_end;
    } else {
      i1 = uint64_t(part[k + 1]);
      j1 = q.a_end + (g1 - q.pb) - (i1 - q.pb);
    }
    if constexpr (MT::PAIRS) {
      MT::run(src_k, src_v, dst_k, dst_v, i0, uint32_t(i1 - i0), j0, uint32_t(j1 - j0), g0, smem);
    } else {
      MT::template run<int>(src_k, nullptr, dst_k, nullptr, i0, uint32_t(i1 - i0), j0, uint32_t(j1 - j0), g0,
                            smem);
    }
    __syncthreads();
  }
}

}  // namespace ms

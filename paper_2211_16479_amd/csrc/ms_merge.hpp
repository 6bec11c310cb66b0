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

// W, the run width of a pass, is the tile size times 2^level: a power of two
// (a merge of two runs of arbitrary length goes through the device-side
// split below instead).
__device__ __forceinline__ PassGeom pass_geom(uint64_t g, uint64_t n, uint64_t W) {
  PassGeom q;
  q.pb = g & ~(2 * W - 1);
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

// G lanes (a power of two dividing 64) share one search: in every round the
// group probes positions of its interval [lo, lo + len) -- all of them when
// len <= G, otherwise G evenly spaced ones -- and a ballot gives the first
// probe whose predicate holds.  probe_pos is lane q's position; the group
// helpers below are called by every lane of the group at the same time.
template <int G>
__device__ __forceinline__ uint64_t probe_pos(uint64_t lo, uint64_t len, uint32_t q) {
  return len <= uint64_t(G) ? lo + q : lo + ((uint64_t(q) + 1) * len) / (G + 1);
}
template <int G>
__device__ __forceinline__ uint64_t group_ballot(bool pred, uint32_t gshift) {
  return (__ballot(pred) >> gshift) & (G == 64 ? ~0ull : ((1ull << G) - 1));
}
__device__ __forceinline__ uint64_t lane_value(uint64_t v, uint32_t src_lane) {
  return uint64_t(__shfl(static_cast<unsigned long long>(v), int(src_lane), 64));
}

// The keys around a two-run split i at diagonal d of pair q (merge tile k):
// head[k] = the pair's merged output at d (the smaller of the two next
// elements), tail[k] = the output just before it (the larger of the two last
// taken; left unwritten at d = 0).  d < the pair's length, so at least one
// next element exists; the index fallbacks only ever name existing elements.
template <class K>
__device__ __forceinline__ void record_split_keys(const K* __restrict__ src, const PassGeom& q, uint64_t d,
                                                  uint64_t i, uint64_t k, K* __restrict__ head,
                                                  K* __restrict__ tail) {
  const uint64_t la = q.a_end - q.pb, lb = q.b_end - q.a_end;
  const bool na = i < la, nb = d - i < lb;
  const K x0 = src[na ? q.pb + i : q.a_end + (d - i)];
  const K x1 = src[nb ? q.a_end + (d - i) : q.pb + i];
  head[k] = x1 < x0 ? x1 : x0;
  const bool pa = i >= 1, pbv = d - i >= 1;
  if (pa || pbv) {
    const K y0 = src[pa ? q.pb + i - 1 : q.a_end + (d - i) - 1];
    const K y1 = src[pbv ? q.a_end + (d - i) - 1 : q.pb + i - 1];
    tail[k] = y0 < y1 ? y1 : y0;
  }
}

// The split of merge tile k (start g = k*Tm < n) of its pair, written to
// part[k], and with head / tail non-null the keys around it.  A group of G
// lanes (lane q, group's first lane gshift) shares the search: each round
// probes G positions of the remaining interval (all of them once it is at
// most G long) and a ballot picks the sub-interval holding the split, which
// is the first m with B[d-1-m] < A[m].  G = 1 is the binary search.
template <class K, int G>
__device__ __forceinline__ void partition_group(const K* __restrict__ src, uint64_t n, uint64_t W, uint32_t Tm,
                                                uint64_t k, const DevCtl& ctl, uint32_t q, uint32_t gshift,
                                                int64_t* __restrict__ part, K* __restrict__ head,
                                                K* __restrict__ tail) {
  const uint64_t g = k * Tm;
  const PassGeom geo = pass_geom(g, n, W, ctl);
  const uint64_t la = geo.a_end - geo.pb, lb = geo.b_end - geo.a_end, d = g - geo.pb;
  const K* A = src + geo.pb;
  const K* B = src + geo.a_end;
  uint64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  if constexpr (G == 1) {
    lo = merge_path_split(A, la, B, lb, d);
  } else {
    while (lo < hi) {  // the same bounds in every lane of the group
      const uint64_t len = hi - lo;
      const uint64_t m = probe_pos<G>(lo, len, q);  // lo <= m < hi
      const bool pred = (len > uint64_t(G) || q < len) && (B[d - 1 - m] < A[m]);
      const uint64_t gm = group_ballot<G>(pred, gshift);
      if (len <= uint64_t(G)) {
        lo = hi = gm ? lo + uint64_t(__builtin_ctzll(gm)) : hi;
      } else if (gm == 0) {
        lo = probe_pos<G>(lo, len, G - 1) + 1;
      } else {
        const uint32_t f = uint32_t(__builtin_ctzll(gm));
        hi = probe_pos<G>(lo, len, f);
        lo = f ? probe_pos<G>(lo, len, f - 1) + 1 : lo;
      }
    }
  }
  if (q == 0) {
    part[k] = int64_t(geo.pb + lo);
    if (head) record_split_keys(src, geo, d, lo, k, head, tail);
  }
}

// One search per merge tile, G lanes each; the loop keeps a wavefront's
// lanes together so that the group ballots see every lane of the group.
template <class K, int G>
__global__ __launch_bounds__(256) void partition_kernel(const K* __restrict__ src, uint64_t n_host, DevCtl ctl,
                                                        uint64_t W, uint32_t Tm, uint64_t num_tiles,
                                                        int64_t* __restrict__ part, K* __restrict__ head = nullptr,
                                                        K* __restrict__ tail = nullptr) {
  static_assert(G >= 1 && G <= 64 && (64 % G) == 0, "group size");
  const int gw = gate_word(ctl);
  if ((gw & 1) == 0) return;
  src = swap_set(ctl, gw) ? global_ptr<const K>(&ctl.other) : rebind(src, ctl.keys);
  const uint64_t n = live_n(ctl, n_host);
  const uint32_t q = threadIdx.x % G, gshift = (__lane_id() / G) * G;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t base = uint64_t(blockIdx.x) * blockDim.x; base < num_tiles * G; base += stride) {
    const uint64_t k = (base + threadIdx.x) / G;
    if (k < num_tiles && k * Tm < n) partition_group<K, G>(src, n, W, Tm, k, ctl, q, gshift, part, head, tail);
  }
}

// Stage 0 of a merge tile made of NP pieces laid back to back in the tile:
// element e (0 <= e < c[NP]) is src[D[p] + e] for c[p] <= e < c[p+1]
// (c[0] = 0; D[p] = piece start - c[p], unsigned wrap-around intended).
// Thread tid stages elements e = tid + r*WG into LDS slot e.  The 64
// consecutive elements a wavefront loads in one step usually lie in one
// piece: the piece is then picked once per wavefront, in scalar registers,
// and the loads are base[lane]; only a chunk that crosses a piece boundary
// or the tile's end picks the piece per lane.  All IPT loads of a thread are
// issued before the first LDS write waits on them.  Slots at or past c[NP]
// receive unspecified values and are never read.
// GAPS > 0 leaves GAPS slots after every piece: element e of piece p goes to
// slot e + p * GAPS, and an element past the tile (e >= c[NP]) to slot
// e + NP * GAPS, beyond the last piece's gap.
template <int NP, int WG, int IPT, int PAD, bool PAIRS, int GAPS = 0, class K, class VV>
__device__ __forceinline__ void stage_pieces(const K* __restrict__ src_k, const VV* __restrict__ src_v,
                                             const uint64_t (&D)[NP], const uint32_t (&c)[NP + 1],
                                             K* __restrict__ sk, VV* __restrict__ sv) {
  static_assert(WG % 64 == 0, "whole wavefronts");
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t wbase = wave_uniform(tid & ~63u);
  K kv[IPT];
  VV vv[PAIRS ? IPT : 1];
  uint32_t gofs[GAPS ? IPT : 1];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint32_t cb = wbase + uint32_t(r) * WG;  // the wavefront's first element of this step
    uint32_t pend = c[1];
    uint64_t Dp = D[0];
    uint32_t gp = 0;
#pragma unroll
    for (int k = 1; k < NP; ++k) {
      if (cb >= c[k]) {
        pend = c[k + 1];
        Dp = D[k];
        gp = uint32_t(k) * GAPS;
      }
    }
    if (cb + 63u < pend) {  // wavefront-uniform: the chunk is inside one piece
      kv[r] = (src_k + (Dp + cb))[lane];
      if constexpr (PAIRS) vv[r] = (src_v + (Dp + cb))[lane];
      if constexpr (GAPS > 0) gofs[r] = gp;
    } else {
      const uint32_t e = cb + lane;
      if (e < c[NP]) {
        uint64_t De = D[0];
#pragma unroll
        for (int k = 1; k < NP; ++k) De = e >= c[k] ? D[k] : De;
        kv[r] = src_k[De + e];
        if constexpr (PAIRS) vv[r] = src_v[De + e];
      }
      if constexpr (GAPS > 0) {
        uint32_t g = 0;
#pragma unroll
        for (int k = 1; k <= NP; ++k) g += e >= c[k] ? uint32_t(GAPS) : 0u;
        gofs[r] = g;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint32_t e = tid + uint32_t(r) * WG;
    if constexpr (GAPS > 0) {
      sk[lds_pad<PAD>(e + gofs[r])] = kv[r];
    } else {
      sk[lds_pad<PAD>(e)] = kv[r];
      if constexpr (PAIRS) sv[lds_pad<PAD>(e)] = vv[r];
    }
  }
}

// Stage 0 of the padded-run form for a tile whose pieces lie within 2^32
// bytes of the first: per lane, in vector registers, with 32-bit offsets
// from the first piece's base (no per-chunk scalar piece selection).
// Element e of piece p (c[p] <= e < c[p+1]) is base[inc[1] + ... + inc[p] + e]
// (inc[k] = D[k] - D[k-1] >= 0) and goes to slot e + p * GAPS; elements past
// the tile go to slot e + 4 * GAPS and are not loaded.
template <int WG, int IPT, int PAD, int GAPS, class K>
__device__ __forceinline__ void stage_pieces_rel(const K* __restrict__ base, const uint32_t (&inc)[4],
                                                 const uint32_t (&c)[5], K* __restrict__ sk) {
  const uint32_t tid = threadIdx.x;
  K kv[IPT];
  auto load = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;  // a whole tile: every element is loaded
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const uint32_t e = tid + uint32_t(r) * WG;
      uint32_t off = e;
#pragma unroll
      for (int k = 1; k < 4; ++k) off += e >= c[k] ? inc[k] : 0u;
      if constexpr (FULL) kv[r] = base[off];
      else kv[r] = e < c[4] ? base[off] : K(0);
    }
  };
  if (c[4] == uint32_t(WG * IPT)) load(std::true_type{}); else load(std::false_type{});
  // slots recomputed here rather than kept from the loads (registers)
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint32_t e = tid + uint32_t(r) * WG;
    uint32_t sl = e;
#pragma unroll
    for (int k = 1; k <= 4; ++k) sl += e >= c[k] ? uint32_t(GAPS) : 0u;
    sk[lds_pad<PAD>(sl)] = kv[r];
  }
}

// Keys-only serial merge of IPT outputs from two runs of s[] that are each
// followed by at least IPT + 1 slots holding the type's largest key: the
// current elements are s[ia] and s[jb], the second run's wins only when
// strictly smaller.  After a run is used up its current element is that
// largest key, which loses to every smaller key; against an equal key either
// choice writes the same value (every output still to come is that key), so
// the loop tests no bounds.  Reads stay within IPT + 1 slots past a run's end.
template <int IPT, int PAD, class K>
__device__ __forceinline__ void merge_run_sentinel(const K* __restrict__ s, uint32_t ia, uint32_t jb,
                                                   K (&ko)[IPT]) {
  K a = s[lds_pad<PAD>(ia)], b = s[lds_pad<PAD>(jb)];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const bool tb = b < a;
    ko[r] = tb ? b : a;
    const uint32_t nx = (tb ? jb : ia) + 1u;
    const K x = s[lds_pad<PAD>(nx)];
    ia = tb ? ia : nx;
    jb = tb ? nx : jb;
    a = tb ? a : x;
    b = tb ? x : b;
  }
}

// Merge-path split at diagonal d of merge(s[pa, pa + la), s[pb, pb + lb))
// (the first run wins ties): the number of its elements among the first d
// outputs.
template <int PAD, class K>
__device__ __forceinline__ uint32_t lds_split(const K* __restrict__ s, uint32_t pa, uint32_t la, uint32_t pb,
                                              uint32_t lb, uint32_t d) {
  uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint32_t m = (lo + hi) >> 1;
    if (s[lds_pad<PAD>(pb + d - 1 - m)] < s[lds_pad<PAD>(pa + m)]) hi = m; else lo = m + 1;
  }
  return lo;
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
    // coalesced staging of both pieces, A then B
    {
      const uint64_t D[2] = {a0, b0 - la};
      const uint32_t c[3] = {0u, la, total};
      stage_pieces<2, WG, IPT, PAD, PAIRS>(src_k, src_v, D, c, sk, sv);
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
  const int gw = gate_word(ctl);
  if ((gw & 1) == 0) return;
  src_k = rebind(src_k, ctl.keys);
  dst_k = rebind(dst_k, ctl.keys);
  {
    const K* sk0 = src_k;
    K* dk0 = dst_k;
    if (swap_set(ctl, gw)) {
      src_k = dk0;
      dst_k = const_cast<K*>(sk0);
      const V* sv0 = src_v;
      src_v = dst_v;
      dst_v = const_cast<V*>(sv0);
    }
  }
  const uint64_t n = live_n(ctl, n_host);
  // workgroup b merges tiles b, b + grid, ... (one each when the grid covers them)
  for (uint64_t k = blockIdx.x; k * MT::TM < n; k += gridDim.x) {
    const uint64_t g0 = k * MT::TM;
    const uint64_t g1 = g0 + MT::TM < n ? g0 + MT::TM : n;
    const PassGeom q = pass_geom(g0, n, W, ctl);
    const uint64_t i0 = wave_uniform(uint64_t(part[k]));
    const uint64_t j0 = q.a_end + (g0 - q.pb) - (i0 - q.pb);
    uint64_t i1, j1;
    if (g1 == q.b_end) {
      i1 = q.a_end;
      j1 = q.b_end;
    } else {
      i1 = wave_uniform(uint64_t(part[k + 1]));
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

// ---------------------------------------------------------------------------
// Fused two-level passes.
//
// Two adjacent levels of the merge tree in one HBM round trip: runs R0..R3 of
// width W (a "quad", clipped to n) become one run of width 4W, computed as
// merge(X, Y) with X = merge(R0, R1) and Y = merge(R2, R3) -- the same two
// tree levels as two passes, so the output is bit-identical (left wins ties
// at both levels), but every element is read and written once instead of
// twice.  A fused pass is three kernels:
//   1. partition_kernel at width W: for every merge tile, the split of its
//      pair at that diagonal (samples of X and Y every Tm outputs);
//   2. partition4_kernel: for every output tile start d of merge(X, Y), the
//      split x of the output between X and Y (a search whose probes need
//      X[m] and Y[p]: O(1) at the samples, one bounded search each in
//      between), and from it the start offsets in R0..R3;
//   3. merge4_kernel: stages the four pieces in LDS, merges R0|R1 and R2|R3
//      in LDS, then the two results, and stores coalesced.

struct QuadGeom {
  uint64_t qb, r1, r2, r3, end;  // starts of R0..R3 and the quad's end
};

__device__ __forceinline__ QuadGeom quad_geom(uint64_t g, uint64_t n, uint64_t W) {
  QuadGeom q;
  q.qb = g & ~(4 * W - 1);  // W is a power of two
  q.r1 = q.qb + W < n ? q.qb + W : n;
  q.r2 = q.qb + 2 * W < n ? q.qb + 2 * W : n;
  q.r3 = q.qb + 3 * W < n ? q.qb + 3 * W : n;
  q.end = q.qb + 4 * W < n ? q.qb + 4 * W : n;
  return q;
}

// Merge-path split at diagonal d of merge(P, Q) (P = src[p0 ...),
// Q = src[q0 ...), P wins ties), searched in [lo, hi], which the caller
// knows to hold it.
template <class K>
__device__ __forceinline__ uint64_t split_in(const K* __restrict__ src, uint64_t p0, uint64_t q0, uint64_t d,
                                             uint64_t lo, uint64_t hi) {
  while (lo < hi) {
    const uint64_t m = (lo + hi) >> 1;
    if (src[q0 + d - 1 - m] < src[p0 + m]) hi = m; else lo = m + 1;
  }
  return lo;
}

// A merge-path split f (f(d) = how many of the first d outputs come from the
// first run) is non-decreasing and so is d - f(d).  Known exactly at dL <= d
// <= dR, it is bounded at d by [max(fL, fR - (dR - d)), min(fR, fL + (d - dL))],
// and always by [max(0, d - lq), min(d, lp)].
struct Bracket {
  uint64_t dL, fL, dR, fR;
  __device__ __forceinline__ void bounds(uint64_t d, uint64_t lp, uint64_t lq, uint64_t* lo, uint64_t* hi) const {
    uint64_t a = fR > dR - d ? fR - (dR - d) : 0;
    a = a > fL ? a : fL;
    const uint64_t g = d > lq ? d - lq : 0;
    *lo = a > g ? a : g;
    uint64_t b = fL + (d - dL);
    b = b < fR ? b : fR;
    *hi = b < d ? (b < lp ? b : lp) : (d < lp ? d : lp);
  }
};

// Split of a pair at a diagonal that is a multiple of Tm (read from the
// two-run partition) or the pair's full length.
__device__ __forceinline__ uint64_t split_at_sample(const int64_t* __restrict__ part, uint64_t p0, uint64_t lp,
                                                    uint64_t L, uint32_t Tm, uint64_t d) {
  return d >= L ? lp : uint64_t(part[(p0 + d) / Tm]) - p0;
}

// For every output tile k (start g = k*Tm < n) of the fused pass at width
// W: the start offsets of its pieces of R0..R3, written as four global
// indices to part4[4k .. 4k+3].  A group of G lanes per tile (lane q,
// group's first lane gshift).  x = the number of X elements among the first
// dl outputs of merge(X, Y) is the first m with Y[dl-1-m] < X[m] (X wins
// ties).
//   coarse: over the sample diagonals m = j*Tm, where X[m] and Y[dl-m-1]
//           are the recorded head and tail keys (one load each per probe);
//   fine:   inside the remaining sample interval; a probe at m finds the
//           R0/R1 split at m and the R2/R3 split at dl - m by searches
//           bounded by the exact splits at the interval ends (brackets);
//           the splits found at the probes next to the chosen
//           sub-interval become its brackets, so later searches are short.
template <class K, int G>
__device__ __forceinline__ void partition4_group(const K* __restrict__ src, uint64_t n, uint64_t W, uint32_t Tm,
                                                 uint64_t k, uint32_t q, uint32_t gshift,
                                                 const int64_t* __restrict__ part, const K* __restrict__ head,
                                                 const K* __restrict__ tail, int64_t* __restrict__ part4) {
  const QuadGeom Q = quad_geom(k * Tm, n, W);
  const uint64_t la = Q.r1 - Q.qb, lb = Q.r2 - Q.r1, lc = Q.r3 - Q.r2, ld = Q.end - Q.r3;
  const uint64_t lx = la + lb, ly = lc + ld;
  const uint64_t dl = k * Tm - Q.qb;
  uint64_t lo = dl > ly ? dl - ly : 0, hi = dl < lx ? dl : lx;
  // coarse: J = the first sample index j in [j0, j1) whose predicate holds
  // (j1 if none); then x lies in ((J-1)*Tm, J*Tm] clipped to [lo, hi]
  {
    const uint64_t j0 = (lo + Tm - 1) / Tm, j1 = (hi + Tm - 1) / Tm;
    uint64_t jlo = j0, jhi = j1;
    while (jlo < jhi) {
      const uint64_t len = jhi - jlo;
      const uint64_t j = probe_pos<G>(jlo, len, q);
      bool pred = false;
      if (len > uint64_t(G) || q < len) {
        const uint64_t m = j * Tm, p = dl - m;  // lo <= m < hi, so 1 <= p <= ly
        const K xk = head[(Q.qb + m) / Tm];
        K yk;
        if (p < ly) {
          yk = tail[(Q.r2 + p) / Tm];
        } else {  // the last element of Y
          const K c = src[lc ? Q.r3 - 1 : Q.end - 1];
          const K e = src[ld ? Q.end - 1 : Q.r3 - 1];
          yk = c < e ? e : c;
        }
        pred = yk < xk;
      }
      const uint64_t gm = group_ballot<G>(pred, gshift);
      if (len <= uint64_t(G)) {
        jlo = jhi = gm ? jlo + uint64_t(__builtin_ctzll(gm)) : jhi;
      } else if (gm == 0) {
        jlo = probe_pos<G>(jlo, len, G - 1) + 1;
      } else {
        const uint32_t f = uint32_t(__builtin_ctzll(gm));
        jhi = probe_pos<G>(jlo, len, f);
        jlo = f ? probe_pos<G>(jlo, len, f - 1) + 1 : jlo;
      }
    }
    const uint64_t wlo = jlo > j0 ? (jlo - 1) * Tm + 1 : lo;
    const uint64_t whi = jlo < j1 ? jlo * Tm : hi;
    lo = wlo;
    hi = whi;
  }
  // fine: [lo, hi] lies inside [mL, mL + Tm]
  const uint64_t mL = (lo / Tm) * Tm;
  const uint64_t mR = mL + Tm < lx ? mL + Tm : lx;
  Bracket bx{mL, split_at_sample(part, Q.qb, la, lx, Tm, mL), mR, split_at_sample(part, Q.qb, la, lx, Tm, mR)};
  const uint64_t pR = dl - mL < ly ? dl - mL : ly;
  const uint64_t pL = dl > mL + Tm ? dl - mL - Tm : 0;
  Bracket by{pL, split_at_sample(part, Q.r2, lc, ly, Tm, pL), pR, split_at_sample(part, Q.r2, lc, ly, Tm, pR)};
  while (lo < hi) {
    const uint64_t len = hi - lo;
    const uint64_t m = probe_pos<G>(lo, len, q);
    uint64_t sx = 0, ty = 0;
    bool pred = false;
    if (len > uint64_t(G) || q < len) {
      const uint64_t p = dl - m;
      uint64_t a0, a1, c0, c1;
      bx.bounds(m, la, lb, &a0, &a1);
      by.bounds(p, lc, ld, &c0, &c1);
      sx = split_in(src, Q.qb, Q.r1, m, a0, a1);
      ty = split_in(src, Q.r2, Q.r3, p, c0, c1);
      // X[m]: the smaller next element; Y[p-1]: the larger last taken one
      const bool xa = sx < la, xb = m - sx < lb;
      const K ka = src[xa ? Q.qb + sx : Q.r1 + (m - sx)];
      const K kb = src[xb ? Q.r1 + (m - sx) : Q.qb + sx];
      const K xk = kb < ka ? kb : ka;
      const bool yc = ty >= 1, yd = p - ty >= 1;
      const K kc = src[yc ? Q.r2 + ty - 1 : Q.r3 + (p - ty) - 1];
      const K kd = src[yd ? Q.r3 + (p - ty) - 1 : Q.r2 + ty - 1];
      const K yk = kc < kd ? kd : kc;
      pred = yk < xk;
    }
    const uint64_t gm = group_ballot<G>(pred, gshift);
    // the probe chosen as the new right end (first true), and the one
    // before it as the new left end (last true: the last probe)
    const uint32_t f = gm ? uint32_t(__builtin_ctzll(gm)) : uint32_t(G);
    const uint32_t fr = f < G ? f : G - 1;
    const uint32_t fl = f ? f - 1 : 0;
    const uint64_t sxr = lane_value(sx, gshift + fr), tyr = lane_value(ty, gshift + fr);
    const uint64_t sxl = lane_value(sx, gshift + fl), tyl = lane_value(ty, gshift + fl);
    if (len <= uint64_t(G)) {
      // every position was probed: x is the first true one, else hi
      if (gm) {
        const uint64_t x = lo + f;
        bx = Bracket{x, sxr, x, sxr};
        by = Bracket{dl - x, tyr, dl - x, tyr};
        lo = hi = x;
      } else {
        lo = hi;
      }
    } else {
      if (gm) {
        const uint64_t mr = probe_pos<G>(lo, len, f);
        bx.dR = mr;
        bx.fR = sxr;
        by.dL = dl - mr;
        by.fL = tyr;
        hi = mr;
      }
      if (f) {
        const uint64_t ml = probe_pos<G>(lo, len, fl);
        bx.dL = ml;
        bx.fL = sxl;
        by.dR = dl - ml;
        by.fR = tyl;
        lo = ml + 1;
      }
    }
  }
  const uint64_t x = lo;
  uint64_t a0, a1, c0, c1;
  bx.bounds(x, la, lb, &a0, &a1);
  by.bounds(dl - x, lc, ld, &c0, &c1);
  const uint64_t a = split_in(src, Q.qb, Q.r1, x, a0, a1);
  const uint64_t c = split_in(src, Q.r2, Q.r3, dl - x, c0, c1);
  if (q == 0) {
    part4[4 * k + 0] = int64_t(Q.qb + a);
    part4[4 * k + 1] = int64_t(Q.r1 + (x - a));
    part4[4 * k + 2] = int64_t(Q.r2 + c);
    part4[4 * k + 3] = int64_t(Q.r3 + (dl - x - c));
  }
}

// G lanes per output tile; the loop keeps a wavefront's lanes together so
// that the group ballots see every lane of the group.
template <class K, int G>
__global__ __launch_bounds__(256) void partition4_kernel(const K* __restrict__ src, uint64_t n_host, DevCtl ctl,
                                                         uint64_t W, uint32_t Tm, uint64_t num_tiles,
                                                         const int64_t* __restrict__ part,
                                                         const K* __restrict__ head, const K* __restrict__ tail,
                                                         int64_t* __restrict__ part4) {
  static_assert(G >= 1 && G <= 64 && (64 % G) == 0, "group size");
  const int gw = gate_word(ctl);
  if ((gw & 1) == 0) return;
  src = swap_set(ctl, gw) ? global_ptr<const K>(&ctl.other) : rebind(src, ctl.keys);
  const uint64_t n = live_n(ctl, n_host);
  const uint32_t q = threadIdx.x % G, gshift = (__lane_id() / G) * G;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t base = uint64_t(blockIdx.x) * blockDim.x; base < num_tiles * G; base += stride) {
    const uint64_t k = (base + threadIdx.x) / G;
    if (k < num_tiles && k * Tm < n) partition4_group<K, G>(src, n, W, Tm, k, q, gshift, part, head, tail, part4);
  }
}

template <class K, class V, int WG, int IPT, int PAD, int REUSE>
struct Merge4Tile {
  static constexpr bool PAIRS = HasVal<V>::value;
  using VV = typename std::conditional<PAIRS, V, int>::type;
  static constexpr int TM = WG * IPT;
  static_assert(TM <= 65536, "buffer-1 positions are 16-bit");
  static constexpr uint32_t SLOTS = lds_padded_size<PAD>(TM);
  static constexpr size_t al16(size_t b) { return (b + 15) / 16 * 16; }
  static constexpr size_t K1_OFF = 0;
  static constexpr size_t V1_OFF = al16(sizeof(K) * SLOTS);
  static constexpr size_t K2_OFF = V1_OFF + (PAIRS ? al16(sizeof(VV) * SLOTS) : 0);
  static constexpr size_t I2_OFF = K2_OFF + (REUSE ? 0 : al16(sizeof(K) * SLOTS));
  static constexpr size_t LDS_BYTES_BOUNDED = I2_OFF + (PAIRS ? al16(sizeof(uint16_t) * SLOTS) : 0);
  // Keys only with separate stage buffers (REUSE = 0): the sentinel form
  // below.  GAP slots of the largest key follow each of the four pieces
  // (buffer 1) and each stage-1 result (buffer 2); GAP >= IPT + 1 and a
  // multiple of 16 bytes, so that the second result stays vector-aligned.
  // (With REUSE the straddling thread would have to hold two output sets
  // across the barrier, which costs 64-bit keys occupancy: those keep the
  // bounded form.)
  static constexpr bool SENTINEL = !PAIRS && !REUSE;
  static constexpr uint32_t GAP = uint32_t(((IPT + 1) * sizeof(K) + 15) / 16 * 16 / sizeof(K));
  static constexpr uint32_t SLOTS1 = lds_padded_size<PAD>(TM + 4 * GAP);
  static constexpr uint32_t SLOTS2 = lds_padded_size<PAD>(TM + 2 * GAP);
  static constexpr size_t KK2_OFF = al16(sizeof(K) * SLOTS1);
  static constexpr size_t LDS_BYTES_SENTINEL = KK2_OFF + al16(sizeof(K) * SLOTS2);
  static constexpr size_t LDS_BYTES = SENTINEL ? LDS_BYTES_SENTINEL : LDS_BYTES_BOUNDED;

  // Keys only, REUSE = 0.  Buffer 1 holds P0..P3 at o[p] = c[p] + p * GAP, each followed
  // by GAP largest keys; X = merge(P0, P1) goes to buffer 2 at [0, c2) and
  // Y = merge(P2, P3) at [c2 + GAP, total + GAP), each followed by GAP largest
  // keys.  Thread t owns outputs e0 = t * IPT .. e0 + IPT of X|Y in stage 1
  // and of merge(X, Y) in stage 2; outputs it computes past its run's end are
  // largest keys and land in that run's gap.  The one thread whose stage-1
  // outputs straddle c2 also computes Y's first IPT outputs (the next thread
  // writes the same values to the ones it owns).
  static __device__ __forceinline__ void run_keys(const K* __restrict__ src_k, K* __restrict__ dst_k,
                                                  const uint64_t (&s)[4], const uint32_t (&l)[4], uint64_t o0,
                                                  unsigned char* smem) {
    const uint32_t tid = threadIdx.x;
    K* k1 = reinterpret_cast<K*>(smem);
    K* k2 = reinterpret_cast<K*>(smem + KK2_OFF);
    const uint32_t c1 = l[0], c2 = c1 + l[1], c3 = c2 + l[2], total = c3 + l[3];
    const uint32_t o1 = c1 + GAP, o2 = c2 + 2 * GAP, o3 = c3 + 3 * GAP;
    const K SENT = key_max<K>();
    // stage 0: P0..P3 into buffer 1, then the gaps
    {
      const uint64_t D[4] = {s[0], s[1] - c1, s[2] - c2, s[3] - c3};
      const uint32_t c[5] = {0u, c1, c2, c3, total};
      if ((D[3] - D[0] + uint64_t(TM)) * sizeof(K) < (uint64_t(1) << 32)) {
        const uint32_t inc[4] = {0u, uint32_t(D[1] - D[0]), uint32_t(D[2] - D[1]), uint32_t(D[3] - D[2])};
        stage_pieces_rel<WG, IPT, PAD, GAP>(src_k + D[0], inc, c, k1);
      } else {
        stage_pieces<4, WG, IPT, PAD, false, GAP>(src_k, static_cast<const int*>(nullptr), D, c, k1,
                                                  static_cast<int*>(nullptr));
      }
      const uint32_t ce[4] = {c1, c2, c3, total};
      for (uint32_t g = tid; g < 4 * GAP; g += WG) {
        const uint32_t p = g / GAP;
        k1[lds_pad<PAD>(ce[p] + p * GAP + (g - p * GAP))] = SENT;
      }
      for (uint32_t g = tid; g < 2 * GAP; g += WG) k2[lds_pad<PAD>(g < GAP ? c2 + g : total + g)] = SENT;
    }
    __syncthreads();
    const uint32_t e0 = tid * IPT;
    // stage 1
    const bool second = e0 >= c2;
    const bool straddle = !second && c2 < e0 + IPT;
    K ko1[IPT], koy[IPT];
    if (e0 < total) {
      const uint32_t pa = second ? o2 : 0u, la = second ? l[2] : l[0];
      const uint32_t pb = second ? o3 : o1, lb = second ? l[3] : l[1];
      const uint32_t d = second ? e0 - c2 : e0;
      const uint32_t x = lds_split<PAD>(k1, pa, la, pb, lb, d);
      merge_run_sentinel<IPT, PAD>(k1, pa + x, pb + d - x, ko1);
      if (straddle) merge_run_sentinel<IPT, PAD>(k1, o2, o3, koy);
    }
    if (e0 < total) {
      const uint32_t w = second ? e0 + GAP : e0;  // buffer-2 slot of output e0
      if constexpr (PAD == 0 && (IPT * sizeof(K)) % 16 == 0 && (GAP * sizeof(K)) % 16 == 0) {
        store_run<K, IPT>(k2 + w, ko1);
      } else {
#pragma unroll
        for (int r = 0; r < IPT; ++r) k2[lds_pad<PAD>(w + r)] = ko1[r];
      }
      if (straddle) {
#pragma unroll
        for (int r = 0; r < IPT; ++r) k2[lds_pad<PAD>(c2 + GAP + r)] = koy[r];
      }
    }
    __syncthreads();
    // stage 2: merge(X, Y) -> global
    if (e0 >= total) return;
    const uint32_t x = lds_split<PAD>(k2, 0u, c2, c2 + GAP, total - c2, e0);
    K ko[IPT];
    merge_run_sentinel<IPT, PAD>(k2, x, c2 + GAP + (e0 - x), ko);
    const uint32_t cnt = total - e0 < uint32_t(IPT) ? total - e0 : uint32_t(IPT);
    K* out = dst_k + o0 + e0;
    if (cnt == IPT && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
      store_run<K, IPT>(out, ko);
    } else {
#pragma unroll
      for (int r = 0; r < IPT; ++r)
        if (uint32_t(r) < cnt) out[r] = ko[r];
    }
  }

  static __device__ __forceinline__ void run(const K* __restrict__ src_k, const VV* __restrict__ src_v,
                                             K* __restrict__ dst_k, VV* __restrict__ dst_v, const uint64_t (&s)[4],
                                             const uint32_t (&l)[4], uint64_t o0, unsigned char* smem) {
    if constexpr (SENTINEL) {
      run_keys(src_k, dst_k, s, l, o0, smem);
      return;
    }
    const uint32_t tid = threadIdx.x;
    K* k1 = reinterpret_cast<K*>(smem + K1_OFF);
    VV* v1 = reinterpret_cast<VV*>(smem + V1_OFF);
    K* k2 = reinterpret_cast<K*>(smem + (REUSE ? K1_OFF : K2_OFF));  // stage-1 results
    uint16_t* i2 = reinterpret_cast<uint16_t*>(smem + I2_OFF);
    const uint32_t c1 = l[0], c2 = c1 + l[1], c3 = c2 + l[2], total = c3 + l[3];
    // stage 0: P0|P1|P2|P3 into buffer 1
    {
      const uint64_t D[4] = {s[0], s[1] - c1, s[2] - c2, s[3] - c3};
      const uint32_t c[5] = {0u, c1, c2, c3, total};
      stage_pieces<4, WG, IPT, PAD, PAIRS>(src_k, src_v, D, c, k1, v1);
    }
    __syncthreads();
    const uint32_t e0 = tid * IPT;
    const uint32_t last = total ? total - 1 : 0;
    // stage 1
    K ko1[REUSE ? IPT : 1];
    uint16_t io1[(REUSE && PAIRS) ? IPT : 1];
    if (e0 < total) {
      // merge state: P = k1[pb, pb + lp), Q = k1[pb + lp, pb + lp + lq)
      const bool second = e0 >= c2;
      const uint32_t pb = second ? c2 : 0u;
      const uint32_t lp = second ? l[2] : l[0];
      const uint32_t lq = second ? l[3] : l[1];
      const uint32_t d = e0 - pb;
      uint32_t lo = d > lq ? d - lq : 0, hi = d < lp ? d : lp;
      while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (k1[lds_pad<PAD>(pb + lp + d - 1 - m)] < k1[lds_pad<PAD>(pb + m)]) hi = m; else lo = m + 1;
      }
      uint32_t i = pb + lo, j = pb + lp + (d - lo);
      uint32_t iend = pb + lp, jend = pb + lp + lq;
      K a = k1[lds_pad<PAD>(i < last ? i : last)];
      K b = k1[lds_pad<PAD>(j < last ? j : last)];
      // position where the second merge starts inside this thread's range
      const uint32_t sw = (!second && c2 > e0 && c2 < e0 + IPT) ? c2 - e0 : uint32_t(IPT);
#pragma unroll
      for (int r = 0; r < IPT; ++r) {
        if (uint32_t(r) == sw) {
          i = c2;
          iend = c3;
          j = c3;
          jend = total;
          a = k1[lds_pad<PAD>(i < last ? i : last)];
          b = k1[lds_pad<PAD>(j < last ? j : last)];
        }
        const uint32_t pos = e0 + uint32_t(r);
        if (pos < total) {
          const bool take_b = (j < jend) && (i >= iend || b < a);
          const uint32_t src = take_b ? j : i;
          if constexpr (REUSE) {
            ko1[r] = take_b ? b : a;
            if constexpr (PAIRS) io1[r] = uint16_t(src);
          } else {
            k2[lds_pad<PAD>(pos)] = take_b ? b : a;
            if constexpr (PAIRS) i2[lds_pad<PAD>(pos)] = uint16_t(src);
          }
          i += take_b ? 0u : 1u;
          j += take_b ? 1u : 0u;
          const uint32_t nx = take_b ? j : i;
          const K x = k1[lds_pad<PAD>(nx < last ? nx : last)];
          a = take_b ? a : x;
          b = take_b ? x : b;
        }
      }
    }
    if constexpr (REUSE) {
      __syncthreads();  // every stage-1 read of buffer 1's keys is done
      if (PAD == 0 && (IPT * sizeof(K)) % 16 == 0 && IPT % 8 == 0 && e0 + uint32_t(IPT) <= total) {
        // unpadded: a thread's IPT results are consecutive, written as 16-byte
        // vectors (scalar writes at a stride of IPT words conflict on banks)
        store_run<K, IPT>(k2 + e0, ko1);
        if constexpr (PAIRS) {
#pragma unroll
          for (int r = 0; r < IPT; r += 8) {
            uint4 w;
            w.x = uint32_t(io1[r]) | (uint32_t(io1[r + 1]) << 16);
            w.y = uint32_t(io1[r + 2]) | (uint32_t(io1[r + 3]) << 16);
            w.z = uint32_t(io1[r + 4]) | (uint32_t(io1[r + 5]) << 16);
            w.w = uint32_t(io1[r + 6]) | (uint32_t(io1[r + 7]) << 16);
            *reinterpret_cast<uint4*>(i2 + e0 + r) = w;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < IPT; ++r)
          if (e0 + uint32_t(r) < total) {
            k2[lds_pad<PAD>(e0 + r)] = ko1[r];
            if constexpr (PAIRS) i2[lds_pad<PAD>(e0 + r)] = io1[r];
          }
      }
    }
    __syncthreads();
    // stage 2: A = k2[0, c2), B = k2[c2, total)
    if (e0 >= total) return;
    const uint32_t la = c2, lb = total - c2, d = e0;
    uint32_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
    while (lo < hi) {
      const uint32_t m = (lo + hi) >> 1;
      if (k2[lds_pad<PAD>(la + d - 1 - m)] < k2[lds_pad<PAD>(m)]) hi = m; else lo = m + 1;
    }
    uint32_t i = lo, j = d - lo;
    K a = k2[lds_pad<PAD>(i < last ? i : last)];
    K b = k2[lds_pad<PAD>(la + j < last ? la + j : last)];
    K ko[IPT];
    uint32_t src_idx[IPT];
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      const bool take_b = (j < lb) && (i >= la || b < a);
      ko[r] = take_b ? b : a;
      src_idx[r] = take_b ? la + j : i;
      i += take_b ? 0u : 1u;
      j += take_b ? 1u : 0u;
      const uint32_t nx = take_b ? la + j : i;
      const K x = k2[lds_pad<PAD>(nx < last ? nx : last)];
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
      for (int r = 0; r < IPT; ++r) {
        const uint32_t p2 = src_idx[r] < last ? src_idx[r] : last;
        vo[r] = v1[lds_pad<PAD>(uint32_t(i2[lds_pad<PAD>(p2)]))];
      }
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

// Output tile k (k*TM < n) of a fused pass: a tile ends at the next tile's
// offsets or, for the quad's last tile, at the run ends.  Every thread of
// the workgroup calls it.
template <class MT, class K, class VV>
__device__ __forceinline__ void merge4_tile(const K* __restrict__ src_k, const VV* __restrict__ src_v,
                                            K* __restrict__ dst_k, VV* __restrict__ dst_v, uint64_t n, uint64_t W,
                                            uint64_t k, const int64_t* __restrict__ part4, unsigned char* smem) {
  const uint64_t g0 = k * MT::TM;
  const uint64_t g1 = g0 + MT::TM < n ? g0 + MT::TM : n;
  const QuadGeom Q = quad_geom(g0, n, W);
  uint64_t s[4], e[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) s[r] = wave_uniform(uint64_t(part4[4 * k + r]));
  if (g1 == Q.end) {
    e[0] = Q.r1;
    e[1] = Q.r2;
    e[2] = Q.r3;
    e[3] = Q.end;
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) e[r] = wave_uniform(uint64_t(part4[4 * (k + 1) + r]));
  }
  // offsets that do not describe four in-run pieces filling the tile are
  // never dereferenced: the tile is left unwritten and the error bit set
  // (exact partitions always pass)
  const uint64_t rs[4] = {Q.qb, Q.r1, Q.r2, Q.r3}, re[4] = {Q.r1, Q.r2, Q.r3, Q.end};
  bool ok = true;
  uint64_t sum = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    ok = ok && rs[r] <= s[r] && s[r] <= e[r] && e[r] <= re[r];
    sum += e[r] - s[r];
  }
  ok = ok && sum == g1 - g0;
  if (!ok && threadIdx.x == 0) raise_dev_error(DEV_ERR_MERGE_OFFSETS);
  uint32_t l[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) l[r] = ok ? uint32_t(e[r] - s[r]) : 0u;
  MT::run(src_k, src_v, dst_k, dst_v, s, l, g0, smem);
}

// Workgroup b merges output tiles b, b + grid, ...
template <class K, class V, int WG, int IPT, int PAD, int REUSE>
__global__ __launch_bounds__(WG) void merge4_kernel(const K* __restrict__ src_k, const V* __restrict__ src_v,
                                                    K* __restrict__ dst_k, V* __restrict__ dst_v, uint64_t n_host,
                                                    DevCtl ctl, uint64_t W, const int64_t* __restrict__ part4) {
  using MT = Merge4Tile<K, V, WG, IPT, PAD, REUSE>;
  using VV = typename MT::VV;
  extern __shared__ __align__(16) unsigned char smem[];
  const int gw = gate_word(ctl);
  if ((gw & 1) == 0) return;
  src_k = rebind(src_k, ctl.keys);
  dst_k = rebind(dst_k, ctl.keys);
  {
    const K* sk0 = src_k;
    K* dk0 = dst_k;
    if (swap_set(ctl, gw)) {
      src_k = dk0;
      dst_k = const_cast<K*>(sk0);
      const V* sv0 = src_v;
      src_v = dst_v;
      dst_v = const_cast<V*>(sv0);
    }
  }
  const uint64_t n = live_n(ctl, n_host);
  for (uint64_t k = blockIdx.x; k * MT::TM < n; k += gridDim.x) {
    if constexpr (MT::PAIRS) {
      merge4_tile<MT>(src_k, src_v, dst_k, dst_v, n, W, k, part4, smem);
    } else {
      merge4_tile<MT>(src_k, static_cast<const VV*>(nullptr), dst_k, static_cast<VV*>(nullptr), n, W, k, part4,
                      smem);
    }
    __syncthreads();
  }
}

}  // namespace ms

// Run-adaptive merging: merge passes that would change nothing are skipped.
//
// After the tile sort every tile is a sorted run.  A merge level is the
// identity when, for every pair of runs it merges, the last key of the left
// run is <= the first key of the right run: the left run wins ties, so the
// merge is the plain concatenation and leaves every element (and value) in
// place.  This is the run detection of the paper's section on Python's
// built-in sort (Timsort finds ordered runs and does not merge inside them),
// applied to whole tree levels.
//
// The first and last keys of every run at every level follow from the
// tiles' first and last keys alone (a merged run starts at the smaller of
// its halves' first keys and ends at the larger of their last keys), so one
// small kernel, run right after the tile sort, decides for every planned HBM
// pass whether all the levels it merges are identities.  Such a pass is
// skipped (its kernels return at once).  The passes that do run alternate
// between the two buffers starting from wherever the data is; a pass whose
// planned direction disagrees reads and writes the buffers the other way
// round (a device-side swap flag), and when an odd number of passes ran the
// result ends in the scratch buffer and a final copy brings it back.
#pragma once
#include "ms_common.hpp"
#include "ms_plan.hpp"

namespace ms {

// Control words (int32): [0] final copy needed, [1 + h] the gate word of
// pass h: bit 0 the pass runs, bit 1 it swaps its buffers.
constexpr int CTL_FINAL = 0;
__host__ __device__ constexpr int ctl_run(int h) { return 1 + h; }

// Tiles per workgroup of the first step (one tile per thread): levels below
// log2(RUN_GROUP) pair tiles inside one group.
constexpr int RUN_GROUP = 256;
constexpr int RUN_GROUP_LEVELS = 8;

// Step 1, one workgroup per group of RUN_GROUP tiles.  keys: the caller's
// buffer, tk: the scratch buffer; the tile sort wrote
// plan.start_in_caller ? keys : tk.  Each thread reads its tile's first and
// last key; the group then runs the levels that pair runs inside it (in LDS)
// and writes its run's first and last key (gf, gl) and a mask of the levels
// at which one of its pairs is out of order (gmask).
template <class K>
__global__ __launch_bounds__(RUN_GROUP) void run_bounds_kernel(const K* __restrict__ keys, const K* __restrict__ tk,
                                                              uint64_t n, uint32_t T, int levels, int start_in_caller,
                                                              K* __restrict__ gf, K* __restrict__ gl,
                                                              uint32_t* __restrict__ gmask) {
  __shared__ K F[RUN_GROUP], L[RUN_GROUP];
  __shared__ uint32_t mask;
  const K* src = start_in_caller ? keys : tk;
  const uint64_t tiles = (n + T - 1) / T;
  const uint64_t g = blockIdx.x, t0 = g * RUN_GROUP;
  const uint32_t i = threadIdx.x;
  const uint64_t t = t0 + i;
  if (i == 0) mask = 0;
  if (t < tiles) {
    const uint64_t e = (t + 1) * T < n ? (t + 1) * T : n;
    F[i] = src[t * T];
    L[i] = src[e - 1];
  }
  __syncthreads();
  const uint64_t in_group = tiles - t0 < uint64_t(RUN_GROUP) ? tiles - t0 : uint64_t(RUN_GROUP);
  const int lv_here = levels < RUN_GROUP_LEVELS ? levels : RUN_GROUP_LEVELS;
  uint64_t runs = in_group;  // runs of 2^p tiles inside the group at level p
  for (int p = 0; p < lv_here; ++p) {
    const uint64_t pairs = (runs + 1) / 2;
    K nf{}, nl{};
    if (i < pairs) {
      const uint32_t a = 2 * i, b = 2 * i + 1;
      nf = F[a];
      nl = L[a];
      if (b < runs) {
        if (F[b] < L[a]) atomicOr(&mask, 1u << p);
        nf = F[b] < nf ? F[b] : nf;
        nl = nl < L[b] ? L[b] : nl;
      }
    }
    __syncthreads();
    if (i < pairs) {
      F[i] = nf;
      L[i] = nl;
    }
    __syncthreads();
    runs = pairs;
  }
  if (i == 0) {
    gf[g] = F[0];
    gl[g] = L[0];
    gmask[g] = mask;
  }
}

// Step 2, one workgroup: the levels that pair whole groups, then the pass
// decisions.  gf/gl hold the groups' first and last keys (ping-ponged with
// hf/hl across levels).
template <class K>
__global__ __launch_bounds__(1024) void run_decide_kernel(uint64_t groups, PassPlan plan, K* __restrict__ gf,
                                                          K* __restrict__ gl, K* __restrict__ hf,
                                                          K* __restrict__ hl, const uint32_t* __restrict__ gmask,
                                                          int* __restrict__ ctl) {
  __shared__ uint32_t unordered_lo;       // levels below RUN_GROUP_LEVELS
  __shared__ int ordered_hi[64];          // levels from RUN_GROUP_LEVELS on
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  int levels = 0;
  for (int h = 0; h < plan.hbm; ++h) levels += plan.levels_in[h];
  if (tid == 0) unordered_lo = 0;
  for (uint32_t i = tid; i < 64; i += nt) ordered_hi[i] = 1;
  __syncthreads();
  uint32_t m = 0;
  for (uint64_t g = tid; g < groups; g += nt) m |= gmask[g];
  if (m) atomicOr(&unordered_lo, m);
  uint64_t runs = groups;
  K *f = gf, *l = gl, *f2 = hf, *l2 = hl;
  for (int p = RUN_GROUP_LEVELS; p < levels; ++p) {
    const uint64_t pairs = (runs + 1) / 2;
    bool ok = true;
    for (uint64_t j = tid; j < pairs; j += nt) {
      const uint64_t a = 2 * j, b = 2 * j + 1;
      if (b < runs) {
        const K fa_ = f[a], la_ = l[a], fb_ = f[b], lb_ = l[b];
        ok = ok && !(fb_ < la_);
        f2[j] = fb_ < fa_ ? fb_ : fa_;
        l2[j] = lb_ < la_ ? la_ : lb_;
      } else {
        f2[j] = f[a];
        l2[j] = l[a];
      }
    }
    if (!ok) ordered_hi[p - RUN_GROUP_LEVELS] = 0;
    __syncthreads();
    K* t0 = f;
    f = f2;
    f2 = t0;
    K* t1 = l;
    l = l2;
    l2 = t1;
    runs = pairs;
  }
  __syncthreads();
  if (tid != 0) return;
  // data location: 0 = caller's buffer, 1 = scratch; pass h as planned reads
  // the buffer the tile sort wrote when h is even, the other when h is odd
  const int start = plan.start_in_caller ? 0 : 1;
  int cur = start;
  for (int h = 0; h < plan.hbm; ++h) {
    bool identity = true;
    for (int q = 0; q < plan.levels_in[h]; ++q) {
      const int p = plan.first_level[h] + q;
      identity = identity && (p < RUN_GROUP_LEVELS ? ((unordered_lo >> p) & 1u) == 0
                                                    : ordered_hi[p - RUN_GROUP_LEVELS] != 0);
    }
    const int planned_src = start ^ (h & 1);
    ctl[ctl_run(h)] = identity ? 0 : (1 | (cur != planned_src ? 2 : 0));
    if (!identity) cur ^= 1;
  }
  ctl[CTL_FINAL] = cur != 0 ? 1 : 0;
}

// The final copy of n keys (and values) from the scratch buffers back to
// the caller's, when the control word says the result ended there.
template <class K, class V>
__global__ __launch_bounds__(256) void copy_back_kernel(const K* __restrict__ tk, const V* __restrict__ tv,
                                                        K* __restrict__ keys, V* __restrict__ vals, uint64_t n,
                                                        const int* __restrict__ ctl) {
  if (ctl[CTL_FINAL] == 0) return;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    keys[i] = tk[i];
    if constexpr (HasVal<V>::value) vals[i] = tv[i];
  }
}

}  // namespace ms

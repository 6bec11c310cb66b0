// Learned-bucket sort: host side (plan, scratch layout, launch sequence) and
// its C ABI (ms_sort_ex and the step-level entry points used by tests).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ms_internal.hpp"
#include "ms_learned.hpp"
#include "ms_plain_cfg.hpp"
#include "ms_plan.hpp"
#include "ms_tuning.hpp"

namespace ms {

__global__ void ls_setup_kernel(LsModel* md, int log_feature, int use_table, int coarse_bits, int fine_bits) {
  if (threadIdx.x != 0) return;
  md->log_feature = log_feature;
  md->use_table = use_table;
  md->coarse_bits = coarse_bits;
  md->fine_bits = fine_bits;
  md->nbins_c = 1u << coarse_bits;
  md->nbins_f = 1u << fine_bits;
  md->fallback = 0;
  md->do_learned = 0;
  md->do_repair = 0;
  md->misordered = 0;
  md->spilled = 0;
  md->kept = 0;
  md->max_bucket = 0;
  md->loss0 = 0.f;
  md->loss_last = 0.f;
  md->off64 = 0;
  md->scale64 = 1.f;
  md->l1_over = 0;
  md->sample_heavy = 0;
  md->sample_run = 0;
  md->sample_fb = 0;
  md->sample_spill = 0;
  md->sample_maxb = 0;
  md->do_train = 1;
}

__global__ void ls_set_theta_kernel(LsModel* md, const float* theta) {
  const int p = threadIdx.x;
  if (p < LS_P) {
    md->theta[0][p] = theta[p];
    md->m[0][p] = 0.f;
    md->v[0][p] = 0.f;
  }
}

__global__ void ls_get_theta_kernel(const LsModel* md, int parity, float* theta) {
  const int p = threadIdx.x;
  if (p < LS_P) theta[p] = md->theta[parity][p];
}

__global__ void ls_get_table_kernel(const LsModel* md, float* t, float* v, int* nt) {
  const int i = threadIdx.x;
  if (i < LS_TAB) {
    t[i] = md->tab_t[i];
    v[i] = md->tab_v[i];
  }
  if (i == 0) *nt = md->tab_n;
}

__global__ __launch_bounds__(256) void ls_bucket_ids_kernel(const uint32_t* __restrict__ keys, uint64_t n,
                                                            const LsModel* md, uint32_t* __restrict__ out) {
  __shared__ LsTable tb;
  ls_load_table(md, &tb);
  __syncthreads();
  const LsUni U = ls_uni(&tb);
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ls_bucket(&tb, U, keys[i]);
}

__global__ void ls_plain_stats_kernel(ms_stats* st) {
  if (threadIdx.x != 0) return;
  *st = ms_stats{};
  st->algo_used = MS_ALGO_MERGE_PATH;
}

__global__ void ls_stats_kernel(const LsModel* md, ms_stats* st, uint64_t buckets, Rebind rs) {
  if (threadIdx.x != 0) return;
  st = rebind(st, rs);
  st->algo_used = md->fallback ? MS_ALGO_MERGE_PATH : MS_ALGO_LEARNED_BUCKET;
  st->fallback_taken = md->fallback;
  st->misordered = md->misordered;
  st->repaired = md->do_repair;
  st->spilled = md->spilled;
  st->max_bucket = md->max_bucket;
  st->buckets = buckets;
  st->loss_initial = md->loss0;
  st->loss_final = md->loss_last;
  st->coarse_recounted = md->l1_over;
  st->sample_fallback = md->sample_fb;
}

// 1 for the log feature, 0 for the linear one.  MS_FEATURE_AUTO: log for
// uint32 keys (the key itself, suited to skewed positive workloads), linear
// for the other types (their feature works on offsets from the sample's
// smallest key, where a log would crowd the lower tail of a symmetric
// distribution into a few buckets).
static int log_feature(int feature, bool uint32_keys) {
  if (feature == MS_FEATURE_AUTO) return uint32_keys ? 1 : 0;
  return feature == MS_FEATURE_LOG ? 1 : 0;
}

// Sizes of one learned sort.
struct LsPlan {
  uint32_t S;          // sample size
  int cb, fb;          // coarse / fine bits
  uint32_t nbc, nbf;   // coarse / fine bins
  uint64_t B;          // buckets
  uint32_t capacity;   // largest bucket sorted in place (the option, at most
                       // the bucket sort's largest small class for the key type)
  uint64_t spill_cap;  // spill that still takes the learned path
  uint64_t chunk_cap;  // bound on level-2 chunks
  bool est;            // first level: regions sized from a random sample
  uint32_t S1, q;      // its sample size, input keys per sampled key
  uint64_t coarse_keys;  // first-level buffer (keys)
  // scratch offsets
  size_t md, sample, sample_tmp, partial, loss, bins, coarse, xr, part, seg, bytes;
  size_t bins_c_off[9], bins_f_off[3];
};

template <class K>
static uint32_t ls_capacity(const ms_options& o) {
  uint32_t bound = 0;
  int ncand = 0;
  seg_class_info<K, NoVal>(seg_num_classes<K, NoVal>() - 1, &bound, &ncand);
  return std::min<uint32_t>(o.bucket_capacity, bound);
}

template <class K>
static LsPlan ls_plan(uint64_t n, const ms_options& o) {
  LsPlan P{};
  P.S = 1u << o.sample_log2;
  P.capacity = ls_capacity<K>(o);
  const uint64_t want = std::max<uint64_t>(1, (n + o.bucket_fill - 1) / o.bucket_fill);
  int tb = 0;
  while ((uint64_t(1) << tb) < want && tb < 20) ++tb;
  P.cb = std::min(tb, 10);
  P.fb = tb - P.cb;
  P.nbc = 1u << P.cb;
  P.nbf = 1u << P.fb;
  P.B = uint64_t(1) << tb;
  P.spill_cap = std::min<uint64_t>(n, uint64_t(std::ceil(double(o.spill_threshold) * double(n))));
  P.chunk_cap = ceil_div(n, ls_chk<K>()) + P.nbc;
  // estimated first level from 2^23 keys: a sample of min(2^20, n / 128)
  // keys (a power of two); the buffer holds the sum of the regions' bounds
  // (ls_plan1_est_kernel), which must stay below 2^32 keys
  P.coarse_keys = n;
  P.est = o.coarse_estimate != 0 && n >= (uint64_t(1) << 23);
  if (P.est) {
    P.S1 = 1u << 16;
    while (P.S1 < (1u << 20) && uint64_t(P.S1) * 2 * 128 <= n) P.S1 *= 2;
    P.q = uint32_t(ceil_div(n, P.S1));
    const uint64_t bound = (uint64_t(5) * P.S1 * P.q) / 4 + uint64_t(P.nbc) * (uint64_t(32) * P.q + 63);
    if (bound < (uint64_t(1) << 32) - 64) P.coarse_keys = std::max<uint64_t>(n, bound); else P.est = false;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off = align_up(off + bytes, 256); return at; };
  P.md = take(sizeof(LsModel));
  P.sample = take(sizeof(K) * P.S);
  P.sample_tmp = take(plain_temp_bytes<K, NoVal>(P.S));
  P.partial = take(sizeof(float) * 2 * LS_TRAIN_G * LS_PS);
  P.loss = take(sizeof(float) * (o.train_steps + 1));
  for (int i = 0; i < 9; ++i) P.bins_c_off[i] = take(sizeof(uint32_t) * (P.nbc + 1));
  for (int i = 0; i < 2; ++i) P.bins_f_off[i] = take(sizeof(uint32_t) * P.B);
  P.bins_f_off[2] = take(sizeof(int64_t) * (P.B + 1));
  P.coarse = take(std::max<size_t>(sizeof(K) * P.coarse_keys, plain_temp_bytes<K, NoVal>(n)));
  P.xr = take(sizeof(K) * n);
  P.part = take(sizeof(int64_t) * (ceil_div(n, PlainCfg<K, NoVal>::MTILE) + 2));  // merge_two_runs
  P.seg = take(seg_temp_bytes<K, NoVal>(P.B, P.capacity));
  P.bytes = off;
  return P;
}

static LsBins ls_bins(char* w, const LsPlan& P) {
  LsBins b;
  uint32_t** c[9] = {&b.cnt_c, &b.off_c, &b.cursor_c, &b.chunk_start, &b.kept_tot, &b.spill_tot,
                     &b.cmaxb, &b.kept_base, &b.spill_base};
  for (int i = 0; i < 9; ++i) *c[i] = reinterpret_cast<uint32_t*>(w + P.bins_c_off[i]);
  b.cnt_f = reinterpret_cast<uint32_t*>(w + P.bins_f_off[0]);
  b.cursor_f = reinterpret_cast<uint32_t*>(w + P.bins_f_off[1]);
  b.seg_off = reinterpret_cast<int64_t*>(w + P.bins_f_off[2]);
  return b;
}

// Tile-sort shape (candidate index) per size class of the bucket sort.  The
// learned buckets (lengths spread around the fill, 512) favour other
// shapes than the batched form's autotuned table, whose segment lengths are
// log-uniform inside each class; measured on the 2^29 mixture, one class
// changed at a time: 256: 64x4, 512: 128x4, 1024: 128x8, 2048: 256x8,
// 4096: 1024x4, 8192: 512x16, 16384: 1024x16.
static const int kLearnedBucketShapes[8] = {0, 1, 0, 0, 2, 0, 0, 0};  // at least the class count

// 64-bit keys: every class's default shape.  Measured on the normal int64
// 2^28 workload's buckets (lengths near the 256-key fill): 8.09 ms per sort,
// against 8.54 ms with the batched form's autotuned row, whose choices are
// made on lengths spread over each class.
static const int kLearnedBucketShapes64[8] = {0, 0, 0, 0, 0, 0, 0, 0};
template <class K>
static const int* learned_bucket_shapes() {
  return sizeof(K) == 4 ? kLearnedBucketShapes : kLearnedBucketShapes64;
}

// Model training on an already sorted sample: start point, then T Adam steps.
template <class K>
static ms_status ls_train_enqueue(const K* sample, uint32_t S, LsModel* md, float* partial, int T, float lr,
                                  float* loss_hist, bool init, hipStream_t s, const int* gate = nullptr) {
  if (init) ls_init_kernel<<<1, 64, 0, s>>>(sample, S, md);
  for (int t = 0; t <= T; ++t) {
    ProfScope ps(PK_LEARN_TRAIN, s);
    ls_train_kernel<<<LS_TRAIN_G, LS_TRAIN_WG, 0, s>>>(sample, S, md, partial, t, T, lr, loss_hist, nullptr, gate);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "training launch");
}

// io_keys / io_stats: if non-null, the caller's key and stats buffers of
// this launch are read from *io_keys and *io_stats at run time (graph
// replays on new buffers).
template <class K>
static ms_status learned_enqueue(K* keys, uint64_t n, const ms_options& o, ms_stats* d_stats, void* ws,
                                 void* const* io_keys, void* const* io_stats, hipStream_t s) {
  const LsPlan P = ls_plan<K>(n, o);
  char* w = static_cast<char*>(ws);
  LsModel* md = reinterpret_cast<LsModel*>(w + P.md);
  K* sample = reinterpret_cast<K*>(w + P.sample);
  float* partial = reinterpret_cast<float*>(w + P.partial);
  float* loss = reinterpret_cast<float*>(w + P.loss);
  K* coarse = reinterpret_cast<K*>(w + P.coarse);
  K* xr = reinterpret_cast<K*>(w + P.xr);
  int64_t* part = reinterpret_cast<int64_t*>(w + P.part);
  const LsBins bn = ls_bins(w, P);
  const DevCtl none{nullptr, nullptr, nullptr};
  const Rebind rk{keys, io_keys};
  const Rebind rs{d_stats, io_stats};

  ls_setup_kernel<<<1, 64, 0, s>>>(md, log_feature(o.feature, std::is_same<K, uint32_t>::value), o.use_network ? 1 : 0, P.cb, P.fb);
  // sample, ranked by the plain merge sort
  ls_sample_kernel<<<dim3(unsigned(ceil_div(P.S, 256))), 256, 0, s>>>(keys, n, P.S, o.seed, sample, rk);
  ms_status st = plain_sort<K, NoVal>(sample, nullptr, P.S, none, s, w + P.sample_tmp);
  if (st != MS_OK) return st;
  ls_feature_range_kernel<K><<<1, 64, 0, s>>>(md, sample, P.S);
  // decision from the sample: runs of T sample keys in one bucket stand for
  // at least twice its capacity (T >= 8, so that a bucket near its capacity
  // rarely shows such a run by chance); equal keys first, before training,
  // then the trained table's buckets
  const uint64_t T = std::max<uint64_t>(8, ceil_div(uint64_t(2) * P.capacity * P.S, n));
  auto sample_check = [&](auto by_key) {
    if (T > P.S) return;
    ls_sample_heavy_kernel<K, decltype(by_key)::value>
        <<<dim3(unsigned(ceil_div(P.S - T + 1, 256))), 256, 0, s>>>(sample, P.S, uint32_t(T), md);
    ls_sample_decide_kernel<<<1, 64, 0, s>>>(md, n, P.S, P.spill_cap);
  };
  sample_check(std::true_type{});
  // train and compile the network (skipped after a fallback decided above)
  st = ls_train_enqueue(sample, P.S, md, partial, int(o.train_steps), o.learning_rate, loss, true, s, &md->do_train);
  if (st != MS_OK) return st;
  ls_compile_kernel<<<1, 64, 0, s>>>(md, int(o.train_steps) & 1, sample, P.S, &md->do_train);
  sample_check(std::false_type{});
  // level 1
  // (gated stages run with a bounded grid: when skipped they cost little)
  const uint64_t gated_grid = uint64_t(device_cu_count()) * 4;
  ls_clear_kernel<<<dim3(unsigned(ceil_div(std::max<uint64_t>(P.B, P.nbc), 256))), 256, 0, s>>>(bn, P.nbc,
                                                                                                 uint32_t(P.B));
  const unsigned chunks1 = unsigned(ceil_div(n, ls_chk<K>()));
  const uint32_t last_len = uint32_t(n - uint64_t(chunks1 - 1) * ls_chk<K>());
  unsigned h1_grid = unsigned(ceil_div(chunks1, LS_H1)), s1_grid = chunks1;
  const int* gate = nullptr;
  if (P.est) {
    // regions sized from a random sample, scatter with a bounds check; the
    // exact pass below runs only if a region was too small
    {
      ProfScope ps(PK_LEARN_EST, s);
      ls_est1_kernel<K><<<P.S1 / (LS_EST * LS_WG), LS_WG, 0, s>>>(keys, n, o.seed, md, bn, rk);
    }
    ls_plan1_est_kernel<<<1, LS_WG, 0, s>>>(md, bn, P.q);
    {
      ProfScope ps(PK_LEARN_SCATTER, s);
      ls_scatter1_kernel<<<chunks1, LS_WG, 0, s>>>(keys, chunks1, last_len, md, bn, coarse, rk, nullptr,
                                                   &md->l1_over);
    }
    ls_fin1_kernel<<<1, LS_WG, 0, s>>>(md, bn, uint32_t(ls_chk<K>()), o.coarse_estimate == 2 ? 1 : 0);
    gate = &md->l1_over;
    h1_grid = unsigned(std::min<uint64_t>(h1_grid, gated_grid));
    s1_grid = unsigned(std::min<uint64_t>(s1_grid, gated_grid));
  }
  // exact: count, plan, scatter
  {
    ProfScope ps(gate ? PK_LEARN_OTHER : PK_LEARN_HIST, s);
    ls_hist1_kernel<<<h1_grid, LS_WG, 0, s>>>(keys, chunks1, last_len, md, bn, rk, gate);
  }
  ls_plan1_kernel<<<1, LS_WG, 0, s>>>(md, bn, uint32_t(ls_chk<K>()), gate);
  {
    ProfScope ps(gate ? PK_LEARN_OTHER : PK_LEARN_SCATTER, s);
    ls_scatter1_kernel<<<s1_grid, LS_WG, 0, s>>>(keys, chunks1, last_len, md, bn, coarse, rk, gate, nullptr);
  }
  // level 2
  {
    ProfScope ps(PK_LEARN_HIST2, s);
    ls_hist2_kernel<<<unsigned(P.chunk_cap), LS_WG, 0, s>>>(coarse, md, bn);
  }
  ls_totals_kernel<<<P.nbc, LS_WG, 0, s>>>(md, bn, P.capacity);
  ls_plan2_kernel<<<1, LS_WG, 0, s>>>(md, bn, n, P.spill_cap, o.force_fallback, keys, xr, rk);
  ls_offsets_kernel<<<P.nbc, LS_WG, 0, s>>>(md, bn, P.capacity);
  {
    ProfScope ps(PK_LEARN_SCATTER2, s);
    ls_scatter2_kernel<<<unsigned(P.chunk_cap), LS_WG, 0, s>>>(coarse, md, bn, P.capacity, xr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "learned bucketing launch");
  // kept buckets: sorted in LDS by the segmented small-class kernels, in the
  // array chosen on the device (*md->r_keys)
  {
    ProfScope ps(PK_LEARN_BUCKET, s);
    st = seg_enqueue<K, NoVal>(keys, nullptr, bn.seg_off, P.B, P.capacity, P.capacity, w + P.seg, s,
                               learned_bucket_shapes<K>(), SegFork{nullptr, nullptr, nullptr},
                               reinterpret_cast<void* const*>(&md->r_keys));
  }
  if (st != MS_OK) return st;
  ls_check_kernel<K><<<dim3(unsigned(ceil_div(P.B, 256))), 256, 0, s>>>(md, bn, P.B);
  // repair: spill sorted by the plain merge sort, then merged with the kept keys
  const uint64_t* spilled = reinterpret_cast<const uint64_t*>(&md->spilled);
  if (P.spill_cap > 0) {
    st = plain_sort<K, NoVal>(xr, nullptr, P.spill_cap, DevCtl{spilled, &md->do_repair, nullptr}, s, coarse,
                              gated_grid);
    if (st != MS_OK) return st;
    st = merge_two_runs<K, NoVal>(xr, keys, n, DevCtl{nullptr, &md->do_repair, spilled, rk}, part, s, gated_grid);
    if (st != MS_OK) return st;
  }
  // fallback: the plain merge sort of the untouched input, on a bounded grid
  // four times wider than the other gated stages'.  Where the fallback runs,
  // 4 workgroups per CU looping over tiles cost it about 5% (2^27 Zipf keys
  // under the automatic choice: 3.86 ms, 3.73 with 16 per CU, plain sort
  // 3.22); skipped, its launches of 16 per CU still cost the learned path
  // nothing measurable (2^29 mixture 7.80 / 7.79 ms).
  const uint64_t fallback_grid = uint64_t(device_cu_count()) * 16;
  st = plain_sort<K, NoVal>(keys, nullptr, n, DevCtl{nullptr, &md->fallback, nullptr, rk}, s, coarse, fallback_grid);
  if (st != MS_OK) return st;
  if (d_stats) ls_stats_kernel<<<1, 64, 0, s>>>(md, d_stats, P.B, rs);
  e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "learned sort launch");
}

static ms_status check_options(const ms_options& o) {
  if (o.algo < MS_ALGO_AUTO || o.algo > MS_ALGO_LEARNED_BUCKET) return MS_ERR_INVALID_ARG;
  if (!(o.spill_threshold >= 0.f && o.spill_threshold <= 0.5f)) return MS_ERR_INVALID_ARG;
  if (o.bucket_capacity != 4096 && o.bucket_capacity != 16384) return MS_ERR_INVALID_ARG;
  if (o.bucket_fill != 0 && (o.bucket_fill < 64 || o.bucket_fill > o.bucket_capacity)) return MS_ERR_INVALID_ARG;
  if (o.train_steps > 100000) return MS_ERR_INVALID_ARG;
  if (!(o.learning_rate >= 0.f && o.learning_rate < 1.f)) return MS_ERR_INVALID_ARG;
  if (o.sample_log2 != 0 && (o.sample_log2 < 10 || o.sample_log2 > 20)) return MS_ERR_INVALID_ARG;
  if (o.feature != MS_FEATURE_LOG && o.feature != MS_FEATURE_LINEAR && o.feature != MS_FEATURE_AUTO)
    return MS_ERR_INVALID_ARG;
  if (o.coarse_estimate < 0 || o.coarse_estimate > 2) return MS_ERR_INVALID_ARG;
  return MS_OK;
}

// The learned sort of one key type: direct enqueue, or the cached graph.
template <class K>
static ms_status learned_sort(K* keys, ms_key_type kt, uint64_t n, const ms_options& o, ms_stats* d_stats,
                              hipStream_t s) {
  const LsPlan P = ls_plan<K>(n, o);
  if (!o.use_graph) {
    void* ws = nullptr;
    ms_status st = get_workspace(s, P.bytes, &ws);
    if (st != MS_OK) return st;
    return learned_enqueue(keys, n, o, d_stats, ws, nullptr, nullptr, s);
  }
  uint32_t lr_bits, th_bits;
  std::memcpy(&lr_bits, &o.learning_rate, 4);
  std::memcpy(&th_bits, &o.spill_threshold, 4);
  // the graph does not depend on the buffers: keys and stats are rebound on
  // every launch
  std::vector<uint64_t> key = {2, uint64_t(kt), n, d_stats ? 1u : 0u, th_bits, o.bucket_capacity, o.bucket_fill,
                               o.train_steps, lr_bits, o.sample_log2, o.seed, uint64_t(o.feature),
                               uint64_t(o.use_network), uint64_t(o.force_fallback),
                               uint64_t(o.coarse_estimate)};
  return cached_graph_launch(
      key, P.bytes, {static_cast<void*>(keys), d_stats},
      [&](void* ws, void* const* io, hipStream_t cs, SegFork) {
        return learned_enqueue(keys, n, o, d_stats, ws, &io[0], &io[1], cs);
      },
      s);
}

// ------------------------------------------------------------ pairs
// Learned pairs: each 32-bit key and its input position are packed into one
// 64-bit key (the key's unsigned image above, the position below), so every
// packed key is distinct and equal keys order by position: the learned sort
// of the packed keys is the stable order.  Then the keys are unpacked and
// the values gathered by position from a copy.
template <class K32>
__global__ __launch_bounds__(256) void lp_pack_kernel(const K32* __restrict__ keys, uint64_t n,
                                                      uint64_t* __restrict__ kp, Rebind rk) {
  keys = rebind(keys, rk);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    kp[i] = (uint64_t(ls_unsigned(keys[i])) << 32) | i;
}

template <class V>
__global__ __launch_bounds__(256) void lp_copy_kernel(const V* __restrict__ vals, uint64_t n, V* __restrict__ out,
                                                      Rebind rv) {
  vals = rebind(vals, rv);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = vals[i];
}

template <class K32, class V>
__global__ __launch_bounds__(256) void lp_unpack_kernel(const uint64_t* __restrict__ kp, const V* __restrict__ vcopy,
                                                        uint64_t n, K32* __restrict__ keys, V* __restrict__ vals,
                                                        Rebind rk, Rebind rv) {
  keys = rebind(keys, rk);
  vals = rebind(vals, rv);
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint64_t p = kp[i];
    const uint32_t u = uint32_t(p >> 32);
    keys[i] = K32(std::is_signed<K32>::value ? u ^ 0x80000000u : u);
    vals[i] = vcopy[uint32_t(p)];
  }
}

// Scratch of one learned pairs sort: packed keys, value copy, then the
// 64-bit learned sort's own scratch.
struct LpPlan {
  size_t kp, vcopy, core, bytes;
};

static LpPlan lp_plan(uint64_t n, size_t vb, const ms_options& o) {
  LpPlan L{};
  L.kp = 0;
  L.vcopy = align_up(sizeof(uint64_t) * n, 256);
  L.core = align_up(L.vcopy + vb * n, 256);
  L.bytes = L.core + ls_plan<uint64_t>(n, o).bytes;
  return L;
}

// io_keys / io_vals / io_stats as for learned_enqueue.
template <class K32, class V>
static ms_status learned_pairs_enqueue(K32* keys, V* vals, uint64_t n, const ms_options& o, ms_stats* d_stats,
                                       void* ws, void* const* io_keys, void* const* io_vals,
                                       void* const* io_stats, hipStream_t s) {
  const LpPlan L = lp_plan(n, sizeof(V), o);
  char* w = static_cast<char*>(ws);
  uint64_t* kp = reinterpret_cast<uint64_t*>(w + L.kp);
  V* vcopy = reinterpret_cast<V*>(w + L.vcopy);
  const unsigned grid = unsigned(std::min<uint64_t>(ceil_div(n, 256), uint64_t(device_cu_count()) * 16));
  lp_pack_kernel<K32><<<grid, 256, 0, s>>>(keys, n, kp, Rebind{keys, io_keys});
  lp_copy_kernel<V><<<grid, 256, 0, s>>>(vals, n, vcopy, Rebind{vals, io_vals});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "pairs pack launch");
  ms_status st = learned_enqueue<uint64_t>(kp, n, o, d_stats, w + L.core, nullptr, io_stats, s);
  if (st != MS_OK) return st;
  lp_unpack_kernel<K32, V><<<grid, 256, 0, s>>>(kp, vcopy, n, keys, vals, Rebind{keys, io_keys},
                                                Rebind{vals, io_vals});
  e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "pairs unpack launch");
}

template <class K32, class V>
static ms_status learned_pairs(K32* keys, V* vals, ms_key_type kt, uint64_t n, const ms_options& o,
                               ms_stats* d_stats, hipStream_t s) {
  const LpPlan L = lp_plan(n, sizeof(V), o);
  if (!o.use_graph) {
    void* ws = nullptr;
    ms_status st = get_workspace(s, L.bytes, &ws);
    if (st != MS_OK) return st;
    return learned_pairs_enqueue(keys, vals, n, o, d_stats, ws, nullptr, nullptr, nullptr, s);
  }
  uint32_t lr_bits, th_bits;
  std::memcpy(&lr_bits, &o.learning_rate, 4);
  std::memcpy(&th_bits, &o.spill_threshold, 4);
  std::vector<uint64_t> key = {3, uint64_t(kt), sizeof(V), n, d_stats ? 1u : 0u, th_bits, o.bucket_capacity,
                               o.bucket_fill, o.train_steps, lr_bits, o.sample_log2, o.seed, uint64_t(o.feature),
                               uint64_t(o.use_network), uint64_t(o.force_fallback),
                               uint64_t(o.coarse_estimate)};
  return cached_graph_launch(
      key, L.bytes, {static_cast<void*>(keys), static_cast<void*>(vals), d_stats},
      [&](void* ws, void* const* io, hipStream_t cs, SegFork) {
        return learned_pairs_enqueue(keys, vals, n, o, d_stats, ws, &io[0], &io[1], &io[2], cs);
      },
      s);
}

// Automatic choice of the learned form (MS_ALGO_AUTO): from the sizes at
// which it was measured faster than the plain sort on one MI355X -- 32-bit
// keys from 2^27 (uniform uint32 and the lognormal mixture 1.20x there;
// 0.85-0.89x at 2^26), 64-bit keys from 2^26 (normal int64 1.19x, uniform
// uint64 1.49x; 0.92x and 1.15x at 2^25).
static bool learned_auto(ms_key_type kt, uint64_t n) {
  const bool wide = kt == MS_KEY_U64 || kt == MS_KEY_I64;
  return n >= (uint64_t(1) << (wide ? 26 : 27));
}

// Options left at 0 take the key type's defaults.  64-bit keys: a 2^18-key
// sample and 256 keys per bucket, since about n / S keys fall beyond each of
// the sample's extremes and share one bucket there, and a workgroup sorts
// at most 4096 such keys in LDS; 32-bit keys: 2^16 and 512 (capacity 16384).
static ms_options resolve_options(ms_options o, ms_key_type kt) {
  const bool wide = kt == MS_KEY_U64 || kt == MS_KEY_I64;
  if (o.sample_log2 == 0) o.sample_log2 = wide ? 18 : 16;
  if (o.bucket_fill == 0) o.bucket_fill = wide ? 256 : 512;
  return o;
}

// A scratch LsModel for the step-level entry points (per device, stream).
static ms_status step_scratch(hipStream_t s, size_t extra, char** w) {
  void* p = nullptr;
  ms_status st = get_workspace(s, align_up(sizeof(LsModel), 256) + align_up(extra, 256), &p);
  *w = static_cast<char*>(p);
  return st;
}

}  // namespace ms

using namespace ms;

extern "C" {

void ms_options_default(ms_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->algo = MS_ALGO_AUTO;
  o->spill_threshold = 0.05f;
  o->bucket_capacity = 16384;
  o->bucket_fill = 0;
  o->train_steps = 16;
  o->learning_rate = 1e-4f;
  o->sample_log2 = 0;
  o->seed = 0;
  o->feature = MS_FEATURE_AUTO;
  o->use_network = 1;
  o->force_fallback = 0;
  o->use_graph = 1;
  o->coarse_estimate = 1;
}

ms_status ms_sort_ex(void* d_keys, size_t n, ms_key_type kt, const ms_options* opt, ms_stats* d_stats, void* stream) {
  ms_options o;
  ms_options_default(&o);
  if (opt) o = *opt;
  if (check_options(o) != MS_OK) {
    set_error("invalid ms_options");
    return MS_ERR_INVALID_ARG;
  }
  if (n > 0 && d_keys == nullptr) {
    set_error("d_keys is NULL with n > 0");
    return MS_ERR_INVALID_ARG;
  }
  if (kt < MS_KEY_U32 || kt > MS_KEY_I64) {
    set_error("unknown key type");
    return MS_ERR_UNSUPPORTED;
  }
  if (n == 0) return MS_OK;
  o = resolve_options(o, kt);
  const bool learned_ok = n >= (uint64_t(4) << o.sample_log2) && n < (uint64_t(1) << 32);
  if (o.algo == MS_ALGO_LEARNED_BUCKET && !learned_ok) {
    set_error("the learned-bucket form needs n >= 4 * sample size and n < 2^32");
    return MS_ERR_UNSUPPORTED;
  }
  // automatic choice: where the learned form was measured faster than the
  // plain sort (see learned_auto)
  const bool learned = learned_ok && o.algo != MS_ALGO_MERGE_PATH &&
                       (o.algo == MS_ALGO_LEARNED_BUCKET || learned_auto(kt, n));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!learned) {
    ms_status st = o.max_workgroups ? plain_sort_capped(d_keys, n, kt, o.max_workgroups, s)
                                    : ms_sort(d_keys, n, kt, stream);
    if (st != MS_OK || !d_stats) return st;
    ls_plain_stats_kernel<<<1, 64, 0, s>>>(d_stats);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MS_OK : hip_fail(e, "stats launch");
  }
  try {
    switch (kt) {
      case MS_KEY_U32: return learned_sort(static_cast<uint32_t*>(d_keys), kt, n, o, d_stats, s);
      case MS_KEY_I32: return learned_sort(static_cast<int32_t*>(d_keys), kt, n, o, d_stats, s);
      case MS_KEY_U64: return learned_sort(static_cast<uint64_t*>(d_keys), kt, n, o, d_stats, s);
      case MS_KEY_I64: return learned_sort(static_cast<int64_t*>(d_keys), kt, n, o, d_stats, s);
    }
    return MS_ERR_UNSUPPORTED;
  } catch (...) {
    set_error("unexpected exception");
    return MS_ERR_INTERNAL;
  }
}

ms_status ms_sort_pairs_ex(void* d_keys, void* d_vals, size_t n, ms_key_type kt, size_t val_bytes,
                           const ms_options* opt, ms_stats* d_stats, void* stream) {
  ms_options o;
  ms_options_default(&o);
  if (opt) o = *opt;
  if (check_options(o) != MS_OK) {
    set_error("invalid ms_options");
    return MS_ERR_INVALID_ARG;
  }
  if (kt < MS_KEY_U32 || kt > MS_KEY_I64) {
    set_error("unknown key type");
    return MS_ERR_UNSUPPORTED;
  }
  if (val_bytes != 4 && val_bytes != 8) {
    set_error("value width must be 4 or 8 bytes");
    return MS_ERR_UNSUPPORTED;
  }
  if (n > 0 && (d_keys == nullptr || d_vals == nullptr)) {
    set_error("d_keys or d_vals is NULL with n > 0");
    return MS_ERR_INVALID_ARG;
  }
  if (n > 0 && d_keys == d_vals) {
    set_error("key and value buffers overlap");
    return MS_ERR_INVALID_ARG;
  }
  if (n == 0) return MS_OK;
  const bool narrow = kt == MS_KEY_U32 || kt == MS_KEY_I32;
  // the packed sort runs on 64-bit keys: their defaults apply, except the
  // feature: the packed key's offset is the key's own offset times 2^32, so
  // uint32 keys keep the log feature they take alone
  o = resolve_options(o, MS_KEY_U64);
  if (o.feature == MS_FEATURE_AUTO) o.feature = kt == MS_KEY_U32 ? MS_FEATURE_LOG : MS_FEATURE_LINEAR;
  const bool learned_ok = narrow && n >= (uint64_t(4) << o.sample_log2) && n < (uint64_t(1) << 32);
  if (o.algo == MS_ALGO_LEARNED_BUCKET && !learned_ok) {
    set_error("learned pairs need 32-bit keys, n >= 4 * sample size and n < 2^32");
    return MS_ERR_UNSUPPORTED;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (o.algo != MS_ALGO_LEARNED_BUCKET) {
    ms_status st = ms_sort_pairs(d_keys, d_vals, n, kt, val_bytes, stream);
    if (st != MS_OK || !d_stats) return st;
    ls_plain_stats_kernel<<<1, 64, 0, s>>>(d_stats);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MS_OK : hip_fail(e, "stats launch");
  }
  try {
    if (kt == MS_KEY_U32) {
      if (val_bytes == 4)
        return learned_pairs(static_cast<uint32_t*>(d_keys), static_cast<uint32_t*>(d_vals), kt, n, o, d_stats, s);
      return learned_pairs(static_cast<uint32_t*>(d_keys), static_cast<uint64_t*>(d_vals), kt, n, o, d_stats, s);
    }
    if (val_bytes == 4)
      return learned_pairs(static_cast<int32_t*>(d_keys), static_cast<uint32_t*>(d_vals), kt, n, o, d_stats, s);
    return learned_pairs(static_cast<int32_t*>(d_keys), static_cast<uint64_t*>(d_vals), kt, n, o, d_stats, s);
  } catch (...) {
    set_error("unexpected exception");
    return MS_ERR_INTERNAL;
  }
}

size_t ms_temp_bytes_learned_pairs(size_t n, ms_key_type kt, size_t val_bytes, const ms_options* opt) {
  ms_options o;
  ms_options_default(&o);
  if (opt) o = *opt;
  if (check_options(o) != MS_OK || n == 0 || (kt != MS_KEY_U32 && kt != MS_KEY_I32) ||
      (val_bytes != 4 && val_bytes != 8))
    return 0;
  o = resolve_options(o, MS_KEY_U64);
  try {
    return graph_bind_bytes() + lp_plan(n, val_bytes, o).bytes;
  } catch (...) {
    return 0;
  }
}

size_t ms_temp_bytes_learned(size_t n, ms_key_type kt, const ms_options* opt) {
  ms_options o;
  ms_options_default(&o);
  if (opt) o = *opt;
  if (check_options(o) != MS_OK || n == 0) return 0;
  o = resolve_options(o, kt);
  try {
    switch (kt) {
      case MS_KEY_U32: return graph_bind_bytes() + ls_plan<uint32_t>(n, o).bytes;
      case MS_KEY_I32: return graph_bind_bytes() + ls_plan<int32_t>(n, o).bytes;
      case MS_KEY_U64: return graph_bind_bytes() + ls_plan<uint64_t>(n, o).bytes;
      case MS_KEY_I64: return graph_bind_bytes() + ls_plan<int64_t>(n, o).bytes;
    }
    return 0;
  } catch (...) {
    return 0;
  }
}

ms_status ms_learned_grad(const uint32_t* d_sample, uint32_t S, int feature, const float* d_theta, float* d_out,
                          void* stream) {
  if (!d_sample || !d_theta || !d_out || S == 0) {
    set_error("NULL pointer or empty sample");
    return MS_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = nullptr;
  ms_status st = step_scratch(s, sizeof(float) * 2 * LS_TRAIN_G * LS_PS, &w);
  if (st != MS_OK) return st;
  LsModel* md = reinterpret_cast<LsModel*>(w);
  float* partial = reinterpret_cast<float*>(w + align_up(sizeof(LsModel), 256));
  ls_setup_kernel<<<1, 64, 0, s>>>(md, log_feature(feature, true), 1, 0, 0);
  ls_set_theta_kernel<<<1, 64, 0, s>>>(md, d_theta);
  ls_train_kernel<<<LS_TRAIN_G, LS_TRAIN_WG, 0, s>>>(d_sample, S, md, partial, 0, 1, 0.f, nullptr, nullptr, nullptr);
  ls_train_kernel<<<LS_TRAIN_G, LS_TRAIN_WG, 0, s>>>(d_sample, S, md, partial, 1, 1, 0.f, nullptr, d_out, nullptr);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "gradient launch");
}

ms_status ms_learned_train(const uint32_t* d_sample, uint32_t S, int feature, uint32_t steps, float learning_rate,
                           const float* d_theta0, float* d_theta_out, float* d_loss_hist, void* stream) {
  if (!d_sample || !d_theta_out || S == 0 || steps > 100000) {
    set_error("NULL pointer, empty sample or too many steps");
    return MS_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = nullptr;
  ms_status st = step_scratch(s, sizeof(float) * 2 * LS_TRAIN_G * LS_PS, &w);
  if (st != MS_OK) return st;
  LsModel* md = reinterpret_cast<LsModel*>(w);
  float* partial = reinterpret_cast<float*>(w + align_up(sizeof(LsModel), 256));
  ls_setup_kernel<<<1, 64, 0, s>>>(md, log_feature(feature, true), 1, 0, 0);
  if (d_theta0) ls_set_theta_kernel<<<1, 64, 0, s>>>(md, d_theta0);
  st = ls_train_enqueue(d_sample, S, md, partial, int(steps), learning_rate, d_loss_hist, d_theta0 == nullptr, s);
  if (st != MS_OK) return st;
  ls_get_theta_kernel<<<1, 64, 0, s>>>(md, int(steps) & 1, d_theta_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "training launch");
}

ms_status ms_learned_table(const float* d_theta, const uint32_t* d_sample, uint32_t S, int feature, float* d_t,
                           float* d_v, int* d_count, void* stream) {
  if (!d_theta || !d_sample || S == 0 || !d_t || !d_v || !d_count) {
    set_error("NULL pointer or empty sample");
    return MS_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = nullptr;
  ms_status st = step_scratch(s, 0, &w);
  if (st != MS_OK) return st;
  LsModel* md = reinterpret_cast<LsModel*>(w);
  ls_setup_kernel<<<1, 64, 0, s>>>(md, log_feature(feature, true), 1, 0, 0);
  ls_set_theta_kernel<<<1, 64, 0, s>>>(md, d_theta);
  ls_compile_kernel<<<1, 64, 0, s>>>(md, 0, d_sample, S, nullptr);
  ls_get_table_kernel<<<1, 64, 0, s>>>(md, d_t, d_v, d_count);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "table launch");
}

ms_status ms_learned_bucket_ids(const uint32_t* d_keys, size_t n, const float* d_theta, const uint32_t* d_sample,
                                uint32_t S, int feature, int use_network, uint32_t log2_buckets, uint32_t* d_out,
                                void* stream) {
  if (n == 0) return MS_OK;
  if (!d_keys || !d_theta || !d_sample || S == 0 || !d_out || log2_buckets > 20) {
    set_error("NULL pointer, empty sample or more than 2^20 buckets");
    return MS_ERR_INVALID_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = nullptr;
  ms_status st = step_scratch(s, 0, &w);
  if (st != MS_OK) return st;
  LsModel* md = reinterpret_cast<LsModel*>(w);
  const int cb = int(std::min<uint32_t>(log2_buckets, 10)), fb = int(log2_buckets) - cb;
  ls_setup_kernel<<<1, 64, 0, s>>>(md, log_feature(feature, true), use_network ? 1 : 0, cb, fb);
  ls_set_theta_kernel<<<1, 64, 0, s>>>(md, d_theta);
  ls_compile_kernel<<<1, 64, 0, s>>>(md, 0, d_sample, S, nullptr);
  ls_bucket_ids_kernel<<<dim3(unsigned(ceil_div(n, 256))), 256, 0, s>>>(d_keys, n, md, d_out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MS_OK : hip_fail(e, "bucket id launch");
}

}  // extern "C"

// Learned-bucket sort (32- and 64-bit keys): device kernels.
//
// The network is this library's small CDF model (the paper has none): a
// two-layer ReLU MLP F(x) = b2 + sum_h w2_h relu(w1_h x + b1_h) of one input
// feature x of the key, trained to map a key to its normalised rank.
//
// Pipeline (all on the device, no host readback):
//   sample  : S keys at seeded positions, sorted by the plain merge sort;
//   init    : closed-form start -- the piecewise-linear interpolant through
//             H sample quantiles;
//   train   : full-batch Adam on the sample's mean squared rank error, one
//             launch per step; every workgroup re-derives the step's
//             parameters from the previous launch's per-workgroup gradient
//             partials, summed in a fixed order (deterministic, no grid-wide
//             barrier);
//   compile : the trained network as a piecewise-linear table with a
//             running-max envelope, so that bucket ids are non-decreasing in
//             the key exactly, FP32 rounding included;
//   bucket  : b = floor(F(x) * B), B = 2^(coarse bits + fine bits);
//   level 1 : coarse histogram (LDS), scan, scatter into coarse buckets
//             through an LDS counting sort per chunk (coalesced runs);
//   level 2 : fine histogram inside each coarse bucket, then per fine bucket
//             either "kept" (at most `capacity` keys: placed contiguously
//             for the LDS bucket sort) or "spilled" (to the spill array);
//   decide  : spilled > tau * n -> the plain merge sort runs instead
//             (device flag; every learned kernel then returns);
//   sort    : kept buckets are sorted in LDS by the segmented small-class
//             kernels;
//   check   : the sorted kept buckets must meet in order (the last key of
//             each <= the first key of the next; it cannot fail
//             for a non-decreasing bucket function, and if it does the plain
//             merge sort sorts the keys, a permutation of the input, again);
//   repair  : the spill is sorted by the plain merge sort and one
//             merge-path pass merges it with the kept keys (exact).
#pragma once
#include "ms_common.hpp"

namespace ms {

constexpr int LS_H = 16;             // hidden units
constexpr int LS_P = 3 * LS_H + 1;   // parameters
constexpr int LS_PS = LS_P + 1;      // parameters + squared-error sum
constexpr int LS_TAB = 32;           // table capacity (>= LS_H + 2)
constexpr int LS_TRAIN_G = 64;       // training workgroups
constexpr int LS_TRAIN_WG = 256;     // training workgroup size
constexpr int LS_WG = 512;           // histogram / scatter workgroup size
constexpr int LS_CHK = 8192;         // keys per histogram / scatter chunk
// keys per chunk for a key type: 8192 for every type (32 KB of 32-bit keys
// staged in LDS, 64 KB of 64-bit keys, which then leave the staged bins out,
// see LsScatterLds; measured on normal int64 2^28: 7.69 -> 7.42 ms per sort
// against 4096-key chunks, whose runs per bin are half as long)
template <class K>
__host__ __device__ constexpr int ls_chk() { return LS_CHK; }
constexpr int LS_MAX_BINS = 1024;    // max coarse or fine bins per level
#ifndef MS_LS_H1
#define MS_LS_H1 4
#endif
constexpr int LS_H1 = MS_LS_H1;      // level-1 histogram chunks per workgroup
constexpr float LS_BETA1 = 0.9f, LS_BETA2 = 0.999f, LS_EPS = 1e-8f;

// Feature of a key (bit-identical to the CPU oracle's float32 computation).
__device__ __forceinline__ float ls_feature(uint32_t k, int log_feature) {
  if (log_feature) {
    const float f = __fadd_rn(__uint2float_rn(k), 1.0f);
    const int bits = __float_as_int(f) - 0x3F800000;
    return __int2float_rn(bits) * 0x1p-28f;
  }
  return __uint2float_rn(k) * 0x1p-32f;
}

// Order-preserving unsigned image of a key (signed types: sign bit flipped).
template <class K>
__device__ __forceinline__ auto ls_unsigned(K k) {
  if constexpr (sizeof(K) == 4) {
    return std::is_signed<K>::value ? uint32_t(k) ^ 0x80000000u : uint32_t(k);
  } else {
    return std::is_signed<K>::value ? uint64_t(k) ^ 0x8000000000000000ull : uint64_t(k);
  }
}

// Feature of a key of any type.  uint32 keys: ls_feature of the key itself
// (bit-identical to the CPU oracle's float32 computation).  Other types: the
// same two forms applied to the offset d of the key's unsigned image from
// off64 (a point just below the sample's smallest image; d = 0 below it):
// linear fl32(d) * scale, log (bits(fl32(fl32(d) + 1)) - bits(1.0)) * 2^-29.  (The
// raw image would not do for signed keys: small keys of either sign sit next
// to 2^31 or 2^63, where a float32 has no resolution left.)  Both forms are
// non-decreasing in the key.
template <class K>
__device__ __forceinline__ float ls_key_feature(K k, int log_feature, uint64_t off64, float scale64) {
  if constexpr (std::is_same<K, uint32_t>::value) {
    return ls_feature(k, log_feature);
  } else {
    const uint64_t u = ls_unsigned(k);
    const uint64_t d = u > off64 ? u - off64 : 0ull;
    const float fd = __ull2float_rn(d);
    if (log_feature) {
      const int bits = __float_as_int(__fadd_rn(fd, 1.0f)) - 0x3F800000;
      return __int2float_rn(bits) * 0x1p-29f;
    }
    return __fmul_rn(fd, scale64);
  }
}

// Model / table / decision record in device memory.
struct LsModel {
  float theta[2][LS_P];  // double-buffered parameters (step parity)
  float m[2][LS_P];      // Adam first moments
  float v[2][LS_P];      // Adam second moments
  float tab_t[LS_TAB];   // breakpoints (ascending; padded with +inf)
  float tab_v[LS_TAB];   // non-decreasing values at the breakpoints
  float tab_s[LS_TAB];   // slope of each segment (>= 0)
  int tab_n;             // number of breakpoints
  int use_table;         // 0: bucket = floor(x * B) (no network)
  int log_feature;
  int fine_bits, coarse_bits;
  uint32_t nbins_c, nbins_f;
  // decision
  int do_learned, do_repair, fallback, misordered;
  unsigned long long spilled, kept, max_bucket;
  void* r_keys;          // key array the kept buckets live in (caller's or scratch)
  uint64_t r_base;       // first kept position in r_keys
  uint32_t total_chunks; // level-2 chunks
  float loss0, loss_last;
  uint64_t off64;        // keys other than uint32: feature offset (the sample's smallest unsigned image)
  float scale64;         // keys other than uint32: linear feature scale
  int l1_over;           // estimated first level: a region was too small (the exact pass runs)
  // decision from the sorted sample, before any pass over the input
  uint32_t sample_heavy; // sample windows that lie in one over-full bucket (ls_sample_heavy_kernel)
  uint32_t sample_run;   // longest run of sample keys in one such bucket
  int sample_fb;         // the sample shows too many keys in over-full buckets: fall back at once
  unsigned long long sample_spill, sample_maxb;  // the windows' and the run's input keys (estimates)
  int do_train;          // training and the table compile run (cleared by a fallback decided before them)
};

// Keys other than uint32: the feature's offset and scale from the sorted
// sample (one thread).  The offset sits 1/64 of the sample's range below its
// smallest key (or at 0), so that keys below the sample still get distinct
// features; the scale is the power of two that maps offset .. the sample's
// largest key into [0, 1].
template <class K>
__global__ void ls_feature_range_kernel(LsModel* md, const K* __restrict__ sample, uint32_t S) {
  if (threadIdx.x != 0) return;
  if constexpr (std::is_same<K, uint32_t>::value) {
    md->off64 = 0;
    md->scale64 = 1.f;
  } else {
    const uint64_t lo = ls_unsigned(sample[0]), hi = ls_unsigned(sample[S - 1]);
    const uint64_t margin = (hi - lo) >> 6;
    const uint64_t off = lo > margin ? lo - margin : 0ull;
    const uint64_t r = hi - off;
    int e = 0;
    while (e < 64 && (r >> e) != 0) ++e;  // bit length of the range
    md->off64 = off;
    md->scale64 = __int_as_float((127 - e) << 23);  // 2^-e
  }
}

// ------------------------------------------------------------ sampling
// Position of draw `idx` in [0, n): the splitmix64 finaliser of a Weyl
// sequence point of (seed, idx), mapped to [0, n) by a 64x64 -> high-64
// product.  The training sample takes draws 0 .. S-1; the first level's
// size estimate takes draws from 2^32 on.
__device__ __forceinline__ uint64_t ls_draw(uint64_t seed, uint64_t idx, uint64_t n) {
  uint64_t z = seed * 0x9E3779B97F4A7C15ull + (idx + 1) * 0xD1B54A32D192ED03ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return __umul64hi(z, n);
}

template <class K>
__global__ __launch_bounds__(256) void ls_sample_kernel(const K* __restrict__ keys, uint64_t n, uint32_t S,
                                                        uint64_t seed, K* __restrict__ out, Rebind rk) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  keys = rebind(keys, rk);
  out[i] = keys[ls_draw(seed, i, n)];
}

// ------------------------------------------------------------ start point
// One thread: knots at sample positions q_i = floor(i (S-1) / H), i = 0..H,
// values (q_i + 0.5) / S; of a run of equal knots only the last is kept;
// unit h is relu(x - k_h) with output weight = slope change at k_h.
template <class K>
__global__ void ls_init_kernel(const K* __restrict__ sample, uint32_t S, LsModel* md) {
  // working arrays in LDS rather than in private (scratch) memory
  __shared__ double k[LS_H + 1], y[LS_H + 1];
  if (threadIdx.x != 0) return;
  // the knots' sample keys, all loads issued before the first is used
  K sk[LS_H + 1];
#pragma unroll
  for (int i = 0; i <= LS_H; ++i) sk[i] = sample[uint32_t((uint64_t(i) * (S - 1)) / LS_H)];
  int m = 0;
#pragma unroll
  for (int i = 0; i <= LS_H; ++i) {
    const uint32_t q = uint32_t((uint64_t(i) * (S - 1)) / LS_H);
    const double kk = double(ls_key_feature(sk[i], md->log_feature, md->off64, md->scale64));
    const double yy = (double(q) + 0.5) / double(S);
    if (m > 0 && k[m - 1] == kk) {
      y[m - 1] = yy;  // keep the last of a run of equal knots
    } else {
      k[m] = kk;
      y[m] = yy;
      ++m;
    }
  }
  float* th = md->theta[0];
  double prev_slope = 0.0;
  for (int h = 0; h < LS_H; ++h) {
    th[h] = 1.0f;                                        // w1
    th[LS_H + h] = float(-(h < m - 1 ? k[h] : k[m - 1]));  // b1
    double w2 = 0.0;
    if (h < m - 1) {
      const double slope = (y[h + 1] - y[h]) / (k[h + 1] - k[h]);
      w2 = slope - prev_slope;
      prev_slope = slope;
    }
    th[2 * LS_H + h] = float(w2);
  }
  th[3 * LS_H] = float(y[0]);
  for (int p = 0; p < LS_P; ++p) {
    md->m[0][p] = 0.f;
    md->v[0][p] = 0.f;
  }
}

// ------------------------------------------------------------ training
// Launch t (t = 0..T): parameters theta_t (for t > 0: one Adam step from
// theta_{t-1} with the gradient summed from partial[(t-1)&1]); workgroup 0
// stores theta_t; for t < T every workgroup then writes its gradient partial
// (and squared-error sum) at theta_t to partial[t&1][blockIdx.x].
// grad_out / loss_out (optional): the summed gradient + squared-error sum of
// the previous launch.
template <class K>
__global__ __launch_bounds__(LS_TRAIN_WG) void ls_train_kernel(const K* __restrict__ sample, uint32_t S,
                                                                LsModel* md, float* __restrict__ partial, int t,
                                                                int T, float lr, float* __restrict__ loss_hist,
                                                                float* __restrict__ grad_out, const int* gate) {
  if (gate && *gate == 0) return;
  constexpr int ROW = LS_PS + 1;  // padded row of the transposed reduction
  __shared__ float th[LS_P];
  __shared__ float red[LS_TRAIN_WG * ROW > LS_TRAIN_G * LS_PS ? LS_TRAIN_WG * ROW : LS_TRAIN_G * LS_PS];
  __shared__ float quart[4][LS_PS];
  __shared__ float gsum[LS_PS];
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  if (t == 0) {
    if (tid < LS_P) th[tid] = md->theta[0][tid];
    __syncthreads();
  } else {
    // previous launch's partials, summed over workgroups in fixed order
    const float* pp = partial + size_t((t - 1) & 1) * G * LS_PS;
    for (int i = tid; i < G * LS_PS; i += LS_TRAIN_WG) red[i] = pp[i];
    __syncthreads();
    if (tid < LS_PS) {
      float acc = 0.f;
      for (int g = 0; g < G; ++g) acc += red[g * LS_PS + tid];
      gsum[tid] = acc;
    }
    __syncthreads();
    if (tid < LS_P) {
      const int pb = (t - 1) & 1, nb = t & 1;
      const float gr = gsum[tid];
      const float m1 = LS_BETA1 * md->m[pb][tid] + (1.f - LS_BETA1) * gr;
      const float v1 = LS_BETA2 * md->v[pb][tid] + (1.f - LS_BETA2) * gr * gr;
      const float mh = m1 / (1.f - powf(LS_BETA1, float(t)));
      const float vh = v1 / (1.f - powf(LS_BETA2, float(t)));
      const float nt = md->theta[pb][tid] - lr * mh / (sqrtf(vh) + LS_EPS);
      th[tid] = nt;
      if (blockIdx.x == 0) {
        md->theta[nb][tid] = nt;
        md->m[nb][tid] = m1;
        md->v[nb][tid] = v1;
      }
    }
    if (blockIdx.x == 0 && tid == 0) {
      const float l = gsum[LS_P] / float(S);
      if (loss_hist) loss_hist[t - 1] = l;
      if (t == 1) md->loss0 = l;
      md->loss_last = l;
    }
    if (blockIdx.x == 0 && grad_out && tid < LS_PS) grad_out[tid] = gsum[tid];
    __syncthreads();
  }
  if (t >= T) return;
  // gradient of the mean squared error at th over this workgroup's samples
  float acc[LS_PS];
#pragma unroll
  for (int p = 0; p < LS_PS; ++p) acc[p] = 0.f;
  const float inv2 = 2.f / float(S);
  for (uint32_t i = blockIdx.x * LS_TRAIN_WG + tid; i < S; i += G * LS_TRAIN_WG) {
    const float x = ls_key_feature(sample[i], md->log_feature, md->off64, md->scale64);
    const float y = (float(i) + 0.5f) / float(S);
    float z[LS_H];
    float F = th[3 * LS_H];
#pragma unroll
    for (int h = 0; h < LS_H; ++h) {
      z[h] = fmaf(th[h], x, th[LS_H + h]);
      F = fmaf(th[2 * LS_H + h], fmaxf(z[h], 0.f), F);
    }
    const float e = F - y;
    const float r = e * inv2;
#pragma unroll
    for (int h = 0; h < LS_H; ++h) {
      const float a = fmaxf(z[h], 0.f);
      const float gz = z[h] > 0.f ? r * th[2 * LS_H + h] : 0.f;
      acc[h] = fmaf(gz, x, acc[h]);           // w1
      acc[LS_H + h] += gz;                   // b1
      acc[2 * LS_H + h] = fmaf(r, a, acc[2 * LS_H + h]);  // w2
    }
    acc[3 * LS_H] += r;        // b2
    acc[LS_P] = fmaf(e, e, acc[LS_P]);
  }
  // workgroup sum in a fixed order: every thread's row into LDS, then for
  // each parameter 4 quarter sums over 64 rows each, then the 4 quarters
  __syncthreads();
#pragma unroll
  for (int p = 0; p < LS_PS; ++p) red[tid * ROW + p] = acc[p];
  __syncthreads();
  if (tid < 4 * LS_PS) {
    const int p = tid % LS_PS, q = tid / LS_PS;
    float s = 0.f;
#pragma unroll 8
    for (int j = 0; j < LS_TRAIN_WG / 4; ++j) s += red[(q * (LS_TRAIN_WG / 4) + j) * ROW + p];
    quart[q][p] = s;
  }
  __syncthreads();
  if (tid < LS_PS)
    partial[size_t(t & 1) * G * LS_PS + size_t(blockIdx.x) * LS_PS + tid] =
        ((quart[0][tid] + quart[1][tid]) + quart[2][tid]) + quart[3][tid];
}

// ------------------------------------------------------------ compile
// One thread: the trained network restricted to the sample's feature range
// [x_min, x_max]: x_min, the breakpoints strictly inside (sorted), x_max;
// F there in double; running maximum clamped into [0.5/S, 1 - 0.5/S], ends
// pinned to those values; interior points that would leave a flat segment
// (FP32 value not above the previous kept point's, or at the upper clamp)
// are dropped, since a flat segment sends all its keys to one bucket; FP32
// table with segment slopes.
template <class K>
__global__ void ls_compile_kernel(LsModel* md, int final_parity, const K* __restrict__ sample, uint32_t S,
                                  const int* gate) {
  // the working arrays in LDS rather than in private (scratch) memory, which
  // the indexed accesses below would otherwise use
  __shared__ double t[LS_H + 2], pts[LS_H + 2], V[LS_H + 2];
  if (gate && *gate == 0) return;
  if (threadIdx.x != 0) return;
  // the parameters in registers: the loops below read each of them many
  // times, and as loads beside the table's stores they would stay loads
  float th[LS_P];
  {
    const float* thg = md->theta[final_parity];
#pragma unroll
    for (int p = 0; p < LS_P; ++p) th[p] = thg[p];
  }
  const double xmin = ls_key_feature(sample[0], md->log_feature, md->off64, md->scale64);
  const double xmax = ls_key_feature(sample[S - 1], md->log_feature, md->off64, md->scale64);
  int nt = 0;
#pragma unroll
  for (int h = 0; h < LS_H; ++h) {
    const double w1 = th[h], b1 = th[LS_H + h];
    if (w1 != 0.0) {
      const double bp = -b1 / w1;
      if (bp > xmin && bp < xmax) t[nt++] = bp;
    }
  }
  for (int i = 1; i < nt; ++i) {  // insertion sort
    const double x = t[i];
    int j = i - 1;
    while (j >= 0 && t[j] > x) { t[j + 1] = t[j]; --j; }
    t[j + 1] = x;
  }
  // ends plus the interior points that are distinct floats strictly inside
  int np = 0;
  pts[np++] = xmin;
  for (int i = 0; i < nt; ++i)
    if (float(t[i]) > float(pts[np - 1]) && float(t[i]) < float(xmax)) pts[np++] = t[i];
  pts[np++] = xmax;
  const double lo = 0.5 / double(S), hi = 1.0 - 0.5 / double(S);
  double run = -1e300;
  for (int i = 0; i < np; ++i) {
    double F = th[3 * LS_H];
#pragma unroll
    for (int h = 0; h < LS_H; ++h) {
      const double z = double(th[h]) * pts[i] + double(th[LS_H + h]);
      if (z > 0.0) F += double(th[2 * LS_H + h]) * z;
    }
    run = F > run ? F : run;
    V[i] = run < lo ? lo : (run > hi ? hi : run);
  }
  V[0] = lo;
  V[np - 1] = hi;
  int m = 1;
  for (int i = 1; i < np - 1; ++i)
    if (float(V[i]) > float(V[m - 1]) && float(V[i]) < float(hi)) {
      pts[m] = pts[i];
      V[m] = V[i];
      ++m;
    }
  pts[m] = pts[np - 1];
  V[m] = V[np - 1];
  np = m + 1;
  for (int i = 0; i < LS_TAB; ++i) {
    if (i < np) {
      md->tab_t[i] = float(pts[i]);
      md->tab_v[i] = float(V[i]);
      const float dv = i + 1 < np ? float(V[i + 1]) - float(V[i]) : 0.f;
      const float dt = i + 1 < np ? float(pts[i + 1]) - float(pts[i]) : 0.f;
      md->tab_s[i] = (i + 1 < np && dt > 0.f && dv > 0.f) ? dv / dt : 0.f;
    } else {
      md->tab_t[i] = __int_as_float(0x7f800000);  // +inf
      md->tab_v[i] = md->tab_v[np - 1];
      md->tab_s[i] = 0.f;
    }
  }
  md->tab_n = np;
}

// Table in LDS for the per-key bucket function: points t, values v, slopes
// s and caps c (c[j] = v[j + 1], and 1 for the last segment).
struct LsTable {
  float t[LS_TAB], v[LS_TAB], s[LS_TAB], c[LS_TAB];
  int n, use_table, log_feature, fine_bits;
  float B;
  uint32_t nb;  // total buckets
  uint64_t off64;
  float scale64;
};

__device__ __forceinline__ void ls_load_table(const LsModel* md, LsTable* tb) {
  const int tid = threadIdx.x;
  if (tid < LS_TAB) {
    tb->t[tid] = md->tab_t[tid];
    tb->v[tid] = md->tab_v[tid];
    tb->s[tid] = md->tab_s[tid];
    tb->c[tid] = tid + 2 < md->tab_n ? md->tab_v[tid + 1] : 1.0f;
  }
  if (tid == 0) {
    tb->n = md->tab_n;
    tb->use_table = md->use_table;
    tb->log_feature = md->log_feature;
    tb->fine_bits = md->fine_bits;
    tb->nb = md->nbins_c << md->fine_bits;
    tb->B = float(tb->nb);
    tb->off64 = md->off64;
    tb->scale64 = md->scale64;
  }
}

// The table's scalar fields, read once per kernel into scalar registers
// (every lane holds the same values), so that branches on them are uniform.
struct LsUni {
  int n, use_table, log_feature, fine_bits;
  float B;
  uint32_t nb;
  uint64_t off64;
  float scale64;
};

__device__ __forceinline__ float uniform_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// After ls_load_table and a barrier.
__device__ __forceinline__ LsUni ls_uni(const LsTable* tb) {
  LsUni u;
  u.n = __builtin_amdgcn_readfirstlane(tb->n);
  u.use_table = __builtin_amdgcn_readfirstlane(tb->use_table);
  u.log_feature = __builtin_amdgcn_readfirstlane(tb->log_feature);
  u.fine_bits = __builtin_amdgcn_readfirstlane(tb->fine_bits);
  u.B = uniform_f(tb->B);
  u.nb = uint32_t(__builtin_amdgcn_readfirstlane(int(tb->nb)));
  u.off64 = wave_uniform(tb->off64);
  u.scale64 = uniform_f(tb->scale64);
  return u;
}

// Bucket id of a key: non-decreasing in the key.  Branch-free per lane: the
// table search takes a fixed number of select steps.  Keys beyond the
// table's range continue its first or last segment (clipped to [0, 1]), so
// the keys past the sample's extremes spread over the end buckets.
template <class K>
__device__ __forceinline__ uint32_t ls_bucket(const LsTable* tb, const LsUni& U, K key) {
  const float x = ls_key_feature(key, U.log_feature, U.off64, U.scale64);
  float u;
  if (U.use_table) {
    int j = 0;  // largest j with t[j] <= x (0 below the range), at most n-2
#pragma unroll
    for (int step = LS_TAB / 2; step >= 1; step >>= 1) j = tb->t[j + step] <= x ? j + step : j;
    j = j < U.n - 2 ? j : U.n - 2;
    // min(value, cap) then max(., 0): the middle of the three, since the
    // caps are positive
    u = __builtin_amdgcn_fmed3f(__fmaf_rn(tb->s[j], __fsub_rn(x, tb->t[j]), tb->v[j]), 0.f, tb->c[j]);
  } else {
    u = fmaxf(x, 0.f);
  }
  const float f = __fmul_rn(u, U.B);
  const uint32_t b = f >= U.B ? U.nb - 1 : uint32_t(f);
  return b < U.nb ? b : U.nb - 1;
}

// ------------------------------------------------------------ scatter
// Bin arrays and decisions of one learned sort (device scratch).
struct LsBins {
  uint32_t* cnt_c;        // [Bc] keys per coarse bucket
  uint32_t* off_c;        // [Bc + 1] exclusive scan of cnt_c
  uint32_t* cursor_c;     // [Bc] coarse scatter cursors
  uint32_t* chunk_start;  // [Bc + 1] first level-2 chunk of each coarse bucket
  uint32_t* cnt_f;        // [B] keys per fine bucket
  uint32_t* cursor_f;     // [B] fine scatter cursors
  int64_t* seg_off;       // [B + 1] kept-bucket segments for the bucket sort
  uint32_t* kept_tot;     // [Bc] per coarse bucket: kept keys
  uint32_t* spill_tot;    // [Bc] spilled keys
  uint32_t* cmaxb;        // [Bc] largest fine bucket
  uint32_t* kept_base;    // [Bc] first kept position of the coarse bucket
  uint32_t* spill_base;   // [Bc] first spill position of the coarse bucket
};

// Exclusive scan of cnt[0, nb) (nb <= 2 * LS_WG) into off[0, nb); *total
// gets the sum.  Whole workgroup; ends with a barrier.
__device__ __forceinline__ void ls_block_scan(const uint32_t* cnt, uint32_t* off, uint32_t nb, uint32_t* tmp,
                                              uint32_t* total) {
  // each thread sums two entries; inclusive scan of those sums inside each
  // wavefront by lane shuffles, then of the wavefront totals by the first
  // wavefront (three barriers in all)
  constexpr int NWV = LS_WG / 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const uint32_t i0 = 2u * tid, i1 = i0 + 1;
  const uint32_t a = i0 < nb ? cnt[i0] : 0u, b = i1 < nb ? cnt[i1] : 0u;
  const uint32_t s = a + b;
  uint32_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t t = lane < NWV ? tmp[lane] : 0u;
#pragma unroll
    for (int d = 1; d < NWV; d <<= 1) {
      const uint32_t y = __shfl_up(t, d, 64);
      if (lane >= d) t += y;
    }
    if (lane < NWV) tmp[NWV + lane] = t;
  }
  __syncthreads();
  const uint32_t incl = (wid ? tmp[NWV + wid - 1] : 0u) + x;
  const uint32_t ex = incl - s;
  if (i0 < nb) off[i0] = ex;
  if (i1 < nb) off[i1] = ex + a;
  if (tid == LS_WG - 1) *total = incl;
  __syncthreads();
}

__global__ __launch_bounds__(256) void ls_clear_kernel(LsBins bn, uint32_t nb_c, uint32_t nb) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) bn.cnt_f[i] = 0;
  if (i < nb_c) bn.cnt_c[i] = 0;
}

// Level 1, exact: coarse histogram of groups of LS_H1 consecutive chunks
// (one flush of LDS counts into the global counters per workgroup, which
// keeps the 1024 global counters from serialising the whole launch); a
// workgroup takes groups blockIdx.x, blockIdx.x + gridDim.x, ...
// The input is nch chunks, all full but the last, of last_len keys; chunk
// lengths come from these 32-bit counts rather than from a 64-bit
// min(n - base, chunk), which this compiler has been seen to lower into a
// select on a stale scalar condition code (every chunk then counted full).
// gate: if non-null, the launch does nothing unless *gate is set.
template <class K>
__global__ __launch_bounds__(LS_WG) void ls_hist1_kernel(const K* __restrict__ keys, uint32_t nch,
                                                         uint32_t last_len, const LsModel* md, LsBins bn,
                                                         Rebind rk, const int* gate) {
  __shared__ LsTable tb;
  __shared__ uint32_t h[LS_MAX_BINS];
  if (md->sample_fb || (gate && *gate == 0)) return;
  keys = rebind(keys, rk);
  ls_load_table(md, &tb);
  const uint32_t nbc = md->nbins_c;
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) h[i] = 0;
  __syncthreads();
  const LsUni U = ls_uni(&tb);
  constexpr int CHK = ls_chk<K>();
  const uint32_t ngroups = (nch + LS_H1 - 1) / LS_H1;
  for (uint32_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const uint32_t c_end = (g + 1) * LS_H1 < nch ? (g + 1) * LS_H1 : nch;
    for (uint32_t ci = g * LS_H1; ci < c_end; ++ci) {  // chunk index (workgroup-uniform)
      const uint32_t lim = ci + 1 < nch ? uint32_t(CHK) : last_len;
      const K* kb = keys + uint64_t(ci) * CHK;
      // full chunks (all but the last) run without per-element bounds checks
      auto body = [&](auto fullc) {
        constexpr bool FULL = decltype(fullc)::value;
        K kv[CHK / LS_WG];
#pragma unroll
        for (int r = 0; r < CHK / LS_WG; ++r) {
          const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
          kv[r] = (FULL || i < lim) ? kb[i] : K(0);
        }
#pragma unroll
        for (int r = 0; r < CHK / LS_WG; ++r) {
          const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
          if (FULL || i < lim) atomicAdd(&h[ls_bucket(&tb, U, kv[r]) >> U.fine_bits], 1u);
        }
      };
      if (lim == uint32_t(CHK)) body(std::true_type{}); else body(std::false_type{});
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG)
    if (h[i]) atomicAdd(&bn.cnt_c[i], h[i]);
}

// Level 1 plan, exact (one workgroup): coarse offsets, cursors, level-2
// chunk map (chunks of `chk` keys).  gate as in ls_hist1_kernel.
__global__ __launch_bounds__(LS_WG) void ls_plan1_kernel(LsModel* md, LsBins bn, uint32_t chk, const int* gate) {
  __shared__ uint32_t cnt[LS_MAX_BINS], off[LS_MAX_BINS], ch[LS_MAX_BINS], choff[LS_MAX_BINS], tmp[LS_WG];
  __shared__ uint32_t total, tch;
  if (md->sample_fb || (gate && *gate == 0)) return;
  const uint32_t nbc = md->nbins_c;
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    cnt[i] = bn.cnt_c[i];
    ch[i] = (cnt[i] + chk - 1) / chk;
  }
  __syncthreads();
  ls_block_scan(cnt, off, nbc, tmp, &total);
  ls_block_scan(ch, choff, nbc, tmp, &tch);
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    bn.off_c[i] = off[i];
    bn.cursor_c[i] = off[i];
    bn.chunk_start[i] = choff[i];
  }
  if (threadIdx.x == 0) {
    bn.off_c[nbc] = total;
    bn.chunk_start[nbc] = tch;
    md->total_chunks = tch;
  }
}

// Decision from the sorted sample, before any pass over the input.  The
// bucket function is non-decreasing, so the T sample keys s[i .. i+T-1] lie
// in one bucket exactly when b(s[i]) == b(s[i+T-1]); the host picks T so that
// T sample keys stand for at least twice a bucket's capacity.  BY_KEY: the
// pass before training, on equal keys (s[i] == s[i+T-1]), which share a
// bucket under any bucket function; else the pass on the compiled table's
// buckets.  Counts such windows (a run of L >= T sample keys gives L - T + 1
// of them) and the longest run, whose first key's thread finds the run's
// end by a binary search.  One thread per window start.
template <bool BY_KEY, class K>
__device__ __forceinline__ auto ls_run_id(const LsTable* tb, const LsUni& U, K key) {
  if constexpr (BY_KEY) return key; else return ls_bucket(tb, U, key);
}
template <class K, bool BY_KEY>
__global__ __launch_bounds__(256) void ls_sample_heavy_kernel(const K* __restrict__ sample, uint32_t S, uint32_t T,
                                                              LsModel* md) {
  __shared__ LsTable tb;
  __shared__ uint32_t cnt;
  if (md->sample_fb) return;  // decided by the pass before
  if constexpr (!BY_KEY) ls_load_table(md, &tb);
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  LsUni U{};
  if constexpr (!BY_KEY) U = ls_uni(&tb);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i + T - 1 < S) {  // T >= 2, S - T + 1 window starts
    const auto b = ls_run_id<BY_KEY>(&tb, U, sample[i]);
    if (b == ls_run_id<BY_KEY>(&tb, U, sample[i + T - 1])) {
      atomicAdd(&cnt, 1u);
      if (i == 0 || ls_run_id<BY_KEY>(&tb, U, sample[i - 1]) != b) {
        uint32_t lo = i + T - 1, hi = S - 1;  // last j with the same id
        while (lo < hi) {
          const uint32_t m = lo + (hi - lo + 1) / 2;
          if (ls_run_id<BY_KEY>(&tb, U, sample[m]) == b) lo = m; else hi = m - 1;
        }
        atomicMax(&md->sample_run, lo - i + 1);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt) atomicAdd(&md->sample_heavy, cnt);
}

// One thread, after each pass: fall back when the windows, each standing
// for n / S input keys, exceed twice the spill limit (a margin over the
// exact decision's limit, so the sample decides only clear cases); a
// fallback decided before training also skips it.  The counters start
// again from zero for the next pass.
__global__ void ls_sample_decide_kernel(LsModel* md, uint64_t n, uint32_t S, uint64_t spill_limit) {
  if (threadIdx.x != 0 || md->sample_fb) return;
  const uint64_t est = uint64_t(md->sample_heavy) * n / S;  // < 2^20 * 2^32
  md->sample_spill = est;
  md->sample_maxb = uint64_t(md->sample_run) * n / S;
  md->sample_fb = est > 2 * spill_limit ? 1 : 0;
  md->do_train = md->sample_fb ? 0 : 1;
  md->sample_heavy = 0;
  md->sample_run = 0;
}

// Level 1, estimated: coarse-bin counts of LS_EST * LS_WG keys per workgroup
// at random positions (draws 2^32 + i), added into cnt_c.
constexpr int LS_EST = 4;
template <class K>
__global__ __launch_bounds__(LS_WG) void ls_est1_kernel(const K* __restrict__ keys, uint64_t n, uint64_t seed,
                                                        const LsModel* md, LsBins bn, Rebind rk) {
  __shared__ LsTable tb;
  __shared__ uint32_t h[LS_MAX_BINS];
  if (md->sample_fb) return;
  keys = rebind(keys, rk);
  ls_load_table(md, &tb);
  const uint32_t nbc = md->nbins_c;
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) h[i] = 0;
  __syncthreads();
  const LsUni U = ls_uni(&tb);
  const uint64_t d0 = (uint64_t(1) << 32) + uint64_t(blockIdx.x) * (LS_EST * LS_WG) + threadIdx.x;
  K kv[LS_EST];
#pragma unroll
  for (int r = 0; r < LS_EST; ++r) kv[r] = keys[ls_draw(seed, d0 + uint64_t(r) * LS_WG, n)];
#pragma unroll
  for (int r = 0; r < LS_EST; ++r) atomicAdd(&h[ls_bucket(&tb, U, kv[r]) >> U.fine_bits], 1u);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG)
    if (h[i]) atomicAdd(&bn.cnt_c[i], h[i]);
}

// Estimated level 1 plan (one workgroup): c sampled keys in bin i, each
// standing for q input keys, give the bin a region of c q + c q / 4 + 32 q
// keys rounded up to a multiple of 64 (a bin that truly holds more than
// that is some 4.5 standard deviations or more out for 64 to 1024 sampled
// keys per bin); cursors at the region starts, region ends in off_c[i + 1].
// The host sizes the buffer for the sum of these bounds.
__global__ __launch_bounds__(LS_WG) void ls_plan1_est_kernel(LsModel* md, LsBins bn, uint32_t q) {
  __shared__ uint32_t r[LS_MAX_BINS], off[LS_MAX_BINS], tmp[LS_WG];
  __shared__ uint32_t total;
  if (md->sample_fb) return;
  const uint32_t nbc = md->nbins_c;
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    const uint64_t e = uint64_t(bn.cnt_c[i]) * q;
    r[i] = uint32_t((e + (e >> 2) + uint64_t(32) * q + 63) & ~uint64_t(63));
  }
  __syncthreads();
  ls_block_scan(r, off, nbc, tmp, &total);
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    bn.off_c[i] = off[i];
    bn.cursor_c[i] = off[i];
  }
  if (threadIdx.x == 0) bn.off_c[nbc] = total;
}

// After the estimated scatter (one workgroup): the exact counts are the
// cursors' advances; level-2 chunk map from them.  If a region was too
// small (or `force`), the counts are cleared instead and *l1_over stays set,
// which opens the gated exact pass that follows.
__global__ __launch_bounds__(LS_WG) void ls_fin1_kernel(LsModel* md, LsBins bn, uint32_t chk, int force) {
  __shared__ uint32_t ch[LS_MAX_BINS], choff[LS_MAX_BINS], tmp[LS_WG];
  __shared__ uint32_t tch;
  if (md->sample_fb) return;  // (l1_over stays clear: the gated exact pass stays off)
  const uint32_t nbc = md->nbins_c;
  if (force || md->l1_over) {  // workgroup-uniform
    for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) bn.cnt_c[i] = 0;
    if (threadIdx.x == 0) md->l1_over = 1;
    return;
  }
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    const uint32_t c = bn.cursor_c[i] - bn.off_c[i];
    bn.cnt_c[i] = c;
    ch[i] = (c + chk - 1) / chk;
  }
  __syncthreads();
  ls_block_scan(ch, choff, nbc, tmp, &tch);
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) bn.chunk_start[i] = choff[i];
  if (threadIdx.x == 0) {
    bn.chunk_start[nbc] = tch;
    md->total_chunks = tch;
  }
}

// Shared body of the two scatters: counting sort of one chunk by bin in LDS,
// one reservation per non-empty bin, then coalesced runs to the destination.
// Without staged bins (ls_sbin<K>() = 0) the write-out recomputes each
// staged key's bin instead of keeping it in LDS (16 KB less LDS per
// workgroup): 64-bit keys, whose 64 KB of staged keys would otherwise leave
// room for one workgroup per CU.
#ifndef MS_LS_SBIN
#define MS_LS_SBIN 1
#endif
template <class K>
__host__ __device__ constexpr int ls_sbin() { return sizeof(K) == 4 ? MS_LS_SBIN : 0; }
template <class K>
struct LsScatterLds {
  uint32_t cnt[LS_MAX_BINS], off[LS_MAX_BINS], gb[LS_MAX_BINS], tmp[LS_WG];
  K stage[ls_chk<K>()];
  uint16_t sbin[ls_sbin<K>() ? ls_chk<K>() : 1];
  uint32_t total;
};

// Level 1 scatter: chunks blockIdx.x, blockIdx.x + gridDim.x, ... of the
// input into coarse buckets (chunks as in ls_hist1_kernel).  gate as in
// ls_hist1_kernel.  over: if non-null the regions are estimated, and a
// reservation that would pass its region's end (off_c[bin + 1]) writes
// nothing and sets *over (the exact pass then redoes the level).
constexpr uint32_t LS_NO_ROOM = 0xFFFFFFFFu;
template <class K>
__global__ __launch_bounds__(LS_WG) void ls_scatter1_kernel(const K* __restrict__ keys, uint32_t nch,
                                                            uint32_t last_len, const LsModel* md, LsBins bn,
                                                            K* __restrict__ out, Rebind rkeys, const int* gate,
                                                            int* over) {
  __shared__ LsTable tb;
  __shared__ LsScatterLds<K> L;
  if (md->sample_fb || (gate && *gate == 0)) return;
  keys = rebind(keys, rkeys);
  ls_load_table(md, &tb);
  const uint32_t nbc = md->nbins_c;
  __syncthreads();
  const LsUni U = ls_uni(&tb);
  constexpr int CHK = ls_chk<K>();
  constexpr int R = CHK / LS_WG;
  for (uint32_t ci = blockIdx.x; ci < nch; ci += gridDim.x) {
    for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) L.cnt[i] = 0;
    __syncthreads();
    const uint32_t lim = ci + 1 < nch ? uint32_t(CHK) : last_len;
    const K* kb = keys + uint64_t(ci) * CHK;
    K kv[R];
    uint32_t bin[R], rk[R];
    // full chunks (all but the last) run without per-element bounds checks
    auto rank = [&](auto fullc) {
      constexpr bool FULL = decltype(fullc)::value;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
        kv[r] = (FULL || i < lim) ? kb[i] : K(0);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
        if (FULL || i < lim) {
          bin[r] = ls_bucket(&tb, U, kv[r]) >> U.fine_bits;
          rk[r] = atomicAdd(&L.cnt[bin[r]], 1u);
        }
      }
    };
    auto stage = [&](auto fullc) {
      constexpr bool FULL = decltype(fullc)::value;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
        if (FULL || i < lim) {
          const uint32_t p = L.off[bin[r]] + rk[r];
          L.stage[p] = kv[r];
          if constexpr (ls_sbin<K>()) L.sbin[p] = uint16_t(bin[r]);
        }
      }
    };
    const bool full = lim == uint32_t(CHK);
    if (full) rank(std::true_type{}); else rank(std::false_type{});
    __syncthreads();
    ls_block_scan(L.cnt, L.off, nbc, L.tmp, &L.total);
    for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
      const uint32_t c = L.cnt[i];
      if (c) {
        const uint32_t g = atomicAdd(&bn.cursor_c[i], c);
        // checked on the keys the bin reserved before this chunk, g - off_c[i]
        // (exact: fewer than n < 2^32), not on g itself, which passes 2^32
        // and wraps when a region near the buffer's end is far too small
        if (over && uint64_t(g - bn.off_c[i]) + c > uint64_t(bn.off_c[i + 1] - bn.off_c[i])) {
          L.gb[i] = LS_NO_ROOM;
          *over = 1;
        } else {
          L.gb[i] = g;
        }
      }
    }
    if (full) stage(std::true_type{}); else stage(std::false_type{});
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < L.total; i += LS_WG) {
      const K x = L.stage[i];
      const uint32_t b = ls_sbin<K>() ? uint32_t(L.sbin[i]) : ls_bucket(&tb, U, x) >> U.fine_bits;
      const uint32_t g = L.gb[b];
      if (g != LS_NO_ROOM) out[g + (i - L.off[b])] = x;
    }
  }
}

// Level-2 chunk w -> coarse bucket c and key range [lo, hi).
__device__ __forceinline__ bool ls_chunk(const LsModel* md, const LsBins& bn, uint32_t w, uint32_t chk,
                                         uint32_t* c, uint32_t* lo, uint32_t* hi) {
  if (w >= md->total_chunks) return false;
  uint32_t a = 0, b = md->nbins_c;  // largest c with chunk_start[c] <= w
  while (b - a > 1) {
    const uint32_t m = (a + b) >> 1;
    if (bn.chunk_start[m] <= w) a = m; else b = m;
  }
  *c = a;
  const uint32_t j = w - bn.chunk_start[a];
  const uint32_t s = bn.off_c[a] + j * chk, e = bn.off_c[a] + bn.cnt_c[a];
  *lo = s;
  *hi = s + chk < e ? s + chk : e;
  return true;
}

// Level 2 histogram: fine-bucket counts of one chunk of a coarse bucket.
template <class K>
__global__ __launch_bounds__(LS_WG) void ls_hist2_kernel(const K* __restrict__ keys, const LsModel* md,
                                                         LsBins bn) {
  __shared__ LsTable tb;
  __shared__ uint32_t h[LS_MAX_BINS];
  if (md->sample_fb) return;  // (the chunk map was not built)
  constexpr int CHK = ls_chk<K>();
  uint32_t c, lo, hi;
  if (!ls_chunk(md, bn, blockIdx.x, CHK, &c, &lo, &hi)) return;
  ls_load_table(md, &tb);
  const uint32_t nbf = md->nbins_f;
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG) h[i] = 0;
  __syncthreads();
  const LsUni U = ls_uni(&tb);
  constexpr int R = CHK / LS_WG;
  const uint32_t lim = hi - lo;
  const K* kb = keys + lo;
  const uint32_t fmask = nbf - 1;
  // full chunks run without per-element bounds checks
  auto body = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
    K kv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
      kv[r] = (FULL || i < lim) ? kb[i] : K(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
      if (FULL || i < lim) atomicAdd(&h[ls_bucket(&tb, U, kv[r]) & fmask], 1u);
    }
  };
  if (lim == uint32_t(CHK)) body(std::true_type{}); else body(std::false_type{});
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG)
    if (h[i]) atomicAdd(&bn.cnt_f[(c << U.fine_bits) | i], h[i]);
}

// Per coarse bucket (one workgroup each): kept / spilled totals and the
// largest bucket.
__global__ __launch_bounds__(LS_WG) void ls_totals_kernel(const LsModel* md, LsBins bn, uint32_t capacity) {
  __shared__ uint32_t kept, spill, maxb;
  const uint32_t c = blockIdx.x;
  const uint32_t nbf = md->nbins_f;
  const uint32_t b0 = c << md->fine_bits;
  if (threadIdx.x == 0) kept = spill = maxb = 0;
  __syncthreads();
  uint32_t k_acc = 0, s_acc = 0, m_acc = 0;
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG) {
    const uint32_t k = bn.cnt_f[b0 + i];
    if (k > capacity) s_acc += k; else k_acc += k;
    m_acc = k > m_acc ? k : m_acc;
  }
  if (k_acc) atomicAdd(&kept, k_acc);
  if (s_acc) atomicAdd(&spill, s_acc);
  if (m_acc) atomicMax(&maxb, m_acc);
  __syncthreads();
  if (threadIdx.x == 0) {
    bn.kept_tot[c] = kept;
    bn.spill_tot[c] = spill;
    bn.cmaxb[c] = maxb;
  }
}

// Decision (one workgroup): kept / spill bases, the order check across coarse
// buckets, fallback and repair flags, where the kept buckets live.
template <class K>
__global__ __launch_bounds__(LS_WG) void ls_plan2_kernel(LsModel* md, LsBins bn, uint64_t n, uint64_t spill_limit,
                                                         int force_fallback, K* d_keys, K* xr, Rebind rk) {
  __shared__ uint32_t k[LS_MAX_BINS], sp[LS_MAX_BINS], kb[LS_MAX_BINS], sb[LS_MAX_BINS], tmp[LS_WG];
  __shared__ uint32_t ktot, stot;
  d_keys = rebind(d_keys, rk);
  const uint32_t nbc = md->nbins_c;
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    k[i] = bn.kept_tot[i];
    sp[i] = bn.spill_tot[i];
  }
  __syncthreads();
  ls_block_scan(k, kb, nbc, tmp, &ktot);
  ls_block_scan(sp, sb, nbc, tmp, &stot);
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) {
    bn.kept_base[i] = kb[i];
    bn.spill_base[i] = sb[i];
  }
  __shared__ uint32_t cm[LS_MAX_BINS];
  for (uint32_t i = threadIdx.x; i < nbc; i += LS_WG) cm[i] = bn.cmaxb[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t maxb = 0;
    for (uint32_t c = 0; c < nbc; ++c) maxb = cm[c] > maxb ? cm[c] : maxb;
    const uint64_t s = stot;
    const int sfb = md->sample_fb;
    const int fb = (sfb || force_fallback || s > spill_limit || uint64_t(ktot) + s != n) ? 1 : 0;
    md->misordered = 0;
    md->fallback = fb;
    md->do_learned = fb ? 0 : 1;
    md->do_repair = (!fb && s > 0) ? 1 : 0;
    // after the sample's decision no key was counted: its estimates instead
    md->spilled = sfb ? md->sample_spill : s;
    md->kept = ktot;
    md->max_bucket = sfb ? md->sample_maxb : maxb;
    md->r_keys = (s == 0) ? static_cast<void*>(d_keys) : static_cast<void*>(xr);
    md->r_base = (s == 0) ? 0 : s;
  }
}

// Fine offsets (one workgroup per coarse bucket): scatter cursors and the
// kept-bucket segments of the bucket sort (all empty on fallback).
__global__ __launch_bounds__(LS_WG) void ls_offsets_kernel(const LsModel* md, LsBins bn, uint32_t capacity) {
  __shared__ uint32_t kc[LS_MAX_BINS], sc[LS_MAX_BINS], ko[LS_MAX_BINS], so[LS_MAX_BINS], tmp[LS_WG];
  __shared__ uint32_t kt, st;
  const uint32_t c = blockIdx.x;
  const uint32_t nbf = md->nbins_f;
  const uint32_t b0 = c << md->fine_bits;
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG) {
    const uint32_t k = bn.cnt_f[b0 + i];
    kc[i] = k <= capacity ? k : 0u;
    sc[i] = k > capacity ? k : 0u;
  }
  __syncthreads();
  ls_block_scan(kc, ko, nbf, tmp, &kt);
  ls_block_scan(sc, so, nbf, tmp, &st);
  const bool on = md->do_learned != 0;
  const uint64_t rb = md->r_base;
  const uint32_t kbase = bn.kept_base[c], sbase = bn.spill_base[c];
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG) {
    const uint32_t kpos = uint32_t(rb) + kbase + ko[i];
    bn.cursor_f[b0 + i] = sc[i] ? sbase + so[i] : kpos;
    bn.seg_off[b0 + i] = on ? int64_t(kpos) : 0;
  }
  if (c == md->nbins_c - 1 && threadIdx.x == 0)
    bn.seg_off[(uint64_t(c) << md->fine_bits) + nbf] = on ? int64_t(rb + md->kept) : 0;
}

// Level 2 scatter: keys of a coarse chunk into their fine buckets, kept
// buckets into the kept array, spilled ones into the spill area.
template <class K>
__global__ __launch_bounds__(LS_WG) void ls_scatter2_kernel(const K* __restrict__ keys, const LsModel* md,
                                                            LsBins bn, uint32_t capacity, K* xr) {
  __shared__ LsTable tb;
  __shared__ LsScatterLds<K> L;
  __shared__ uint8_t kept[LS_MAX_BINS];
  if (md->do_learned == 0) return;
  constexpr int CHK = ls_chk<K>();
  uint32_t c, lo, hi;
  if (!ls_chunk(md, bn, blockIdx.x, CHK, &c, &lo, &hi)) return;
  ls_load_table(md, &tb);
  const uint32_t nbf = md->nbins_f;
  const uint32_t b0 = c << md->fine_bits;
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG) L.cnt[i] = 0;
  __syncthreads();
  const LsUni U = ls_uni(&tb);
  constexpr int R = CHK / LS_WG;
  const uint32_t fmask = nbf - 1;
  const uint32_t lim = hi - lo;
  const K* kb = keys + lo;
  K kv[R];
  uint32_t bin[R], rk[R];
  // full chunks run without per-element bounds checks
  auto rank = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
      kv[r] = (FULL || i < lim) ? kb[i] : K(0);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
      if (FULL || i < lim) {
        bin[r] = ls_bucket(&tb, U, kv[r]) & fmask;
        rk[r] = atomicAdd(&L.cnt[bin[r]], 1u);
      }
    }
  };
  auto stage = [&](auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t i = threadIdx.x + uint32_t(r) * LS_WG;
      if (FULL || i < lim) {
        const uint32_t p = L.off[bin[r]] + rk[r];
        L.stage[p] = kv[r];
        if constexpr (ls_sbin<K>()) L.sbin[p] = uint16_t(bin[r]);
      }
    }
  };
  const bool full = lim == uint32_t(CHK);
  if (full) rank(std::true_type{}); else rank(std::false_type{});
  __syncthreads();
  ls_block_scan(L.cnt, L.off, nbf, L.tmp, &L.total);
  for (uint32_t i = threadIdx.x; i < nbf; i += LS_WG)
    if (L.cnt[i]) {
      L.gb[i] = atomicAdd(&bn.cursor_f[b0 + i], L.cnt[i]);
      kept[i] = bn.cnt_f[b0 + i] <= capacity ? 1 : 0;
    }
  if (full) stage(std::true_type{}); else stage(std::false_type{});
  __syncthreads();
  K* rk_arr = global_ptr<K>(&md->r_keys);
  for (uint32_t i = threadIdx.x; i < L.total; i += LS_WG) {
    const K x = L.stage[i];
    const uint32_t b = ls_sbin<K>() ? uint32_t(L.sbin[i]) : (ls_bucket(&tb, U, x) & fmask);
    K* dst = kept[b] ? rk_arr : xr;
    dst[L.gb[b] + (i - L.off[b])] = x;
  }
}

// The order check: after the bucket sort, the kept buckets (each sorted, laid out
// in bucket order from r_base) must meet in order.  One thread per bucket
// compares the key before the bucket's first position with its first key;
// a failure sends the keys (a permutation of the input) to the plain merge
// sort.
template <class K>
__global__ __launch_bounds__(256) void ls_check_kernel(LsModel* md, LsBins bn, uint64_t nb) {
  if (md->do_learned == 0) return;
  const uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t lo = bn.seg_off[b], hi = bn.seg_off[b + 1];
  if (hi <= lo || uint64_t(lo) <= md->r_base) return;
  const K* rk = global_ptr<const K>(&md->r_keys);
  if (rk[lo] < rk[lo - 1]) {
    md->misordered = 1;
    md->fallback = 1;
  }
}

}  // namespace ms

/*
 * msort.h -- C ABI of the gfx950 (MI355X) stable merge sort library.
 *
 * The operation is the stable merge sort of integer arrays that the paper
 * "Approaches to the Parallelization of Merge Sort in Python" (arXiv
 * 2211.16479) parallelises on CPUs: sections "Sequential Merge Sort" (what a
 * merge sort computes), "Multiprocessing Merge Sort" (independent sorts of
 * equal chunks) and "Merging the subarrays" (a tree of pairwise merges).
 * Here the chunks are GPU tiles and every tree level is one merge pass.
 *
 * Result (every entry point): ascending order; unsigned comparison for
 * MS_KEY_U32 / MS_KEY_U64, signed for MS_KEY_I32 / MS_KEY_I64; stable -- equal
 * keys keep their input order and values move with their keys.  Because the
 * sort is stable the result is unique, and it is bit-identical on every run.
 *
 * Conventions shared by all entry points
 *  - Pointers named d_* are device pointers on the current HIP device.  The
 *    caller owns them; the library never frees or retains them.  Key and
 *    value buffers must not overlap.  Results overwrite the inputs.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls only enqueue work on it and return; results are valid once the
 *    stream has been synchronised.  Calls on different streams may run
 *    concurrently (each stream gets its own library scratch).
 *  - Arguments are checked before anything is enqueued: a failed check
 *    enqueues nothing.  n == 0 (or num_segments == 0) is a no-op returning
 *    MS_OK.  A NULL pointer with n > 0 is MS_ERR_INVALID_ARG; an unknown key
 *    type or a value width other than 4 or 8 is MS_ERR_UNSUPPORTED.  HIP
 *    launch or allocation failures return MS_ERR_HIP / MS_ERR_OUT_OF_MEMORY.
 *    No C++ exception crosses this ABI.  ms_last_error() describes the last
 *    failure on the calling thread.
 *  - Scratch: by default the library allocates device scratch itself, in
 *    stream order (hipMallocAsync), once per (device, stream), and keeps it
 *    for reuse until ms_release_workspace() or process exit.
 */
#ifndef MSORT_H
#define MSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ms_key_type {
  MS_KEY_U32 = 0,
  MS_KEY_I32 = 1,
  MS_KEY_U64 = 2,
  MS_KEY_I64 = 3
} ms_key_type;

typedef enum ms_status {
  MS_OK = 0,
  MS_ERR_INVALID_ARG = 1,
  MS_ERR_UNSUPPORTED = 2,
  MS_ERR_OUT_OF_MEMORY = 3,
  MS_ERR_HIP = 4,
  MS_ERR_INTERNAL = 5
} ms_status;

/* Library version as major * 10000 + minor * 100 + patch. */
int ms_version(void);

/* Number of hipGraphs captured so far by this process (the segmented and
 * learned forms capture one per device, stream and size/option set and
 * replay it on any buffers); for tests and diagnostics. */
uint64_t ms_graph_captures(void);

/*
 * ms_device_errors -- internal-consistency checks done by the kernels of the
 * current device since the last call (then cleared): bit 0 (value 1) = a
 * fused merge tile received partition offsets that do not describe its
 * pieces and was left unwritten.  Nonzero means a library bug, never a
 * property of the input.  Synchronises the device.  flags may be NULL.
 */
ms_status ms_device_errors(uint32_t* flags);

/* Static text for a status code; never NULL. */
const char* ms_status_string(ms_status s);

/* Text of the last failure reported on the calling thread ("" if none).
 * The pointer stays valid until the next library call on this thread. */
const char* ms_last_error(void);

/*
 * ms_sort -- sort n keys in place, ascending.
 *   d_keys : device array of n keys of type kt (4-byte keys for U32/I32,
 *            8-byte keys for U64/I64), any alignment of the element type.
 * Keys only: equal keys are identical bits, so stability is unobservable and
 * the result is the unique sorted sequence.
 * Method: tile sort (one workgroup per tile), then ceil(log2(n / tile))
 * merge-path passes; each pass is a partition kernel and a merge kernel.
 * Keys-only sorts of at most 2^22 keys replay a cached hipGraph from the
 * second call with the same key type and n on a stream (the buffer is
 * bound per launch; the graph owns ms_temp_bytes(n, kt, 0) bytes of
 * scratch); other sizes, and first calls, enqueue the kernels directly.
 */
ms_status ms_sort(void* d_keys, size_t n, ms_key_type kt, void* stream);

/*
 * ms_sort_pairs -- stable sort of (key, value) pairs by key.
 *   d_keys    : n keys of type kt, sorted in place.
 *   d_vals    : n values of val_bytes bytes each (4 or 8), moved with their
 *               keys; values are opaque bits, never compared.
 * Equal keys keep their input order (left run wins ties in every merge).
 */
ms_status ms_sort_pairs(void* d_keys, void* d_vals, size_t n, ms_key_type kt, size_t val_bytes,
                        void* stream);

/*
 * ms_segmented_sort -- sort many independent arrays with one graph launch.
 *   d_keys          : n_total keys of type kt; segment s is
 *                     d_keys[d_offsets[s], d_offsets[s+1]) and is sorted in
 *                     place, ascending and stable, independently of the others.
 *   d_vals          : NULL when val_bytes == 0 (keys only), otherwise n_total
 *                     values of val_bytes (4 or 8) bytes moved with their keys.
 *   d_offsets       : device array of num_segments + 1 int64 offsets,
 *                     non-decreasing, d_offsets[0] == 0 and
 *                     d_offsets[num_segments] == n_total.  Empty segments are
 *                     allowed.  The library does not check these conditions
 *                     (they live on the device); violating them is undefined.
 *   max_segment_len : a hint: an upper bound on segment lengths, or 0 if
 *                     unknown (then n_total).  Merge passes up to the hint
 *                     run over every reserved tile at full width; the passes
 *                     that longer segments (up to n_total) would need are in
 *                     the graph too, with a small grid, and return at once
 *                     unless the device finds such a segment.  A hint that is
 *                     too small therefore costs time, never correctness.
 * Limits: fewer than 2^26 segments and n_total < 2^32 per call, otherwise
 * MS_ERR_UNSUPPORTED.
 * Segments are binned by length on the device into small classes, each sorted
 * by a persistent kernel entirely in LDS (per-class workgroup size and items
 * per thread from the tuning table), and a large class sorted by tiles plus
 * merge passes that stay inside the segment.  The whole pipeline is captured
 * once into a hipGraph (cached per device, stream, num_segments, n_total,
 * max_segment_len, key/value type and tuning table; up to 8 graphs, each
 * owning its scratch of ms_temp_bytes_segmented bytes) and replayed with one
 * hipGraphLaunch on `stream`, preceded by a one-thread kernel that binds this
 * call's buffers: new buffers of the same sizes replay the same graph.  This
 * is the batched form of the paper's chunk-parallel sort (section
 * "Multiprocessing Merge Sort"), with each array a chunk.
 */
ms_status ms_segmented_sort(void* d_keys, void* d_vals, const int64_t* d_offsets, size_t num_segments,
                            size_t n_total, size_t max_segment_len, ms_key_type kt, size_t val_bytes,
                            void* stream);

/*
 * Size classes and the autotuned per-class shapes of ms_segmented_sort.
 * A family is (kt, val_bytes with 0 = keys only).  Class c holds segments of
 * length <= max_len (class bounds increase with c); longer segments form the
 * large class.  Each small class has num_candidates compiled shapes
 * (workgroup size wg, items per thread ipt, wg * ipt == max_len); the tuning
 * table picks one per class (candidate 0 until set).  All host-only.
 *   ms_seg_num_classes : number of small classes of the family.
 *   ms_seg_class_info  : bound and candidate count of class cls.
 *   ms_seg_candidate   : shape of candidate idx of class cls.
 *   ms_tuning_set      : select the candidate with shape (wg, ipt) for cls;
 *                        MS_ERR_UNSUPPORTED if no such shape is compiled.
 *   ms_tuning_get      : the shape currently selected for cls.
 *   ms_tuning_load     : apply a tuning file: lines "arch key_type value_bytes
 *                        class wg ipt" (key_type u32|i32|u64|i64, '#' starts a
 *                        comment line); only lines whose arch equals `arch`
 *                        (NULL = the current device's, e.g. "gfx950") are
 *                        applied; *applied (may be NULL) gets their count.
 * Changing the table makes later calls capture new graphs.
 */
ms_status ms_seg_num_classes(ms_key_type kt, size_t val_bytes, int* num_classes);
ms_status ms_seg_class_info(ms_key_type kt, size_t val_bytes, int cls, uint32_t* max_len, int* num_candidates);
ms_status ms_seg_candidate(ms_key_type kt, size_t val_bytes, int cls, int idx, int* wg, int* ipt);
ms_status ms_tuning_set(ms_key_type kt, size_t val_bytes, int cls, int wg, int ipt);
ms_status ms_tuning_get(ms_key_type kt, size_t val_bytes, int cls, int* wg, int* ipt);
ms_status ms_tuning_load(const char* path, const char* arch, int* applied);

/* ------------------------------------------------------------------------
 * Learned-bucket form (all four key types).  A small two-layer ReLU MLP
 *   F(x) = b2 + sum_h w2_h * relu(w1_h * x + b1_h),   H = 16 hidden units,
 * of a feature x of the key is trained on the GPU to map keys to normalised
 * ranks.  Features: uint32 keys u, MS_FEATURE_LOG a monotone
 * piecewise-linear log2(1 + u) / 32 computed from the float bits and
 * MS_FEATURE_LINEAR u * 2^-32; the other types, with u the key's
 * order-preserving unsigned image (the sign bit flipped for signed types),
 * the same two forms of the offset d = u - u0 (0 below u0), where u0 lies
 * 1/64 of the sample's range below the sample's smallest u (or is 0):
 * (float bits of 1 + d minus those of 1.0) * 2^-29, and d * 2^-e with e the
 * bit length of (the sample's largest u) - u0.  Training runs on a
 * sample of 2^sample_log2 keys that the plain merge sort ranks: closed-form
 * start at the piecewise-linear interpolant through 16 sample quantiles,
 * then full-batch Adam on the mean squared rank error.  The trained network
 * is evaluated as the piecewise-linear function it is, on the sample's
 * feature range with the ends pinned to the sample's extreme mid-ranks,
 * through a running-max envelope, and beyond that range along its first and
 * last segments (clipped to [0, 1]), so bucket ids floor(F(x) * B) are
 * non-decreasing in the key.
 * Keys are scattered (two levels) into B ~ n / bucket_fill buckets (the
 * first level into regions sized from a random sample, see coarse_estimate);
 * buckets of at most bucket_capacity keys (64-bit keys: at most 4096, the
 * largest bucket one workgroup sorts in LDS) are sorted in LDS; larger ones
 * spill.  The spill is sorted by the plain merge sort and merged back with
 * one exact merge-path pass.  If more than spill_threshold * n keys spill, or
 * the order check of the buckets fails, the plain merge sort sorts the input
 * instead (decided on the device); where the sorted sample already shows
 * more than twice that many keys in over-full buckets (heavy ties), the plain
 * sort runs before any pass over the input (stats.sample_fallback).  The
 * output is the same bytes as ms_sort's.
 * ------------------------------------------------------------------------ */
typedef enum ms_algo {
  MS_ALGO_AUTO = 0,            /* learned for 32-bit keys from n = 2^27 and 64-bit keys from 2^26
                                  (where it measured faster), else merge path */
  MS_ALGO_MERGE_PATH = 1,
  MS_ALGO_LEARNED_BUCKET = 2
} ms_algo;

/* MS_FEATURE_AUTO: log for uint32 keys, linear for the other types (a log
 * of the offset from the sample's smallest key crowds the lower tail of a
 * symmetric distribution into a few buckets). */
typedef enum ms_feature { MS_FEATURE_LOG = 0, MS_FEATURE_LINEAR = 1, MS_FEATURE_AUTO = 2 } ms_feature;

typedef struct ms_options {
  int algo;                  /* ms_algo */
  float spill_threshold;     /* fall back when spilled keys > this * n; [0, 0.5], default 0.05 */
  uint32_t bucket_capacity;  /* keys sorted per LDS bucket: 4096 or 16384 (default) */
  uint32_t bucket_fill;      /* target mean keys per bucket, 64..capacity; 0 (default): 512 for
                                32-bit keys, 256 for 64-bit keys */
  uint32_t train_steps;      /* Adam steps, default 16 */
  float learning_rate;       /* default 1e-4 */
  uint32_t sample_log2;      /* log2 of the sample size, 10..20; 0 (default): 16 for 32-bit keys,
                                18 for 64-bit keys (about n / 2^sample_log2 keys fall beyond each
                                of the sample's extremes and share one end bucket) */
  uint64_t seed;             /* sample positions, default 0 */
  int feature;               /* ms_feature, default MS_FEATURE_AUTO */
  int use_network;           /* 1 (default); 0: bucket = floor(x * B) with no network */
  int force_fallback;        /* 1: always take the plain merge sort (testing) */
  int use_graph;             /* 1 (default): replay a cached hipGraph of the pipeline */
  uint32_t max_workgroups;   /* merge path only, measurement support: at most this many workgroups per
                                launch, each looping over tiles (the worker count of a scaling study);
                                0 (default) = one workgroup per tile */
  int coarse_estimate;       /* learned form, first scatter level: 1 (default) sizes each coarse
                                bucket's region from a random sample of the input (n >= 2^23:
                                min(2^20, n / 128) keys) instead of counting every key first; a
                                region found too small during the scatter is detected and the exact
                                count-then-scatter pass runs instead (stats.coarse_recounted);
                                0: always the exact pass; 2: estimate, then always recount (testing) */
} ms_options;

/* Written on the device when the sort completes (valid after the stream). */
typedef struct ms_stats {
  int32_t algo_used;         /* MS_ALGO_MERGE_PATH or MS_ALGO_LEARNED_BUCKET */
  int32_t fallback_taken;    /* the learned path handed over to the plain sort */
  int32_t misordered;        /* the bucket order check failed */
  int32_t repaired;          /* a spill was sorted and merged back */
  uint64_t spilled;          /* keys in over-full buckets (estimated from the sample when
                                sample_fallback is set) */
  uint64_t max_bucket;       /* largest bucket (likewise) */
  uint64_t buckets;          /* number of buckets B */
  float loss_initial;        /* training loss at the start point */
  float loss_final;          /* training loss before the last step */
  int32_t coarse_recounted;  /* the estimated first-level regions were replaced by the exact pass */
  int32_t sample_fallback;   /* the sorted sample already showed more than twice spill_threshold * n
                                keys in over-full buckets (runs of sample keys that stand for at
                                least twice a bucket's capacity each), so the plain sort ran with no
                                pass of the learned form over the input */
} ms_stats;

/* Default options (as documented above). */
void ms_options_default(ms_options* opt);

/*
 * ms_sort_ex -- ms_sort with a choice of algorithm.  opt may be NULL
 * (defaults); d_stats may be NULL, otherwise a device pointer to one
 * ms_stats.  MS_ALGO_LEARNED_BUCKET requires n >= 4 * 2^sample_log2 (the
 * resolved value: 2^20 keys for 64-bit keys by default) and
 * n < 2^32 (else MS_ERR_UNSUPPORTED); invalid options give
 * MS_ERR_INVALID_ARG.  The learned pipeline is replayed from a cached
 * hipGraph (use_graph = 1) keyed by the key type, n, whether d_stats is NULL
 * and the options (not by the buffers, which are bound per launch); the
 * graph owns ms_temp_bytes_learned(n, kt, opt) bytes of scratch.
 */
ms_status ms_sort_ex(void* d_keys, size_t n, ms_key_type kt, const ms_options* opt, ms_stats* d_stats,
                     void* stream);
size_t ms_temp_bytes_learned(size_t n, ms_key_type kt, const ms_options* opt);

/*
 * ms_sort_pairs_ex -- ms_sort_pairs with a choice of algorithm (stable, as
 * ms_sort_pairs).  MS_ALGO_LEARNED_BUCKET (32-bit keys, values of 4 or 8
 * bytes, n >= 4 * 2^sample_log2 with the 64-bit keys' default 2^18 when 0,
 * n < 2^32; else MS_ERR_UNSUPPORTED): each key and its input position are
 * packed into one 64-bit key (the key's order-preserving unsigned image
 * above, the position below), the packed keys are sorted by the learned
 * form for 64-bit keys (options as for ms_sort_ex, their 64-bit defaults;
 * MS_FEATURE_AUTO: log for uint32 keys, linear for int32),
 * then the keys are unpacked and the values gathered by position.  Packed
 * keys are distinct, so equal keys keep their input order.  Heavy ties
 * (one key over a bucket's capacity) spill or fall back to the plain sort,
 * exact either way.  MS_ALGO_AUTO and MS_ALGO_MERGE_PATH run ms_sort_pairs.
 * d_stats as for ms_sort_ex.  The cached graph (use_graph = 1) is keyed by
 * key type, value width, n, whether d_stats is NULL and the options, and
 * owns ms_temp_bytes_learned_pairs(n, kt, val_bytes, opt) bytes of scratch
 * (0 for unsupported arguments).
 */
ms_status ms_sort_pairs_ex(void* d_keys, void* d_vals, size_t n, ms_key_type kt, size_t val_bytes,
                           const ms_options* opt, ms_stats* d_stats, void* stream);
size_t ms_temp_bytes_learned_pairs(size_t n, ms_key_type kt, size_t val_bytes, const ms_options* opt);

/*
 * Steps of the learned form on uint32 keys, for tests and inspection (all device pointers;
 * parameters theta are 49 floats laid out [w1 x16, b1 x16, w2 x16, b2]):
 *   ms_learned_grad   : at theta, over the sorted sample (S keys, target of
 *                       position i = (i + 0.5) / S), write the gradient of the
 *                       mean squared error (49 floats) and the sum of squared
 *                       errors (1 float) to d_out[50].
 *   ms_learned_train  : from d_theta0 (NULL: the quantile start point) run
 *                       `steps` Adam steps; write the parameters to
 *                       d_theta_out[49] and, if d_loss_hist is not NULL, the
 *                       loss before each step to d_loss_hist[steps].
 *   ms_learned_table  : the inference table of theta on the sorted sample's
 *                       feature range: points d_t[32] (ascending, +inf
 *                       padded), values d_v[32], count d_count[1].
 *   ms_learned_bucket_ids : bucket id in [0, 2^log2_buckets) of each of n
 *                       keys under theta and the sorted sample's table
 *                       (use_network = 0: floor(x * B)).
 */
ms_status ms_learned_grad(const uint32_t* d_sample, uint32_t S, int feature, const float* d_theta, float* d_out,
                          void* stream);
ms_status ms_learned_train(const uint32_t* d_sample, uint32_t S, int feature, uint32_t steps, float learning_rate,
                           const float* d_theta0, float* d_theta_out, float* d_loss_hist, void* stream);
ms_status ms_learned_table(const float* d_theta, const uint32_t* d_sample, uint32_t S, int feature, float* d_t,
                           float* d_v, int* d_count, void* stream);
ms_status ms_learned_bucket_ids(const uint32_t* d_keys, size_t n, const float* d_theta, const uint32_t* d_sample,
                                uint32_t S, int feature, int use_network, uint32_t log2_buckets, uint32_t* d_out,
                                void* stream);

/*
 * ms_temp_bytes -- device scratch (bytes) that a plain sort of n keys with
 * values of val_bytes (0 = keys only) uses.  Host arithmetic only.
 * Returns 0 for an unsupported kt / val_bytes.
 *
 * ms_temp_bytes_segmented -- scratch that one ms_segmented_sort graph of
 * num_segments segments and n_total keys owns (0 for an unsupported type).
 *
 * ms_temp_bytes_learned -- scratch that one ms_sort_ex learned-bucket graph
 * of n keys of type kt owns under options opt (NULL = defaults); 0 if the
 * options or the key type are invalid.  Host arithmetic only.
 */
size_t ms_temp_bytes(size_t n, ms_key_type kt, size_t val_bytes);
size_t ms_temp_bytes_segmented(size_t num_segments, size_t n_total, ms_key_type kt, size_t val_bytes);

/*
 * ms_plan_query -- the plan ms_sort / ms_sort_pairs would use for n keys:
 * tile size; two-run merge tile size; number of merge-tree levels after the
 * tile sort (ceil(log2(ceil(n / tile)))); whether the tile sort writes the
 * caller's buffer (1) or the scratch buffer (0) so that the last pass lands
 * in the caller's buffer; the number of HBM merge passes (pairs of levels
 * run as one fused four-run pass, an odd level count adds one two-run pass);
 * and the fused pass's merge tile (0 when passes are not fused).  Host
 * arithmetic only; any output pointer may be NULL.
 */
ms_status ms_plan_query(size_t n, ms_key_type kt, size_t val_bytes, int* tile, int* merge_tile,
                        int* passes, int* tile_sort_in_place, int* hbm_passes, int* merge4_tile);

/*
 * ms_sort_noalloc -- ms_sort that allocates nothing, for callers that cannot
 * allocate device memory (code under hipGraph stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * kernels as ms_sort; its scratch is a fixed __device__ array of
 * MS_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held from the
 * first call on that GPU until the process ends (its address is looked up
 * with hipGetSymbolAddress on that first call; no hipMalloc, hipFree or
 * allocating routine runs, and the event profiler records nothing here).
 * Limit: n with ms_temp_bytes(n, kt, 0) <= MS_NOALLOC_SCRATCH_BYTES (about
 * 16.7 million 32-bit keys or 8.4 million 64-bit keys); larger n returns
 * MS_ERR_INVALID_ARG and enqueues nothing.
 * Every call on one GPU shares that GPU's array: calls that may overlap in
 * time on one GPU (different streams, or host threads on one stream without
 * ordering) race on it and give undefined results.  Calls ordered on one
 * stream are safe; no part of the array needs to start at zero.
 */
#define MS_NOALLOC_SCRATCH_BYTES (64u << 20)
ms_status ms_sort_noalloc(void* d_keys, size_t n, ms_key_type kt, void* stream);

/* Free the library's scratch buffers and cached segmented-sort graphs of the
 * current device (all streams).  Synchronises the device first. */
ms_status ms_release_workspace(void);

/*
 * Event profiler (measurement support).  While enabled, every kernel launch
 * of the library is bracketed by a pair of HIP events recorded on the launch
 * stream (launches recorded into a graph are not timed).  ms_profile_read()
 * synchronises those events and returns, for the kernel class `kernel`
 * (0 tile sort, 1 two-run partition, 2 two-run merge, 3 segment classify,
 * 4 small-segment sort, 5 large-segment passes, 6 MLP training, 7 learned
 * level-1 histogram, 8 learned level-1 scatter, 9 bucket sort, 10 other
 * learned kernels, 11 four-way partition, 12 fused four-run merge,
 * 13 learned level-2 histogram, 14 learned level-2 scatter, 15 the sampling
 * two-run partition of a fused pass, 16 learned level-1 size estimate; the
 * level-1 exact pass counts as class 10 when it only runs after an estimate
 * proved too small), the number of launches and their summed duration in
 * milliseconds since the last ms_profile_reset().
 */
ms_status ms_profile_enable(int on);
/* Time only the kernel classes whose bit (1 << class) is set in class_mask
 * (default: all); fewer events per sort disturb the timed run less. */
ms_status ms_profile_select(uint32_t class_mask);
ms_status ms_profile_reset(void);
ms_status ms_profile_read(int kernel, uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* MSORT_H */

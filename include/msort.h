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
 * ms_temp_bytes -- device scratch (bytes) that a plain sort of n keys with
 * values of val_bytes (0 = keys only) uses.  Host arithmetic only.
 * Returns 0 for an unsupported kt / val_bytes.
 */
size_t ms_temp_bytes(size_t n, ms_key_type kt, size_t val_bytes);

/*
 * ms_plan_query -- the plan ms_sort / ms_sort_pairs would use for n keys:
 * tile size, merge tile size, number of merge passes, and whether the tile
 * sort writes the caller's buffer (1) or the scratch buffer (0) so that the
 * last pass lands in the caller's buffer.  Host arithmetic only; any output
 * pointer may be NULL.
 */
ms_status ms_plan_query(size_t n, ms_key_type kt, size_t val_bytes, int* tile, int* merge_tile,
                        int* passes, int* tile_sort_in_place);

/* Free the library's scratch buffers of the current device (all streams).
 * Synchronises the device first. */
ms_status ms_release_workspace(void);

/*
 * Event profiler (measurement support).  While enabled, every kernel launch
 * of the library is bracketed by a pair of HIP events recorded on the launch
 * stream.  ms_profile_read() synchronises those events and returns, for the
 * kernel class `kernel` (0 tile sort, 1 partition, 2 merge, 3 segment
 * classify, 4 small-segment sort, 5 large-segment passes, 6 MLP training,
 * 7 learned histograms, 8 learned scatters, 9 bucket sort, 10 other learned
 * kernels), the number of launches and their summed duration in
 * milliseconds since the last ms_profile_reset().
 */
ms_status ms_profile_enable(int on);
ms_status ms_profile_reset(void);
ms_status ms_profile_read(int kernel, uint64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* MSORT_H */

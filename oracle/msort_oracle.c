/*
 * CPU oracle for the stable merge sort -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU library never links it, and it shares no
 * code, header or table with the GPU path.
 *
 * What it computes (the plain definition): for keys k[0..n) and optional
 * values v[0..n), the stable ascending sort, i.e. the unique permutation p
 * such that the pairs (k[p(i)], p(i)) are strictly increasing, keys compared
 * unsigned for U32/U64 and signed for I32/I64; keys_out[i] = k[p(i)],
 * vals_out[i] = v[p(i)].
 *
 * How: the paper's sequential merge sort (section "Sequential Merge Sort",
 * its four-step description and the mergesort figure), top-down and
 * recursive, with two readings of that section made explicit:
 *   - the right half is array[mid:] (the printed figure repeats array[:mid]);
 *   - merge(), which the paper never defines, takes from the right run only
 *     when its head is strictly smaller, so the left run wins ties and the
 *     sort is stable.
 * No small-array cutoff (the hybrid variant's SMALLEST_ARRAY_SIZE is left
 * out) and no library sort anywhere.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_U32 = 0, K_I32 = 1, K_U64 = 2, K_I64 = 3 };

/* One recursive merge sort per (key type, value width).  The macro only
 * stamps out the same plain code for each element type: NAME##_merge is the
 * merge step (step 4), NAME the recursion (steps 1-3), and NAME##_sort /
 * NAME##_mergev the same two with untyped pointers for the threaded driver
 * below. */
#define DEFINE_MERGESORT(NAME, KT, VT)                                         \
  /* step 4: merge a[0, mid) with a[mid, n) through t; the right head is     \
   * taken only if strictly smaller, so the left run wins ties */            \
  static void NAME##_merge(KT *a, VT *va, KT *t, VT *vt, size_t n,             \
                           size_t mid, int has_v) {                            \
    size_t i = 0, j = mid, k = 0;                                              \
    while (i < mid && j < n) {                                                 \
      if (a[j] < a[i]) {                                                       \
        t[k] = a[j];                                                           \
        if (has_v) vt[k] = va[j];                                              \
        j++;                                                                   \
      } else {                                                                 \
        t[k] = a[i];                                                           \
        if (has_v) vt[k] = va[i];                                              \
        i++;                                                                   \
      }                                                                        \
      k++;                                                                     \
    }                                                                          \
    while (i < mid) {                                                          \
      t[k] = a[i];                                                             \
      if (has_v) vt[k] = va[i];                                                \
      i++, k++;                                                                \
    }                                                                          \
    while (j < n) {                                                            \
      t[k] = a[j];                                                             \
      if (has_v) vt[k] = va[j];                                                \
      j++, k++;                                                                \
    }                                                                          \
    memcpy(a, t, n * sizeof(KT));                                              \
    if (has_v) memcpy(va, vt, n * sizeof(VT));                                 \
  }                                                                            \
  static void NAME(KT *a, VT *va, KT *t, VT *vt, size_t n, int has_v) {        \
    if (n < 2) return; /* step 1: fewer than two elements */                   \
    size_t mid = n / 2; /* step 2: left = a[:mid], right = a[mid:] */          \
    NAME(a, va, t, vt, mid, has_v); /* step 3: sort both halves */             \
    NAME(a + mid, has_v ? va + mid : va, t, vt, n - mid, has_v);               \
    NAME##_merge(a, va, t, vt, n, mid, has_v);                                 \
  }                                                                            \
  static void NAME##_sort(void *a, void *va, void *t, void *vt, size_t n,      \
                          int has_v) {                                         \
    NAME((KT *)a, (VT *)va, (KT *)t, (VT *)vt, n, has_v);                      \
  }                                                                            \
  static void NAME##_mergev(void *a, void *va, void *t, void *vt, size_t n,    \
                            size_t mid, int has_v) {                           \
    NAME##_merge((KT *)a, (VT *)va, (KT *)t, (VT *)vt, n, mid, has_v);         \
  }

DEFINE_MERGESORT(ms_u32_v32, uint32_t, uint32_t)
DEFINE_MERGESORT(ms_u32_v64, uint32_t, uint64_t)
DEFINE_MERGESORT(ms_i32_v32, int32_t, uint32_t)
DEFINE_MERGESORT(ms_i32_v64, int32_t, uint64_t)
DEFINE_MERGESORT(ms_u64_v32, uint64_t, uint32_t)
DEFINE_MERGESORT(ms_u64_v64, uint64_t, uint64_t)
DEFINE_MERGESORT(ms_i64_v32, int64_t, uint32_t)
DEFINE_MERGESORT(ms_i64_v64, int64_t, uint64_t)

static size_t key_bytes(int kt) { return (kt == K_U32 || kt == K_I32) ? 4 : 8; }

/* Sort keys (and values when val_bytes is 4 or 8; 0 = keys only) in place.
 * Returns 0 on success, -1 on bad arguments, -2 when scratch cannot be
 * allocated. */
int oracle_sort(void *keys, void *vals, size_t n, int kt, size_t val_bytes) {
  if (n < 2) return 0;
  if (kt < 0 || kt > 3) return -1;
  if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return -1;
  int has_v = val_bytes != 0 && vals != NULL;
  size_t vb = val_bytes ? val_bytes : 4;
  void *t = malloc(n * key_bytes(kt));
  void *vt = has_v ? malloc(n * vb) : NULL;
  if (!t || (has_v && !vt)) {
    free(t);
    free(vt);
    return -2;
  }
  /* Keys-only sorts pass a dummy value array that is never touched. */
  void *va = has_v ? vals : keys;
  void *vtt = has_v ? vt : t;
  switch (kt * 2 + (vb == 8)) {
    case K_U32 * 2 + 0: ms_u32_v32(keys, va, t, vtt, n, has_v); break;
    case K_U32 * 2 + 1: ms_u32_v64(keys, va, t, vtt, n, has_v); break;
    case K_I32 * 2 + 0: ms_i32_v32(keys, va, t, vtt, n, has_v); break;
    case K_I32 * 2 + 1: ms_i32_v64(keys, va, t, vtt, n, has_v); break;
    case K_U64 * 2 + 0: ms_u64_v32(keys, va, t, vtt, n, has_v); break;
    case K_U64 * 2 + 1: ms_u64_v64(keys, va, t, vtt, n, has_v); break;
    case K_I64 * 2 + 0: ms_i64_v32(keys, va, t, vtt, n, has_v); break;
    case K_I64 * 2 + 1: ms_i64_v64(keys, va, t, vtt, n, has_v); break;
  }
  free(t);
  free(vt);
  return 0;
}

/* The same sort with its top recursion levels on threads, for timing the
 * CPU baseline on many cores (the paper's multiprocessing merge sort,
 * section "Multiprocessing Merge Sort": independent sorts of chunks, then a
 * tree of merges; here the chunks are the halves the recursion cuts at its
 * top levels, so merges pair adjacent runs).  At depth d > 0 the left half
 * is sorted on a new thread while the calling thread sorts the right half,
 * then the calling thread merges; the halves use disjoint parts of the
 * scratch arrays.  Every merge is the sequential one above, so the output is
 * identical to oracle_sort's. */
typedef void (*sort_fn)(void *, void *, void *, void *, size_t, int);
typedef void (*merge_fn)(void *, void *, void *, void *, size_t, size_t, int);

struct par_job {
  sort_fn sort;
  merge_fn merge;
  char *a, *va, *t, *vt;
  size_t kb, vb, n;
  int depth, has_v;
  int rc;
};

static void *par_sort(void *arg) {
  struct par_job *j = (struct par_job *)arg;
  j->rc = 0;
  if (j->n < 2) return NULL;
  if (j->depth == 0) {
    j->sort(j->a, j->va, j->t, j->vt, j->n, j->has_v);
    return NULL;
  }
  size_t mid = j->n / 2;
  size_t vs = j->has_v ? j->vb : 0;
  struct par_job left = *j, right = *j;
  left.n = mid;
  left.depth = right.depth = j->depth - 1;
  right.a = j->a + mid * j->kb;
  right.va = j->va + mid * vs;
  right.t = j->t + mid * j->kb;
  right.vt = j->vt + mid * vs;
  right.n = j->n - mid;
  pthread_t th;
  int spawned = pthread_create(&th, NULL, par_sort, &left) == 0;
  if (!spawned) par_sort(&left); /* no thread available: same result */
  par_sort(&right);
  if (spawned) pthread_join(th, NULL);
  if (left.rc || right.rc) {
    j->rc = left.rc ? left.rc : right.rc;
    return NULL;
  }
  j->merge(j->a, j->va, j->t, j->vt, j->n, mid, j->has_v);
  return NULL;
}

/* Sort like oracle_sort with `threads` threads (1 = oracle_sort's own
 * recursion); depth = ceil(log2(threads)) levels run in parallel. */
int oracle_sort_parallel(void *keys, void *vals, size_t n, int kt, size_t val_bytes, int threads) {
  if (n < 2) return 0;
  if (kt < 0 || kt > 3 || threads < 1) return -1;
  if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return -1;
  int depth = 0;
  while ((1 << depth) < threads && depth < 16) depth++;
  int has_v = val_bytes != 0 && vals != NULL;
  size_t vb = val_bytes ? val_bytes : 4;
  size_t kb = key_bytes(kt);
  void *t = malloc(n * kb);
  void *vt = has_v ? malloc(n * vb) : NULL;
  if (!t || (has_v && !vt)) {
    free(t);
    free(vt);
    return -2;
  }
  struct par_job j;
  memset(&j, 0, sizeof j);
  switch (kt * 2 + (vb == 8)) {
    case K_U32 * 2 + 0: j.sort = ms_u32_v32_sort; j.merge = ms_u32_v32_mergev; break;
    case K_U32 * 2 + 1: j.sort = ms_u32_v64_sort; j.merge = ms_u32_v64_mergev; break;
    case K_I32 * 2 + 0: j.sort = ms_i32_v32_sort; j.merge = ms_i32_v32_mergev; break;
    case K_I32 * 2 + 1: j.sort = ms_i32_v64_sort; j.merge = ms_i32_v64_mergev; break;
    case K_U64 * 2 + 0: j.sort = ms_u64_v32_sort; j.merge = ms_u64_v32_mergev; break;
    case K_U64 * 2 + 1: j.sort = ms_u64_v64_sort; j.merge = ms_u64_v64_mergev; break;
    case K_I64 * 2 + 0: j.sort = ms_i64_v32_sort; j.merge = ms_i64_v32_mergev; break;
    case K_I64 * 2 + 1: j.sort = ms_i64_v64_sort; j.merge = ms_i64_v64_mergev; break;
  }
  /* keys-only sorts pass the key arrays as (never touched) value arrays */
  j.a = (char *)keys;
  j.va = has_v ? (char *)vals : (char *)keys;
  j.t = (char *)t;
  j.vt = has_v ? (char *)vt : (char *)t;
  j.kb = kb;
  j.vb = vb;
  j.n = n;
  j.depth = depth;
  j.has_v = has_v;
  par_sort(&j);
  free(t);
  free(vt);
  return j.rc;
}

/* Segmented form: every segment [off[s], off[s+1]) is sorted on its own with
 * the same merge sort (positions relative to the segment).  Offsets must be
 * non-decreasing with off[0] = 0 and off[nseg] = total length. */
int oracle_segmented_sort(void *keys, void *vals, const int64_t *off,
                          size_t nseg, int kt, size_t val_bytes) {
  size_t kb = key_bytes(kt);
  for (size_t s = 0; s < nseg; s++) {
    if (off[s + 1] < off[s]) return -1;
    size_t b = (size_t)off[s], len = (size_t)(off[s + 1] - off[s]);
    void *vk = (char *)keys + b * kb;
    void *vv = vals ? (char *)vals + b * val_bytes : NULL;
    int rc = oracle_sort(vk, vv, len, kt, vals ? val_bytes : 0);
    if (rc) return rc;
  }
  return 0;
}

/* Rank bounds of probe values by definition: lt[q] = #{i : k[i] < probe[q]},
 * le[q] = #{i : k[i] <= probe[q]}.  A sorted output o is correct at position
 * r exactly when lt(o[r]) <= r < le(o[r]); this lets a test verify sampled
 * positions of an output too large to sort on the CPU in a test's time. */
#define DEFINE_RANKS(NAME, KT)                                                 \
  static void NAME(const KT *k, size_t n, const KT *probe, size_t np,          \
                   uint64_t *lt, uint64_t *le) {                               \
    for (size_t q = 0; q < np; q++) lt[q] = le[q] = 0;                         \
    for (size_t i = 0; i < n; i++) {                                           \
      KT x = k[i];                                                             \
      for (size_t q = 0; q < np; q++) {                                        \
        lt[q] += x < probe[q];                                                 \
        le[q] += x <= probe[q];                                                \
      }                                                                        \
    }                                                                          \
  }
DEFINE_RANKS(rk_u32, uint32_t)
DEFINE_RANKS(rk_i32, int32_t)
DEFINE_RANKS(rk_u64, uint64_t)
DEFINE_RANKS(rk_i64, int64_t)

int oracle_rank_bounds(const void *keys, size_t n, int kt, const void *probe,
                       size_t np, uint64_t *lt, uint64_t *le) {
  switch (kt) {
    case K_U32: rk_u32(keys, n, probe, np, lt, le); return 0;
    case K_I32: rk_i32(keys, n, probe, np, lt, le); return 0;
    case K_U64: rk_u64(keys, n, probe, np, lt, le); return 0;
    case K_I64: rk_i64(keys, n, probe, np, lt, le); return 0;
  }
  return -1;
}

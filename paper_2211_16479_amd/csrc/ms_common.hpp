// Shared device-side building blocks of the gfx950 merge sort.
//
// Ordering used everywhere: ascending, stable.  Keys compare as unsigned
// (u32/u64) or signed (i32/i64).  Whenever two runs are merged, the run that
// came first in the input (the left run) wins ties; this is the reading of the
// paper's undefined merge() that makes the sort stable (section "Sequential
// Merge Sort").
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ms {

// ---------------------------------------------------------------- value tag
struct NoVal {};  // keys-only sorts

template <class V>
struct HasVal { static constexpr bool value = true; };
template <>
struct HasVal<NoVal> { static constexpr bool value = false; };

// ------------------------------------------------------------- sort items
// Inside one tile the block sort orders "items".  Keys-only: the key itself
// (equal keys are identical bits, so the order among them is unobservable).
// Key/value pairs: the key together with its tile-local input position, so
// that the (key, position) order -- a strict total order -- is exactly the
// stable order; the value is fetched by position at the end.
template <class K>
struct KeyBits;
template <>
struct KeyBits<uint32_t> { static __device__ __forceinline__ uint32_t ord(uint32_t k) { return k; } static __device__ __forceinline__ uint32_t unord(uint32_t b) { return b; } };
template <>
struct KeyBits<int32_t> { static __device__ __forceinline__ uint32_t ord(int32_t k) { return uint32_t(k) ^ 0x80000000u; } static __device__ __forceinline__ int32_t unord(uint32_t b) { return int32_t(b ^ 0x80000000u); } };

template <class K>
__device__ __forceinline__ K key_max();
template <> __device__ __forceinline__ uint32_t key_max<uint32_t>() { return 0xFFFFFFFFu; }
template <> __device__ __forceinline__ int32_t key_max<int32_t>() { return 0x7FFFFFFF; }
template <> __device__ __forceinline__ uint64_t key_max<uint64_t>() { return ~0ull; }
template <> __device__ __forceinline__ int64_t key_max<int64_t>() { return 0x7FFFFFFFFFFFFFFFll; }

struct Key64Pos {
  uint64_t k;    // key bits (the key type decides how they compare)
  uint32_t pos;  // tile-local input position
  uint32_t pad;
};

template <class K, bool PAIRS, bool WIDE = (sizeof(K) == 8)>
struct Item;

// Median of three 32-bit integers (v_med3): with c the smallest key it is
// min(a, b), with c the largest max(a, b) -- one instruction for the
// lane-dependent min-or-max of a bitonic exchange.
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ int32_t med3_i32(int32_t a, int32_t b, int32_t c) {
  int32_t r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// keys only: the key
template <class K, bool WIDE>
struct Item<K, false, WIDE> {
  using T = K;
  // 32-bit keys: keep(v, p, side(lower)) = lower ? min(v, p) : max(v, p)
  static constexpr bool MED3 = sizeof(K) == 4;
  static constexpr bool WITH_POS = false;
  static __device__ __forceinline__ T side(bool lower) {  // the smallest or the largest key
    if constexpr (sizeof(K) == 4 && K(0) < K(-1)) return lower ? K(0) : key_max<K>();
    else return lower ? K(-key_max<K>() - 1) : key_max<K>();
  }
  static __device__ __forceinline__ T keep(const T& v, const T& p, const T& sd) {
    if constexpr (sizeof(K) == 4 && K(0) < K(-1)) return T(med3_u32(uint32_t(v), uint32_t(p), uint32_t(sd)));
    else if constexpr (sizeof(K) == 4) return T(med3_i32(int32_t(v), int32_t(p), int32_t(sd)));
    else return v;  // unused: MED3 is false
  }
  static __device__ __forceinline__ T make(K k, uint32_t) { return k; }
  static __device__ __forceinline__ T pad(uint32_t) { return key_max<K>(); }
  static __device__ __forceinline__ K key(const T& t) { return t; }
  static __device__ __forceinline__ uint32_t pos(const T&) { return 0; }
  static __device__ __forceinline__ bool less(const T& a, const T& b) { return a < b; }
  static __device__ __forceinline__ T vmin(const T& a, const T& b) { return a < b ? a : b; }
  static __device__ __forceinline__ T vmax(const T& a, const T& b) { return a < b ? b : a; }
};

// 32-bit keys with values: (order-preserving key bits << 32) | position
template <class K>
struct Item<K, true, false> {
  using T = uint64_t;
  static constexpr bool MED3 = false;
  static constexpr bool WITH_POS = true;
  static __device__ __forceinline__ T make(K k, uint32_t p) { return (uint64_t(KeyBits<K>::ord(k)) << 32) | p; }
  static __device__ __forceinline__ T pad(uint32_t p) { return (0xFFFFFFFFull << 32) | p; }
  static __device__ __forceinline__ K key(const T& t) { return KeyBits<K>::unord(uint32_t(t >> 32)); }
  static __device__ __forceinline__ uint32_t pos(const T& t) { return uint32_t(t); }
  static __device__ __forceinline__ bool less(const T& a, const T& b) { return a < b; }
  static __device__ __forceinline__ T vmin(const T& a, const T& b) { return a < b ? a : b; }
  static __device__ __forceinline__ T vmax(const T& a, const T& b) { return a < b ? b : a; }
};

// 64-bit keys with values: key and position side by side
template <class K>
struct Item<K, true, true> {
  using T = Key64Pos;
  static constexpr bool MED3 = false;
  static constexpr bool WITH_POS = true;
  static __device__ __forceinline__ T make(K k, uint32_t p) { T t; t.k = uint64_t(k); t.pos = p; t.pad = 0; return t; }
  static __device__ __forceinline__ T pad(uint32_t p) { return make(key_max<K>(), p); }
  static __device__ __forceinline__ K key(const T& t) { return K(t.k); }
  static __device__ __forceinline__ uint32_t pos(const T& t) { return t.pos; }
  static __device__ __forceinline__ bool less(const T& a, const T& b) {
    K ka = K(a.k), kb = K(b.k);
    return ka < kb || (ka == kb && a.pos < b.pos);
  }
  static __device__ __forceinline__ T vmin(const T& a, const T& b) { return less(b, a) ? b : a; }
  static __device__ __forceinline__ T vmax(const T& a, const T& b) { return less(a, b) ? b : a; }
};

// ------------------------------------------------------- cross-lane xor moves
// xor_lane<M>(v): the value v held by lane (lane ^ M) of the same wavefront.
// Each mask uses the cheapest gfx950 route: DPP quad permutes for 1, 2, 3,
// DPP row_half_mirror / row_mirror for 7 / 15, ds_swizzle (bit mode, xor
// within 32 lanes) for 4, 8, 16, 31 and ds_bpermute for the full-wave 63.
template <int M>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t v) {
  if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(int(v), 0xB1, 0xF, 0xF, false);
  else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(int(v), 0x4E, 0xF, 0xF, false);
  else if constexpr (M == 3) return __builtin_amdgcn_mov_dpp(int(v), 0x1B, 0xF, 0xF, false);
  else if constexpr (M == 7) return __builtin_amdgcn_mov_dpp(int(v), 0x141, 0xF, 0xF, false);
  else if constexpr (M == 15) return __builtin_amdgcn_mov_dpp(int(v), 0x140, 0xF, 0xF, false);
  else if constexpr (M == 4 || M == 8 || M == 16 || M == 31)
    return __builtin_amdgcn_ds_swizzle(int(v), (M << 10) | 0x1F);
  else {
    static_assert(M > 0 && M < 64, "lane mask");
    const int lane = __lane_id();
    return __builtin_amdgcn_ds_bpermute((lane ^ M) << 2, int(v));
  }
}

template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) { return xor_lane32<M>(v); }
template <int M>
__device__ __forceinline__ int32_t xor_lane(int32_t v) { return int32_t(xor_lane32<M>(uint32_t(v))); }
template <int M>
__device__ __forceinline__ uint64_t xor_lane(uint64_t v) {
  uint32_t lo = xor_lane32<M>(uint32_t(v)), hi = xor_lane32<M>(uint32_t(v >> 32));
  return (uint64_t(hi) << 32) | lo;
}
template <int M>
__device__ __forceinline__ int64_t xor_lane(int64_t v) { return int64_t(xor_lane<M>(uint64_t(v))); }
template <int M>
__device__ __forceinline__ Key64Pos xor_lane(const Key64Pos& v) {
  Key64Pos r;
  r.k = xor_lane<M>(v.k);
  r.pos = xor_lane32<M>(v.pos);
  r.pad = 0;
  return r;
}

// ---------------------------------------------------- small helpers
__host__ __device__ constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// LDS index with one pad slot every 2^S elements (S = 0: no padding).
// Merge-path threads read positions about IPT/2 apart, and blocked writes are
// IPT apart; with power-of-two strides those land in a few of the 64 LDS
// banks.  The pad spreads them.
template <int S>
__host__ __device__ constexpr uint32_t lds_pad(uint32_t e) {
  return S ? e + (e >> S) : e;
}
template <int S>
__host__ __device__ constexpr uint32_t lds_padded_size(uint32_t n) {
  return S ? n + (n >> S) + 1 : n;
}

// Vector store of N consecutive 32- or 64-bit elements when the address is
// aligned for it; element count N is a compile-time multiple of the vector.
template <class E, int N>
__device__ __forceinline__ void store_run(E* __restrict__ dst, const E (&v)[N]) {
  if constexpr (sizeof(E) == 4 && N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      uint4 w;
      w.x = __builtin_bit_cast(uint32_t, v[i]);
      w.y = __builtin_bit_cast(uint32_t, v[i + 1]);
      w.z = __builtin_bit_cast(uint32_t, v[i + 2]);
      w.w = __builtin_bit_cast(uint32_t, v[i + 3]);
      *reinterpret_cast<uint4*>(dst + i) = w;
    }
  } else if constexpr (sizeof(E) == 8 && N % 2 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 2) {
      uint4 w;
      uint64_t a = __builtin_bit_cast(uint64_t, v[i]), b = __builtin_bit_cast(uint64_t, v[i + 1]);
      w.x = uint32_t(a); w.y = uint32_t(a >> 32); w.z = uint32_t(b); w.w = uint32_t(b >> 32);
      *reinterpret_cast<uint4*>(dst + i) = w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) dst[i] = v[i];
  }
}

template <class E, int N>
__device__ __forceinline__ void load_run(const E* __restrict__ src, E (&v)[N]) {
  if constexpr (sizeof(E) == 4 && N % 4 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      uint4 w = *reinterpret_cast<const uint4*>(src + i);
      v[i] = __builtin_bit_cast(E, w.x); v[i + 1] = __builtin_bit_cast(E, w.y);
      v[i + 2] = __builtin_bit_cast(E, w.z); v[i + 3] = __builtin_bit_cast(E, w.w);
    }
  } else if constexpr (sizeof(E) == 8 && N % 2 == 0) {
#pragma unroll
    for (int i = 0; i < N; i += 2) {
      uint4 w = *reinterpret_cast<const uint4*>(src + i);
      v[i] = __builtin_bit_cast(E, uint64_t(w.x) | (uint64_t(w.y) << 32));
      v[i + 1] = __builtin_bit_cast(E, uint64_t(w.z) | (uint64_t(w.w) << 32));
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = src[i];
  }
}

// Internal-consistency error bits of this code object's kernels (each
// translation unit has its own word; the host reads and clears them all
// through ms_device_errors()).  A kernel that detects an inconsistency sets
// a bit and writes nothing it cannot vouch for.
constexpr unsigned int DEV_ERR_MERGE_OFFSETS = 1u;  // fused merge tile: offsets do not describe its pieces
static __device__ unsigned int g_dev_errors;
__device__ __forceinline__ void raise_dev_error(unsigned int bits) { atomicOr(&g_dev_errors, bits); }

// Host side: read and clear this translation unit's error word (blocking).
#define MS_DEFINE_DEV_ERRORS(fn)                                                    \
  unsigned int fn() {                                                              \
    unsigned int v = 0, z = 0;                                                     \
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_dev_errors), sizeof v) != hipSuccess) \
      return 0x80000000u;                                                          \
    if (v && hipMemcpyToSymbol(HIP_SYMBOL(g_dev_errors), &z, sizeof z) != hipSuccess) \
      return v | 0x80000000u;                                                      \
    return v;                                                                      \
  }

// A device pointer read from memory.  Typed as a global-memory pointer, the
// loads and stores through it stay global instructions; read as a plain
// void*, it would make the compiler fall back to flat instructions for every
// access that might use it (slower, and they wait on LDS traffic too).
template <class T>
__device__ __forceinline__ T* global_ptr(const void* const* slot) {
  typedef __attribute__((address_space(1))) void* gvoid;
  const gvoid p = *(const gvoid*)(slot);
  return (T*)(__attribute__((address_space(1))) T*)p;
}

// A caller's buffer that a cached hipGraph sees at launch time.  The graph's
// kernels keep the pointer of the call that captured them (`token`); before
// every replay the library writes the current call's pointer to *cur, and a
// kernel argument equal to the token is replaced by it.  cur == nullptr: no
// rebinding (plain launches).
struct Rebind {
  const void* token;
  void* const* cur;
};

template <class T>
__device__ __forceinline__ T* rebind(T* p, const Rebind& r) {
  return (r.cur && static_cast<const void*>(p) == r.token) ? global_ptr<T>(r.cur) : p;
}

// Optional device-side controls shared by the sort kernels: an element count
// that lives in device memory (set by an earlier kernel), a gate flag that
// lets a kernel return at once when its stage is not needed, and the
// rebinding of the caller's key buffer under graph replay.
struct DevCtl {
  const uint64_t* n_dev;      // if non-null, the element count (<= the host bound)
  const int* gate;            // if non-null and bit 0 of *gate is clear, the kernel does nothing
  const uint64_t* split_dev;  // if non-null: one merge of run [0, split) with [split, n)
  Rebind keys = {nullptr, nullptr};  // key-buffer arguments equal to keys.token read *keys.cur
  int swap_bit = 0;  // 1: bit 1 of *gate set means the pass reads the buffers the other way round
  const void* other = nullptr;  // with swap_bit: the planned destination keys (a partition kernel's source then)
};

// The gate word, 1 (run, no swap) when there is none: one load per kernel.
__device__ __forceinline__ int gate_word(const DevCtl& c) { return c.gate ? *c.gate : 1; }
__device__ __forceinline__ bool swap_set(const DevCtl& c, int gw) { return c.swap_bit && (gw & 2); }

__device__ __forceinline__ bool gated_off(const DevCtl& c) { return c.gate && (*c.gate & 1) == 0; }

// A value the caller knows to be the same in every lane of the wavefront
// (a tile's offsets, read at a workgroup-uniform address), moved to scalar
// registers: the arithmetic on it then runs on the scalar unit, and branches
// on it are uniform rather than exec-masked.
__device__ __forceinline__ uint64_t wave_uniform(uint64_t x) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(x))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(x >> 32))));
  return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_uniform(uint32_t x) {
  return uint32_t(__builtin_amdgcn_readfirstlane(int(x)));
}
__device__ __forceinline__ uint64_t live_n(const DevCtl& c, uint64_t n_host) {
  return c.n_dev ? *c.n_dev : n_host;
}

}  // namespace ms

// Device-side building blocks shared by the RSKA kernels (gfx950, wave64).
//
// Cross-workgroup exchange. The persistent kernels never use a fenced grid
// barrier: a release/acquire fence at agent scope writes back and invalidates
// the XCD's L2, which costs tens of microseconds per step on an 8-XCD part.
// Instead every value that crosses workgroups travels as 64-bit words
// (tag << 32 | 32 payload bits) written and read with relaxed agent-scope
// atomics. Those bypass the non-coherent per-XCD L2 state by themselves, and
// a 64-bit atomic store is single-copy atomic, so a reader that sees the tag
// of the current exchange also sees its payload. Tags count exchanges within
// one launch (the host zeroes the exchange area first), so no stale word can
// match. Every wait is bounded: an expired wait reports RSK_ERR_ABORTED and
// the kernel runs to its end.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsk {

typedef unsigned long long u64;

enum : int { ST_OK = 0, ST_ZERO_ROW = 5, ST_INDEX = 6, ST_NONFINITE = 7, ST_ABORTED = 8 };

// About 2^22 polls of roughly a microsecond each: seconds, far beyond any
// legitimate wait between two steps.
constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ void xstore(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 xload(const u64* p) {
  return __hip_atomic_load(const_cast<u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads from device (global) memory through a generic pointer. A pointer read
// from memory (a batch descriptor) is otherwise accessed with FLAT
// instructions, which count against the LDS counter as well, so that every LDS
// wait and barrier would also wait for them. Scalars and vectors only: an
// aggregate copy binds a generic reference and loses the address space.
template <typename T>
__device__ __forceinline__ T load_global(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T, int N>
__device__ __forceinline__ void load_global_vec(const T* p, T (&out)[N]) {
  typedef T vt __attribute__((ext_vector_type(N)));
  const vt v = *(const __attribute__((address_space(1))) vt*)p;
#pragma unroll
  for (int e = 0; e < N; ++e) out[e] = v[e];
}

__device__ __forceinline__ float4 load_global_f4(const float* p) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 v = *(const __attribute__((address_space(1))) v4*)p;
  return make_float4(v[0], v[1], v[2], v[3]);
}
template <typename T>
__device__ __forceinline__ void store_global(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

template <typename T> struct Words;
template <> struct Words<float> { static constexpr int N = 1; };
template <> struct Words<double> { static constexpr int N = 2; };

__device__ __forceinline__ void put_tagged(u64* s, float v, unsigned tag) {
  xstore(s, ((u64)tag << 32) | (u64)__float_as_uint(v));
}
__device__ __forceinline__ void put_tagged(u64* s, double v, unsigned tag) {
  const u64 bits = (u64)__double_as_longlong(v);
  xstore(s, ((u64)tag << 32) | (bits & 0xffffffffull));
  xstore(s + 1, ((u64)tag << 32) | (bits >> 32));
}
__device__ __forceinline__ bool try_tagged(const u64* s, unsigned tag, float& v) {
  const u64 w = xload(s);
  if ((unsigned)(w >> 32) != tag) return false;
  v = __uint_as_float((unsigned)w);
  return true;
}
__device__ __forceinline__ bool try_tagged(const u64* s, unsigned tag, double& v) {
  const u64 lo = xload(s), hi = xload(s + 1);
  if ((unsigned)(lo >> 32) != tag || (unsigned)(hi >> 32) != tag) return false;
  v = __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
  return true;
}
// Spin until the slot carries `tag`; on expiry set `err` and return 0. Once
// `err` is set every later wait returns at once, so a broken exchange ends
// the launch after one expired wait rather than one per slot.
template <typename T>
__device__ __forceinline__ T wait_tagged(const u64* s, unsigned tag, int& err) {
  T v;
  if (err) return T(0);
  unsigned spins = 0;
  while (!try_tagged(s, tag, v)) {
    if (++spins > kSpinLimit) { err = ST_ABORTED; return T(0); }
    __builtin_amdgcn_s_sleep(1);
  }
  return v;
}

// Wait until the `cnt` (<= N) float slots base[i*stride] all carry `tag`.
// All pending slots are loaded before any is checked, so the waits of one
// lane overlap instead of costing one round trip each.
template <int N>
__device__ __forceinline__ void wait_tagged_batch(const u64* base, size_t stride, int cnt, unsigned tag,
                                                  float (&v)[N], int& err) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = 0.f;
  if (err || cnt <= 0) return;
  unsigned pending = cnt >= 32 ? 0xffffffffu : ((1u << cnt) - 1u);
  unsigned spins = 0;
  for (;;) {
    u64 w[N];
#pragma unroll
    for (int i = 0; i < N; ++i) w[i] = ((pending >> i) & 1u) ? xload(base + (size_t)i * stride) : 0ull;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (((pending >> i) & 1u) && (unsigned)(w[i] >> 32) == tag) {
        v[i] = __uint_as_float((unsigned)w[i]);
        pending &= ~(1u << i);
      }
    }
    if (!pending) return;
    if (++spins > kSpinLimit) { err = ST_ABORTED; return; }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Block OR in one barrier (HIP's __syncthreads_or costs three and waits for every outstanding
// load): the bits go into the word of this step's parity, read after the barrier; the other
// word, last read before an earlier barrier, is cleared for the next step.
__device__ __forceinline__ int block_or(int* words, int v, int64_t k) {
  if (v) atomicOr(&words[k & 1], v);
  __syncthreads();
  const int r = words[k & 1];
  if (threadIdx.x == 0) words[(k + 1) & 1] = 0;
  return r;
}

// First error wins.
__device__ __forceinline__ void set_status(int* status, int code) {
  if (code) atomicCAS(status, 0, code);
}

// ||a_i||^2 / w_i: the row norm with the row's weight of Definition 1 folded in (variants
// v3/v4 of Sec. 5), so that (alpha/eta)(r - b)/(||a||^2/w) relaxes the row by alpha w. A zero
// row stays 0 (reported as such); w = 0 gives an infinite norm, i.e. no update from the row.
template <typename T>
__device__ __forceinline__ T weighted_rn(const T* r2, const T* row_w, int64_t i) {
  const T rn = load_global(r2 + i);
  return (row_w && rn != T(0)) ? rn / load_global(row_w + i) : rn;
}

template <typename T>
__device__ __forceinline__ T shrink(T v, T lambda) {
  // S_lambda(v) = max(|v| - lambda, 0) sign(v); |v| == lambda gives 0.
  const T a = fabs(v) - lambda;
  return a > T(0) ? (v > T(0) ? a : -a) : T(0);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum within aligned groups of `width` lanes (width a power of two <= 64),
// butterfly offsets width/2, ..., 1. Unrolled with a wave-uniform predicate,
// so no loop back-edge makes the compiler drain outstanding memory operations.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
    if (off < width) v += __shfl_xor(v, off);
  return v;
}

// Workgroup g -> slice index such that the 8 XCDs (dispatch is round-robin
// over XCDs by workgroup id) each own one contiguous range of columns; a
// boundary cache line is then shared inside one XCD's L2 rather than fetched
// by two. Only performance depends on this mapping, never correctness.
__device__ __forceinline__ int xcd_slice(int g, int G) {
  if (G % 8 != 0) return g;
  return (g % 8) * (G / 8) + g / 8;
}

template <typename T, int N>
struct __attribute__((aligned(sizeof(T) * N))) Vec {
  T v[N];
};

}  // namespace rsk

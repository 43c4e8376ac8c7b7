// Device-side helpers shared by the truss kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace truss {

constexpr int kWave = 64;

// ---- lane / wave helpers --------------------------------------------------

__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of `mask` strictly below this lane
__device__ __forceinline__ int rank_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p ? 1 : 0); }

// Orders LDS traffic between lanes of one wavefront (no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T x) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    T y = __shfl_xor(x, d, kWave);
    x = y < x ? y : x;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) {
    T y = __shfl_xor(x, d, kWave);
    x = y > x ? y : x;
  }
  return x;
}

// first lane (lowest id) of a non-empty mask broadcasts `x`
template <typename T>
__device__ __forceinline__ T wave_bcast(T x, int src) {
  return __shfl(x, src, kWave);
}

// ---- device-scope atomics ---------------------------------------------------

__device__ __forceinline__ int atomic_load_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated append: every lane with `want` gets a distinct slot from
// *counter; returns the slot (undefined for lanes without `want`).
__device__ __forceinline__ int wave_append(int* counter, bool want) {
  const uint64_t m = ballot(want);
  if (m == 0) return 0;
  const int leader = __builtin_ctzll(m);
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader, kWave);
  return base + rank_below(m);
}

// ---- ordering of vertices for the orientation --------------------------------
// u precedes v iff (deg u, u) < (deg v, v); edges point from earlier to later.
__device__ __forceinline__ bool vertex_before(int64_t du, int u, int64_t dv, int v) {
  return du < dv || (du == dv && u < v);
}

// lower_bound of `key` in the sorted range a[lo, hi)
template <typename IdxT>
__device__ __forceinline__ IdxT lower_bound_i32(const int* __restrict__ a, IdxT lo, IdxT hi, int key) {
  while (lo < hi) {
    IdxT mid = lo + ((hi - lo) >> 1);
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---- edge hash table ------------------------------------------------------------
// The membership test of Algorithm 2 (is (v, w) an edge of E_G?) through a
// hashtable over E_G (Section 3.2): open addressing with linear probing, key
// (min << 32 | max), value the canonical edge id.  At most half full.
struct EdgeSlot {
  unsigned long long key;
  int eid;
  int pad;
};
constexpr unsigned long long kEmptyKey = ~0ULL;

__device__ __forceinline__ unsigned long long mix64(unsigned long long k) {
  // MurmurHash3 64-bit finaliser
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ unsigned long long edge_key(int a, int b) {
  const unsigned lo = (unsigned)(a < b ? a : b), hi = (unsigned)(a < b ? b : a);
  return ((unsigned long long)lo << 32) | hi;
}

// edge id of {a, b}, or -1 if it is not an edge
__device__ __forceinline__ int edge_lookup(const EdgeSlot* __restrict__ tab, unsigned long long mask, int a, int b) {
  const unsigned long long key = edge_key(a, b);
  unsigned long long h = mix64(key) & mask;
  for (;;) {
    const unsigned long long k = tab[h].key;
    if (k == key) return tab[h].eid;
    if (k == kEmptyKey) return -1;
    h = (h + 1) & mask;
  }
}

}  // namespace truss

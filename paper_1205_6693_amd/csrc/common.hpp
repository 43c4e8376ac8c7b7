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

// ---- row hash tables ------------------------------------------------------------
// The membership test of Algorithm 2 (is (v, w) an edge of E_G?) through a
// hash table over E_G (Section 3.2), kept per vertex: the table of v holds
// v's neighbours w with the edge id of (v, w), open addressing with linear
// probing, 2^lg >= 2 deg(v) slots (at most half full); an empty slot has
// w = -1.  The tables of all vertices lie back to back (offsets rtoff), so a
// walk whose entries all look up the same vertex's neighbours touches one
// compact region, which stays in cache, instead of lines scattered over one
// table of all edges.
__device__ __forceinline__ int row_table_lg(int64_t slots) { return 63 - __builtin_clzll((unsigned long long)slots); }

__device__ __forceinline__ uint32_t row_slot(int32_t w, int lg) {
  return lg == 0 ? 0u : ((uint32_t)w * 2654435769u) >> (32 - lg);
}

// edge id of (v, w) from v's table at rtab[off, off + 2^lg), or -1
__device__ __forceinline__ int row_lookup(const int2* __restrict__ rtab, int64_t off, int lg, int32_t w) {
  const uint32_t mask = (1u << lg) - 1u;
  uint32_t h = row_slot(w, lg);
  for (;;) {
    const int2 x = rtab[off + h];
    if (x.x == w) return x.y;
    if (x.x < 0) return -1;
    h = (h + 1) & mask;
  }
}

}  // namespace truss

// Exclusive prefix sums (reduce-then-scan over 2048-element tiles) and an LSD
// radix sort with 8-bit digits and stable in-tile ranking by wavefront match.
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T block_exclusive_sum(T x, T* wave_tot, T* total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_sum(x);
  if (lane == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  T base = 0, all = 0;
  for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
    T v = wave_tot[i];
    if (i < w) base += v;
    all += v;
  }
  *total = all;
  __syncthreads();
  return base + inc - x;
}

template <typename InT, typename OutT>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const InT* __restrict__ in, int64_t n,
                                                               OutT* __restrict__ partial) {
  __shared__ OutT wt[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  OutT s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j * kScanThreads + threadIdx.x;
    if (i < n) s += (OutT)in[i];
  }
  s = wave_sum(s);
  if (lane_id() == 0) wt[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    OutT t = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) t += wt[i];
    partial[blockIdx.x] = t;
  }
}

// one block: exclusive scan of partial[0..ntiles), total into partial[ntiles]
template <typename OutT>
__global__ void __launch_bounds__(1024) k_scan_partials(OutT* __restrict__ partial, int64_t ntiles) {
  __shared__ OutT wt[1024 / kWave];
  const int64_t per = (ntiles + blockDim.x - 1) / blockDim.x;
  const int64_t lo = threadIdx.x * per;
  const int64_t hi = lo + per < ntiles ? lo + per : ntiles;
  OutT s = 0;
  for (int64_t i = lo; i < hi; ++i) s += partial[i];
  OutT total;
  OutT run = block_exclusive_sum(s, wt, &total);
  for (int64_t i = lo; i < hi; ++i) {
    OutT v = partial[i];
    partial[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) partial[ntiles] = total;
}

template <typename InT, typename OutT>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const InT* __restrict__ in, OutT* __restrict__ out,
                                                              int64_t n, const OutT* __restrict__ partial) {
  __shared__ OutT tile[kTile + kTile / 32];
  __shared__ OutT wt[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  auto pad = [](int i) { return i + (i >> 5); };
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int li = j * kScanThreads + threadIdx.x;
    int64_t i = base + li;
    tile[pad(li)] = i < n ? (OutT)in[i] : (OutT)0;
  }
  __syncthreads();
  OutT v[kScanItems];
  OutT s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = tile[pad(threadIdx.x * kScanItems + j)];
    s += v[j];
  }
  OutT total;
  OutT run = block_exclusive_sum(s, wt, &total) + partial[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    tile[pad(threadIdx.x * kScanItems + j)] = run;
    run += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int li = j * kScanThreads + threadIdx.x;
    int64_t i = base + li;
    if (i < n) out[i] = tile[pad(li)];
  }
}

template <typename OutT>
__global__ void k_store_total(OutT* out, int64_t n, const OutT* partial, int64_t ntiles) {
  out[n] = partial[ntiles];
}

template <typename OutT>
__global__ void k_zero1(OutT* out) { out[0] = 0; }

template <typename InT, typename OutT>
void scan_impl(const InT* in, OutT* out, int64_t n, OutT* tmp, hipStream_t s) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_zero1<OutT>, dim3(1), dim3(1), 0, s, out);
    return;
  }
  const int64_t ntiles = (n + kTile - 1) / kTile;
  hipLaunchKernelGGL((k_scan_reduce<InT, OutT>), dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_partials<OutT>, dim3(1), dim3(1024), 0, s, tmp, ntiles);
  hipLaunchKernelGGL((k_scan_apply<InT, OutT>), dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, out, n, tmp);
  hipLaunchKernelGGL(k_store_total<OutT>, dim3(1), dim3(1), 0, s, out, n, tmp, ntiles);
}

// ---- radix sort -------------------------------------------------------------------

constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixThreads * kRadixItems;
constexpr int kRadixWaves = kRadixThreads / kWave;

template <typename K>
__global__ void __launch_bounds__(kRadixThreads) k_rs_hist(const K* __restrict__ keys, int64_t n, int shift,
                                                            int32_t* __restrict__ counts, int64_t ntiles) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int j = 0; j < kRadixItems; ++j) {
    int64_t i = base + j * kRadixThreads + threadIdx.x;
    if (i < n) atomicAdd(&hist[(int)((keys[i] >> shift) & 255)], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter of one tile.  Wavefront w owns the tile's elements
// [w * kWave * kRadixItems, (w + 1) * kWave * kRadixItems), item j of lane l
// being element w * kWave * kRadixItems + j * kWave + l, so (wavefront, item,
// lane) is the input order.  Each wavefront ranks its items one after another
// by wavefront match (eight ballots) against its own per-digit counters, with
// no workgroup barrier between items; one barrier later the per-digit
// prefix over the wavefronts places every element.
template <typename K>
__global__ void __launch_bounds__(kRadixThreads) k_rs_scatter(const K* __restrict__ keys, const int32_t* __restrict__ vals,
                                                               int64_t n, int shift, const int32_t* __restrict__ offs,
                                                               int64_t ntiles, K* __restrict__ keys_out,
                                                               int32_t* __restrict__ vals_out) {
  __shared__ int run[256];
  __shared__ int wcnt[kRadixWaves][256];
  const int w = threadIdx.x / kWave, lane = lane_id();
  run[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  for (int q = 0; q < kRadixWaves; ++q) wcnt[q][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile + (int64_t)w * kWave * kRadixItems;
  K k[kRadixItems];
  int32_t val[kRadixItems];
  int rk[kRadixItems];  // position among the wavefront's elements of the same digit
#pragma unroll
  for (int j = 0; j < kRadixItems; ++j) {
    const int64_t i = base + j * kWave + lane;
    k[j] = i < n ? keys[i] : (K)0;
    val[j] = i < n ? vals[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < kRadixItems; ++j) {
    const bool valid = base + j * kWave + lane < n;
    const int d = (int)((k[j] >> shift) & 255);
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    rk[j] = 0;
    if (valid) rk[j] = wcnt[w][d] + rank_below(peers);
    wave_sync();
    if (valid && rank_below(peers) == 0) wcnt[w][d] += __popcll(peers);
    wave_sync();
  }
  __syncthreads();
  // thread t: digit t's start for each wavefront
  {
    int acc = run[threadIdx.x];
    for (int q = 0; q < kRadixWaves; ++q) {
      const int c = wcnt[q][threadIdx.x];
      wcnt[q][threadIdx.x] = acc;
      acc += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kRadixItems; ++j) {
    if (base + j * kWave + lane < n) {
      const int d = (int)((k[j] >> shift) & 255);
      const int pos = wcnt[w][d] + rk[j];
      keys_out[pos] = k[j];
      vals_out[pos] = val[j];
    }
  }
}

template <typename K>
bool radix_impl(K* keys, int32_t* vals, K* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                int32_t* tmp, hipStream_t s) {
  if (n <= 1 || bits <= 0) return false;
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  int32_t* counts = tmp;
  int32_t* offs = counts + 256 * ntiles;
  int32_t* stmp = offs + 256 * ntiles + 1;
  K* kin = keys;
  int32_t* vin = vals;
  K* kout = keys_alt;
  int32_t* vout = vals_alt;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)ntiles), dim3(kRadixThreads), 0, s, kin, n, shift, counts, ntiles);
    scan_impl<int32_t, int32_t>(counts, offs, 256 * ntiles, stmp, s);
    hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)ntiles), dim3(kRadixThreads), 0, s, kin, vin, n, shift, offs,
                       ntiles, kout, vout);
    K* tk = kin; kin = kout; kout = tk;
    int32_t* tv = vin; vin = vout; vout = tv;
  }
  return kin != keys;
}

}  // namespace

size_t scan_tmp_elems(int64_t count) { return (size_t)((count + kTile - 1) / kTile) + 2; }

void scan_exclusive_i32_to_i64(const int32_t* in, int64_t* out, int64_t count, int64_t* tmp, hipStream_t s) {
  scan_impl<int32_t, int64_t>(in, out, count, tmp, s);
}

void scan_exclusive_i32_to_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* tmp, hipStream_t s) {
  scan_impl<int32_t, int32_t>(in, out, count, tmp, s);
}

size_t radix_tmp_elems(int64_t n) {
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  return (size_t)(2 * 256 * ntiles + 1) + scan_tmp_elems(256 * ntiles);
}

bool radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                    int32_t* tmp, hipStream_t s) {
  return radix_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s);
}

bool radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt, int64_t n, int bits,
                    int32_t* tmp, hipStream_t s) {
  return radix_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s);
}

}  // namespace truss

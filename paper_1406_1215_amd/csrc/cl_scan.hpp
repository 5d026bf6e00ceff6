// Device-wide exclusive prefix sums (reduce / scan-of-partials / down-sweep),
// generic over the element type and over how elements are produced and
// consumed.  Tiles of kScanThreads x kScanItems consecutive elements.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cl_plan.hpp"

namespace cl {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr uint64_t kScanTile = static_cast<uint64_t>(kScanThreads) * kScanItems;

__device__ __forceinline__ uint64_t shfl_up64(uint64_t x, int d) {
  const int lo = __shfl_up(static_cast<int>(static_cast<uint32_t>(x)), d, 64);
  const int hi = __shfl_up(static_cast<int>(static_cast<uint32_t>(x >> 32)), d, 64);
  return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t shfl_idx64(uint64_t x, int src) {
  const int lo = __shfl(static_cast<int>(static_cast<uint32_t>(x)), src, 64);
  const int hi = __shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), src, 64);
  return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

template <class T>
struct ScanTraits;

template <>
struct ScanTraits<uint64_t> {
  __device__ static uint64_t zero() { return 0; }
  __device__ static uint64_t add(uint64_t a, uint64_t b) { return a + b; }
  __device__ static uint64_t shfl_up(uint64_t a, int d) { return shfl_up64(a, d); }
  __device__ static uint64_t shfl_idx(uint64_t a, int src) { return shfl_idx64(a, src); }
};

template <>
struct ScanTraits<Triple> {
  __device__ static Triple zero() { return Triple{0, 0, 0}; }
  __device__ static Triple add(Triple a, Triple b) { return Triple{a.c + b.c, a.k + b.k, a.h + b.h}; }
  __device__ static Triple shfl_up(Triple a, int d) {
    return Triple{shfl_up64(a.c, d), shfl_up64(a.k, d), shfl_up64(a.h, d)};
  }
  __device__ static Triple shfl_idx(Triple a, int src) {
    return Triple{shfl_idx64(a.c, src), shfl_idx64(a.k, src), shfl_idx64(a.h, src)};
  }
};

// Exclusive scan of one value per thread across a block of kScanThreads.
// Returns the exclusive prefix; *total gets the block total.
template <class T>
__device__ __forceinline__ T block_exclusive(T v, T* total) {
  using Tr = ScanTraits<T>;
  __shared__ T wave_tot[kScanThreads / 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  T inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = Tr::shfl_up(inc, d);
    if (lane >= d) inc = Tr::add(inc, o);
  }
  if (lane == 63) wave_tot[wave] = inc;
  __syncthreads();
  T wbase = Tr::zero();
  T all = Tr::zero();
#pragma unroll
  for (int i = 0; i < kScanThreads / 64; ++i) {
    if (i < wave) wbase = Tr::add(wbase, wave_tot[i]);
    all = Tr::add(all, wave_tot[i]);
  }
  __syncthreads();
  *total = all;
  // exclusive = inclusive - v, formed as wbase + (inclusive of lanes before)
  T prev = Tr::shfl_up(inc, 1);
  if (lane == 0) prev = Tr::zero();
  return Tr::add(wbase, prev);
}

// Element producers and consumers.  An In provides
//   uint32_t graph_of(i)      which graph element i belongs to (0 if one),
//   Ctx context(g)            that graph's parameters,
//   T load(i, ctx)            element i;
// an Out provides Ctx context(g) and store(i, ctx, value, exclusive prefix).
// A tile whose elements all belong to one graph binds the context once, in
// wave-uniform registers; a tile that straddles graphs looks it up per element.
struct OneGraph {
  using Ctx = uint32_t;
  __device__ uint32_t graph_of(uint64_t) const { return 0; }
  __device__ Ctx context(uint32_t) const { return 0; }
};

// inclusive scan across the 64 lanes of a wavefront
template <class T>
__device__ __forceinline__ T wave_inclusive(T v) {
  using Tr = ScanTraits<T>;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T o = Tr::shfl_up(v, d);
    if (lane >= d) v = Tr::add(v, o);
  }
  return v;
}

// Phase 1: per-tile totals (striped, coalesced loads; the order of the
// additions does not matter for the integer types scanned on the plan path).
template <class T, class In>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(In in, uint64_t N, T* partials) {
  using Tr = ScanTraits<T>;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
  const uint64_t end = (base + kScanTile < N) ? base + kScanTile : N;
  const uint32_t g0 = __builtin_amdgcn_readfirstlane(in.graph_of(base));
  const uint32_t g1 = __builtin_amdgcn_readfirstlane(in.graph_of(end - 1));
  T s = Tr::zero();
  if (g0 == g1) {
    const typename In::Ctx c = in.context(g0);
    for (int r = 0; r < kScanItems; ++r) {
      const uint64_t idx = base + static_cast<uint64_t>(r) * kScanThreads + threadIdx.x;
      if (idx < end) s = Tr::add(s, in.load(idx, c));
    }
  } else {
    for (int r = 0; r < kScanItems; ++r) {
      const uint64_t idx = base + static_cast<uint64_t>(r) * kScanThreads + threadIdx.x;
      if (idx < end) s = Tr::add(s, in.load(idx, in.context(in.graph_of(idx))));
    }
  }
  T tot;
  (void)block_exclusive<T>(s, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Phase 2: exclusive scan of the tile totals in place (one block; each
// thread owns kScanItems consecutive totals of a chunk).
template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_partials(T* partials, uint64_t ntiles) {
  using Tr = ScanTraits<T>;
  T carry = Tr::zero();
  for (uint64_t chunk = 0; chunk < ntiles; chunk += kScanTile) {
    const uint64_t base = chunk + static_cast<uint64_t>(threadIdx.x) * kScanItems;
    T vals[kScanItems];
    T s = Tr::zero();
    for (int i = 0; i < kScanItems; ++i) {
      const uint64_t idx = base + i;
      vals[i] = (idx < ntiles) ? partials[idx] : Tr::zero();
      s = Tr::add(s, vals[i]);
    }
    T tot;
    T ex = Tr::add(carry, block_exclusive<T>(s, &tot));
    for (int i = 0; i < kScanItems; ++i) {
      const uint64_t idx = base + i;
      if (idx < ntiles) partials[idx] = ex;
      ex = Tr::add(ex, vals[i]);
    }
    carry = Tr::add(carry, tot);
  }
}

// Phase 3: per-tile exclusive scan plus the tile's carry-in; out.store(idx,
// ctx, value, exclusive prefix) for every element.  Each wavefront owns a
// contiguous quarter of the tile and walks it 64 elements at a time, so loads
// and stores are coalesced; its carry-in is the tile's plus the totals of the
// wavefronts before it.
template <class T, class In, class Out>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(In in, Out out, uint64_t N, const T* partials) {
  using Tr = ScanTraits<T>;
  constexpr int kWaves = kScanThreads / 64;
  constexpr uint64_t kWaveSpan = static_cast<uint64_t>(kScanItems) * 64;
  __shared__ T wave_tot[kWaves];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
  const uint64_t end = (base + kScanTile < N) ? base + kScanTile : N;
  const uint64_t wbase = base + wave * kWaveSpan;
  const uint32_t g0 = __builtin_amdgcn_readfirstlane(in.graph_of(base));
  const uint32_t g1 = __builtin_amdgcn_readfirstlane(in.graph_of(end - 1));
  const bool one = (g0 == g1);
  const typename In::Ctx ci = in.context(g0);
  const typename Out::Ctx co = out.context(g0);
  T vals[kScanItems];
  T s = Tr::zero();
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint64_t idx = wbase + static_cast<uint64_t>(r) * 64 + lane;
    T v = Tr::zero();
    if (idx < end) v = one ? in.load(idx, ci) : in.load(idx, in.context(in.graph_of(idx)));
    vals[r] = v;
    s = Tr::add(s, v);
  }
  s = wave_inclusive<T>(s);
  if (lane == 63) wave_tot[wave] = s;
  __syncthreads();
  T carry = partials[blockIdx.x];
  for (int w = 0; w < kWaves; ++w)
    if (w < wave) carry = Tr::add(carry, wave_tot[w]);
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const uint64_t idx = wbase + static_cast<uint64_t>(r) * 64 + lane;
    const T incl = wave_inclusive<T>(vals[r]);
    T prev = Tr::shfl_up(incl, 1);
    if (lane == 0) prev = Tr::zero();
    if (idx < end) {
      const T ex = Tr::add(carry, prev);
      if (one)
        out.store(idx, co, vals[r], ex);
      else
        out.store(idx, out.context(in.graph_of(idx)), vals[r], ex);
    }
    carry = Tr::add(carry, Tr::shfl_idx(incl, 63));
  }
}

inline uint64_t scan_tiles(uint64_t N) { return (N + kScanTile - 1) / kScanTile; }

// Runs the three phases on `stream`; `partials` must hold scan_tiles(N) T's.
template <class T, class In, class Out>
inline hipError_t device_scan(In in, Out out, uint64_t N, T* partials, hipStream_t stream) {
  if (N == 0) return hipSuccess;
  const uint64_t nt = scan_tiles(N);
  hipLaunchKernelGGL((k_scan_reduce<T, In>), dim3(static_cast<uint32_t>(nt)), dim3(kScanThreads), 0, stream,
                     in, N, partials);
  hipLaunchKernelGGL((k_scan_partials<T>), dim3(1), dim3(kScanThreads), 0, stream, partials, nt);
  hipLaunchKernelGGL((k_scan_down<T, In, Out>), dim3(static_cast<uint32_t>(nt)), dim3(kScanThreads), 0, stream,
                     in, out, N, partials);
  return hipGetLastError();
}

}  // namespace cl

// Device-wide exclusive prefix sums (reduce / scan-of-partials / down-sweep),
// generic over the element type and over how elements are produced and
// consumed.  Tiles of kScanThreads x kScanItems consecutive elements; each
// thread owns kScanItems consecutive elements of its tile.
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
};

template <>
struct ScanTraits<Triple> {
  __device__ static Triple zero() { return Triple{0, 0, 0}; }
  __device__ static Triple add(Triple a, Triple b) { return Triple{a.c + b.c, a.k + b.k, a.h + b.h}; }
  __device__ static Triple shfl_up(Triple a, int d) {
    return Triple{shfl_up64(a.c, d), shfl_up64(a.k, d), shfl_up64(a.h, d)};
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

// Phase 1: per-tile totals.
template <class T, class In>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(In in, uint64_t N, T* partials) {
  using Tr = ScanTraits<T>;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile +
                        static_cast<uint64_t>(threadIdx.x) * kScanItems;
  T s = Tr::zero();
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t idx = base + i;
    if (idx < N) s = Tr::add(s, in.load(idx));
  }
  T tot;
  (void)block_exclusive<T>(s, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Phase 2: exclusive scan of the tile totals in place (one block).
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
// value, exclusive prefix) for every element.
template <class T, class In, class Out>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(In in, Out out, uint64_t N, const T* partials) {
  using Tr = ScanTraits<T>;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile +
                        static_cast<uint64_t>(threadIdx.x) * kScanItems;
  T vals[kScanItems];
  T s = Tr::zero();
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t idx = base + i;
    vals[i] = (idx < N) ? in.load(idx) : Tr::zero();
    s = Tr::add(s, vals[i]);
  }
  T tot;
  T ex = Tr::add(partials[blockIdx.x], block_exclusive<T>(s, &tot));
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t idx = base + i;
    if (idx < N) out.store(idx, vals[i], ex);
    ex = Tr::add(ex, vals[i]);
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

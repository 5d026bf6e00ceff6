// Device-wide exclusive prefix sums (reduce / scan-of-partials / down-sweep),
// generic over the element type and over how elements are produced and
// consumed.  Tiles of kScanThreads x ScanItems<T> consecutive elements.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cl_plan.hpp"

namespace cl {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;

// elements per thread of a tile: kScanItems, or 8 for the 24-byte Triple,
// whose down-sweep holds its tile in registers (fewer registers, more waves)
template <class T>
struct ScanItems {
  static constexpr int value = kScanItems;
};
template <>
struct ScanItems<Triple> {
  static constexpr int value = 8;
};
template <class T>
constexpr uint64_t scan_tile() {
  return static_cast<uint64_t>(kScanThreads) * ScanItems<T>::value;
}

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

// DPP move of both halves of a 64-bit value: lanes outside the row / bank
// masks, and lanes whose source lies outside the row (or the wavefront),
// read 0.  kCtrl is the DPP control word (row_shr:n = 0x110 + n,
// wave_shr:1 = 0x138, row_bcast:15 = 0x142, row_bcast:31 = 0x143).
template <int kCtrl, int kRowMask, int kBankMask>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(x)), kCtrl, kRowMask,
                                             kBankMask, true);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(x >> 32)), kCtrl, kRowMask,
                                             kBankMask, true);
  return (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ __forceinline__ uint64_t lane63_64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(x)), 63);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(x >> 32)), 63);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

template <class T>
struct ScanTraits;

template <>
struct ScanTraits<uint64_t> {
  __device__ static uint64_t zero() { return 0; }
  __device__ static uint64_t add(uint64_t a, uint64_t b) { return a + b; }
  __device__ static uint64_t shfl_up(uint64_t a, int d) { return shfl_up64(a, d); }
  __device__ static uint64_t shfl_idx(uint64_t a, int src) { return shfl_idx64(a, src); }
  template <int kCtrl, int kRowMask, int kBankMask>
  __device__ static uint64_t dpp(uint64_t a) { return dpp64<kCtrl, kRowMask, kBankMask>(a); }
  __device__ static uint64_t lane63(uint64_t a) { return lane63_64(a); }
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
  template <int kCtrl, int kRowMask, int kBankMask>
  __device__ static Triple dpp(Triple a) {
    return Triple{dpp64<kCtrl, kRowMask, kBankMask>(a.c), dpp64<kCtrl, kRowMask, kBankMask>(a.k),
                  dpp64<kCtrl, kRowMask, kBankMask>(a.h)};
  }
  __device__ static Triple lane63(Triple a) { return Triple{lane63_64(a.c), lane63_64(a.k), lane63_64(a.h)}; }
};

// Inclusive scan across the 64 lanes of a wavefront with DPP moves (no LDS
// traffic): three row shifts sum each lane's group of four, shifts by 4 and
// 8 complete the scan of each row of 16 lanes, and the broadcasts of lanes
// 15 and 31 carry the row totals into the rows above.
template <class T>
__device__ __forceinline__ T wave_inclusive(T v) {
  using Tr = ScanTraits<T>;
  const T v0 = v;
  v = Tr::add(v, Tr::template dpp<0x111, 0xf, 0xf>(v0));   // row_shr:1
  v = Tr::add(v, Tr::template dpp<0x112, 0xf, 0xf>(v0));   // row_shr:2
  v = Tr::add(v, Tr::template dpp<0x113, 0xf, 0xf>(v0));   // row_shr:3
  v = Tr::add(v, Tr::template dpp<0x114, 0xf, 0xe>(v));    // row_shr:4 into lanes 4..15 of a row
  v = Tr::add(v, Tr::template dpp<0x118, 0xf, 0xc>(v));    // row_shr:8 into lanes 8..15 of a row
  v = Tr::add(v, Tr::template dpp<0x142, 0xa, 0xf>(v));    // lane 15 of rows 0, 2 into rows 1, 3
  v = Tr::add(v, Tr::template dpp<0x143, 0xc, 0xf>(v));    // lane 31 into rows 2, 3
  return v;
}

// the value of the lane below (0 in lane 0)
template <class T>
__device__ __forceinline__ T wave_prev(T v) {
  return ScanTraits<T>::template dpp<0x138, 0xf, 0xf>(v);   // wave_shr:1
}

// Exclusive scan of one value per thread across a block of kScanThreads.
// Returns the exclusive prefix; *total gets the block total.
template <class T>
__device__ __forceinline__ T block_exclusive(T v, T* total) {
  using Tr = ScanTraits<T>;
  __shared__ T wave_tot[kScanThreads / 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const T inc = wave_inclusive<T>(v);
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
  // exclusive = wbase + (inclusive of the lanes before)
  return Tr::add(wbase, wave_prev<T>(inc));
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

// Phase 1: per-tile totals (striped, coalesced loads; the order of the
// additions does not matter for the integer types scanned on the plan path).
template <class T, class In>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(In in, uint64_t N, T* partials) {
  using Tr = ScanTraits<T>;
  constexpr int kItems = ScanItems<T>::value;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * scan_tile<T>();
  const uint64_t end = (base + scan_tile<T>() < N) ? base + scan_tile<T>() : N;
  const uint32_t g0 = __builtin_amdgcn_readfirstlane(in.graph_of(base));
  const uint32_t g1 = __builtin_amdgcn_readfirstlane(in.graph_of(end - 1));
  T s = Tr::zero();
  if (g0 == g1) {
    const typename In::Ctx c = in.context(g0);
    for (int r = 0; r < kItems; ++r) {
      const uint64_t idx = base + static_cast<uint64_t>(r) * kScanThreads + threadIdx.x;
      if (idx < end) s = Tr::add(s, in.load(idx, c));
    }
  } else {
    for (int r = 0; r < kItems; ++r) {
      const uint64_t idx = base + static_cast<uint64_t>(r) * kScanThreads + threadIdx.x;
      if (idx < end) s = Tr::add(s, in.load(idx, in.context(in.graph_of(idx))));
    }
  }
  T tot;
  (void)block_exclusive<T>(s, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Phase 2: exclusive scan of the tile totals in place (one block; each
// thread owns kPartItems consecutive totals of a chunk: 24, so that the
// 2048-element Triple tiles of 1e7 sources fit one chunk).
constexpr int kPartItems = 24;

template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_partials(T* partials, uint64_t ntiles) {
  using Tr = ScanTraits<T>;
  constexpr uint64_t kChunk = static_cast<uint64_t>(kScanThreads) * kPartItems;
  T carry = Tr::zero();
  for (uint64_t chunk = 0; chunk < ntiles; chunk += kChunk) {
    const uint64_t base = chunk + static_cast<uint64_t>(threadIdx.x) * kPartItems;
    T vals[kPartItems];
    T s = Tr::zero();
    for (int i = 0; i < kPartItems; ++i) {
      const uint64_t idx = base + i;
      vals[i] = (idx < ntiles) ? partials[idx] : Tr::zero();
      s = Tr::add(s, vals[i]);
    }
    T tot;
    T ex = Tr::add(carry, block_exclusive<T>(s, &tot));
    for (int i = 0; i < kPartItems; ++i) {
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
// wavefronts before it.  A tile inside one graph (kOne) runs an instance with
// no per-element context loads: with them, every wait for a load in the store
// loop would also wait for the stores issued before it.
template <bool kOne, class T, class In, class Out>
__device__ __forceinline__ void scan_down_tile(In in, Out out, uint64_t base, uint64_t end, uint32_t g0,
                                               const T* partials) {
  using Tr = ScanTraits<T>;
  constexpr int kItems = ScanItems<T>::value;
  constexpr int kWaves = kScanThreads / 64;
  constexpr uint64_t kWaveSpan = static_cast<uint64_t>(kItems) * 64;
  __shared__ T wave_tot[kWaves];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t wbase = base + wave * kWaveSpan;
  const typename In::Ctx ci = in.context(g0);
  const typename Out::Ctx co = out.context(g0);
  T vals[kItems];
  T s = Tr::zero();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const uint64_t idx = wbase + static_cast<uint64_t>(r) * 64 + lane;
    T v = Tr::zero();
    if (idx < end) v = kOne ? in.load(idx, ci) : in.load(idx, in.context(in.graph_of(idx)));
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
  for (int r = 0; r < kItems; ++r) {
    const uint64_t idx = wbase + static_cast<uint64_t>(r) * 64 + lane;
    const T incl = wave_inclusive<T>(vals[r]);
    const T prev = wave_prev<T>(incl);
    if (idx < end) {
      const T ex = Tr::add(carry, prev);
      if (kOne)
        out.store(idx, co, vals[r], ex);
      else
        out.store(idx, out.context(in.graph_of(idx)), vals[r], ex);
    }
    carry = Tr::add(carry, Tr::lane63(incl));
  }
}

template <class T, class In, class Out>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(In in, Out out, uint64_t N, const T* partials) {
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * scan_tile<T>();
  const uint64_t end = (base + scan_tile<T>() < N) ? base + scan_tile<T>() : N;
  const uint32_t g0 = __builtin_amdgcn_readfirstlane(in.graph_of(base));
  const uint32_t g1 = __builtin_amdgcn_readfirstlane(in.graph_of(end - 1));
  if (g0 == g1) scan_down_tile<true, T>(in, out, base, end, g0, partials);
  else scan_down_tile<false, T>(in, out, base, end, g0, partials);
}

template <class T = uint64_t>
inline uint64_t scan_tiles(uint64_t N) {
  return (N + scan_tile<T>() - 1) / scan_tile<T>();
}

// Runs the three phases on `stream`; `partials` must hold scan_tiles<T>(N) T's.
template <class T, class In, class Out>
inline hipError_t device_scan(In in, Out out, uint64_t N, T* partials, hipStream_t stream) {
  if (N == 0) return hipSuccess;
  const uint64_t nt = scan_tiles<T>(N);
  hipLaunchKernelGGL((k_scan_reduce<T, In>), dim3(static_cast<uint32_t>(nt)), dim3(kScanThreads), 0, stream,
                     in, N, partials);
  hipLaunchKernelGGL((k_scan_partials<T>), dim3(1), dim3(kScanThreads), 0, stream, partials, nt);
  hipLaunchKernelGGL((k_scan_down<T, In, Out>), dim3(static_cast<uint32_t>(nt)), dim3(kScanThreads), 0, stream,
                     in, out, N, partials);
  return hipGetLastError();
}

}  // namespace cl

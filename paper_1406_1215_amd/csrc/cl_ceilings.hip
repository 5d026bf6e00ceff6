// Measured memory-system ceilings for the roofline of the generation kernel
// (a measurement probe next to the generator, not part of it; C ABI in
// include/clceil.h).
//
// The generation kernel reads one float64 weight w_v per visited candidate,
// at positions that jump by geometric skips, and writes 4-byte slot words in
// whole 64-byte chunks.  Its ceilings on this GPU are therefore
//   * the rate of independent 8-byte loads at random positions of the same
//     weight array (uniform positions, or a caller-supplied list of positions
//     drawn with the candidates' density), and
//   * the rate of plain coalesced 16-byte stores.
// Each kernel keeps kInFlight loads (or stores) in flight per thread and
// writes one value per thread so that nothing is optimised away.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "clceil.h"

namespace {

constexpr int kThreads = 256;
constexpr int kInFlight = 8;

// splitmix64's output function (Steele, Lea, Flood 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// load i of the launch: position floor(mix(seed + i) n / 2^64), uniform on [0, n)
__global__ void __launch_bounds__(kThreads) k_gather_uniform(const double* __restrict__ w, uint64_t n, uint64_t count,
                                                             uint64_t seed, double* __restrict__ out) {
  const uint64_t nt = static_cast<uint64_t>(gridDim.x) * kThreads;
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  double acc = 0.0;
  for (uint64_t base = tid; base < count; base += nt * kInFlight) {
    double v[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const uint64_t i = base + static_cast<uint64_t>(k) * nt;
      const uint64_t pos = __umul64hi(mix64(seed + i), n);
      v[k] = (i < count) ? w[pos] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) acc += v[k];
  }
  out[tid] = acc;
}

// load i of the launch: position idx[i] (idx read coalesced)
__global__ void __launch_bounds__(kThreads) k_gather_list(const double* __restrict__ w, uint64_t n,
                                                          const uint32_t* __restrict__ idx, uint64_t count,
                                                          double* __restrict__ out) {
  const uint64_t nt = static_cast<uint64_t>(gridDim.x) * kThreads;
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  double acc = 0.0;
  for (uint64_t base = tid; base < count; base += nt * kInFlight) {
    uint32_t p[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const uint64_t i = base + static_cast<uint64_t>(k) * nt;
      p[k] = (i < count) ? idx[i] : 0u;
    }
    double v[kInFlight];
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) {
      const uint64_t i = base + static_cast<uint64_t>(k) * nt;
      v[k] = (i < count && p[k] < n) ? w[p[k]] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kInFlight; ++k) acc += v[k];
  }
  out[tid] = acc;
}

// 16-byte stores, consecutive threads to consecutive addresses
__global__ void __launch_bounds__(kThreads) k_store(uint4* __restrict__ buf, uint64_t n16) {
  const uint64_t nt = static_cast<uint64_t>(gridDim.x) * kThreads;
  const uint64_t tid = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  for (uint64_t i = tid; i < n16; i += nt) {
    const uint32_t x = static_cast<uint32_t>(i);
    buf[i] = make_uint4(x, x + 1u, x + 2u, x + 3u);
  }
}

inline int launch_status() { return hipGetLastError() == hipSuccess ? 0 : -8; }

}  // namespace

extern "C" {

int clc_gather_uniform(const double* w, uint64_t n, uint64_t count, uint64_t seed, uint32_t blocks, double* out,
                       void* stream) {
  if (!w || !out || n == 0 || n > 0xFFFFFFFFull || blocks == 0) return -1;
  hipLaunchKernelGGL(k_gather_uniform, dim3(blocks), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream), w,
                     n, count, seed, out);
  return launch_status();
}

int clc_gather_list(const double* w, uint64_t n, const uint32_t* idx, uint64_t count, uint32_t blocks, double* out,
                    void* stream) {
  if (!w || !out || (count > 0 && !idx) || n == 0 || blocks == 0) return -1;
  hipLaunchKernelGGL(k_gather_list, dim3(blocks), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream), w, n,
                     idx, count, out);
  return launch_status();
}

int clc_store(void* buf, uint64_t bytes, uint32_t blocks, void* stream) {
  if (!buf || (reinterpret_cast<uintptr_t>(buf) & 15) || blocks == 0) return -1;
  hipLaunchKernelGGL(k_store, dim3(blocks), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream),
                     static_cast<uint4*>(buf), bytes / 16);
  return launch_status();
}

}  // extern "C"

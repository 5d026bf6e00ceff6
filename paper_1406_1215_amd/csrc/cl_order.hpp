// Processing order of the work units of a single-graph plan (the default
// for one graph; cl_tuning unit_order = 2).  The units are handed out by the
// prefix position where their first segment starts (in the quantised prefix
// Q of w), in kOrderBands bands of equal Q-mass (the graded tail units form a
// second run after the first, the padding units come last), so that the lanes
// in flight at any time visit candidates in a narrow stretch of v and gather
// the same lines of w.
//
// The order decides nothing about the output: every unit writes its own slot
// (or its own count), and every draw is keyed by (seed, u, k, t).  Inside a
// (band, block) cell the order is that of LDS atomics and may differ from run
// to run; the permutation is a permutation either way.
//
// Three kernels, after the lane plan and the heavy-segment table (the
// histogram cleared before them):
//   k_order_count    each unit's bin -> order_keys[unit]; the block's counts
//                    per bin (LDS), added to the global histogram (one atomic
//                    per bin the block uses)
//   k_order_offsets  exclusive scan of the histogram -> each bin's first place
//   k_order_scatter  the block's counts per bin again; one global atomic per
//                    bin reserves the block's places in it; each unit goes to
//                    perm[reserved start + its rank in the block (LDS atomic)]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cl_kernels.hpp"
#include "cl_plan.hpp"
#include "cl_scan.hpp"

namespace cl {

constexpr uint32_t kOrderBands = 512;
constexpr uint32_t kOrderBins = 2 * kOrderBands + 1;   // equal-cost units, graded units, padding
constexpr int kOrderThreads = 256;
constexpr int kOrderItems = 16;
constexpr uint64_t kOrderTile = static_cast<uint64_t>(kOrderThreads) * kOrderItems;
constexpr int kOrderScanItems = (kOrderBins + kOrderThreads - 1) / kOrderThreads;

inline uint64_t order_blocks(uint64_t nl) { return (nl + kOrderTile - 1) / kOrderTile; }

struct OrderCtx {
  gptr<uint32_t> lane_seg;
  gptr<u32x4> hseg;
  gptr<uint64_t> Q;     // the graph's quantised prefix (n + 1 slots)
  gptr<uint64_t> SB;    // the graph's per-source segment prefix (index u - u_begin)
  uint64_t Qbase, Qend;
  double scale;         // kOrderBands / (Q mass of the graph)
  uint64_t L, Lm, nl;   // units carrying work, units before the graded tail, units incl. padding
  double iscale;        // kOrderBands / n
  uint32_t NH, nseg, u_begin, u_light;   // heavy segments, segments, first source, first one-segment source
};

__device__ __forceinline__ OrderCtx order_ctx(const WsHeader* hdr) {
  const GraphDesc& d = hdr->desc[0];
  OrderCtx c;
  c.lane_seg = to_global(hdr->lane_seg);
  c.hseg = to_global(reinterpret_cast<const u32x4*>(hdr->hseg + d.hs_off));
  c.Q = to_global(hdr->Q + d.q_off);
  c.SB = to_global(hdr->SB + d.r_off);
  c.Qbase = d.Qbase;
  c.Qend = d.Qend;
  const uint64_t mass = d.Qend - d.Qbase;
  c.scale = mass ? static_cast<double>(kOrderBands) / static_cast<double>(mass) : 0.0;
  c.L = d.L;
  c.Lm = (d.graded && d.Lm < d.L) ? d.Lm : d.L;
  c.nl = hdr->total_nl;
  c.NH = static_cast<uint32_t>(d.NH);
  c.nseg = static_cast<uint32_t>(d.SB1 - d.SB0);
  c.u_begin = static_cast<uint32_t>(d.u_begin);
  c.u_light = static_cast<uint32_t>(d.u_begin + d.H);
  c.iscale = d.n ? static_cast<double>(kOrderBands) / static_cast<double>(d.n) : 0.0;
  return c;
}

// bins of the kOrderItems units base + r * kOrderThreads + threadIdx.x: the
// band of the prefix position where each unit's first segment starts, plus
// kOrderBands for a graded unit; padding units and units past the last
// segment in the last bin.  A heavy segment k of K_u starts at the share k/K_u
// of its source's prefix mass past Q_{u+1} (its boundary search targets that
// mass), so only per-source values are read, which neighbouring units share,
// and no gather at the candidate itself.  A unit that starts at a
// one-segment source u is placed by u / n (its candidates spread over all of
// [u + 1, n); reading Q_{u+1} would cost one cache line per unit).  The rounds of loads are
// each issued for all items before any is used.
__device__ __forceinline__ void unit_bins(const OrderCtx& c, uint64_t base, uint32_t (&bin)[kOrderItems]) {
  uint32_t s[kOrderItems];
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const uint64_t l = base + static_cast<uint64_t>(r) * kOrderThreads + threadIdx.x;
    s[r] = (l < c.nl) ? c.lane_seg[l] : c.nseg;
  }
  uint32_t u[kOrderItems], k[kOrderItems];
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const u32x4 h = (s[r] < c.NH) ? c.hseg[s[r]] : u32x4{c.u_begin, 0u, 0u, 0u};
    u[r] = h.x;
    k[r] = h.y;
  }
  uint64_t q[kOrderItems], K[kOrderItems];
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const bool heavy = s[r] < c.NH;
    const uint32_t i = u[r] - c.u_begin;
    q[r] = heavy ? c.Q[u[r] + 1] : c.Qbase;
    K[r] = heavy ? c.SB[i + 1] - c.SB[i] : 1;
  }
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const uint64_t l = base + static_cast<uint64_t>(r) * kOrderThreads + threadIdx.x;
    const double at = static_cast<double>(q[r] - c.Qbase) +
                      static_cast<double>(k[r]) / static_cast<double>(K[r]) * static_cast<double>(c.Qend - q[r]);
    const double x = (s[r] < c.NH) ? at * c.scale
                                   : static_cast<double>(c.u_light + (s[r] - c.NH)) * c.iscale;
    uint32_t b = (x < static_cast<double>(kOrderBands)) ? static_cast<uint32_t>(x) : kOrderBands - 1;
    if (l >= c.Lm) b += kOrderBands;
    bin[r] = (l >= c.L || s[r] >= c.nseg) ? kOrderBins - 1 : b;
  }
}

// LDS counter updates of one wavefront, one item per lane (the live lanes are
// a prefix of the wave, since the units of a round are consecutive).
// Neighbouring units mostly share a bin, so when every live lane holds lane
// 0's bin one lane adds them all, instead of 64 atomics on one address; the
// branch is wave-uniform.  wave_add counts; wave_rank returns each live lane's
// place among the additions (old count + rank among the live lanes, or the
// old count of its own atomic).
__device__ __forceinline__ bool wave_same_bin(uint32_t b, bool live, uint64_t* act) {
  *act = __ballot(live);
  const uint32_t b0 = __builtin_amdgcn_readfirstlane(b);
  return __ballot(live && b == b0) == *act;
}

__device__ __forceinline__ void wave_add(uint32_t* cnt, uint32_t b, bool live) {
  uint64_t act;
  if (wave_same_bin(b, live, &act)) {
    if ((threadIdx.x & 63) == 0 && act) atomicAdd(&cnt[b], static_cast<uint32_t>(__popcll(act)));
  } else if (live) {
    atomicAdd(&cnt[b], 1u);
  }
}

__device__ __forceinline__ uint32_t wave_rank(uint32_t* cnt, uint32_t b, bool live) {
  uint64_t act;
  if (wave_same_bin(b, live, &act)) {
    uint32_t old = 0;
    if ((threadIdx.x & 63) == 0 && act) old = atomicAdd(&cnt[b], static_cast<uint32_t>(__popcll(act)));
    old = __builtin_amdgcn_readfirstlane(old);
    return old + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(act >> 32),
                                           __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(act), 0u));
  }
  return live ? atomicAdd(&cnt[b], 1u) : 0u;
}

// each unit's bin, and the number of units per bin (the histogram
// order_hist, cleared before)
__global__ void __launch_bounds__(kOrderThreads) k_order_count(const WsHeader* hdr) {
  __shared__ uint32_t cnt[kOrderBins];
  if (hdr->status) return;
  const OrderCtx c = order_ctx(hdr);
  uint32_t* hist = hdr->order_hist;
  uint16_t* keys = hdr->order_keys;
  for (uint32_t b = threadIdx.x; b < kOrderBins; b += kOrderThreads) cnt[b] = 0;
  __syncthreads();
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kOrderTile;
  uint32_t bin[kOrderItems];
  unit_bins(c, base, bin);
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const uint64_t l = base + static_cast<uint64_t>(r) * kOrderThreads + threadIdx.x;
    const bool live = l < c.nl;
    if (live) keys[l] = static_cast<uint16_t>(bin[r]);
    wave_add(cnt, bin[r], live);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < kOrderBins; b += kOrderThreads)
    if (cnt[b]) atomicAdd(&hist[b], cnt[b]);
}

// exclusive scan of the histogram into the bins' first places (one block;
// each thread owns kOrderScanItems consecutive bins)
__global__ void __launch_bounds__(kOrderThreads) k_order_offsets(const WsHeader* hdr) {
  if (hdr->status) return;
  uint32_t* hist = hdr->order_hist;
  uint32_t* first = hdr->order_hist + kOrderBins;
  uint64_t v[kOrderScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kOrderScanItems; ++i) {
    const uint32_t b = threadIdx.x * kOrderScanItems + i;
    v[i] = (b < kOrderBins) ? hist[b] : 0u;
    sum += v[i];
  }
  uint64_t tot;
  uint64_t ex = block_exclusive<uint64_t>(sum, &tot);
#pragma unroll
  for (int i = 0; i < kOrderScanItems; ++i) {
    const uint32_t b = threadIdx.x * kOrderScanItems + i;
    if (b < kOrderBins) first[b] = static_cast<uint32_t>(ex);   // < nl < 2^32
    ex += v[i];
  }
}

__global__ void __launch_bounds__(kOrderThreads) k_order_scatter(const WsHeader* hdr) {
  __shared__ uint32_t cnt[kOrderBins];
  __shared__ uint32_t start[kOrderBins];
  if (hdr->status) return;
  const uint64_t nl = hdr->total_nl;
  const uint16_t* keys = hdr->order_keys;
  uint32_t* first = hdr->order_hist + kOrderBins;
  uint32_t* perm = hdr->perm;
  for (uint32_t b = threadIdx.x; b < kOrderBins; b += kOrderThreads) cnt[b] = 0;
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kOrderTile;
  uint32_t bin[kOrderItems];
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const uint64_t l = base + static_cast<uint64_t>(r) * kOrderThreads + threadIdx.x;
    bin[r] = (l < nl) ? keys[l] : 0u;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const uint64_t l = base + static_cast<uint64_t>(r) * kOrderThreads + threadIdx.x;
    wave_add(cnt, bin[r], l < nl);
  }
  __syncthreads();
  // the block's places in each bin it uses, then the counts restart as ranks
  for (uint32_t b = threadIdx.x; b < kOrderBins; b += kOrderThreads) {
    start[b] = cnt[b] ? atomicAdd(&first[b], cnt[b]) : 0u;
    cnt[b] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kOrderItems; ++r) {
    const uint64_t l = base + static_cast<uint64_t>(r) * kOrderThreads + threadIdx.x;
    const uint32_t rank = wave_rank(cnt, bin[r], l < nl);
    if (l < nl) perm[start[bin[r]] + rank] = static_cast<uint32_t>(l);
  }
}

inline hipError_t launch_order(const WsHeader* dhdr, const WsHeader& h, hipStream_t s) {
  const uint64_t blocks = h.order_blocks;
  if (!h.perm || blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, reinterpret_cast<unsigned long long*>(h.order_hist),
                     static_cast<uint64_t>(kOrderBins + 1) / 2);
  hipLaunchKernelGGL(k_order_count, dim3(static_cast<uint32_t>(blocks)), dim3(kOrderThreads), 0, s, dhdr);
  hipLaunchKernelGGL(k_order_offsets, dim3(1), dim3(kOrderThreads), 0, s, dhdr);
  hipLaunchKernelGGL(k_order_scatter, dim3(static_cast<uint32_t>(blocks)), dim3(kOrderThreads), 0, s, dhdr);
  return hipGetLastError();
}

}  // namespace cl

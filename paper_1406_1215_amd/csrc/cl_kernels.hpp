// Chung-Lu edge generation kernels for gfx950: validation, exact weight sum, quantised
// prefix, per-source costs and segments, lane plan (uniform-cost chunking),
// count pass, offsets, write pass, digest.
//
// Sec. 3, Alg. 1 (Create-Edges) is the per-lane loop in run_lane(); Sec. 4,
// Eq. 1-6 and Alg. 2 (uniform consecutive partition) become the lane plan:
// every lane of every wavefront receives a consecutive run of source
// segments of equal expected cost.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cl_device.hpp"
#include "cl_plan.hpp"
#include "cl_scan.hpp"

namespace cl {

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------
// largest g in [0, G) with off(g) <= i (offsets non-decreasing, off(0) = 0)
template <class F>
__device__ __forceinline__ uint32_t find_graph(uint32_t G, uint64_t i, F off) {
  uint32_t lo = 0, hi = G;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off(mid) <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// first v in [lo, hi] with Qrel(v) >= target; Qrel(hi) >= target is assumed
__device__ __forceinline__ uint64_t q_lower_bound(const uint64_t* Q, uint64_t q_off, uint64_t Qbase,
                                                  uint64_t lo, uint64_t hi, uint64_t target) {
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (Q[q_off + mid] - Qbase >= target) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v) { *p = v; }

__global__ void k_zero_u64(unsigned long long* p, uint64_t count) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0ull;
}

// --------------------------------------------------------------------------
// validation (+ exponent-binned exact sum for single arrays)
// --------------------------------------------------------------------------
// Every non-negative finite double is mant * 2^(b - 1075) with b = max(e, 1)
// (e the biased exponent, mant the 53-bit significand incl. the hidden bit for
// normals).  Summing mant per b in two 64-bit halves is exact; the finaliser
// assembles sum_b mant_b 2^(b-1) as a big integer and rounds it once.
constexpr int kBins = 2048;

__device__ __forceinline__ void bin_flush(unsigned long long* lds, int b, uint64_t lo, uint64_t hi) {
  if (b >= 0 && (lo | hi)) {
    atomicAdd(&lds[2 * b], static_cast<unsigned long long>(lo));
    atomicAdd(&lds[2 * b + 1], static_cast<unsigned long long>(hi));
  }
}

// Validates every weight of every graph (slot space of the Q prefix: n + 1
// slots per graph, the last one of each graph ignored).  With bins != null
// (single graph), also accumulates the exact sum.
template <bool want_sum>
__global__ void __launch_bounds__(256) k_validate(GraphDesc* desc, uint32_t G, uint64_t total_slots,
                                                  unsigned long long* bins) {
  __shared__ unsigned long long lbins[want_sum ? 2 * kBins : 2];
  if (want_sum) {
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) lbins[i] = 0ull;
    __syncthreads();
  }
  int cur_b = -1;
  uint64_t acc_lo = 0, acc_hi = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total_slots; i += stride) {
    const uint32_t g = find_graph(G, i, [&](uint32_t x) { return desc[x].q_off; });
    const GraphDesc& d = desc[g];
    const uint64_t v = i - d.q_off;
    if (v >= d.n) continue;
    const double x = d.w[v];
    const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t ex = static_cast<uint32_t>((bits >> 52) & 0x7FF);
    uint32_t flag = 0;
    if (ex == 0x7FF) {
      flag |= kStNonfinite;
    } else if (x < 0.0) {
      flag |= kStNegative;
    } else {
      if (v + 1 < d.n) {
        const double y = d.w[v + 1];
        if (x < y) flag |= kStUnsorted;
      }
      if (v == 0) {
        if (x > d.S || (x > 0.0 && x < 0x1.0p-960)) flag |= kStBadS;
      }
      if (want_sum) {
        const int b = (ex == 0) ? 1 : static_cast<int>(ex);
        uint64_t mant = bits & 0x000FFFFFFFFFFFFFull;
        if (ex != 0) mant |= 0x0010000000000000ull;
        if (b != cur_b) {
          bin_flush(lbins, cur_b, acc_lo, acc_hi);
          cur_b = b;
          acc_lo = 0;
          acc_hi = 0;
        }
        acc_lo += mant & 0xFFFFFFFFull;
        acc_hi += mant >> 32;
      }
    }
    if (flag) atomicOr(&desc[g].status, flag);
  }
  if (want_sum) {
    bin_flush(lbins, cur_b, acc_lo, acc_hi);
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) {
      const unsigned long long val = lbins[i];
      if (val) atomicAdd(&bins[i], val);
    }
  }
}

// Rounds sum_b (hi_b 2^32 + lo_b) 2^(b-1) * 2^-1074 to the nearest double
// (ties to even).  One thread.  35 limbs of 64 bits cover 2^2240.
constexpr int kLimbs = 36;

__global__ void k_sum_finalize(const unsigned long long* bins, double* S_out, uint32_t* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t T[kLimbs];
  for (int i = 0; i < kLimbs; ++i) T[i] = 0;
  auto add_shifted = [&](uint64_t val, int sh) {
    // T += val << sh
    if (!val) return;
    int li = sh >> 6;
    const int bs = sh & 63;
    uint64_t lo = val << bs;
    uint64_t hi = bs ? (val >> (64 - bs)) : 0;
    uint64_t old = T[li];
    T[li] = old + lo;
    uint64_t carry = (T[li] < old) ? 1 : 0;
    ++li;
    uint64_t add = hi + carry;           // hi < 2^63, no overflow
    while (add && li < kLimbs) {
      old = T[li];
      T[li] = old + add;
      add = (T[li] < old) ? 1 : 0;
      ++li;
    }
  };
  for (int b = 1; b < kBins; ++b) {
    add_shifted(bins[2 * b], b - 1);
    add_shifted(bins[2 * b + 1], b - 1 + 32);
  }
  int top = -1;
  for (int li = kLimbs - 1; li >= 0; --li) {
    if (T[li]) {
      top = li * 64 + 63 - __clzll(static_cast<long long>(T[li]));
      break;
    }
  }
  auto bit_at = [&](int p) -> uint64_t { return (T[p >> 6] >> (p & 63)) & 1ull; };
  double S;
  if (top < 0) {
    S = 0.0;
  } else if (top <= 52) {
    S = __longlong_as_double(static_cast<long long>(T[0]));   // value = T * 2^-1074, bits = T
  } else {
    const int shift = top - 52;
    uint64_t mant = 0;
    for (int p = top; p >= shift; --p) mant = (mant << 1) | bit_at(p);
    const uint64_t half = bit_at(shift - 1);
    bool sticky = false;
    for (int p = shift - 2; p >= 0 && !sticky; --p) sticky = bit_at(p) != 0;
    int e = shift + 1;
    if (half && (sticky || (mant & 1ull))) {
      ++mant;
      if (mant == (1ull << 53)) {
        mant >>= 1;
        ++e;
      }
    }
    if (e >= 2047) {
      S = __longlong_as_double(0x7FF0000000000000ll);
      atomicOr(status, kStNonfinite);
    } else {
      S = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(e) << 52) |
                                                      (mant & 0x000FFFFFFFFFFFFFull)));
    }
  }
  *S_out = S;
}

// status words are cleared at the start of every plan (a replayed graph
// starts from a clean state)
__global__ void k_reset_status(WsHeader* hdr) {
  for (uint32_t g = threadIdx.x; g < hdr->G; g += blockDim.x) hdr->desc[g].status = 0;
  if (threadIdx.x == 0) {
    hdr->status = 0;
    hdr->total_cand = 0;
  }
}

// --------------------------------------------------------------------------
// quantised prefix Q, all graphs in one scan
// --------------------------------------------------------------------------
__global__ void k_graph_init(GraphDesc* desc, uint32_t G) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  GraphDesc& d = desc[g];
  const double w0 = (d.n > 0) ? d.w[0] : 0.0;
  d.qscale = (w0 > 0.0) ? (4294967296.0 / w0) : 0.0;
}

struct QIn {
  const GraphDesc* desc;
  uint32_t G;
  __device__ uint64_t load(uint64_t i) const {
    const uint32_t g = find_graph(G, i, [&](uint32_t x) { return desc[x].q_off; });
    const GraphDesc& d = desc[g];
    const uint64_t v = i - d.q_off;
    if (v >= d.n || d.qscale == 0.0) return 0;
    return quantise(d.w[v], d.qscale);
  }
};

struct QOut {
  GraphDesc* desc;
  uint32_t G;
  uint64_t* Q;
  __device__ void store(uint64_t i, uint64_t, uint64_t ex) const {
    Q[i] = ex;
    const uint32_t g = find_graph(G, i, [&](uint32_t x) { return desc[x].q_off; });
    GraphDesc& d = desc[g];
    const uint64_t v = i - d.q_off;
    if (v == 0) d.Qbase = ex;
    if (v == d.n) d.Qend = ex;
  }
};

// --------------------------------------------------------------------------
// per-source (cost units, segments, heavy flag)
// --------------------------------------------------------------------------
// The cost of a source is Eq. 2 applied to each of its segments:
// (expected edges) + (one unit per segment), in units of 1/16.
struct NodeIn {
  const GraphDesc* desc;
  uint32_t G;
  const uint64_t* Q;
  __device__ Triple load(uint64_t i) const {
    const uint32_t g = find_graph(G, i, [&](uint32_t x) { return desc[x].r_off; });
    const GraphDesc& d = desc[g];
    const uint64_t r = i - d.r_off;
    const uint64_t nr = d.u_end - d.u_begin;
    if (r >= nr) return Triple{0, 0, 0};
    const uint64_t u = d.u_begin + r;
    uint32_t K = 1;
    double eh = 0.0;
    if (d.qscale != 0.0 && u + 1 < d.n) {
      const double a = d.w[u] / d.S;
      const uint64_t Qn = d.Qend - d.Qbase;
      const uint64_t D = Qn - (Q[d.q_off + u + 1] - d.Qbase);
      eh = ehat_of(a, D, d.qscale);
      K = nseg_of(eh, d.n, u);
    }
    double ce = eh * static_cast<double>(kCostUnit);
    if (ce > 0x1.0p36) ce = 0x1.0p36;
    const uint64_t c = static_cast<uint64_t>(ce) + static_cast<uint64_t>(kCostUnit) * K;
    return Triple{c, K, (K > 1) ? 1ull : 0ull};
  }
};

struct NodeOut {
  GraphDesc* desc;
  uint32_t G;
  uint64_t* C;
  uint64_t* SB;
  __device__ void store(uint64_t i, Triple, Triple ex) const {
    C[i] = ex.c;
    SB[i] = ex.k;
    const uint32_t g = find_graph(G, i, [&](uint32_t x) { return desc[x].r_off; });
    GraphDesc& d = desc[g];
    const uint64_t r = i - d.r_off;
    if (r == 0) {
      d.C0 = ex.c;
      d.SB0 = ex.k;
      d.H0 = ex.h;
    }
    if (r == d.u_end - d.u_begin) {
      d.C1 = ex.c;
      d.SB1 = ex.k;
      d.H1 = ex.h;
    }
  }
};

// --------------------------------------------------------------------------
// per-graph sizes, offsets over graphs (one block)
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_plan_sizes(WsHeader* hdr) {
  GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  uint64_t carry_nh = 0, carry_nl = 0, carry_cost = 0;
  for (uint32_t base = 0; base < G; base += blockDim.x) {
    const uint32_t g = base + threadIdx.x;
    uint64_t nh = 0, nl = 0, cost = 0;
    if (g < G) {
      GraphDesc& d = desc[g];
      const uint64_t nr = d.u_end - d.u_begin;
      d.H = d.H1 - d.H0;
      const uint64_t Z = d.C1 - d.C0;
      const uint64_t nseg = d.SB1 - d.SB0;
      nh = (d.H > 0) ? (hdr->SB[d.r_off + d.H] - d.SB0) : 0;
      uint64_t L = 0;
      if (nr > 0 && d.qscale != 0.0 && d.status == 0) {
        L = (Z + d.budget - 1) / d.budget;
        if (L > nseg) L = nseg;
        if (L == 0) L = 1;
      }
      d.L = L;
      d.NH = nh;
      cost = (L > 0) ? Z : 0;
      nl = (L + kLaneGroup - 1) / kLaneGroup * kLaneGroup;
      d.NL = nl;
    }
    uint64_t tot_nh, tot_nl, tot_cost;
    const uint64_t ex_nh = block_exclusive<uint64_t>(nh, &tot_nh);
    const uint64_t ex_nl = block_exclusive<uint64_t>(nl, &tot_nl);
    (void)block_exclusive<uint64_t>(cost, &tot_cost);
    carry_cost += tot_cost;
    if (g < G) {
      desc[g].hs_off = carry_nh + ex_nh;
      desc[g].lane_off = carry_nl + ex_nl;
    }
    carry_nh += tot_nh;
    carry_nl += tot_nl;
  }
  if (threadIdx.x == 0) {
    hdr->total_nh = carry_nh;
    hdr->total_nl = carry_nl;
    hdr->total_cost = carry_cost;
    uint32_t st = 0;
    for (uint32_t g = 0; g < G; ++g) st |= desc[g].status;
    if (hdr->cap_nl != 0 && (carry_nh > hdr->cap_nh || carry_nl > hdr->cap_nl)) st |= kStCapacity;
    hdr->status |= st;
  }
}

// --------------------------------------------------------------------------
// heavy-segment starts b_k (one thread per heavy segment)
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_heavy_table(const WsHeader* hdr) {
  if (hdr->status) return;
  const GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  const uint64_t NH = hdr->total_nh;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t h = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; h < NH; h += stride) {
    const uint32_t g = find_graph(G, h, [&](uint32_t x) { return desc[x].hs_off; });
    const GraphDesc& d = desc[g];
    const uint64_t hl = h - d.hs_off;
    // heavy source: last r in [0, H) with SB(r) - SB0 <= hl
    uint64_t lo = 0, hi = d.H;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (hdr->SB[d.r_off + mid] - d.SB0 <= hl) lo = mid; else hi = mid;
    }
    const uint64_t r = lo;
    const uint64_t sb = hdr->SB[d.r_off + r] - d.SB0;
    const uint64_t K = hdr->SB[d.r_off + r + 1] - hdr->SB[d.r_off + r];
    const uint64_t k = hl - sb;
    const uint64_t u = d.u_begin + r;
    uint64_t b;
    if (k == 0) {
      b = u + 1;
    } else {
      const uint64_t base = hdr->Q[d.q_off + u + 1] - d.Qbase;
      const uint64_t Dm = (d.Qend - d.Qbase) - base;
      const uint64_t target = k * (Dm / K) + (k * (Dm % K)) / K;
      b = q_lower_bound(hdr->Q, d.q_off, d.Qbase, u + 1, d.n, base + target);
    }
    hdr->hseg[h] = static_cast<uint32_t>(b);
  }
}

// --------------------------------------------------------------------------
// lane plan.  Lane i of a graph starts at the first segment whose
// inclusive cumulative cost reaches i Z / L (Eq. 5 with P = L lanes), where a
// segment of source u carries cost c_u / K_u.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t lane_floor(uint64_t C, uint64_t L, uint64_t Z) {
  return static_cast<uint64_t>(floor(static_cast<double>(C) * static_cast<double>(L) / static_cast<double>(Z)));
}

__global__ void __launch_bounds__(256) k_lane_plan(const WsHeader* hdr) {
  if (hdr->status) return;
  const GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  const uint64_t total_r = hdr->total_r;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total_r; i += stride) {
    const uint32_t g = find_graph(G, i, [&](uint32_t x) { return desc[x].r_off; });
    const GraphDesc& d = desc[g];
    const uint64_t r = i - d.r_off;
    const uint64_t nr = d.u_end - d.u_begin;
    if (r >= nr) continue;
    hdr->A[i] = d.w[d.u_begin + r] / d.S;  // a_u of Alg. 1, once per source
    if (d.L == 0) continue;
    const uint64_t L = d.L;
    const uint64_t Z = d.C1 - d.C0;
    const uint64_t cex = hdr->C[i] - d.C0;
    const uint64_t cin = hdr->C[i + 1] - d.C0;
    const uint64_t K = hdr->SB[i + 1] - hdr->SB[i];
    uint64_t ilo = (r == 0) ? 0 : lane_floor(cex, L, Z) + 1;
    uint64_t ihi = lane_floor(cin, L, Z);
    if (ihi > L - 1) ihi = L - 1;
    const double cnode = static_cast<double>(cin - cex);
    for (uint64_t li = ilo; li <= ihi; ++li) {
      const double Ti = static_cast<double>(li) * static_cast<double>(Z) / static_cast<double>(L);
      double kk = ceil((Ti - static_cast<double>(cex)) * static_cast<double>(K) / cnode) - 1.0;
      if (!(kk > 0.0)) kk = 0.0;
      if (kk > static_cast<double>(K - 1)) kk = static_cast<double>(K - 1);
      hdr->lane_start[d.lane_off + li] =
          make_uint2(static_cast<uint32_t>(d.u_begin + r), static_cast<uint32_t>(kk));
      if (hdr->lane_cum) {
        // plan cost before the lane's first segment (segments of a source share its cost equally)
        const double before = static_cast<double>(cex) + kk * cnode / static_cast<double>(K);
        uint64_t cb = static_cast<uint64_t>(before);
        if (cb > cin) cb = cin;
        hdr->lane_cum[d.lane_off + li] = cb;
      }
    }
  }
}

// group -> graph map, and the padding lanes (empty: start = (u_end, 0))
__global__ void __launch_bounds__(256) k_lane_groups(const WsHeader* hdr) {
  if (hdr->status) return;
  const GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  const uint64_t ngroups = hdr->total_nl / kLaneGroup;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t q = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < ngroups; q += stride) {
    const uint64_t l0 = q * kLaneGroup;
    const uint32_t g = find_graph(G, l0, [&](uint32_t x) { return desc[x].lane_off; });
    const GraphDesc& d = desc[g];
    hdr->group_graph[q] = g;
    for (uint64_t li = (l0 - d.lane_off); li < (l0 - d.lane_off) + kLaneGroup; ++li) {
      if (li >= d.L) {
        hdr->lane_start[d.lane_off + li] = make_uint2(static_cast<uint32_t>(d.u_end), 0u);
        if (hdr->lane_cum) hdr->lane_cum[d.lane_off + li] = d.C1 - d.C0;
      }
    }
  }
}

// --------------------------------------------------------------------------
// the per-lane Create-Edges loop
// --------------------------------------------------------------------------
// pointers into global memory (address space 1), so that loads through them
// are global loads rather than generic ones
template <class T>
using gptr = const T __attribute__((address_space(1)))*;

template <class T>
__device__ __forceinline__ gptr<T> to_global(const T* p) {
  return (gptr<T>)(p);
}

// wave-uniform copies of values that are equal on every lane (they then live
// in scalar registers)
__device__ __forceinline__ uint32_t uni32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return (static_cast<uint64_t>(uni32(static_cast<uint32_t>(x >> 32))) << 32) | uni32(static_cast<uint32_t>(x));
}
__device__ __forceinline__ double unif64(double x) {
  return __longlong_as_double(static_cast<long long>(uni64(static_cast<uint64_t>(__double_as_longlong(x)))));
}
template <class T>
__device__ __forceinline__ const T* uniptr(const T* p) {
  return reinterpret_cast<const T*>(uni64(reinterpret_cast<uint64_t>(p)));
}

struct LaneCtx {
  gptr<double> w;
  gptr<double> A;                 // a_u = w_u / S of the range's sources (index u - u_begin)
  uint32_t n;
  uint32_t u_begin, u_heavy_end;  // sources [u_begin, u_heavy_end) are heavy
  gptr<uint64_t> SB;              // source prefix of segment counts (graph's r_off applied)
  uint64_t SB0;
  gptr<uint32_t> hseg;            // graph's heavy table
};

// Runs the segments of one lane from (u, k) up to (ue, ke) (exclusive) and
// reports each kept edge through emit(u, v); emit returns false to stop.
// All lanes of the wavefront iterate together; a lane that has finished its
// segment opens the next one at the top of the loop.
template <class Emit>
__device__ __forceinline__ void run_lane(const LaneCtx& cx, const RoundKeys& rk, const Series& sr, uint32_t u,
                                         uint32_t k, uint32_t ue, uint32_t ke, Emit& emit, uint32_t& visits) {
  bool more = (u < ue) || (u == ue && k < ke);
  bool inseg = false;
  uint32_t su = 0, sk = 0;   // source and segment of the open segment
  uint32_t j = 0, send = 0, t = 0;
  double a = 0.0, p = 0.0;
  while (true) {
    if (!inseg && more) {
      su = u;
      sk = k;
      const uint32_t r = u - cx.u_begin;
      a = cx.A[r];
      uint32_t K = 1;
      if (u < cx.u_heavy_end) {
        const uint64_t sb = cx.SB[r] - cx.SB0;
        K = static_cast<uint32_t>(cx.SB[r + 1] - cx.SB[r]);
        j = cx.hseg[sb + k];
        send = (k + 1 < K) ? cx.hseg[sb + k + 1] : cx.n;
      } else {
        j = u + 1;
        send = cx.n;
      }
      t = 0;
      p = (j < send) ? cap1(a * cx.w[j]) : 0.0;
      inseg = (p > 0.0);
      ++k;
      if (k >= K) {
        k = 0;
        ++u;
      }
      more = (u < ue) || (u == ue && k < ke);
    }
    if (!__any(inseg || more)) break;
    if (inseg) {
      // candidate step of Alg. 1: skip, then accept with probability q/p
      const bool capped = (p == 1.0);
      double wv_c = 0.0;
      if (capped) wv_c = cx.w[j];
      const bool need_rng = !capped || !(a * wv_c >= 1.0);
      Block4 x{0u, 0u, 0u, 0u};
      if (need_rng) x = philox10(t, sk, su, 0u, rk);
      ++t;
      bool stop = false;
      uint32_t v = j;
      double q;
      if (capped) {
        q = cap1(a * wv_c);
      } else {
        const double r_skip = unit53(x.x1, x.x0);
        const double ratio = ln_unit(r_skip, sr) / ln_one_minus(p, sr);
        if (!(ratio < static_cast<double>(send - j))) {
          stop = true;
          q = 0.0;
        } else {
          v = j + static_cast<uint32_t>(ratio);
          q = cap1(a * cx.w[v]);
        }
      }
      if (!stop) {
        ++visits;
        const double r_acc = unit53(x.x3, x.x2);
        const bool keep = capped ? (q == 1.0 || r_acc * p < q) : (r_acc * p < q);
        if (keep) {
          if (!emit(su, v)) {
            inseg = false;
            more = false;
            continue;
          }
        }
        p = q;
        j = v + 1;
        if (j >= send || !(p > 0.0)) stop = true;
      }
      if (stop) inseg = false;
    }
  }
}

struct CountEmit {
  uint32_t c;
  __device__ bool operator()(uint32_t, uint32_t) {
    ++c;
    return true;
  }
};

// Write-pass output through LDS: every lane stages its edges in 64-byte
// chunks of the output (8 pairs, aligned to the window start) and stores a
// chunk once it is complete, as four 16-byte stores, so that HBM receives
// whole 64-byte sectors instead of the 8-byte pieces of 64 interleaved lane
// streams.  Chunks a lane shares with its neighbours (its first and last) are
// stored pair by pair.  LDS layout [slot][thread] keeps the per-emission
// stores of a wavefront free of bank conflicts.
constexpr int kStageSlots = 8;

struct WriteEmit {
  uint2* stage;      // LDS, kStageSlots x blockDim entries
  uint32_t tid;      // thread in block
  uint32_t nthr;     // blockDim.x
  uint2* out;        // output window: out[i] is position lo + i
  uint64_t pos, lo, hi, first;
  __device__ uint2& slot(uint64_t q) { return stage[(q & (kStageSlots - 1)) * nthr + tid]; }
  __device__ void flush(uint64_t q0, uint64_t qend) {
    // chunk [q0, q0 + 8) of the window; the lane owns entries [max(q0, first), qend)
    const uint64_t f = (first > lo) ? first - lo : 0;
    const uint64_t s0 = (q0 > f) ? q0 : f;
    if (s0 == q0 && qend == q0 + kStageSlots) {
      uint4* dst = reinterpret_cast<uint4*>(out + q0);
#pragma unroll
      for (int i = 0; i < kStageSlots / 2; ++i) {
        const uint2 x0 = stage[(2 * i) * nthr + tid];
        const uint2 x1 = stage[(2 * i + 1) * nthr + tid];
        dst[i] = make_uint4(x0.x, x0.y, x1.x, x1.y);
      }
    } else {
      for (uint64_t q = s0; q < qend; ++q) out[q] = slot(q);
    }
  }
  __device__ bool operator()(uint32_t u, uint32_t v) {
    if (pos >= hi) return false;
    if (pos >= lo) {
      const uint64_t q = pos - lo;
      slot(q) = make_uint2(u, v);
      if ((q & (kStageSlots - 1)) == kStageSlots - 1) flush(q - (kStageSlots - 1), q + 1);
    }
    ++pos;
    return true;
  }
  // the lane's last, incomplete chunk
  __device__ void finish() {
    const uint64_t end = (pos < hi) ? pos : hi;
    if (end > lo) {
      const uint64_t q = end - lo;
      if (q & (kStageSlots - 1)) flush(q & ~static_cast<uint64_t>(kStageSlots - 1), q);
    }
  }
};

// One-pass output: the lane counts every kept edge and writes the first
// `cap` of them into its slot (64-byte aligned), staged like WriteEmit.
struct SlotEmit {
  WriteEmit wr;      // window = the slot
  uint32_t c;
  __device__ bool operator()(uint32_t u, uint32_t v) {
    ++c;
    if (wr.pos < wr.hi) wr(u, v);
    return true;
  }
};

// kMode 0: count pass.  kMode 1: write pass (replay into the output window;
// in one-pass plans only the lanes that overflowed their slot).  kMode 2:
// one pass, count and write into slots.
template <int kMode>
__global__ void __launch_bounds__(256) k_lanes(WsHeader* hdr, uint2* out, uint64_t e_lo, uint64_t e_hi) {
  constexpr bool kWrite = (kMode != 0);
  __shared__ uint2 stage[kWrite ? kStageSlots * 256 : 1];
  if (hdr->status || hdr->magic != kWsMagic) return;
  if (kMode == 1 && !hdr->planned) return;
  const bool only_overflow = (kMode == 1) && (uni32(hdr->mode) == 1);
  if (only_overflow && uni32(hdr->overflow) == 0) return;
  const GraphDesc* desc = hdr->desc;
  const uint64_t ngroups = uni64(hdr->total_nl) / kLaneGroup;
  const Series sr = load_series();
  const int lane = threadIdx.x & 63;
  uint64_t visited = 0;   // candidates visited by this lane over all its work items (count pass)
  // The loop body has no lane-divergent region that is not closed inside it:
  // the ticket is fetched by lane 0, broadcast to every lane (so the value is
  // uniform before readfirstlane marks it so for the compiler), and the only
  // other single-lane action (the candidate total) is done after the loop.
  while (true) {
    uint32_t grp = 0;
    if (lane == 0) grp = atomicAdd(&hdr->queue, 1u);
    grp = static_cast<uint32_t>(__shfl(static_cast<int>(grp), 0, 64));
    grp = uni32(grp);
    if (grp >= ngroups) break;
    const uint32_t g = uni32(hdr->group_graph[grp]);
    const GraphDesc& d = desc[g];
    const uint64_t lane_off = uni64(d.lane_off), NL = uni64(d.NL);
    const uint32_t u_end = uni32(static_cast<uint32_t>(d.u_end));
    const uint64_t l = static_cast<uint64_t>(grp) * kLaneGroup + lane;
    const uint2 st = hdr->lane_start[l];
    uint2 en = make_uint2(u_end, 0u);
    if (l + 1 < lane_off + NL) en = hdr->lane_start[l + 1];
    LaneCtx cx;
    cx.w = to_global(uniptr(d.w));
    cx.n = uni32(static_cast<uint32_t>(d.n));
    cx.u_begin = uni32(static_cast<uint32_t>(d.u_begin));
    cx.u_heavy_end = cx.u_begin + uni32(static_cast<uint32_t>(d.H));
    const uint64_t r_off = uni64(d.r_off);
    cx.A = to_global(uniptr(hdr->A) + r_off);
    cx.SB = to_global(uniptr(hdr->SB) + r_off);
    cx.SB0 = uni64(d.SB0);
    cx.hseg = to_global(uniptr(hdr->hseg) + uni64(d.hs_off));
    const RoundKeys rk = philox_round_keys(uni64(d.seed));
    if (kMode == 2) {
      const uint64_t s0 = hdr->slot_off[l];
      const uint64_t s1 = hdr->slot_off[l + 1];
      // the writer indexes its window from the window start: out[i] is slot position s0 + i
      SlotEmit em{WriteEmit{stage, threadIdx.x, blockDim.x, hdr->slots + s0, s0, s0, s1, s0}, 0u};
      uint32_t visits = 0;
      run_lane(cx, rk, sr, st.x, st.y, en.x, en.y, em, visits);
      em.wr.finish();
      hdr->lane_cnt[l] = em.c;
      if (em.c > s1 - s0) atomicAdd(&hdr->overflow, 1u);
      visited += visits;
    } else if (kMode == 1) {
      const uint64_t pos0 = hdr->lane_pos[l];
      const uint64_t cnt = hdr->lane_cnt[l];
      bool touches = (pos0 < e_hi) && (pos0 + cnt > e_lo);
      if (only_overflow) touches = touches && (cnt > hdr->slot_off[l + 1] - hdr->slot_off[l]);
      if (__any(touches)) {
        WriteEmit em{stage, threadIdx.x, blockDim.x, out, pos0, e_lo, e_hi, pos0};
        uint32_t su = st.x, sk = st.y, eu = en.x, ek = en.y;
        if (!touches) {
          eu = su;
          ek = sk;
        }
        uint32_t visits = 0;
        run_lane(cx, rk, sr, su, sk, eu, ek, em, visits);
        if (touches) em.finish();
      }
    } else {
      CountEmit em{0u};
      uint32_t visits = 0;
      run_lane(cx, rk, sr, st.x, st.y, en.x, en.y, em, visits);
      hdr->lane_cnt[l] = em.c;
      visited += visits;
    }
  }
  if (kMode != 1) {
    // candidates visited by the wavefront (statistics of the cost model)
    for (int dd = 32; dd >= 1; dd >>= 1) visited += shfl_idx64(visited, lane ^ dd);
    if (lane == 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&hdr->total_cand), static_cast<unsigned long long>(visited));
  }
}

// --------------------------------------------------------------------------
// one-pass slots: capacity of a lane = its plan cost mu (in expected
// candidates, which bounds its expected edges) + 8 sqrt(mu) + 24, rounded up
// to whole 64-byte chunks; a lane above it (probability < 1e-14 by the
// Chernoff bound used in Sec. 4, Theorem 2) is replayed by the write kernel.
// --------------------------------------------------------------------------
struct SlotIn {
  const WsHeader* hdr;
  uint64_t nl;
  __device__ uint64_t load(uint64_t l) const {
    if (l >= nl) return 0;
    const GraphDesc& d = hdr->desc[hdr->group_graph[l / kLaneGroup]];
    const uint64_t i = l - d.lane_off;
    if (i >= d.L) return 0;
    const uint64_t c1 = (i + 1 < d.L) ? hdr->lane_cum[l + 1] : (d.C1 - d.C0);
    const uint64_t c0 = hdr->lane_cum[l];
    const double mu = static_cast<double>(c1 > c0 ? c1 - c0 : 0) / static_cast<double>(kCostUnit);
    const double cap = (hdr->slot_margin == 1) ? mu : (mu + 8.0 * sqrt(mu) + 24.0);
    const uint64_t c = static_cast<uint64_t>(ceil(cap));
    return (c + kStageSlots - 1) / kStageSlots * kStageSlots;
  }
};

struct SlotOut {
  uint64_t* off;
  __device__ void store(uint64_t i, uint64_t, uint64_t ex) const { off[i] = ex; }
};

__global__ void k_slot_check(WsHeader* hdr) {
  if (hdr->slot_off[hdr->total_nl] > hdr->slot_cap) atomicOr(&hdr->status, kStCapacity);
}

// copies every lane's slot to its place in the output window [lo, hi); one
// wavefront per 64 lanes, 64 edges per step
__global__ void __launch_bounds__(256) k_compact(const WsHeader* hdr, uint2* out, uint64_t lo, uint64_t hi) {
  if (hdr->status || hdr->mode != 1 || !hdr->planned) return;
  const uint64_t ngroups = uni64(hdr->total_nl) / kLaneGroup;
  const int lane = threadIdx.x & 63;
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / 64);
  gptr<uint64_t> slots = to_global(uniptr(reinterpret_cast<const uint64_t*>(hdr->slots)));
  uint64_t* out64 = reinterpret_cast<uint64_t*>(out);
  for (uint64_t grp = uni64(static_cast<uint64_t>(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6));
       grp < ngroups; grp += nwaves) {
    const uint64_t l = grp * kLaneGroup + lane;
    const uint64_t my_pos = hdr->lane_pos[l];
    const uint64_t my_cnt = hdr->lane_cnt[l];
    const uint64_t my_s0 = hdr->slot_off[l];
    const uint64_t my_cap = hdr->slot_off[l + 1] - my_s0;
    for (int j = 0; j < 64; ++j) {
      const uint64_t pos = uni64(shfl_idx64(my_pos, j));
      const uint64_t cnt = uni64(shfl_idx64(my_cnt, j));
      const uint64_t s0 = uni64(shfl_idx64(my_s0, j));
      const uint64_t cap = uni64(shfl_idx64(my_cap, j));
      if (cnt == 0 || cnt > cap || pos >= hi || pos + cnt <= lo) continue;
      const uint64_t a = (pos > lo) ? pos : lo;
      const uint64_t b = (pos + cnt < hi) ? pos + cnt : hi;
      for (uint64_t e = a + lane; e < b; e += 64) out64[e - lo] = slots[s0 + (e - pos)];
    }
  }
}

// --------------------------------------------------------------------------
// offsets of the lanes' output
// --------------------------------------------------------------------------
struct CntIn {
  const uint32_t* cnt;
  uint64_t n;
  __device__ uint64_t load(uint64_t i) const { return (i < n) ? cnt[i] : 0; }
};

struct OffOut {
  uint64_t* off;
  __device__ void store(uint64_t i, uint64_t, uint64_t ex) const { off[i] = ex; }
};

__global__ void __launch_bounds__(256) k_graph_edges(WsHeader* hdr, uint64_t* m_dev) {
  GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
    GraphDesc& d = desc[g];
    if (hdr->status || d.NL == 0) {
      d.m = 0;
      d.edge_off = (d.NL == 0 && !hdr->status) ? hdr->lane_pos[d.lane_off] : 0;
    } else {
      d.edge_off = hdr->lane_pos[d.lane_off];
      d.m = hdr->lane_pos[d.lane_off + d.NL] - d.edge_off;
    }
    if (m_dev) m_dev[g] = d.m;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->total_m = hdr->status ? 0 : hdr->lane_pos[hdr->total_nl];
}

__global__ void __launch_bounds__(256) k_graph_offsets(const WsHeader* hdr, uint64_t* go) {
  const uint32_t G = hdr->G;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g <= G; g += gridDim.x * blockDim.x)
    go[g] = (g < G) ? hdr->desc[g].edge_off : hdr->total_m;
}

// --------------------------------------------------------------------------
// digest of an edge list (position keyed, order independent reduction)
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_hash(const uint2* e, uint64_t m, uint64_t base,
                                               unsigned long long* acc) {
  uint64_t h = 0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint2 x = e[i];
    const uint64_t key = (static_cast<uint64_t>(x.x) << 32) | x.y;
    h += mix64(mix64(base + i) ^ key);
  }
  // wave reduction, then one atomic per wave
  for (int d = 32; d >= 1; d >>= 1) h += shfl_idx64(h, (threadIdx.x & 63) ^ d);
  if ((threadIdx.x & 63) == 0) atomicAdd(acc, static_cast<unsigned long long>(h));
}

}  // namespace cl

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
// pointers into global memory (address space 1), so that loads through them
// are global loads rather than generic ones
template <class T>
using gptr = const T __attribute__((address_space(1)))*;

template <class T>
__device__ __forceinline__ gptr<T> to_global(const T* p) {
  return (gptr<T>)(p);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// writable global pointers (stores with immediate offsets, no LDS aperture check)
template <class T>
using gout = T __attribute__((address_space(1)))*;

template <class T>
__device__ __forceinline__ gout<T> to_global_mut(T* p) {
  return (gout<T>)(p);
}

// wave-uniform copies of values that are equal on every lane (they then live
// in scalar registers)
__device__ __forceinline__ uint32_t uni32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
  return (static_cast<uint64_t>(uni32(static_cast<uint32_t>(x >> 32))) << 32) | uni32(static_cast<uint32_t>(x));
}
template <class T>
__device__ __forceinline__ const T* uniptr(const T* p) {
  return reinterpret_cast<const T*>(uni64(reinterpret_cast<uint64_t>(p)));
}
template <class T>
__device__ __forceinline__ T* uniptr_mut(T* p) {
  return reinterpret_cast<T*>(uni64(reinterpret_cast<uint64_t>(p)));
}

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

// largest g in [lo, hi] with off(g) <= i (off(lo) <= i)
template <class F>
__device__ __forceinline__ uint32_t find_graph_in(uint32_t lo, uint32_t hi, uint64_t i, F off) {
  uint32_t h = hi + 1;
  while (h - lo > 1) {
    const uint32_t mid = (lo + h) >> 1;
    if (off(mid) <= i) lo = mid; else h = mid;
  }
  return lo;
}

// largest g >= from with off(g) <= i, for off(from) <= i: a few steps forward
// one graph at a time (a tile walk meets a new graph rarely), then a search
// of the rest (many small graphs)
template <class F>
__device__ __forceinline__ uint32_t advance_graph(uint32_t G, uint32_t from, uint64_t i, F off) {
  for (int step = 0; step < 4; ++step) {
    if (from + 1 >= G || off(from + 1) > i) return from;
    ++from;
  }
  return find_graph_in(from, G - 1, i, off);
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
// (single graph), also accumulates the exact sum.  A single graph's fields
// are read once and its flags ORed once per thread; each thread handles
// kValUnroll slots of a tile per step, their loads issued together.
constexpr int kValUnroll = 4;
constexpr uint64_t kValTile = 256 * kValUnroll;   // slots per tile (several graphs)

struct ValView {
  const double* w;
  uint64_t q_off, n;
  double S;
  uint32_t g;
};

template <bool want_sum>
__global__ void __launch_bounds__(256) k_validate(GraphDesc* desc, uint32_t G, uint64_t total_slots,
                                                  unsigned long long* bins) {
  __shared__ unsigned long long lbins[want_sum ? 2 * kBins : 2];
  if (want_sum) {
    for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) lbins[i] = 0ull;
    __syncthreads();
  }
  auto view = [&](uint32_t g) {
    const GraphDesc& d = desc[g];
    return ValView{d.w, d.q_off, d.n, d.S, g};
  };
  const ValView v0 = view(0);
  uint32_t flags0 = 0;     // single graph: its flags, ORed at the end
  int cur_b = -1;
  uint64_t acc_lo = 0, acc_hi = 0;
  // kValUnroll slots idx[r] of graphs dv[r] (idx >= total_slots: none), their
  // loads issued together
  auto step = [&](const uint64_t (&idx)[kValUnroll], const ValView (&dv)[kValUnroll]) {
    double x[kValUnroll], y[kValUnroll];
    bool live[kValUnroll];
#pragma unroll
    for (int r = 0; r < kValUnroll; ++r) {
      const uint64_t v = idx[r] - dv[r].q_off;
      live[r] = (idx[r] < total_slots) && (v < dv[r].n);
      x[r] = live[r] ? dv[r].w[v] : 0.0;
      y[r] = (live[r] && v + 1 < dv[r].n) ? dv[r].w[v + 1] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kValUnroll; ++r) {
      if (!live[r]) continue;
      const uint64_t v = idx[r] - dv[r].q_off;
      const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x[r]));
      const uint32_t ex = static_cast<uint32_t>((bits >> 52) & 0x7FF);
      uint32_t flag = 0;
      if (ex == 0x7FF) {
        flag |= kStNonfinite;
      } else if (x[r] < 0.0) {
        flag |= kStNegative;
      } else {
        if (x[r] < y[r]) flag |= kStUnsorted;   // y = 0 past the last weight
        if (v == 0) {
          if (x[r] > dv[r].S || (x[r] > 0.0 && x[r] < 0x1.0p-960)) flag |= kStBadS;
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
      if (flag) {
        if (G == 1) flags0 |= flag;
        else atomicOr(&desc[dv[r].g].status, flag);
      }
    }
  };
  // each block walks a run of consecutive tiles of kValTile slots (with the
  // weights sorted, a thread's items then mostly share an exponent, so its
  // sum accumulator rarely flushes); with several graphs, a tile inside one
  // graph reads that graph's fields once, by block-uniform loads, and a tile
  // across graphs searches only the graphs it spans
  uint64_t idx[kValUnroll];
  ValView dv[kValUnroll];
  auto qoff = [&](uint32_t q) { return desc[q].q_off; };
  const uint64_t ntiles = (total_slots + kValTile - 1) / kValTile;
  const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;   // consecutive tiles per block
  const uint64_t t_end = ((blockIdx.x + 1) * per < ntiles) ? (blockIdx.x + 1) * per : ntiles;
  uint32_t gc = 0;   // graph of the last tile's end (the walk only moves forward)
  bool first = true;
  for (uint64_t tile = blockIdx.x * per; tile < t_end; ++tile) {
    const uint64_t tb = tile * kValTile;
    const uint64_t te = ((tb + kValTile < total_slots) ? tb + kValTile : total_slots) - 1;
#pragma unroll
    for (int r = 0; r < kValUnroll; ++r) idx[r] = tb + static_cast<uint64_t>(r) * blockDim.x + threadIdx.x;
    if (G == 1) {
#pragma unroll
      for (int r = 0; r < kValUnroll; ++r) dv[r] = v0;
    } else {
      const uint32_t g0 = uni32(first ? find_graph(G, tb, qoff) : advance_graph(G, gc, tb, qoff));
      const uint32_t g1 = uni32(advance_graph(G, g0, te, qoff));
      gc = g1;
      first = false;
      if (g0 == g1) {
        const ValView vg = view(g0);
#pragma unroll
        for (int r = 0; r < kValUnroll; ++r) dv[r] = vg;
      } else {
#pragma unroll
        for (int r = 0; r < kValUnroll; ++r) dv[r] = view(find_graph_in(g0, g1, idx[r] < te ? idx[r] : te, qoff));
      }
    }
    step(idx, dv);
  }
  if (flags0) atomicOr(&desc[0].status, flags0);
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
// (ties to even).  One wavefront: lane L owns limb L (bits [64 L, 64 L + 64))
// of the big integer T; 36 limbs cover 2^2304.  Zero bins are skipped.
// S_out[0] gets S and S_out[1] (as a 64-bit word) the status flags.
constexpr int kLimbs = 36;

__global__ void __launch_bounds__(64) k_sum_finalize(const unsigned long long* bins, double* S_out,
                                                     uint32_t* status) {
  if (blockIdx.x != 0) return;
  const int L = threadIdx.x;   // limb
  uint64_t acc = 0, carry = 0;  // limb value acc + carry 2^64
  auto add_at = [&](uint64_t val, int sh) {
    const int li = sh >> 6;
    const int bs = sh & 63;
    uint64_t part = 0;
    if (L == li) part = val << bs;
    if (L == li + 1 && bs != 0) part = val >> (64 - bs);
    acc += part;
    carry += (acc < part) ? 1 : 0;
  };
  // all bin words are loaded first (one round trip instead of one per chunk)
  constexpr int kChunks = 2 * kBins / 64;
  uint64_t words[kChunks];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) words[c] = bins[c * 64 + L];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int b0 = c * 64;
    const uint64_t mine = words[c];
    uint64_t nz = __ballot(mine != 0);
    while (nz) {
      const int k = __ffsll(static_cast<long long>(nz)) - 1;
      nz &= nz - 1;
      const int idx = b0 + k;                // bin b = idx / 2, half idx & 1
      const int b = idx >> 1;
      if (b == 0) continue;                  // bin 0 is never filled
      add_at(shfl_idx64(mine, k), (b - 1) + ((idx & 1) ? 32 : 0));
    }
  }
  // carry propagation, limb by limb
  uint64_t T = 0, cin = 0;
  for (int l = 0; l < kLimbs; ++l) {
    const uint64_t a = shfl_idx64(acc, l);
    const uint64_t c = shfl_idx64(carry, l);
    const uint64_t t = a + cin;
    if (L == l) T = t;
    cin = c + ((t < cin) ? 1 : 0);
  }
  auto limb = [&](int l) -> uint64_t { return (l >= 0 && l < kLimbs) ? shfl_idx64(T, l) : 0ull; };
  const uint64_t nzl = __ballot(L < kLimbs && T != 0);
  double S;
  bool inf_sum = false;   // the sum rounds past the largest double
  if (nzl == 0) {
    S = 0.0;
  } else {
    const int topL = 63 - __clzll(static_cast<long long>(nzl));
    const uint64_t tv = limb(topL);
    const int top = topL * 64 + 63 - __clzll(static_cast<long long>(tv));
    if (top <= 52) {
      S = __longlong_as_double(static_cast<long long>(limb(0)));   // value = T 2^-1074, bits = T
    } else {
      const int shift = top - 52;   // mant = bits [shift, top]
      auto bits_from = [&](int p) -> uint64_t {
        // 64 bits of T starting at bit p (p >= 0)
        const int l = p >> 6, o = p & 63;
        const uint64_t lo = limb(l), hi = limb(l + 1);
        return o ? ((lo >> o) | (hi << (64 - o))) : lo;
      };
      uint64_t mant = bits_from(shift) & ((1ull << 53) - 1);
      const int hp = shift - 1;    // half bit
      const uint64_t half = (bits_from(hp) & 1ull);
      bool sticky = false;
      if (hp > 0) {
        const int ls = hp >> 6, os = hp & 63;
        sticky = (os != 0) && ((limb(ls) & ((1ull << os) - 1)) != 0);
        const uint64_t below = (ls > 0) ? (nzl & ((1ull << ls) - 1)) : 0ull;
        sticky = sticky || (below != 0);
      }
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
        inf_sum = true;
      } else {
        S = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(e) << 52) |
                                                        (mant & 0x000FFFFFFFFFFFFFull)));
      }
    }
  }
  if (L == 0) {
    // the validation kernel's flags (an earlier launch) and this one's; the
    // status word is also stored beside S, so that one read returns both
    uint32_t st = *status;
    if (inf_sum) {
      st |= kStNonfinite;
      atomicOr(status, kStNonfinite);
    }
    S_out[0] = S;
    reinterpret_cast<unsigned long long*>(S_out)[1] = st;
  }
}

// a graph's quantisation scale 2^32 / w_0 (0 when w_0 = 0)
__device__ __forceinline__ void graph_init(GraphDesc& d) {
  const double w0 = (d.n > 0) ? d.w[0] : 0.0;
  d.qscale = (w0 > 0.0) ? (4294967296.0 / w0) : 0.0;
}

__global__ void k_graph_init(GraphDesc* desc, uint32_t G) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  graph_init(desc[g]);
}

// the start of a plan: cleared status words and counters (a replayed graph
// starts from a clean state) and each graph's quantisation scale
__global__ void k_plan_init(WsHeader* hdr) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g == 0) {
    hdr->status = 0;
    hdr->total_cand = 0;
    hdr->total_words = 0;
    hdr->queue = 0;      // the unit queue of the plan's lane kernel
    hdr->overflow = 0;
  }
  if (g >= hdr->G) return;
  hdr->desc[g].status = 0;
  graph_init(hdr->desc[g]);
}

// --------------------------------------------------------------------------
// quantised prefix Q, all graphs in one scan
// --------------------------------------------------------------------------
struct QIn {
  const GraphDesc* desc;
  uint32_t G;
  struct Ctx {
    const double* w;
    uint64_t n, q_off;
    double qscale;
  };
  __device__ uint32_t graph_of(uint64_t i) const {
    return find_graph(G, i, [&](uint32_t x) { return desc[x].q_off; });
  }
  __device__ Ctx context(uint32_t g) const {
    const GraphDesc& d = desc[g];
    return Ctx{d.w, d.n, d.q_off, d.qscale};
  }
  __device__ uint64_t load(uint64_t i, const Ctx& c) const {
    const uint64_t v = i - c.q_off;
    if (v >= c.n || c.qscale == 0.0) return 0;
    return quantise(c.w[v], c.qscale);
  }
};

struct QOut {
  GraphDesc* desc;
  uint32_t G;
  uint64_t* Q;
  struct Ctx {
    GraphDesc* d;
    uint64_t n, q_off;
  };
  __device__ Ctx context(uint32_t g) const { return Ctx{desc + g, desc[g].n, desc[g].q_off}; }
  __device__ void store(uint64_t i, const Ctx& c, uint64_t, uint64_t ex) const {
    Q[i] = ex;
    const uint64_t v = i - c.q_off;
    if (v == 0) c.d->Qbase = ex;
    if (v == c.n) c.d->Qend = ex;
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
  struct Ctx {
    const double* w;
    const uint64_t* Qg;   // the graph's quantised prefix relative to Qbase
    double S, qscale;
    uint64_t n, u_begin, nr, r_off, Qbase, Qn;
  };
  __device__ uint32_t graph_of(uint64_t i) const {
    return find_graph(G, i, [&](uint32_t x) { return desc[x].r_off; });
  }
  __device__ Ctx context(uint32_t g) const {
    const GraphDesc& d = desc[g];
    return Ctx{d.w, Q + d.q_off, d.S, d.qscale, d.n, d.u_begin, d.u_end - d.u_begin, d.r_off, d.Qbase,
               d.Qend - d.Qbase};
  }
  __device__ Triple load(uint64_t i, const Ctx& c) const {
    const uint64_t r = i - c.r_off;
    if (r >= c.nr) return Triple{0, 0, 0};
    const uint64_t u = c.u_begin + r;
    uint32_t K = 1;
    double eh = 0.0;
    if (c.qscale != 0.0 && u + 1 < c.n) {
      const double a = c.w[u] / c.S;
      const uint64_t D = c.Qn - (c.Qg[u + 1] - c.Qbase);
      eh = ehat_of(a, D, c.qscale);
      K = nseg_of(eh, c.n, u);
    }
    double ce = eh * static_cast<double>(kCostUnit);
    if (ce > 0x1.0p36) ce = 0x1.0p36;
    const uint64_t cost = static_cast<uint64_t>(ce) + static_cast<uint64_t>(kCostUnit) * K;
    return Triple{cost, K, (K > 1) ? 1ull : 0ull};
  }
};

struct NodeOut {
  GraphDesc* desc;
  uint32_t G;
  uint64_t* C;
  uint64_t* SB;
  struct Ctx {
    GraphDesc* d;
    uint64_t r_off, nr;
  };
  __device__ Ctx context(uint32_t g) const {
    return Ctx{desc + g, desc[g].r_off, desc[g].u_end - desc[g].u_begin};
  }
  __device__ void store(uint64_t i, const Ctx& c, Triple, Triple ex) const {
    C[i] = ex.c;
    SB[i] = ex.k;
    const uint64_t r = i - c.r_off;
    if (r == 0) {
      c.d->C0 = ex.c;
      c.d->SB0 = ex.k;
      c.d->H0 = ex.h;
    }
    if (r == c.nr) {
      c.d->C1 = ex.c;
      c.d->SB1 = ex.k;
      c.d->H1 = ex.h;
    }
  }
};

// --------------------------------------------------------------------------
// per-graph sizes, offsets over graphs (one block)
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_plan_sizes(WsHeader* hdr) {
  GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  uint64_t carry_nh = 0, carry_nl = 0, carry_cost = 0, carry_seg = 0;
  for (uint32_t base = 0; base < G; base += blockDim.x) {
    const uint32_t g = base + threadIdx.x;
    uint64_t nh = 0, nl = 0, cost = 0, sg = 0;
    if (g < G) {
      GraphDesc& d = desc[g];
      const uint64_t nr = d.u_end - d.u_begin;
      d.H = d.H1 - d.H0;
      const uint64_t Z = d.C1 - d.C0;
      const uint64_t nseg = d.SB1 - d.SB0;
      nh = (d.H > 0) ? (hdr->SB[d.r_off + d.H] - d.SB0) : 0;
      uint64_t L = 0, Lm = 0, Zm = Z;
      if (nr > 0 && d.qscale != 0.0 && d.status == 0) {
        L = (Z + d.budget - 1) / d.budget;
        if (L > nseg) L = nseg;
        if (d.policy == 1 && L > nr) L = nr;   // equal source counts: at most one unit per source
        if (L == 0) L = 1;
        Lm = L;
        const uint64_t bt = d.budget / kTailDiv;
        if (d.policy == 0 && d.graded && L >= kTailMinUnits && bt > 0) {
          const uint64_t Zt = Z / kTailShare;
          const uint64_t m = (Z - Zt + d.budget - 1) / d.budget;
          const uint64_t t = (Zt + bt - 1) / bt;
          if (m > 0 && t > 0 && m + t <= nseg) {
            Zm = Z - Zt;
            Lm = m;
            L = m + t;
          }
        }
      }
      // segment and unit indices are 32-bit: a graph above 2^32 - 1 segments
      // is refused (n < 2^32 sources leaves room for ~1e9 heavy segments)
      if (nseg > 0xFFFFFFFFull) atomicOr(&d.status, kStCapacity);
      // round-robin units step by L <= nseg: keep sg + L below 2^32
      if (d.policy == 2 && nseg > 0x80000000ull) atomicOr(&d.status, kStCapacity);
      d.L = L;
      d.Lm = Lm;
      d.Zm = Zm;
      d.um = (Zm > 0) ? static_cast<double>(Lm) / static_cast<double>(Zm) : 0.0;
      d.ut = (Z > Zm) ? static_cast<double>(L - Lm) / static_cast<double>(Z - Zm) : 0.0;
      d.NH = nh;
      sg = nseg;
      cost = (L > 0) ? Z : 0;
      nl = (L + kLaneGroup - 1) / kLaneGroup * kLaneGroup;
      d.NL = nl;
    }
    uint64_t tot_nh, tot_nl, tot_cost, tot_seg;
    const uint64_t ex_nh = block_exclusive<uint64_t>(nh, &tot_nh);
    const uint64_t ex_nl = block_exclusive<uint64_t>(nl, &tot_nl);
    (void)block_exclusive<uint64_t>(cost, &tot_cost);
    (void)block_exclusive<uint64_t>(sg, &tot_seg);
    carry_cost += tot_cost;
    carry_seg += tot_seg;
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
    hdr->total_seg = carry_seg;
    uint32_t st = 0;
    for (uint32_t g = 0; g < G; ++g) st |= desc[g].status;
    if (hdr->cap_nl != 0 && (carry_nh > hdr->cap_nh || carry_nl > hdr->cap_nl)) st |= kStCapacity;
    if (carry_nl > 0xFFFFFFFFull) st |= kStCapacity;   // units are numbered in 32 bits
    hdr->status |= st;
  }
}

// --------------------------------------------------------------------------
// lane plan.  Lane i of a graph starts at the first segment whose
// inclusive cumulative cost reaches T_i (Eq. 5 with P = L lanes), where a
// segment of source u carries cost c_u / K_u; T_i = i Zm / Lm for i <= Lm and
// Zm + (i - Lm) (Z - Zm) / (L - Lm) after (uniform units when Lm = L).
// A segment with cost share (b, b'] holds the starts of the units i with
// b < T_i <= b' (the graph's first segment also holds unit 0).  The plan
// only schedules: the rates Lm / Zm, ... are rounded once per graph and
// multiplied here.  The count of unit starts up to x is monotone in x and
// neighbouring segments compute their common bound identically, so every
// unit is claimed by exactly one segment and the lane starts stay in order.
// The starts inside heavy sources are claimed by the heavy-segment table
// (one thread per segment, so a source with many units is spread over
// threads); those of the one-segment sources by the lane-plan kernel.
// --------------------------------------------------------------------------
struct PlanCtx {
  const double* w;
  double S;
  uint64_t r_off, nr, u_begin, L, C0, SB0, lane_off, Lm, Zm, H, NH;
  double um, ut;
  uint32_t policy;
  // the last unit whose start is at most x, as an integral double
  __device__ double unit_at(double x) const {
    const double zm = static_cast<double>(Zm);
    if (x < zm || Lm == L) return floor(x * um);
    return static_cast<double>(Lm) + floor((x - zm) * ut);
  }
  // units of equal cost whose starts are claimed here
  __device__ bool equal_cost_units() const { return L != 0 && policy == 0; }
};

__device__ __forceinline__ PlanCtx plan_ctx(const GraphDesc& d) {
  return PlanCtx{d.w,  d.S,  d.r_off, d.u_end - d.u_begin, d.u_begin, d.L, d.C0, d.SB0, d.lane_off, d.Lm, d.Zm,
                 d.H,  d.NH, d.um,    d.ut,                d.policy};
}

// Units (flo, min(fhi, L - 1)] start at graph-relative segment seg, with plan
// cost cum before it.
__device__ __forceinline__ void claim_units(const PlanCtx& p, double flo, double fhi, uint64_t seg, uint64_t cum,
                                            gout<uint32_t> lane_seg, gout<uint64_t> lane_cum) {
  fhi = fmin(fhi, static_cast<double>(p.L - 1));
  if (!(flo < fhi)) return;
  const uint64_t ihi = static_cast<uint64_t>(fhi);
  for (uint64_t li = static_cast<uint64_t>(flo + 1.0); li <= ihi; ++li) {
    lane_seg[p.lane_off + li] = static_cast<uint32_t>(seg);
    if (lane_cum) lane_cum[p.lane_off + li] = cum;
  }
}

// --------------------------------------------------------------------------
// heavy-segment table (one thread per heavy segment), and the unit starts
// inside heavy segments.  The graph's fields are read once per thread into
// registers (before any store).  Each thread searches its segment's start;
// the end comes from the next lane, except in a wavefront's last lane, whose
// two searches advance in lockstep.
// --------------------------------------------------------------------------
struct HeavyCtx {
  uint64_t hs_off, H, r_off, SB0, u_begin, q_off, Qbase, Qn, n;
};

__device__ __forceinline__ HeavyCtx heavy_ctx(const GraphDesc& d) {
  return HeavyCtx{d.hs_off, d.H, d.r_off, d.SB0, d.u_begin, d.q_off, d.Qbase, d.Qend - d.Qbase, d.n};
}

__global__ void __launch_bounds__(256) k_heavy_table(const WsHeader* hdr) {
  if (hdr->status) return;
  const GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  const uint64_t NH = hdr->total_nh;
  const gptr<uint64_t> SB = to_global(hdr->SB);
  const gptr<uint64_t> Q = to_global(hdr->Q);
  const gout<u32x4> hseg = to_global_mut(reinterpret_cast<u32x4*>(hdr->hseg));   // HSeg {u, k, j, send}
  const gptr<uint64_t> C = to_global(hdr->C);
  const gout<uint32_t> lane_seg = to_global_mut(hdr->lane_seg);
  const gout<uint64_t> lane_cum = to_global_mut(hdr->lane_cum);
  const HeavyCtx c0 = heavy_ctx(desc[0]);
  const PlanCtx p0 = plan_ctx(desc[0]);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t h = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; h < NH; h += stride) {
    const uint32_t g = (G == 1) ? 0u : find_graph(G, h, [&](uint32_t x) { return desc[x].hs_off; });
    const HeavyCtx c = (G == 1) ? c0 : heavy_ctx(desc[g]);
    const uint64_t hl = h - c.hs_off;
    // heavy source: last r in [0, H) with SB(r) - SB0 <= hl
    uint64_t lo = 0, hi = c.H;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (SB[c.r_off + mid] - c.SB0 <= hl) lo = mid; else hi = mid;
    }
    const uint64_t r = lo;
    const uint64_t sbr = SB[c.r_off + r];
    const uint64_t K = SB[c.r_off + r + 1] - sbr;
    const uint64_t cex = C[c.r_off + r], cin = C[c.r_off + r + 1];   // used after the searches
    const uint64_t k = hl - (sbr - c.SB0);
    const uint64_t u = c.u_begin + r;
    const gptr<uint64_t> Qg = Q + c.q_off;
    const uint64_t base = Qg[u + 1] - c.Qbase;
    const uint64_t Dm = c.Qn - base;
    // b_kk = first v in [u+1, n] with Q_v - Q_{u+1} >= kk floor(D/K) + floor(kk (D mod K) / K)
    // (b_0 = u + 1; the last segment ends at n)
    auto target = [&](uint64_t kk) { return base + kk * (Dm / K) + (kk * (Dm % K)) / K; };
    const uint64_t t0 = target(k), t1 = target(k + 1);
    // The end of segment k is the start of segment k + 1, which the next lane
    // searches (table entry h + 1) unless this is the wavefront's last lane or
    // the table's last entry; the last segment of a source ends at n.
    const int lane = threadIdx.x & 63;
    const bool own_end = (k + 1 < K) && (lane == 63 || h + 1 >= NH);
    uint64_t lo0 = u + 1, hi0 = c.n, lo1 = u + 1, hi1 = c.n;
    if (k == 0) hi0 = lo0;
    if (!own_end) lo1 = hi1;
    while (lo0 < hi0 || lo1 < hi1) {
      const uint64_t m0 = lo0 + ((hi0 - lo0) >> 1);
      const uint64_t m1 = lo1 + ((hi1 - lo1) >> 1);
      const uint64_t q0 = (lo0 < hi0) ? Qg[m0] - c.Qbase : 0;
      const uint64_t q1 = (lo1 < hi1) ? Qg[m1] - c.Qbase : 0;
      if (lo0 < hi0) {
        if (q0 >= t0) hi0 = m0; else lo0 = m0 + 1;
      }
      if (lo1 < hi1) {
        if (q1 >= t1) hi1 = m1; else lo1 = m1 + 1;
      }
    }
    const uint32_t next_start = static_cast<uint32_t>(__shfl_down(static_cast<int>(lo0), 1, 64));
    const uint32_t send = (k + 1 >= K) ? static_cast<uint32_t>(c.n) : own_end ? static_cast<uint32_t>(lo1) : next_start;
    hseg[h] = u32x4{static_cast<uint32_t>(u), static_cast<uint32_t>(k), static_cast<uint32_t>(lo0), send};
    const PlanCtx p = (G == 1) ? p0 : plan_ctx(desc[g]);
    if (p.equal_cost_units()) {
      // segment k's share (b_k, b_k+1] of the source's cost (C_u, C_u+1]
      const double ce = static_cast<double>(cex - p.C0), ci = static_cast<double>(cin - p.C0);
      const double per_seg = (ci - ce) / static_cast<double>(K);
      auto bound = [&](uint64_t kk) {
        return (kk == 0) ? ce : (kk == K) ? ci : ce + static_cast<double>(kk) * per_seg;
      };
      const double b0 = bound(k);
      const double flo = (r == 0 && k == 0) ? -1.0 : p.unit_at(b0);
      const uint64_t cum = static_cast<uint64_t>(b0);
      claim_units(p, flo, p.unit_at(bound(k + 1)), hl, cum < cin - p.C0 ? cum : cin - p.C0, lane_seg, lane_cum);
    }
  }
}

// Each thread takes kPlanUnroll sources per step, their loads (weight and
// cost prefixes) issued together before any of them is used.  A single
// graph has its own instance (kOne) with no per-source descriptor loads,
// whose waits would also wait for the stores in flight.  Several graphs are
// walked in tiles of kPlanTile consecutive sources, a run of consecutive
// tiles per block: a tile inside one graph reads that graph's fields once, by
// block-uniform loads; a tile across graphs searches only the graphs it spans.
constexpr int kPlanUnroll = 4;
constexpr uint64_t kPlanTile = 256 * kPlanUnroll;

// the workspace arrays the lane plan reads and writes, read once per thread
struct PlanArrays {
  uint64_t total_r;
  gptr<uint64_t> C, SB;
  gout<double> A;
  gout<uint32_t> lane_seg;
  gout<uint64_t> lane_cum;
};

// one step over the sources idx[q] (idx >= total_r: none); ctx(q) gives
// item q's graph fields
template <class Ctx>
__device__ __forceinline__ void plan_sources_step(const PlanArrays& pa, const uint64_t (&idx)[kPlanUnroll], Ctx ctx) {
  const uint64_t total_r = pa.total_r;
  const gptr<uint64_t> C = pa.C;
  const gptr<uint64_t> SB = pa.SB;
  const gout<double> A = pa.A;
  const gout<uint32_t> lane_seg = pa.lane_seg;
  const gout<uint64_t> lane_cum = pa.lane_cum;
  bool live[kPlanUnroll];
  double wu[kPlanUnroll];
  uint64_t cl[kPlanUnroll], ch[kPlanUnroll];
#pragma unroll
  for (int q = 0; q < kPlanUnroll; ++q) {
    const uint64_t i = idx[q];
    const PlanCtx d = ctx(q);
    const uint64_t r = i - d.r_off;
    live[q] = (i < total_r) && (r < d.nr);   // r < nr: C[i + 1] is the graph's own
    wu[q] = live[q] ? to_global(d.w)[d.u_begin + r] : 0.0;
    cl[q] = live[q] ? C[i] : 0;
    ch[q] = live[q] ? C[i + 1] : 0;
  }
  // the unit starts of the one-segment sources (graph-relative segment
  // NH + r - H), computed before any store: a wait for a load also waits
  // for the stores issued before it
  double flo[kPlanUnroll], fhi[kPlanUnroll];
  uint64_t seg[kPlanUnroll];
#pragma unroll
  for (int q = 0; q < kPlanUnroll; ++q) {
    flo[q] = 0.0;
    fhi[q] = 0.0;
    seg[q] = 0;
    if (!live[q]) continue;
    const uint64_t i = idx[q];
    const PlanCtx d = ctx(q);
    const uint64_t r = i - d.r_off;
    if (d.equal_cost_units()) {
      if (r < d.H) continue;   // claimed segment by segment with the heavy table
      flo[q] = (r == 0) ? -1.0 : d.unit_at(static_cast<double>(cl[q] - d.C0));
      fhi[q] = d.unit_at(static_cast<double>(ch[q] - d.C0));
      seg[q] = d.NH + (r - d.H);
    } else if (d.L != 0 && d.policy == 1) {
      // equal source counts: unit li starts at source floor(li nr / L), segment 0
      // (L <= nr, so a source starts at most one unit); round-robin starts
      // (policy 2) are set with the groups
      const uint64_t L = d.L;
      const uint64_t li = (r * L + d.nr - 1) / d.nr;          // ceil(r L / nr)
      if (li < L && (li * d.nr) / L == r) {
        flo[q] = static_cast<double>(li) - 1.0;
        fhi[q] = static_cast<double>(li);
        seg[q] = SB[i] - d.SB0;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kPlanUnroll; ++q) {
    const PlanCtx d = ctx(q);
    if (flo[q] < fhi[q]) claim_units(d, flo[q], fhi[q], seg[q], cl[q] - d.C0, lane_seg, lane_cum);
    if (live[q]) A[idx[q]] = wu[q] / d.S;   // a_u of Alg. 1, once per source
  }
}

template <bool kOne>
__device__ __forceinline__ void lane_plan_sources(const WsHeader* hdr) {
  const GraphDesc* desc = hdr->desc;
  const uint64_t total_r = hdr->total_r;
  const PlanArrays pa{total_r, to_global(hdr->C), to_global(hdr->SB), to_global_mut(hdr->A),
                      to_global_mut(hdr->lane_seg), to_global_mut(hdr->lane_cum)};
  uint64_t idx[kPlanUnroll];
  if constexpr (kOne) {
    const PlanCtx c0 = plan_ctx(desc[0]);
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i0 < total_r;
         i0 += kPlanUnroll * stride) {
#pragma unroll
      for (int q = 0; q < kPlanUnroll; ++q) idx[q] = i0 + q * stride;
      plan_sources_step(pa, idx, [&](int) { return c0; });
    }
  } else {
    const uint32_t G = hdr->G;
    auto roff = [&](uint32_t x) { return desc[x].r_off; };
    const uint64_t ntiles = (total_r + kPlanTile - 1) / kPlanTile;
    const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;   // consecutive tiles per block
    const uint64_t t_end = ((blockIdx.x + 1) * per < ntiles) ? (blockIdx.x + 1) * per : ntiles;
    uint32_t gc = 0;   // graph of the last tile's end (the walk only moves forward)
    bool first = true;
    for (uint64_t tile = blockIdx.x * per; tile < t_end; ++tile) {
      const uint64_t tb = tile * kPlanTile;
      const uint64_t te = ((tb + kPlanTile < total_r) ? tb + kPlanTile : total_r) - 1;
      const uint32_t g0 = uni32(first ? find_graph(G, tb, roff) : advance_graph(G, gc, tb, roff));
      const uint32_t g1 = uni32(advance_graph(G, g0, te, roff));
      gc = g1;
      first = false;
#pragma unroll
      for (int q = 0; q < kPlanUnroll; ++q) idx[q] = tb + static_cast<uint64_t>(q) * blockDim.x + threadIdx.x;
      if (g0 == g1) {
        const PlanCtx dg = plan_ctx(desc[g0]);
        plan_sources_step(pa, idx, [&](int) { return dg; });
      } else {
        uint32_t gq[kPlanUnroll];
#pragma unroll
        for (int q = 0; q < kPlanUnroll; ++q) gq[q] = find_graph_in(g0, g1, idx[q] < te ? idx[q] : te, roff);
        plan_sources_step(pa, idx, [&](int q) { return plan_ctx(desc[gq[q]]); });
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_lane_plan(const WsHeader* hdr) {
  if (hdr->status) return;
  if (hdr->G == 1) lane_plan_sources<true>(hdr);
  else lane_plan_sources<false>(hdr);
}

// group -> graph map, the padding lanes (empty: start = (u_end, 0)) and the
// starts of round-robin units; one thread per lane (lane_off is a multiple
// of the group size, so a group's first lane is a graph-relative multiple)
__global__ void __launch_bounds__(256) k_lane_groups(const WsHeader* hdr) {
  if (hdr->status) return;
  const GraphDesc* desc = hdr->desc;
  const uint32_t G = hdr->G;
  const uint64_t nl = hdr->total_nl;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t l = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; l < nl; l += stride) {
    const uint32_t g = (G == 1) ? 0u : find_graph(G, l, [&](uint32_t x) { return desc[x].lane_off; });
    const GraphDesc& d = desc[g];
    const uint64_t li = l - d.lane_off;
    if (l % kLaneGroup == 0) hdr->group_graph[l / kLaneGroup] = g;
    if (li < d.L && d.policy == 2) {
      hdr->lane_seg[l] = static_cast<uint32_t>(li);   // round robin: first segment i
    } else if (li >= d.L) {
      hdr->lane_seg[l] = static_cast<uint32_t>(d.SB1 - d.SB0);
      if (hdr->lane_cum) hdr->lane_cum[l] = d.C1 - d.C0;
    }
  }
}

// --------------------------------------------------------------------------
// the per-lane Create-Edges loop
// --------------------------------------------------------------------------
struct LaneCtx {
  gptr<double> w;
  gptr<double> A;                 // a_u = w_u / S of the range's sources (index u - u_begin)
  uint32_t n;
  uint32_t u_begin, u_heavy_end;  // sources [u_begin, u_heavy_end) are heavy
  uint32_t NH;                    // heavy segments; segment index NH + i is light source u_heavy_end + i
  uint32_t stride;                // segment step inside a unit: 1, or L for round-robin units
  gptr<u32x4> hseg;               // graph's heavy segments (u, k, j, send)
};

// State of one lane inside its current work unit: the unit is the run of
// segments [sg, sg_end) of the lane plan (graph-relative segment indices),
// taken with step cx.stride (1; L for round-robin units);
// (u, k) is the open segment, j its next candidate, send its end, t the index
// of its next draw.
struct LaneRun {
  uint32_t sg, sg_end;
  uint32_t u, k, j, send, t;
  double a, p;
  bool inseg;
  __device__ bool more() const { return sg < sg_end; }
};

// Opens segment sg (Alg. 1 set-up of source u, segment k).
__device__ __forceinline__ void open_segment(LaneRun& s, const LaneCtx& cx) {
  const uint32_t sg = s.sg;
  if (sg < cx.NH) {
    const u32x4 d = cx.hseg[sg];
    s.u = d.x;
    s.k = d.y;
    s.j = d.z;
    s.send = d.w;
  } else {
    s.u = cx.u_heavy_end + (sg - cx.NH);
    s.k = 0;
    s.j = s.u + 1;
    s.send = cx.n;
  }
  s.a = cx.A[s.u - cx.u_begin];
  const bool any = s.j < s.send;
  const double wj = cx.w[any ? s.j : 0u];
  s.p = any ? cap1(s.a * wj) : 0.0;
  s.inseg = (s.p > 0.0);
  s.t = 0;
  s.sg += cx.stride;
}

// ln(1 - p) of ln_one_minus without the branch: both forms share one division
// and one series evaluation, the operands are selected.  Bit-identical to
// ln_one_minus for p in (0, 1); for p = 1 it returns a finite value.
__device__ __forceinline__ double ln_one_minus_sel(double p, const Series& sr) {
  const bool small = p < 0.25;
  double m;
  int e;
  log_reduce(1.0 - p, m, e);
  const double f = m - 1.0;
  const double num = small ? -p : f;
  const double den = small ? 2.0 - p : 2.0 + f;
  const double l = two_s_series(num / den, sr);
  return small ? l : (static_cast<double>(e) * 0x1.62e42fefa39efp-1) + l;
}

// One candidate step of Alg. 1 on the open segment: geometric skip with
// r_skip, then accept with probability q/p using r_acc (draw t of segment
// (u, k)); a capped segment (p = 1) takes the next candidate without a skip.
// Straight-line apart from the emission.  Kept edges go to emit(u, v); emit
// returns false to end the unit.
template <class Emit>
__device__ __forceinline__ void candidate_step(LaneRun& s, const LaneCtx& cx, const RoundKeys& rk,
                                               const Series& sr, Emit& emit, uint32_t& visits) {
  const bool capped = (s.p == 1.0);
  const Block4 x = philox10(s.t, s.k, s.u, 0u, rk);
  ++s.t;
  const double lr = ln_unit(unit53(x.x1, x.x0), sr);
  const double ratio = lr / ln_one_minus_sel(s.p, sr);
  const bool leaves = !capped && !(ratio < static_cast<double>(s.send - s.j));   // the skip leaves the segment
  const uint32_t v = s.j + ((capped || leaves) ? 0u : static_cast<uint32_t>(ratio));
  const double q = cap1(s.a * cx.w[v]);    // v < send <= n, or v = j < send
  const double r_acc = unit53(x.x3, x.x2);
  const bool keep = !leaves && ((capped && q == 1.0) || (r_acc * s.p < q));
  if (keep && !emit(s.u, v)) {
    s.inseg = false;
    s.sg = s.sg_end;
    return;
  }
  if (!leaves) {
    ++visits;
    s.p = q;
    s.j = v + 1;
  }
  s.inseg = !(leaves || s.j >= s.send || !(s.p > 0.0));
}

struct CountEmit {
  uint32_t c;
  __device__ bool operator()(uint32_t, uint32_t) {
    ++c;
    return true;
  }
};

// Write-pass output through LDS: every lane stages its edges in 64-byte
// chunks of the output (8 pairs, aligned to the window start lo) and stores
// a chunk once it is complete, as four 16-byte stores, so that HBM receives
// whole 64-byte sectors instead of the 8-byte pieces of 64 interleaved lane
// streams.  Chunks a lane shares with its neighbours (the first and last of
// a unit) are stored pair by pair.  LDS layout [slot][thread] keeps the
// per-emission stores of a wavefront free of bank conflicts.
constexpr int kStageSlots = 8;
constexpr int kLaneThreads = 256;   // block size of the lane kernels

struct WriteEmit {
  uint2* stage;      // LDS, kStageSlots x kLaneThreads entries
  gout<uint2> out;   // output window: out[i] is position lo + i (uniform)
  uint64_t lo;       // window start (uniform)
  uint64_t pos, hi;  // next position, end of the unit's range
  uint32_t run;      // entries staged by this unit (saturates at kStageSlots)
  __device__ uint2& slot(uint64_t q) { return stage[(q & (kStageSlots - 1)) * kLaneThreads + threadIdx.x]; }
  // stores the lane's entries of the chunk that ends at qend (exclusive):
  // the whole chunk if the lane staged all of it, else its last `own` entries
  __device__ void flush(uint64_t qend, uint32_t own) {
    const uint64_t q0 = (qend - 1) & ~static_cast<uint64_t>(kStageSlots - 1);
    if (own == kStageSlots) {
      gout<u32x4> dst = reinterpret_cast<gout<u32x4>>(out + q0);
#pragma unroll
      for (int i = 0; i < kStageSlots / 2; ++i) {
        const uint2 x0 = stage[(2 * i) * kLaneThreads + threadIdx.x];
        const uint2 x1 = stage[(2 * i + 1) * kLaneThreads + threadIdx.x];
        dst[i] = u32x4{x0.x, x0.y, x1.x, x1.y};
      }
    } else {
      gout<uint64_t> o = reinterpret_cast<gout<uint64_t>>(out);
      for (uint64_t q = qend - own; q < qend; ++q) {
        const uint2 x = slot(q);
        o[q] = (static_cast<uint64_t>(x.y) << 32) | x.x;
      }
    }
  }
  __device__ bool operator()(uint32_t u, uint32_t v) {
    if (pos >= hi) return false;
    if (pos >= lo) {
      const uint64_t q = pos - lo;
      slot(q) = make_uint2(u, v);
      if (run < kStageSlots) ++run;
      if ((q & (kStageSlots - 1)) == kStageSlots - 1) {
        // a chunk the lane started mid-way holds only its last `run` entries
        flush(q + 1, run);
        run = kStageSlots;
      }
    }
    ++pos;
    return true;
  }
  // the unit's last, incomplete chunk
  __device__ void finish() {
    const uint64_t end = (pos < hi) ? pos : hi;
    if (end > lo) {
      const uint64_t q = end - lo;
      const uint32_t part = static_cast<uint32_t>(q & (kStageSlots - 1));
      if (part) flush(q, (run < part) ? run : part);
    }
  }
};

// One-pass output: the lane counts every kept edge and writes the unit's
// edges into its slot as 32-bit words: v for each edge, preceded by the pair
// (kSourceMark, u) whenever the source changes (a vertex id is at most
// 2^32 - 2, so kSourceMark is never a v).  Half the bytes of (u, v) pairs; the
// compaction expands them.  Words are staged in LDS like WriteEmit and stored
// as whole 64-byte chunks (16 words).  Words beyond the slot are counted, not
// written; the unit then overflowed and the write kernel replays it.
constexpr uint32_t kSourceMark = 0xFFFFFFFFu;
constexpr int kWordSlots = 16;   // words per 64-byte chunk

struct WordEmit {
  uint32_t* stage;      // LDS, kWordSlots x kLaneThreads words (the pair stage's bytes)
  gout<uint32_t> out;   // all slots, word-indexed
  uint64_t start, pos, hi;  // the unit's slot [start, hi), next word position
  uint32_t run;         // words staged by this unit (saturates at kWordSlots)
  uint32_t cur;         // source of the last edge (kSourceMark: none yet)
  uint32_t c;           // edges
  uint64_t words;       // words the unit needs (its slot holds min(words, hi - start))
  __device__ bool over() const { return words > hi - start; }
  __device__ uint32_t& slot(uint64_t q) { return stage[(q & (kWordSlots - 1)) * kLaneThreads + threadIdx.x]; }
  __device__ void flush(uint64_t qend, uint32_t own) {
    const uint64_t q0 = (qend - 1) & ~static_cast<uint64_t>(kWordSlots - 1);
    if (own == kWordSlots) {
      gout<u32x4> dst = reinterpret_cast<gout<u32x4>>(out + q0);
#pragma unroll
      for (int i = 0; i < kWordSlots / 4; ++i)
        dst[i] = u32x4{stage[(4 * i) * kLaneThreads + threadIdx.x], stage[(4 * i + 1) * kLaneThreads + threadIdx.x],
                       stage[(4 * i + 2) * kLaneThreads + threadIdx.x], stage[(4 * i + 3) * kLaneThreads + threadIdx.x]};
    } else {
      for (uint64_t q = qend - own; q < qend; ++q) out[q] = slot(q);
    }
  }
  __device__ void push(uint32_t x) {
    ++words;
    if (pos >= hi) return;
    slot(pos) = x;
    if (run < kWordSlots) ++run;
    if ((pos & (kWordSlots - 1)) == kWordSlots - 1) {
      flush(pos + 1, run);
      run = kWordSlots;
    }
    ++pos;
  }
  __device__ bool operator()(uint32_t u, uint32_t v) {
    ++c;
    if (u != cur) {
      push(kSourceMark);
      push(u);
      cur = u;
    }
    push(v);
    return true;
  }
  // the unit's last, incomplete chunk
  __device__ void finish() {
    const uint32_t part = static_cast<uint32_t>(pos & (kWordSlots - 1));
    if (part) flush(pos, (run < part) ? run : part);
  }
};

// CSR write pass: every kept edge (u, v) writes v at its batch position of
// the column array (staged in 64-byte chunks of 16 words like WordEmit, the
// chunks aligned to position 0) and counts one edge for row u; the count of
// a run of equal u is kept in a register and added to rows[u] once.
struct CsrEmit {
  uint32_t* stage;                // LDS, kWordSlots x kLaneThreads words
  gout<uint32_t> col;             // column array: col[i] is batch position i
  unsigned long long* rows;       // per-source edge counts of the bound graph
  uint64_t pos, hi;               // next position, end of the unit's range
  uint32_t run;                   // words staged by this unit (saturates at kWordSlots)
  uint32_t cur, cnt;              // source of the current run and its edges so far
  __device__ uint32_t& slot(uint64_t q) { return stage[(q & (kWordSlots - 1)) * kLaneThreads + threadIdx.x]; }
  __device__ void store(uint64_t qend, uint32_t own) {
    const uint64_t q0 = (qend - 1) & ~static_cast<uint64_t>(kWordSlots - 1);
    if (own == kWordSlots) {
      gout<u32x4> dst = reinterpret_cast<gout<u32x4>>(col + q0);
#pragma unroll
      for (int i = 0; i < kWordSlots / 4; ++i)
        dst[i] = u32x4{stage[(4 * i) * kLaneThreads + threadIdx.x], stage[(4 * i + 1) * kLaneThreads + threadIdx.x],
                       stage[(4 * i + 2) * kLaneThreads + threadIdx.x], stage[(4 * i + 3) * kLaneThreads + threadIdx.x]};
    } else {
      for (uint64_t q = qend - own; q < qend; ++q) col[q] = slot(q);
    }
  }
  __device__ void count_flush() {
    if (cnt) atomicAdd(&rows[cur], static_cast<unsigned long long>(cnt));
    cnt = 0;
  }
  __device__ bool operator()(uint32_t u, uint32_t v) {
    if (pos >= hi) return false;
    if (u != cur) {
      count_flush();
      cur = u;
    }
    ++cnt;
    slot(pos) = v;
    if (run < kWordSlots) ++run;
    if ((pos & (kWordSlots - 1)) == kWordSlots - 1) {
      store(pos + 1, run);
      run = kWordSlots;
    }
    ++pos;
    return true;
  }
  // the unit's last, incomplete chunk and its last run
  __device__ void finish() {
    const uint32_t part = static_cast<uint32_t>(pos & (kWordSlots - 1));
    if (part) store(pos, (run < part) ? run : part);
    count_flush();
  }
};

// Degree consumer: every kept edge (u, v) adds 1 to the degrees of u and v,
// and no edge is stored.  The source's count is kept in a register and added
// once per run of equal u; integer additions commute, so the result does not
// depend on the schedule.
struct DegEmit {
  uint32_t* deg;      // degrees of the bound graph's nodes
  uint32_t cur, cnt;  // source whose edges are being counted, and how many so far
  __device__ void flush() {
    if (cnt) atomicAdd(&deg[cur], cnt);
    cnt = 0;
  }
  __device__ bool operator()(uint32_t u, uint32_t v) {
    atomicAdd(&deg[v], 1u);
    if (u != cur) {
      flush();
      cur = u;
    }
    ++cnt;
    return true;
  }
};

template <int kMode>
struct EmitOf;
template <>
struct EmitOf<2> {
  using type = WordEmit;
};
template <>
struct EmitOf<3> {
  using type = DegEmit;
};
template <>
struct EmitOf<0> {
  using type = CountEmit;
};
template <>
struct EmitOf<1> {
  using type = WriteEmit;
};
template <>
struct EmitOf<4> {
  using type = CsrEmit;
};

// The lane kernel.  kMode 0: count pass.  kMode 1: write pass (replay into
// the output window; in one-pass plans only the units that overflowed their
// slot).  kMode 2: one pass, count and write slot words.  kMode 3: degrees
// only (adds into deg at each graph's node offset q_off; no edge output).
//
// Scheduling: the work units of the lane plan (Eq. 5 applied to lanes) are
// handed out dynamically.  A wavefront takes chunks of 64 consecutive units
// (all of one graph) from a global ticket counter, and each of its lanes takes
// the next unit of the chunk as soon as it has finished its previous one, so a
// lane never waits for the slowest lane of a fixed group.  With a processing
// order (perm, single-graph plans) the t-th unit handed out is perm[t].  The lanes of a
// wavefront work on one graph at a time (its parameters live in scalar
// registers); a chunk of another graph is handed out once every lane is idle.
//
// kStats (count pass only): each unit's record goes to stats[unit] (its lane,
// the wave clock when it was taken and finished, its plan cost, candidates
// and edges), for the comparison of unit policies; the header's candidate
// total is left alone.
template <int kMode, bool kStats = false>
__global__ void __launch_bounds__(kLaneThreads) k_lanes(WsHeader* hdr, uint2* out, uint64_t e_lo, uint64_t e_hi,
                                                       uint32_t* deg, unsigned long long* rows, UnitStat* stats) {
  static_assert(!kStats || kMode == 0, "statistics are recorded by the count pass");
  using Emit = typename EmitOf<kMode>::type;
  constexpr bool kWrite = (kMode == 1 || kMode == 2 || kMode == 4);
  constexpr bool kReplay = (kMode == 1 || kMode == 4);
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  __shared__ uint2 stage[kWrite ? kStageSlots * kLaneThreads : 1];
  if (hdr->status || hdr->magic != kWsMagic) return;
  if (kReplay && hdr->planned != 1) return;   // the write passes need the counts
  if (kMode == 3 && !hdr->planned) return;
  const bool only_overflow = kReplay && (uni32(hdr->mode) == 1);
  if (only_overflow && uni32(hdr->overflow) == 0) return;
  const GraphDesc* desc = hdr->desc;
  const uint32_t ngroups = uni32(static_cast<uint32_t>(uni64(hdr->total_nl) / kLaneGroup));
  const Series sr = load_series();
  const int lane = threadIdx.x & 63;
  // workspace arrays, read once into scalar registers
  const gptr<uint32_t> lane_seg = to_global(uniptr(hdr->lane_seg));
  const gout<uint32_t> lane_cnt = to_global_mut(uniptr_mut(hdr->lane_cnt));
  const gptr<uint64_t> slot_off = to_global(uniptr(hdr->slot_off));
  const gptr<uint64_t> lane_pos = to_global(uniptr(hdr->lane_pos));
  const gptr<uint32_t> group_graph = to_global(uniptr(hdr->group_graph));
  const gout<uint32_t> slots = to_global_mut(uniptr_mut(hdr->slots));
  const gout<uint32_t> lane_words = to_global_mut(uniptr_mut(hdr->lane_words));
  const gout<uint2> outw = to_global_mut(uniptr_mut(out));
  const uint32_t* perm_p = uniptr(hdr->perm);   // processing order (null: index order)
  const gptr<uint32_t> perm = to_global(perm_p);
  unsigned int* overflow = &hdr->overflow;

  // wave-uniform: the graph bound to the wavefront, its parameters, the chunk
  uint32_t g_cur = kNone;
  LaneCtx cx{};
  RoundKeys rk{};
  uint64_t unit_end = 0;     // one past the graph's last (padded) unit
  uint32_t nseg = 0;         // segments of the graph
  bool rr = false;           // round-robin units
  uint32_t* degp = nullptr;  // degree mode: the graph's degree array
  unsigned long long* rowp = nullptr;   // CSR mode: the graph's row counts
  uint32_t cnext = 0, cend = 0, cgraph = kNone;
  bool queue_done = false;
  gptr<uint64_t> costp{}, segp{};   // statistics: the graph's cost and segment prefixes

  // per lane
  uint32_t unit = kNone;
  bool touched = false;      // write pass: the unit writes into the window
  uint32_t visits = 0;
  uint64_t words_acc = 0;    // one pass: slot words of the lane's units
  LaneRun s{};
  s.sg = 0;
  s.sg_end = 0;
  s.inseg = false;
  Emit em{};
  uint64_t st_t0 = 0;        // statistics of the lane's current unit
  uint32_t st_v0 = 0;
  double st_cost = 0.0;

  while (true) {
    // (1) a lane that has finished its unit closes it
    const bool idle = !(s.inseg || s.more());
    if (idle && unit != kNone) {
      if constexpr (kMode == 0) {
        lane_cnt[unit] = em.c;
        if constexpr (kStats) {
          const uint32_t wave = blockIdx.x * (kLaneThreads / 64) + threadIdx.x / 64;
          stats[unit] = UnitStat{st_t0, __builtin_amdgcn_s_memrealtime(),
                                 static_cast<uint32_t>(st_cost + 0.5), visits - st_v0, em.c,
                                 wave * 64u + static_cast<uint32_t>(lane)};
        }
      } else if constexpr (kMode == 2) {
        em.finish();
        lane_cnt[unit] = em.c;
        lane_words[unit] = static_cast<uint32_t>(em.words);
        words_acc += em.words;
        if (em.over()) atomicAdd(overflow, 1u);
      } else if constexpr (kMode == 3) {
        em.flush();
      } else {
        if (touched) em.finish();
      }
      unit = kNone;
    }
    // (2) idle lanes take the next units of the wavefront's chunk
    const uint64_t idle_mask = __ballot(idle);
    if (idle_mask != 0 && !(queue_done && cnext >= cend)) {
      if (cnext >= cend) {
        uint32_t grp = 0;
        if (lane == 0) grp = atomicAdd(&hdr->queue, 1u);
        grp = uni32(static_cast<uint32_t>(__shfl(static_cast<int>(grp), 0, 64)));
        if (grp >= ngroups) {
          queue_done = true;
        } else {
          cnext = grp * kLaneGroup;
          cend = cnext + kLaneGroup;
          cgraph = uni32(group_graph[grp]);
        }
      }
      if (cnext < cend && (cgraph == g_cur || idle_mask == ~0ull)) {
        if (cgraph != g_cur) {
          g_cur = cgraph;
          const GraphDesc& d = desc[g_cur];
          cx.w = to_global(uniptr(d.w));
          cx.n = uni32(static_cast<uint32_t>(d.n));
          cx.u_begin = uni32(static_cast<uint32_t>(d.u_begin));
          cx.u_heavy_end = cx.u_begin + uni32(static_cast<uint32_t>(d.H));
          cx.NH = uni32(static_cast<uint32_t>(d.NH));
          rr = (uni32(d.policy) == 2);
          cx.stride = rr ? uni32(static_cast<uint32_t>(d.L)) : 1u;
          cx.A = to_global(uniptr(hdr->A) + uni64(d.r_off));
          cx.hseg = to_global(reinterpret_cast<const u32x4*>(uniptr(hdr->hseg) + uni64(d.hs_off)));
          rk = philox_round_keys(uni64(d.seed));
          unit_end = uni64(d.lane_off) + uni64(d.NL);
          nseg = uni32(static_cast<uint32_t>(d.SB1 - d.SB0));
          if constexpr (kMode == 3) degp = uniptr_mut(deg) + uni64(d.q_off);
          if constexpr (kMode == 4) rowp = uniptr_mut(rows) + uni64(d.q_off);
          if constexpr (kStats) {
            costp = to_global(uniptr(hdr->C) + uni64(d.r_off));
            segp = to_global(uniptr(hdr->SB) + uni64(d.r_off));
          }
        }
        // rank of this lane among the idle lanes
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(idle_mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(idle_mask), 0u));
        const uint32_t mine = cnext + rank;
        if (idle && mine < cend) {
          unit = perm_p ? perm[mine] : mine;
          s.sg = lane_seg[unit];
          s.sg_end = (rr || unit + 1 >= unit_end) ? nseg : lane_seg[unit + 1];
          if (s.sg > s.sg_end || s.sg_end > nseg) {   // never for a valid plan: flagged, nothing read
            atomicOr(&hdr->status, static_cast<uint32_t>(kStPlan));
            s.sg = s.sg_end = 0;
          }
          s.inseg = false;
          if constexpr (kStats) {
            st_t0 = __builtin_amdgcn_s_memrealtime();
            st_v0 = visits;
            st_cost = 0.0;
          }
          if constexpr (kMode == 0) {
            em = Emit{0u};
          } else if constexpr (kMode == 2) {
            const uint64_t s0 = slot_off[unit];
            const uint64_t s1 = slot_off[unit + 1];
            em = WordEmit{reinterpret_cast<uint32_t*>(stage), slots, s0, s0, s1, 0u, kSourceMark, 0u, 0ull};
          } else if constexpr (kMode == 3) {
            em = DegEmit{degp, kNone, 0u};
          } else {
            const uint64_t pos0 = lane_pos[unit];
            const uint64_t cnt = lane_cnt[unit];
            touched = (pos0 < e_hi) && (pos0 + cnt > e_lo);
            // one-pass plans: only the units whose words did not fit their slot
            if (only_overflow) touched = touched && (lane_words[unit] > slot_off[unit + 1] - slot_off[unit]);
            if constexpr (kMode == 4)
              em = CsrEmit{reinterpret_cast<uint32_t*>(stage), to_global_mut(reinterpret_cast<uint32_t*>(out)), rowp,
                           pos0, e_hi, 0u, kNone, 0u};
            else
              em = WriteEmit{stage, outw, e_lo, pos0, e_hi, 0u};
            if (!touched) s.sg_end = s.sg;
          }
        }
        const uint32_t handed = static_cast<uint32_t>(__popcll(idle_mask));
        cnext = (cend - cnext > handed) ? cnext + handed : cend;
      }
    }
    // (3) open the next segment of the unit
    if (!s.inseg && s.more()) {
      open_segment(s, cx);
      if constexpr (kStats) {   // the segment's share c_u / K_u of its source's plan cost
        const uint32_t r = s.u - cx.u_begin;
        st_cost += static_cast<double>(costp[r + 1] - costp[r]) / static_cast<double>(segp[r + 1] - segp[r]);
      }
    }
    if (!__any(s.inseg || s.more() || unit != kNone) && queue_done && cnext >= cend) break;
    // (4) one candidate step
    if (s.inseg) candidate_step(s, cx, rk, sr, em, visits);
  }
  if ((kMode == 0 && !kStats) || kMode == 2) {
    // candidates visited by the wavefront (statistics of the cost model)
    uint64_t visited = visits;
    for (int dd = 32; dd >= 1; dd >>= 1) visited += shfl_idx64(visited, lane ^ dd);
    if (lane == 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&hdr->total_cand), static_cast<unsigned long long>(visited));
  }
  if (kMode == 2) {
    for (int dd = 32; dd >= 1; dd >>= 1) words_acc += shfl_idx64(words_acc, lane ^ dd);
    if (lane == 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(&hdr->total_words), static_cast<unsigned long long>(words_acc));
  }
}
// --------------------------------------------------------------------------
// one-pass slots: capacity of a lane = its plan cost mu (in expected
// candidates, which bounds its expected edges) + 8 sqrt(mu) + 24 edge words,
// plus two words per segment for the source marks, rounded up to whole
// 64-byte chunks; a lane above it (probability < 1e-14 by the Chernoff bound
// used in Sec. 4, Theorem 2) is replayed by the write kernel.
// --------------------------------------------------------------------------
struct SlotIn {
  const WsHeader* hdr;
  struct Ctx {
    uint64_t nl;        // lanes of all graphs (padded)
    uint64_t lane_off, L, Z, nseg;
  };
  __device__ uint32_t graph_of(uint64_t l) const {
    return (l < hdr->total_nl) ? hdr->group_graph[l / kLaneGroup] : 0u;
  }
  __device__ Ctx context(uint32_t g) const {
    const GraphDesc& d = hdr->desc[g];
    return Ctx{hdr->total_nl, d.lane_off, d.L, d.C1 - d.C0, d.SB1 - d.SB0};
  }
  __device__ uint64_t load(uint64_t l, const Ctx& c) const {
    if (l >= c.nl) return 0;
    const uint64_t i = l - c.lane_off;
    if (i >= c.L) return 0;
    const uint64_t c1 = (i + 1 < c.L) ? hdr->lane_cum[l + 1] : c.Z;
    const uint64_t c0 = hdr->lane_cum[l];
    const double mu = static_cast<double>(c1 > c0 ? c1 - c0 : 0) / static_cast<double>(kCostUnit);
    const double cap = (hdr->slot_margin == 1) ? mu : (mu + 8.0 * sqrt(mu) + 24.0);
    // words: one per edge, plus a (mark, u) pair per source, at most one per segment
    const uint64_t g0 = hdr->lane_seg[l];
    const uint64_t g1 = (i + 1 < c.L) ? hdr->lane_seg[l + 1] : c.nseg;
    const uint64_t cc = static_cast<uint64_t>(ceil(cap)) + 2 * (g1 > g0 ? g1 - g0 : 0);
    return (cc + kWordSlots - 1) / kWordSlots * kWordSlots;
  }
};

// the slot offsets; the total (offset at unit total_nl) is checked against
// the slots' capacity (the offsets are non-decreasing, so only offsets above
// the capacity look up total_nl)
struct SlotOut : OneGraph {
  uint64_t* off;
  uint64_t slot_cap;
  WsHeader* hdr;
  __device__ void store(uint64_t i, Ctx, uint64_t, uint64_t ex) const {
    off[i] = ex;
    if (ex > slot_cap && i == hdr->total_nl) atomicOr(&hdr->status, kStCapacity);
  }
};

// Expands every unit's slot words into (u, v) pairs at the unit's place in
// the output window [lo, hi).  One wavefront per group of 64 units, which it
// reads as one stream: the words of the group's units one after the other
// (units whose slot overflowed, or that miss the window, left out; the
// replay writes the overflowed ones), 64 consecutive words per instruction
// and kCompactSteps instructions in flight per lane, whatever the unit sizes.
// Each unit's words begin with a mark and its source id, so the decoding runs
// across unit boundaries unchanged: a lane learns from ballots whether its
// word is a mark, a source id (the word after a mark) or an edge, takes u from
// the nearest source id at or below it (or the one carried from the previous
// instruction), and numbers its edge by the edges before it in the stream.
// The unit of a word comes from the group's word prefix in LDS (a lane's
// unit index only moves forward); edge k of the stream lies in unit j and
// goes to position lane_pos[j] + (k - edges of the stream before unit j).
constexpr int kCompactSteps = 8;

//
// With kCsr the output is the column array of the compressed sparse rows
// form: v alone at the edge's position (4 bytes), and each run of edges of one
// source inside an instruction adds its length to rows[q_g + u] (the first
// lane of the run does, a run being a stretch of consecutive edge lanes).
template <bool kCsr>
__global__ void __launch_bounds__(256) k_compact(WsHeader* hdr, uint2* out, uint64_t lo, uint64_t hi,
                                                 unsigned long long* rows) {
  __shared__ uint64_t sh_wpre[4][kLaneGroup + 1];   // stream position of each unit's first word, then the total
  __shared__ uint64_t sh_src[4][kLaneGroup];        // slot index of stream word t of unit j: sh_src[j] + t
  __shared__ uint64_t sh_dst[4][kLaneGroup];        // output position of stream edge k of unit j: sh_dst[j] + k
  // the unit queue of the replay kernel that follows (no lane kernel runs
  // during this one), reset for every plan kind
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->queue = 0;
  if (hdr->status || hdr->mode != 1 || !hdr->planned) return;
  const uint64_t ngroups = uni64(hdr->total_nl) / kLaneGroup;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;       // lanes under this one
  const uint64_t upto = below | (1ull << lane);    // lanes up to this one
  const uint64_t nwaves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / 64);
  gptr<uint32_t> slots = to_global(uniptr(static_cast<const uint32_t*>(hdr->slots)));
  const gout<uint64_t> out64 = to_global_mut(uniptr_mut(reinterpret_cast<uint64_t*>(out)));
  const gout<uint32_t> out32 = to_global_mut(uniptr_mut(reinterpret_cast<uint32_t*>(out)));
  for (uint64_t grp = uni64(static_cast<uint64_t>(blockIdx.x) * (blockDim.x / 64) + wv); grp < ngroups;
       grp += nwaves) {
    unsigned long long* rowp = nullptr;   // CSR: the group's graph's row counts
    if constexpr (kCsr) rowp = uniptr_mut(rows) + uni64(hdr->desc[uni32(hdr->group_graph[grp])].q_off);
    const uint64_t l = grp * kLaneGroup + lane;
    const uint64_t pos = hdr->lane_pos[l];
    const uint64_t cnt = hdr->lane_cnt[l];
    const uint64_t words = hdr->lane_words[l];
    const uint64_t s0 = hdr->slot_off[l];
    const uint64_t cap = hdr->slot_off[l + 1] - s0;
    const bool in = cnt > 0 && words <= cap && pos < hi && pos + cnt > lo;
    const uint64_t wn = in ? words : 0, en = in ? cnt : 0;
    const uint64_t wincl = wave_inclusive<uint64_t>(wn);
    const uint64_t eincl = wave_inclusive<uint64_t>(en);
    const uint64_t total = lane63_64(wincl);
    sh_wpre[wv][lane] = wincl - wn;
    if (lane == 63) sh_wpre[wv][kLaneGroup] = total;
    sh_src[wv][lane] = s0 - (wincl - wn);
    sh_dst[wv][lane] = pos - (eincl - en);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t j = 0;            // this lane's unit (moves forward only), and its fields
    uint64_t j_end = sh_wpre[wv][1], j_src = sh_src[wv][0], j_dst = sh_dst[wv][0];
    uint32_t carry_u = 0;      // source id carried from the previous instruction
    bool carry_mark = false;   // the previous instruction ended with a mark
    uint64_t ebase = 0;        // stream edges before the current instruction
    for (uint64_t t0 = 0; t0 < total; t0 += 64 * kCompactSteps) {
      uint32_t x[kCompactSteps];
      uint64_t dst[kCompactSteps];
#pragma unroll
      for (int r = 0; r < kCompactSteps; ++r) {
        const uint64_t t = t0 + r * 64 + lane;
        x[r] = 0u;
        dst[r] = 0;
        if (t < total) {
          if (t >= j_end) {
            do {
              ++j;   // t < total, so j stays below 64
            } while (t >= sh_wpre[wv][j + 1]);
            j_end = sh_wpre[wv][j + 1];
            j_src = sh_src[wv][j];
            j_dst = sh_dst[wv][j];
          }
          dst[r] = j_dst;
          x[r] = slots[j_src + t];
        }
      }
#pragma unroll
      for (int r = 0; r < kCompactSteps; ++r) {
        const bool valid = t0 + r * 64 + lane < total;
        const bool mark = valid && x[r] == kSourceMark;
        const uint64_t mmask = __ballot(mark);
        const bool after_mark = (lane == 0) ? carry_mark : ((mmask >> (lane - 1)) & 1ull) != 0;
        const bool is_u = valid && after_mark;
        const bool edge = valid && !mark && !is_u;
        const uint64_t umask = __ballot(is_u);
        const uint64_t emask = __ballot(edge);
        const uint64_t mine = umask & upto;
        const uint32_t u_here = static_cast<uint32_t>(
            __shfl(static_cast<int>(x[r]), mine ? 63 - __clzll(static_cast<long long>(mine)) : 0, 64));
        const uint32_t u = mine ? u_here : carry_u;
        if (edge) {
          const uint64_t e = dst[r] + ebase + static_cast<uint64_t>(__popcll(emask & below));
          if constexpr (kCsr) {
            if (e >= lo && e < hi) out32[e - lo] = x[r];
            if (lane == 0 || ((emask >> (lane - 1)) & 1ull) == 0) {   // first lane of a run
              const uint64_t rest = emask >> lane;
              const uint32_t len = (rest == ~0ull) ? 64u : static_cast<uint32_t>(__builtin_ctzll(~rest));
              atomicAdd(&rowp[u], static_cast<unsigned long long>(len));
            }
          } else {
            if (e >= lo && e < hi) out64[e - lo] = (static_cast<uint64_t>(x[r]) << 32) | u;
          }
        }
        if (umask) {
          const int top = 63 - __clzll(static_cast<long long>(umask));
          carry_u = static_cast<uint32_t>(__shfl(static_cast<int>(x[r]), top, 64));
        }
        carry_mark = (mmask >> 63) != 0;
        ebase += static_cast<uint64_t>(__popcll(emask));
      }
    }
    __builtin_amdgcn_wave_barrier();   // the next group rewrites this wavefront's LDS
  }
}

// --------------------------------------------------------------------------
// offsets of the lanes' output
// --------------------------------------------------------------------------
struct CntIn : OneGraph {
  const uint32_t* cnt;
  uint64_t n;
  __device__ uint64_t load(uint64_t i, Ctx) const { return (i < n) ? cnt[i] : 0; }
};

struct OffOut : OneGraph {
  uint64_t* off;
  __device__ void store(uint64_t i, Ctx, uint64_t, uint64_t ex) const { off[i] = ex; }
};

// CSR rows: per-source edge counts in, exclusive prefix (row offsets) out,
// in place (every element is read before the same thread writes it)
struct RowIn : OneGraph {
  const unsigned long long* c;
  uint64_t n;
  __device__ uint64_t load(uint64_t i, Ctx) const { return (i < n) ? c[i] : 0; }
};

struct RowOut : OneGraph {
  unsigned long long* r;
  __device__ void store(uint64_t i, Ctx, uint64_t, uint64_t ex) const { r[i] = ex; }
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
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->total_m = hdr->status ? 0 : hdr->lane_pos[hdr->total_nl];
    hdr->planned = hdr->status ? 0u : 1u;   // counted: the write kernels may run
  }
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

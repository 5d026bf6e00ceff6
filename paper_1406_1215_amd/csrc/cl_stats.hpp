// Model statistics and the uniform consecutive partition.
//
//  * E[m] and Var[m] of the capped model (Eq. 1 with min(., 1)); for sorted
//    weights the capped candidates of a source u are a prefix of v > u, so
//    e_u = (J_u - u - 1) + a_u sum_{v >= J_u} w_v with J_u the first
//    uncapped candidate.
//  * Sec. 4, Eq. 2 / Eq. 5 / Alg. 2: fixed-point costs c_u = floor(256 e_u) +
//    256 (e_u from Eq. 6 on the quantised prefix), their exact prefix C, and
//    n_k = min{u : C_u >= k Z / P}.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cl_device.hpp"
#include "cl_kernels.hpp"
#include "cl_plan.hpp"
#include "cl_scan.hpp"

namespace cl {

struct Dbl2 {
  double a, b;
};

template <>
struct ScanTraits<Dbl2> {
  __device__ static Dbl2 zero() { return Dbl2{0.0, 0.0}; }
  __device__ static Dbl2 add(Dbl2 x, Dbl2 y) { return Dbl2{x.a + y.a, x.b + y.b}; }
  __device__ static Dbl2 shfl_up(Dbl2 x, int d) {
    return Dbl2{__longlong_as_double(static_cast<long long>(shfl_up64(static_cast<uint64_t>(__double_as_longlong(x.a)), d))),
                __longlong_as_double(static_cast<long long>(shfl_up64(static_cast<uint64_t>(__double_as_longlong(x.b)), d)))};
  }
  __device__ static Dbl2 shfl_idx(Dbl2 x, int src) {
    return Dbl2{__longlong_as_double(static_cast<long long>(shfl_idx64(static_cast<uint64_t>(__double_as_longlong(x.a)), src))),
                __longlong_as_double(static_cast<long long>(shfl_idx64(static_cast<uint64_t>(__double_as_longlong(x.b)), src)))};
  }
  template <int kCtrl, int kRowMask, int kBankMask>
  __device__ static Dbl2 dpp(Dbl2 x) {   // lanes that read nothing get +0.0
    auto one = [](double v) {
      return __longlong_as_double(static_cast<long long>(
          dpp64<kCtrl, kRowMask, kBankMask>(static_cast<uint64_t>(__double_as_longlong(v)))));
    };
    return Dbl2{one(x.a), one(x.b)};
  }
  __device__ static Dbl2 lane63(Dbl2 x) {
    return Dbl2{__longlong_as_double(static_cast<long long>(lane63_64(static_cast<uint64_t>(__double_as_longlong(x.a))))),
                __longlong_as_double(static_cast<long long>(lane63_64(static_cast<uint64_t>(__double_as_longlong(x.b)))))};
  }
};

// suffix sums of w and w^2: element i is w[n-1-i]; exclusive prefix at i is
// sum_{y > n-1-i} w_y, i.e. the suffix from v = n - i.
struct SufIn : OneGraph {
  const double* w;
  uint64_t n;
  __device__ Dbl2 load(uint64_t i, Ctx) const {
    if (i >= n) return Dbl2{0.0, 0.0};
    const double x = w[n - 1 - i];
    return Dbl2{x, x * x};
  }
};

struct SufOut : OneGraph {
  Dbl2* suf;  // suf[v] = (sum_{y >= v} w_y, sum_{y >= v} w_y^2), v in [0, n]
  uint64_t n;
  __device__ void store(uint64_t i, Ctx, Dbl2, Dbl2 ex) const { suf[n - i] = ex; }
};

// per-source terms, reduced per block into partials
__global__ void __launch_bounds__(256) k_expected_edges(const double* w, uint64_t n, double S, const Dbl2* suf,
                                                        Dbl2* partials) {
  double E = 0.0, V = 0.0;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t u = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride) {
    const double a = w[u] / S;
    // J = first v in [u+1, n] with a * w_v < 1 (the sampler's own product)
    uint64_t lo = u + 1, hi = n;
    while (lo < hi) {
      const uint64_t mid = lo + ((hi - lo) >> 1);
      if (a * w[mid] >= 1.0) lo = mid + 1; else hi = mid;
    }
    const Dbl2 s = suf[lo];
    E += static_cast<double>(lo - u - 1) + a * s.a;
    V += a * s.a - a * a * s.b;
  }
  Dbl2 tot;
  (void)block_exclusive<Dbl2>(Dbl2{E, V}, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_reduce_dbl2(const Dbl2* partials, uint32_t np, Dbl2* out) {
  Dbl2 s{0.0, 0.0};
  for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) s = ScanTraits<Dbl2>::add(s, partials[i]);
  Dbl2 tot;
  (void)block_exclusive<Dbl2>(s, &tot);
  if (threadIdx.x == 0) *out = tot;
}

// ------------------------------------------------------------- partition
struct PartIn : OneGraph {
  const GraphDesc* desc;
  const uint64_t* Q;
  __device__ uint64_t load(uint64_t u, Ctx) const {
    const GraphDesc& d = desc[0];
    if (u >= d.n) return 0;
    double e = 0.0;
    if (d.qscale != 0.0) {
      const double a = d.w[u] / d.S;
      const uint64_t D = (d.Qend - d.Qbase) - (Q[u + 1] - d.Qbase);
      e = ehat_of(a, D, d.qscale);
    }
    double s = e * 256.0;
    if (s > 0x1.0p40) s = 0x1.0p40;
    return static_cast<uint64_t>(floor(s)) + 256ull;
  }
};

struct PartOut : OneGraph {
  uint64_t* C;
  __device__ void store(uint64_t i, Ctx, uint64_t, uint64_t ex) const { C[i] = ex; }
};

// n_k = first u with C_incl(u) = C[u+1] >= ceil(k Z / P), for k in [1, P-1]
__global__ void __launch_bounds__(256) k_part_bounds(const uint64_t* C, uint64_t n, uint32_t P, uint64_t* bounds) {
  const uint64_t Z = C[n];
  const uint64_t q = Z / P, rr = Z % P;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= P; k += gridDim.x * blockDim.x) {
    uint64_t b;
    if (k == 0) {
      b = 0;
    } else if (k == P) {
      b = n;
    } else {
      const uint64_t kr = static_cast<uint64_t>(k) * rr;  // < P^2 < 2^64
      const uint64_t Tk = static_cast<uint64_t>(k) * q + kr / P + ((kr % P) ? 1 : 0);
      uint64_t lo = 0, hi = n - 1;   // C[n] = Z >= Tk, so u = n-1 qualifies
      while (lo < hi) {
        const uint64_t mid = lo + ((hi - lo) >> 1);
        if (C[mid + 1] >= Tk) hi = mid; else lo = mid + 1;
      }
      b = lo;
    }
    bounds[k] = b;
  }
}

}  // namespace cl

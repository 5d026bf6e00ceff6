// Expected degree of the capped Chung-Lu model and its adjoint.
//
//   d_i = sum_{j != i} min(x_ij, 1),  x_ij = a_i w_j,  a_i = fl32(w_i / S)
//
// (Sec. 3 gives the uncapped form w_i - w_i^2/S.)  Tiles: a workgroup owns
// kEdLanes R rows (R per lane, kEdLanes lanes) and one tile of C columns
// (R, C: template parameters); the column weights are wave-uniform, so they come through
// the scalar cache, sixteen at a time, and each pair costs two vector ops:
// the product with the clamp output modifier (min(x, 1) of a product that
// is >= 0, as weights are non-negative: fmed3(x, 0, 1) folds into the
// multiply) and the add.  Every row keeps four float32 accumulators over the
// tile; tile partials are summed per row in float64 by a second kernel, which
// also removes the j = i term.
//
// Adjoint, for g = dL/dd:
//   dL/dw_k = (g_k A_k + B_k - T) / S,  A_k = sum_{j != k, x_kj < 1} w_j,
//   B_k = sum_{j != k, x_kj < 1} g_j w_j,  T = sum_i g_i U_i,  U_i = a_i A_i,
// the T term being the dependence of S = sum w on w_k (optional).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cl_scan.hpp"
#include "cl_stats.hpp"

namespace cl {

// Tile shape: kEdLanes threads per workgroup, R rows per thread, C columns
// per tile.  R and C are schedule knobs (tile shapes of the instantiations
// below; the default 2 x 1024); they change the float32 summation order of
// the partials only within a tile of C columns.
constexpr int kEdLanes = 256;
constexpr int kEdRowsDefault = 2;
constexpr int kEdColsDefault = 1024;
constexpr int kEdColsMin = 512;   // the workspace holds the partials of the smallest tile width
constexpr int kEdUnroll = 16;

__global__ void __launch_bounds__(256) k_rowscale(const float* __restrict__ w, uint64_t n, double S,
                                                  float* __restrict__ a) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = static_cast<float>(static_cast<double>(w[i]) / S);
}

// Smallest float32 t with fl(a * t) >= 1.  Rounding is monotone in w, so for
// every finite w >= 0 the capped test fl(a * w) < 1 holds exactly when w < t;
// the adjoint tile then compares against t instead of forming the product.
__device__ inline float cap_threshold(float a) {
  if (!(a > 0.0f)) return __builtin_inff();
  float t = 1.0f / a;
  if (__builtin_isinf(t)) {
    if (a * __FLT_MAX__ < 1.0f) return __builtin_inff();
    t = __FLT_MAX__;
  }
  // a few ulps at most from the true boundary; walk to it
  for (int it = 0; it < 64 && t > 0.0f && a * __uint_as_float(__float_as_uint(t) - 1u) >= 1.0f; ++it)
    t = __uint_as_float(__float_as_uint(t) - 1u);
  for (int it = 0; it < 64 && a * t < 1.0f; ++it) t = __uint_as_float(__float_as_uint(t) + 1u);
  return t;
}

__global__ void __launch_bounds__(256) k_threshold(const float* __restrict__ a, uint64_t n, float* __restrict__ t) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) t[i] = cap_threshold(a[i]);
}

// forward tile: part[tile * n + i] = sum_{j in tile} min(a_i w_j, 1) (float32).
// Row i = blockIdx.x * kEdLanes R + r * kEdLanes + lane; column j of the tile
// goes to accumulator j mod 4 of every row.
template <int R, int C>
__global__ void __launch_bounds__(kEdLanes) k_expdeg_tile(const float* __restrict__ w, const float* __restrict__ a,
                                                          uint64_t n, float* __restrict__ part) {
  static_assert(C % kEdUnroll == 0, "whole unrolled steps per tile");
  const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * (kEdLanes * R) + threadIdx.x;
  const uint64_t j0 = static_cast<uint64_t>(blockIdx.y) * C;
  const uint64_t jn = (n - j0 < static_cast<uint64_t>(C)) ? (n - j0) : C;
  float ai[R], s[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = i0 + static_cast<uint64_t>(r) * kEdLanes;
    ai[r] = (i < n) ? a[i] : 0.0f;
    s[r][0] = s[r][1] = s[r][2] = s[r][3] = 0.0f;
  }
  const float* __restrict__ wc = w + j0;
  uint64_t jj = 0;
  for (; jj + kEdUnroll <= jn; jj += kEdUnroll) {
    float wv[kEdUnroll];
#pragma unroll
    for (int q = 0; q < kEdUnroll; ++q) wv[q] = wc[jj + q];
#pragma unroll
    for (int q = 0; q < kEdUnroll; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) s[r][q & 3] += __builtin_amdgcn_fmed3f(ai[r] * wv[q], 0.0f, 1.0f);
  }
  // ragged tail of the last tile (kEdUnroll divides C)
#pragma unroll
  for (int q = 0; q < kEdUnroll; ++q)
    if (jj + q < jn)
#pragma unroll
      for (int r = 0; r < R; ++r) s[r][q & 3] += __builtin_amdgcn_fmed3f(ai[r] * wc[jj + q], 0.0f, 1.0f);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = i0 + static_cast<uint64_t>(r) * kEdLanes;
    if (i < n) part[static_cast<uint64_t>(blockIdx.y) * n + i] = (s[r][0] + s[r][1]) + (s[r][2] + s[r][3]);
  }
}

// row sums of the tile partials in float64, minus the own term
__global__ void __launch_bounds__(256) k_expdeg_rows(const float* __restrict__ w, const float* __restrict__ a,
                                                     uint64_t n, uint32_t ntiles, const float* __restrict__ part,
                                                     double* __restrict__ d) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (uint32_t t = 0; t < ntiles; ++t) s += static_cast<double>(part[static_cast<uint64_t>(t) * n + i]);
  s -= static_cast<double>(__builtin_amdgcn_fmed3f(a[i] * w[i], 0.0f, 1.0f));
  d[i] = s;
}

// Mask of the adjoint as one clamped multiply-add.  For a row with threshold
// t = 1.x * 2^e (cap_threshold) and k = 2^(24 - e), the exact value (t - w) k
// is >= 1 whenever w < t: either w >= t/2, where t and w are both multiples
// of 2^(e - 24), or w < t/2 and the difference exceeds 2^(e - 1).  It is <= 0
// when w >= t, and a fused multiply-add rounds it once, so clamping to [0, 1]
// yields exactly 1.0 or 0.0.  k stays a normal float for e >= -100 and for
// t = inf (then t k = inf and every finite w passes); a wave holding a row
// with a smaller threshold takes the plain comparison instead.
struct MaskRow {
  float k, tk;
};

__device__ inline bool mask_row(float t, MaskRow* m) {
  const int e = static_cast<int>((__float_as_uint(t) >> 23) & 0xFFu) - 127;
  m->k = __uint_as_float(static_cast<uint32_t>(127 + 24 - e) << 23);
  m->tk = t * m->k;
  return e >= -100;
}

template <bool kFma>
__device__ inline float mask_of(float wj, float t, const MaskRow& m) {
  if constexpr (kFma) return __builtin_amdgcn_fmed3f(__builtin_fmaf(-wj, m.k, m.tk), 0.0f, 1.0f);
  return wj < t ? 1.0f : 0.0f;
}

// adjoint tile: partA = sum_{j in tile, x_ij < 1} w_j, partB = sum ... g_j w_j.
// The mask (0.0 or 1.0) is applied with a fused multiply-add: w * 1 and g * 0
// are exact, so each step rounds as the plain masked sum does (for finite g).
// Column j goes to accumulator j mod 2 of every row.
template <bool kFma, int R>
__device__ inline void bwd_columns(const float* __restrict__ wc, const float* __restrict__ gc, uint64_t jn,
                                   const float (&ti)[R], const MaskRow (&mr)[R], float (&A)[R][2], float (&B)[R][2]) {
  uint64_t jj = 0;
  for (; jj + kEdUnroll <= jn; jj += kEdUnroll) {
    float wv[kEdUnroll], gv[kEdUnroll];
#pragma unroll
    for (int q = 0; q < kEdUnroll; ++q) {
      wv[q] = wc[jj + q];
      gv[q] = gc[jj + q];
    }
#pragma unroll
    for (int q = 0; q < kEdUnroll; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float m = mask_of<kFma>(wv[q], ti[r], mr[r]);
        A[r][q & 1] = __builtin_fmaf(wv[q], m, A[r][q & 1]);
        B[r][q & 1] = __builtin_fmaf(gv[q], m, B[r][q & 1]);
      }
  }
#pragma unroll
  for (int q = 0; q < kEdUnroll; ++q)
    if (jj + q < jn)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float m = mask_of<kFma>(wc[jj + q], ti[r], mr[r]);
        A[r][q & 1] = __builtin_fmaf(wc[jj + q], m, A[r][q & 1]);
        B[r][q & 1] = __builtin_fmaf(gc[jj + q], m, B[r][q & 1]);
      }
}

template <int R, int C>
__global__ void __launch_bounds__(kEdLanes) k_expdeg_bwd_tile(const float* __restrict__ w, const float* __restrict__ thr,
                                                              const float* __restrict__ gw, uint64_t n,
                                                              float* __restrict__ partA, float* __restrict__ partB) {
  static_assert(C % kEdUnroll == 0, "whole unrolled steps per tile");
  const uint64_t i0 = static_cast<uint64_t>(blockIdx.x) * (kEdLanes * R) + threadIdx.x;
  const uint64_t j0 = static_cast<uint64_t>(blockIdx.y) * C;
  const uint64_t jn = (n - j0 < static_cast<uint64_t>(C)) ? (n - j0) : C;
  float ti[R], A[R][2], B[R][2];
  MaskRow mr[R];
  bool fast = true;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = i0 + static_cast<uint64_t>(r) * kEdLanes;
    ti[r] = (i < n) ? thr[i] : 1.0f;  // rows past n: any normal threshold, never stored
    fast = mask_row(ti[r], &mr[r]) && fast;
    A[r][0] = A[r][1] = B[r][0] = B[r][1] = 0.0f;
  }
  if (__builtin_amdgcn_ballot_w64(!fast) == 0)
    bwd_columns<true, R>(w + j0, gw + j0, jn, ti, mr, A, B);
  else
    bwd_columns<false, R>(w + j0, gw + j0, jn, ti, mr, A, B);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = i0 + static_cast<uint64_t>(r) * kEdLanes;
    if (i < n) {
      partA[static_cast<uint64_t>(blockIdx.y) * n + i] = A[r][0] + A[r][1];
      partB[static_cast<uint64_t>(blockIdx.y) * n + i] = B[r][0] + B[r][1];
    }
  }
}

// g_j w_j in float32 (the column operand of B)
__global__ void __launch_bounds__(256) k_gw(const float* __restrict__ w, const double* __restrict__ g, uint64_t n,
                                            float* __restrict__ gw) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) gw[i] = static_cast<float>(g[i] * static_cast<double>(w[i]));
}

// A_k, B_k in float64 (own term removed), and per-block partials of T
__global__ void __launch_bounds__(256) k_expdeg_bwd_rows(const float* __restrict__ w, const float* __restrict__ a,
                                                         const double* __restrict__ g, const float* __restrict__ gw,
                                                         uint64_t n, uint32_t ntiles, const float* __restrict__ partA,
                                                         const float* __restrict__ partB, double* __restrict__ A,
                                                         double* __restrict__ B, double* __restrict__ tpart) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double t = 0.0;
  if (i < n) {
    double sa = 0.0, sb = 0.0;
    for (uint32_t tt = 0; tt < ntiles; ++tt) {
      sa += static_cast<double>(partA[static_cast<uint64_t>(tt) * n + i]);
      sb += static_cast<double>(partB[static_cast<uint64_t>(tt) * n + i]);
    }
    if (a[i] * w[i] < 1.0f) {
      sa -= static_cast<double>(w[i]);
      sb -= static_cast<double>(gw[i]);
    }
    A[i] = sa;
    B[i] = sb;
    t = g[i] * static_cast<double>(a[i]) * sa;
  }
  Dbl2 td;
  (void)block_exclusive<Dbl2>(Dbl2{t, 0.0}, &td);
  if (threadIdx.x == 0) tpart[blockIdx.x] = td.a;
}

__global__ void __launch_bounds__(256) k_sum_dbl(const double* __restrict__ x, uint32_t m, double* __restrict__ out) {
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) s += x[i];
  Dbl2 td;
  (void)block_exclusive<Dbl2>(Dbl2{s, 0.0}, &td);
  if (threadIdx.x == 0) *out = td.a;
}

__global__ void __launch_bounds__(256) k_expdeg_grad(const double* __restrict__ g, const double* __restrict__ A,
                                                     const double* __restrict__ B, const double* __restrict__ T,
                                                     int use_T, uint64_t n, double S, float* __restrict__ grad) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double tt = use_T ? *T : 0.0;
  grad[i] = static_cast<float>((g[i] * A[i] + B[i] - tt) / S);
}

}  // namespace cl

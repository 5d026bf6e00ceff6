// Expected degree of the capped Chung-Lu model and its adjoint.
//
//   d_i = sum_{j != i} min(x_ij, 1),  x_ij = a_i w_j,  a_i = fl32(w_i / S)
//
// (Sec. 3 gives the uncapped form w_i - w_i^2/S.)  Tiles: a workgroup owns
// kEdRows rows (one per lane) and one tile of kEdCols columns; the column
// weights are wave-uniform, so they come through the scalar cache and each
// pair costs three vector ops (multiply, min, add).  Every lane keeps four
// float32 accumulators over the tile; tile partials are summed per row in
// float64 by a second kernel, which also removes the j = i term.
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

constexpr int kEdRows = 256;
constexpr int kEdCols = 1024;

__global__ void __launch_bounds__(256) k_rowscale(const float* __restrict__ w, uint64_t n, double S,
                                                  float* __restrict__ a) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = static_cast<float>(static_cast<double>(w[i]) / S);
}

// forward tile: part[tile * n + i] = sum_{j in tile} min(a_i w_j, 1) (float32)
__global__ void __launch_bounds__(kEdRows) k_expdeg_tile(const float* __restrict__ w, const float* __restrict__ a,
                                                         uint64_t n, float* __restrict__ part) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kEdRows + threadIdx.x;
  const uint64_t j0 = static_cast<uint64_t>(blockIdx.y) * kEdCols;
  const uint64_t jn = (n - j0 < static_cast<uint64_t>(kEdCols)) ? (n - j0) : kEdCols;
  const float ai = (i < n) ? a[i] : 0.0f;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  const float* __restrict__ wc = w + j0;
  uint64_t jj = 0;
  for (; jj + 4 <= jn; jj += 4) {
    s0 += fminf(ai * wc[jj + 0], 1.0f);
    s1 += fminf(ai * wc[jj + 1], 1.0f);
    s2 += fminf(ai * wc[jj + 2], 1.0f);
    s3 += fminf(ai * wc[jj + 3], 1.0f);
  }
  for (; jj < jn; ++jj) s0 += fminf(ai * wc[jj], 1.0f);
  if (i < n) part[static_cast<uint64_t>(blockIdx.y) * n + i] = (s0 + s1) + (s2 + s3);
}

// row sums of the tile partials in float64, minus the own term
__global__ void __launch_bounds__(256) k_expdeg_rows(const float* __restrict__ w, const float* __restrict__ a,
                                                     uint64_t n, uint32_t ntiles, const float* __restrict__ part,
                                                     double* __restrict__ d) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (uint32_t t = 0; t < ntiles; ++t) s += static_cast<double>(part[static_cast<uint64_t>(t) * n + i]);
  s -= static_cast<double>(fminf(a[i] * w[i], 1.0f));
  d[i] = s;
}

// adjoint tile: partA = sum_{j in tile, x_ij < 1} w_j, partB = sum ... g_j w_j
__global__ void __launch_bounds__(kEdRows) k_expdeg_bwd_tile(const float* __restrict__ w, const float* __restrict__ a,
                                                             const float* __restrict__ gw, uint64_t n,
                                                             float* __restrict__ partA, float* __restrict__ partB) {
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kEdRows + threadIdx.x;
  const uint64_t j0 = static_cast<uint64_t>(blockIdx.y) * kEdCols;
  const uint64_t jn = (n - j0 < static_cast<uint64_t>(kEdCols)) ? (n - j0) : kEdCols;
  const float ai = (i < n) ? a[i] : 0.0f;
  float A0 = 0.0f, A1 = 0.0f, B0 = 0.0f, B1 = 0.0f;
  const float* __restrict__ wc = w + j0;
  const float* __restrict__ gc = gw + j0;
  uint64_t jj = 0;
  for (; jj + 2 <= jn; jj += 2) {
    const float w0 = wc[jj], w1 = wc[jj + 1];
    const bool m0 = ai * w0 < 1.0f, m1 = ai * w1 < 1.0f;
    A0 += m0 ? w0 : 0.0f;
    B0 += m0 ? gc[jj] : 0.0f;
    A1 += m1 ? w1 : 0.0f;
    B1 += m1 ? gc[jj + 1] : 0.0f;
  }
  for (; jj < jn; ++jj) {
    const float w0 = wc[jj];
    const bool m0 = ai * w0 < 1.0f;
    A0 += m0 ? w0 : 0.0f;
    B0 += m0 ? gc[jj] : 0.0f;
  }
  if (i < n) {
    partA[static_cast<uint64_t>(blockIdx.y) * n + i] = A0 + A1;
    partB[static_cast<uint64_t>(blockIdx.y) * n + i] = B0 + B1;
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
  uint64_t tot;
  Dbl2 td;
  (void)block_exclusive<Dbl2>(Dbl2{t, 0.0}, &td);
  (void)tot;
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

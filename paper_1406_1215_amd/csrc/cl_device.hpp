// Device primitives of the Chung-Lu sampler (gfx950).
//
// The sampling rule is Alg. 1 of Sec. 3 (Create-Edges) with its open points
// fixed: a Philox4x32-10 counter-based stream, 53-bit uniforms in (0,1), and
// binary64 logarithms built from IEEE basic operations only, so that every
// rounding is determined.  Everything here compiles with contraction off
// (-ffp-contract=off); fused multiply-adds appear only where written.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cl {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 3.2): ten rounds of
//   (x0,x1,x2,x3) -> (hi(B*x2) ^ x1 ^ k0, lo(B*x2), hi(A*x0) ^ x3 ^ k1, lo(A*x0))
// with A = 0xD2511F53, B = 0xCD9E8D57, and the key advanced by the Weyl
// increments (0x9E3779B9, 0xBB67AE85) between rounds.
// ---------------------------------------------------------------------------
struct RoundKeys {
  uint32_t k0[10];
  uint32_t k1[10];
};

__device__ __forceinline__ RoundKeys philox_round_keys(uint64_t seed) {
  RoundKeys rk;
  uint32_t a = static_cast<uint32_t>(seed);
  uint32_t b = static_cast<uint32_t>(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    rk.k0[r] = a;
    rk.k1[r] = b;
    a += 0x9E3779B9u;
    b += 0xBB67AE85u;
  }
  return rk;
}

struct Block4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           const RoundKeys& rk) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t y0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ rk.k0[r];
    const uint32_t y2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ rk.k1[r];
    c1 = static_cast<uint32_t>(pb);
    c3 = static_cast<uint32_t>(pa);
    c0 = y0;
    c2 = y2;
  }
  return Block4{c0, c1, c2, c3};
}

// 53-bit uniform in (0,1) from two 32-bit words (hi:lo): the odd integer
// 2*(x >> 12) + 1 < 2^53 times 2^-53; both steps are exact.
__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  const uint64_t x = (static_cast<uint64_t>(hi) << 32) | lo;
  const uint64_t odd = ((x >> 12) << 1) | 1ull;
  return static_cast<double>(odd) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Logarithms.  ln(m) = 2 atanh(s), s = (m - 1)/(m + 1), and
// atanh(s)/s = sum_{j>=0} s^{2j}/(2j+1); eleven terms in Horner/FMA form are
// enough for |s| <= 0.1716.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double atanh_series(double z) {
  // coefficients 1/(2j+1) rounded to nearest, j = 10 down to 0
  double r = 1.0 / 21.0;
  r = __builtin_fma(r, z, 1.0 / 19.0);
  r = __builtin_fma(r, z, 1.0 / 17.0);
  r = __builtin_fma(r, z, 1.0 / 15.0);
  r = __builtin_fma(r, z, 1.0 / 13.0);
  r = __builtin_fma(r, z, 1.0 / 11.0);
  r = __builtin_fma(r, z, 1.0 / 9.0);
  r = __builtin_fma(r, z, 1.0 / 7.0);
  r = __builtin_fma(r, z, 1.0 / 5.0);
  r = __builtin_fma(r, z, 1.0 / 3.0);
  r = __builtin_fma(r, z, 1.0);
  return r;
}

// natural log of a normal x in (0, 1]: split x = m 2^e (m in [1,2)); fold m
// above sqrt(2) into (0.707, 1] with e + 1; then e ln2 + 2 s P(s^2).
__device__ __forceinline__ double ln_unit(double x) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x));
  int e = static_cast<int>((bits >> 52) & 0x7FF) - 1023;
  double m = __longlong_as_double(static_cast<long long>((bits & 0x000FFFFFFFFFFFFFull) |
                                                         0x3FF0000000000000ull));
  if (m > 0x1.6a09e667f3bcdp+0) {  // sqrt(2) rounded to nearest
    m = m * 0.5;
    e = e + 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  const double l = (2.0 * s) * atanh_series(z);
  return (static_cast<double>(e) * 0x1.62e42fefa39efp-1) + l;  // ln 2 rounded to nearest
}

// ln(1 - p) for p in (0,1): for p < 1/4, -2 atanh(p/(2-p)) (no cancellation);
// otherwise ln of the rounded 1 - p.
__device__ __forceinline__ double ln_one_minus(double p) {
  if (p < 0.25) {
    const double s = p / (2.0 - p);
    const double z = s * s;
    return -((2.0 * s) * atanh_series(z));
  }
  return ln_unit(1.0 - p);
}

__device__ __forceinline__ double cap1(double x) { return (x < 1.0) ? x : 1.0; }

// ---------------------------------------------------------------------------
// Quantised weight mass (exact integers): q_v = floor(w_v * 2^32 / w_0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t quantise(double wv, double qscale) {
  return static_cast<uint64_t>(floor(wv * qscale));
}

// expected edges of source u on the quantised mass: (a_u * D_u) / qscale
__device__ __forceinline__ double ehat_of(double a, uint64_t D, double qscale) {
  return (a * static_cast<double>(D)) / qscale;
}

// segments of a source: 1 unless ehat > 256, else min(ceil(ehat/256), n-u-1)
__device__ __forceinline__ uint32_t nseg_of(double eh, uint64_t n, uint64_t u) {
  if (!(eh > 256.0) || u + 2 >= n) return 1u;
  const uint64_t capk = n - u - 1;
  const double kd = ceil(eh / 256.0);
  if (kd >= static_cast<double>(capk)) return static_cast<uint32_t>(capk);
  return static_cast<uint32_t>(kd);
}

// splitmix64's output function (Steele, Lea, Flood, OOPSLA 2014)
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace cl

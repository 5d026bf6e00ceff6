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

// three-way exclusive or in one v_bitop3_b32 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Block4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           const RoundKeys& rk) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t y0 = xor3(static_cast<uint32_t>(pb >> 32), c1, rk.k0[r]);
    const uint32_t y2 = xor3(static_cast<uint32_t>(pa >> 32), c3, rk.k1[r]);
    c1 = static_cast<uint32_t>(pb);
    c3 = static_cast<uint32_t>(pa);
    c0 = y0;
    c2 = y2;
  }
  return Block4{c0, c1, c2, c3};
}

// 53-bit uniform in (0,1) from two 32-bit words (hi:lo): (2*(x >> 12) + 1) * 2^-53.
// Formed exactly as (1 + k 2^-52) - (1 - 2^-53), k = x >> 12: the first term
// is k placed in the mantissa of 1.0 and the subtraction is exact (Sterbenz).
// The two words of 1 + k 2^-52 are funnel shifts: (hi:lo) >> 12 and
// (0x3FF:hi) >> 12.
__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo) {
  const uint32_t mlo = __builtin_amdgcn_alignbit(hi, lo, 12);
  const uint32_t mhi = __builtin_amdgcn_alignbit(0x3FFu, hi, 12);
  const double one_k = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(mhi) << 32) | mlo));
  return one_k - 0x1.fffffffffffffp-1;
}

// ---------------------------------------------------------------------------
// Logarithms.  ln(m) = 2 atanh(s), s = (m - 1)/(m + 1), and
// atanh(s)/s = sum_{j>=0} s^{2j}/(2j+1); eleven terms in Horner/FMA form are
// enough for |s| <= 0.1716.
//
// The coefficients 1/(2j+1) (rounded to nearest) live in constant memory and
// are read once per kernel into scalar registers, so each Horner step is one
// v_fma_f64 with a scalar addend.
// ---------------------------------------------------------------------------
__constant__ double kSeries[11] = {1.0,        1.0 / 3.0,  1.0 / 5.0,  1.0 / 7.0,  1.0 / 9.0, 1.0 / 11.0,
                                   1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0};

struct Series {
  double c[11];
};

__device__ __forceinline__ Series load_series() {
  Series sr;
#pragma unroll
  for (int j = 0; j < 11; ++j) sr.c[j] = kSeries[j];
  return sr;
}

// 2 s P(s^2), P the 11-term series in Horner form from the top coefficient
__device__ __forceinline__ double two_s_series(double s, const Series& sr) {
  const double z = s * s;
  double r = sr.c[10];
#pragma unroll
  for (int j = 9; j >= 0; --j) r = __builtin_fma(r, z, sr.c[j]);
  return (2.0 * s) * r;
}

// split a normal x into m in (0.707, 1.414] and e with x = m 2^e
__device__ __forceinline__ void log_reduce(double x, double& m, int& e) {
  const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(x));
  e = static_cast<int>((bits >> 52) & 0x7FF) - 1023;
  m = __longlong_as_double(static_cast<long long>((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  if (m > 0x1.6a09e667f3bcdp+0) {  // sqrt(2) rounded to nearest
    m = m * 0.5;
    e = e + 1;
  }
}

// natural log of a normal x in (0, 1]: e ln2 + 2 s P(s^2), s = (m-1)/(2+(m-1))
__device__ __forceinline__ double ln_unit(double x, const Series& sr) {
  double m;
  int e;
  log_reduce(x, m, e);
  const double f = m - 1.0;
  const double l = two_s_series(f / (2.0 + f), sr);
  return (static_cast<double>(e) * 0x1.62e42fefa39efp-1) + l;  // ln 2 rounded to nearest
}

// ln(1 - p) for p in (0,1): for p < 1/4, -2 atanh(p/(2-p)) (no cancellation);
// otherwise ln of the rounded 1 - p.  The small-p quotient is formed as
// (-p)/(2-p), exactly the negated p/(2-p), so 2 s P(s^2) carries the sign of
// -2 atanh without a separate negation.
__device__ __forceinline__ double ln_one_minus(double p, const Series& sr) {
  if (p < 0.25) return two_s_series((-p) / (2.0 - p), sr);
  return ln_unit(1.0 - p, sr);
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

// Device Wiener increments: Philox4x32-10 and the polar normal map.
//
// The paper draws one N(0, dt) increment per sample, step and direction,
// shared by all nodes of the sample (Sec. 5.2 after eq. def_dx; the
// Conclusions report per-node or per-element increments as unstable).  The
// generator is Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11):
// counter (step, sample, attempt, stream), key (seed lo, seed hi).
//
// Every floating-point operation below is an explicit round-to-nearest
// intrinsic so that an independent implementation doing the same operations
// in the same order reproduces the same bits:
//   k  = (r0 >> 6) * 2^26 + (r1 >> 6),  v = (2k + 1 - 2^52) * 2^-52   (exact)
//   s  = va*va + vb*vb; accept s < 1 (else next attempt, at most 64)
//   z  = v * sqrt((-2 * log(s)) / s)
// log(s): s = m 2^e with m in [sqrt(1/2), sqrt(2)) (exact), t = (m-1)/(m+1),
// log m = 2 (t + t (t^2 P(t^2))), P(x) = sum_{k=1..11} x^(k-1)/(2k+1) by
// Horner, log s = e*LN2_HI + (e*LN2_LO + log m) (Cody-Waite split: LN2_HI
// is ln 2 rounded to 33 significant bits, LN2_LO = ln 2 - LN2_HI rounded).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "sl_internal.hpp"

namespace sl {

struct Normal2 {
  double a, b;
};

__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

__device__ __forceinline__ double own_log(double s) {
  const double kLn2Hi = 0x1.62e42fef00000p-1;
  const double kLn2Lo = 0x1.473de6af278edp-34;
  const double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
  int e0;
  const double m0 = frexp(s, &e0);   // s = m0 * 2^e0, m0 in [0.5, 1)
  double m = m0;
  int e = e0;
  if (m0 < kSqrtHalf) {
    m = __dmul_rn(m0, 2.0);
    e = e0 - 1;
  }
  const double f = __dadd_rn(m, -1.0);
  const double den = __dadd_rn(m, 1.0);
  const double t = __ddiv_rn(f, den);
  const double t2 = __dmul_rn(t, t);
  double p = 1.0 / 23.0;
  p = __dadd_rn(1.0 / 21.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 19.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 17.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 15.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 13.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 11.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 9.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 7.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 5.0, __dmul_rn(t2, p));
  p = __dadd_rn(1.0 / 3.0, __dmul_rn(t2, p));
  const double a = __dmul_rn(t2, p);
  const double b = __dmul_rn(t, a);
  const double c = __dadd_rn(t, b);
  const double lm = __dmul_rn(2.0, c);
  const double ef = (double)e;
  const double a1 = __dmul_rn(ef, kLn2Lo);
  const double a2 = __dadd_rn(a1, lm);
  const double a3 = __dmul_rn(ef, kLn2Hi);
  return __dadd_rn(a3, a2);
}

__device__ __forceinline__ double philox_v(uint32_t hi_word, uint32_t lo_word) {
  const int64_t k = ((int64_t)(hi_word >> 6) << 26) + (int64_t)(lo_word >> 6);
  const int64_t num = 2 * k + 1 - ((int64_t)1 << 52);
  return __dmul_rn((double)num, 0x1p-52);
}

// Standard normal pair for (step, sample) of a handle; bounded retry loop.
__device__ __forceinline__ Normal2 normal_pair(uint64_t seed, uint32_t stream, uint64_t step, uint64_t sample) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  Normal2 out{0.0, 0.0};
  for (uint32_t att = 0; att < (uint32_t)kMaxAttempts; ++att) {
    uint32_t c0 = (uint32_t)step, c1 = (uint32_t)sample, c2 = att, c3 = stream;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    const double va = philox_v(c0, c1);
    const double vb = philox_v(c2, c3);
    const double s = __dadd_rn(__dmul_rn(va, va), __dmul_rn(vb, vb));
    if (s < 1.0) {
      const double lg = own_log(s);
      const double q = __ddiv_rn(__dmul_rn(-2.0, lg), s);
      const double r = __dsqrt_rn(q);
      out.a = __dmul_rn(va, r);
      out.b = __dmul_rn(vb, r);
      break;
    }
  }
  return out;
}

// Moved reference coordinate of one node in one direction (position contract):
// xi* = xi + (A + B z), three round-to-nearest operations, no fused multiply-add.
__device__ __forceinline__ double moved_coord(double xi, double A, double B, double z) {
  return __dadd_rn(xi, __dadd_rn(A, __dmul_rn(B, z)));
}

// Displacement A + B z of a moved edge point, rounded as in moved_coord, so the
// sign that picks the upwind side agrees with the moved positions.  Defined
// here, outside the fit code that enables contraction.
__device__ __forceinline__ double edge_disp(double A, double B, double z) {
  return __dadd_rn(A, __dmul_rn(B, z));
}

}  // namespace sl

// Binary64 log(1 + y) for 0 <= y <= 1, the one logarithm of the FP64 path:
// log cosh(u) + ln 2 = |u| + log(1 + e^{-2|u|}).
//
// Written for this range only, from the series
//   log(1 + f) = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = f / (2 + f),
// arranged so that f itself is the leading term (the arrangement
// f - (f^2/2 - s (f^2/2 + R)) of the classic Sun fdlibm log and log1p; the
// coefficients here are the plain series terms 2/(2k+1), not a minimax fit),
// after the reduction 1 + y = m 2^e with m in [sqrt(1/2), sqrt(2)) and
// e in {0, 1}, so |s| <= 0.1716 and s^2 <= 0.02944; the terms through s^19
// leave a truncation below 2^-56 of the result.  The rounding error of the
// sum 1 + y is carried separately and added back, so small y keep their
// relative accuracy.  Accuracy: below 2 units in the last place over
// [0, 1] (checked on the host against a long double reference).  It is a plain
// function of binary64 arithmetic, so the same source compiles for the host
// and for gfx950.
#pragma once

#if !defined(__HIPCC__)
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

#include <cmath>

namespace lingam {

// log1p_unit_with(y, rcp) takes the reciprocal estimate as a parameter (the
// host test runs it with deliberately perturbed ones); log1p_unit uses the
// hardware estimate on the device and a division on the host.  Every
// product-sum is an explicit fused multiply-add and nothing else is
// contracted, so both builds perform the same operations in the same order.
template <class Rcp>
__host__ __device__ inline double log1p_unit_with(double y, Rcp rcp) {
#if defined(__clang__)
#pragma clang fp contract(off)
#endif
  const double z = 1.0 + y;            // in [1, 2]
  const double c = (1.0 - z) + y;      // exact: z + c = 1 + y (|y| <= 1)
  const bool hi = z > 1.4142135623730951;
  const double m = hi ? 0.5 * z : z;   // exact
  const double f = m - 1.0;            // exact (m within a factor 2 of 1)
  // s = f / (2 + f) from a reciprocal estimate r0 of relative error e0 and
  // two Newton steps on the quotient, each multiplying its relative error
  // by e0: 2^-24 (the hardware estimate on this range) -> 2^-48 -> 2^-72
  const double dd = 2.0 + f;           // exact
  const double r0 = rcp(dd);
  double s = f * r0;
  s = std::fma(r0, std::fma(-s, dd, f), s);
  s = std::fma(r0, std::fma(-s, dd, f), s);
  const double w = s * s;
  // q = 2/3 + 2/5 w + ... + 2/19 w^8, Horner from the highest power
  double q = 2.0 / 19.0;
  q = std::fma(q, w, 2.0 / 17.0);
  q = std::fma(q, w, 2.0 / 15.0);
  q = std::fma(q, w, 2.0 / 13.0);
  q = std::fma(q, w, 2.0 / 11.0);
  q = std::fma(q, w, 2.0 / 9.0);
  q = std::fma(q, w, 2.0 / 7.0);
  q = std::fma(q, w, 2.0 / 5.0);
  q = std::fma(q, w, 2.0 / 3.0);
  // 2 atanh(s) = 2 s + s w q, and 2 s = f - s f with s f = hfsq (1 - s),
  // hfsq = f^2 / 2: log(m) = f - (hfsq - s (hfsq + w q)), whose leading term
  // f is exact and whose correction is at most f / 2 of the result
  const double hfsq = (0.5 * f) * f;
  const double lm = f - std::fma(-s, std::fma(w, q, hfsq), hfsq);   // log(m)
  // log(z + c) = log z + c / z to first order; 1.5 - z / 2 is within 13%
  // of 1/z on [1, 2], far more than c (at most half an ulp of z) needs
  const double corr = c * std::fma(-0.5, z, 1.5);
  return (hi ? lm + 0.6931471805599453 : lm) + corr;
}

struct RcpEstimate {
  __host__ __device__ double operator()(double x) const {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(x);    // v_rcp_f64
#else
    return 1.0 / x;
#endif
  }
};

__host__ __device__ inline double log1p_unit(double y) { return log1p_unit_with(y, RcpEstimate{}); }

}  // namespace lingam

// Device math for kernel-entry evaluation on gfx950.
//
// Kernel entries need kappa(r) for r = |x - y| >= 0 and an argument of exp
// that is never positive, so the general-purpose libm paths (denormal
// rescaling, overflow and NaN handling) are unnecessary.  These routines are
// written from the textbook constructions:
//   sqrt: hardware reciprocal-square-root estimate, one Goldschmidt step
//         (simultaneous iteration for sqrt and 1/(2 sqrt)) and one Newton
//         correction of the residual r2 - s^2; r2 == 0 maps to ~3e-151.
//   exp2: split t = n + f with n = rint(t), |f| <= 1/2; 2^f from the Taylor
//         series of exp(f ln 2) to degree 12 (truncation < 2^-52 relative on
//         |f| <= 1/2), evaluated by Horner; scale by 2^n with ldexp, which
//         underflows to 0 for very negative n.
// Their error is a few ulps, far below any construction tolerance; the
// parity tests compare with the oracle's libm values at 1e-13 relative.
#pragma once

#include <hip/hip_runtime.h>

namespace h2dev {

__device__ __forceinline__ double sqrt_nonneg(double r2) {
  // A floor far below the ulp of any squared distance that is not exactly 0
  // keeps the estimate finite at r2 == 0 (sqrt(2^-1000) ~ 3e-151 -> kappa = 1).
  r2 += 0x1p-1000;
  const double y = __builtin_amdgcn_rsq(r2);  // ~ 1/sqrt(r2)
  double s = r2 * y;                         // ~ sqrt(r2)
  double h = 0.5 * y;                        // ~ 1/(2 sqrt(r2))
  const double e = __builtin_fma(-h, s, 0.5);
  s = __builtin_fma(s, e, s);
  h = __builtin_fma(h, e, h);
  const double d = __builtin_fma(-s, s, r2);
  return __builtin_fma(d, h, s);
}

// 2^t for t <= 0 (any finite t <= 0; results below the smallest subnormal are 0).
// Coefficients c_k = (ln 2)^k / k!, k = 0..12, correctly rounded to double.
__device__ __forceinline__ double exp2_nonpos(double t) {
  const double n = __builtin_rint(t);
  const double f = t - n;  // exact, |f| <= 1/2
  double p = 0x1.c3bd650fc2986p-36;     // k = 12
  p = __builtin_fma(p, f, 0x1.e8cac7351bb25p-32);  // 11
  p = __builtin_fma(p, f, 0x1.e4cf5158b8ecap-28);  // 10
  p = __builtin_fma(p, f, 0x1.b5253d395e7c4p-24);  // 9
  p = __builtin_fma(p, f, 0x1.62c0223a5c824p-20);  // 8
  p = __builtin_fma(p, f, 0x1.ffcbfc588b0c7p-17);  // 7
  p = __builtin_fma(p, f, 0x1.430912f86c787p-13);  // 6
  p = __builtin_fma(p, f, 0x1.5d87fe78a6731p-10);  // 5
  p = __builtin_fma(p, f, 0x1.3b2ab6fba4e77p-7);   // 4
  p = __builtin_fma(p, f, 0x1.c6b08d704a0c0p-5);   // 3
  p = __builtin_fma(p, f, 0x1.ebfbdff82c58fp-3);   // 2
  p = __builtin_fma(p, f, 0x1.62e42fefa39efp-1);   // 1
  p = __builtin_fma(p, f, 1.0);                    // 0
  return __builtin_amdgcn_ldexp(p, static_cast<int>(__builtin_fmax(n, -2048.0)));
}

// log2(e)
constexpr double kLog2e = 0x1.71547652b82fep+0;

}  // namespace h2dev

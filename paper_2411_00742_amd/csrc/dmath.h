// FP64 exp and log for the per-step rate laws, written for register economy
// inside long time loops on gfx950.
//
// Both use textbook constructions:
//   exp(x): x = k ln2 + r with |r| <= ln2/2 (Cody-Waite two-term ln2), then
//           the Taylor series of e^r to degree 13 (truncation < 1e-17
//           relative), scaled by 2^k with v_ldexp_f64;
//   log(x): x = m 2^e with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1),
//           log m = 2 atanh(s) = 2 (s + s^3/3 + ... + s^23/23) (truncation
//           < 1e-17 relative), plus e ln2 in two terms.
// Coefficients are 1/n! and 1/(2n+1), held in a __constant__ table and read
// through a pointer the optimizer cannot see through, so each call loads them
// with scalar loads instead of the compiler hoisting ~40 FP64 constants into
// vector registers for the whole enclosing loop (gfx9 VOP3 instructions take
// no 64-bit literal operands).
#pragma once

#include <hip/hip_runtime.h>

namespace pbe {
namespace dev {

struct DMathTable {
    double inv_fact[14];     // 1/0!, 1/1!, ..., 1/13!
    double inv_odd[12];      // 1/1, 1/3, ..., 1/23
    double ln2_hi, ln2_lo, log2e, pad;
};

__constant__ DMathTable g_dmath = {
    {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040, 1.0 / 40320, 1.0 / 362880,
     1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600, 1.0 / 6227020800.0},
    {1.0, 1.0 / 3, 1.0 / 5, 1.0 / 7, 1.0 / 9, 1.0 / 11, 1.0 / 13, 1.0 / 15, 1.0 / 17, 1.0 / 19, 1.0 / 21, 1.0 / 23},
    // ln2_hi = ln 2 truncated to 32 significant bits (k*ln2_hi exact for |k| < 2^21),
    // ln2_lo = ln 2 - ln2_hi rounded to double; log2e = 1/ln 2 rounded
    0.6931471803691238, 1.9082149292705877e-10, 1.4426950408889634, 0.0};

__device__ __forceinline__ const DMathTable* dmath_table() {
    const DMathTable* t = &g_dmath;
    asm volatile("" : "+s"(t));
    return t;
}

// e^x for finite x; underflows to 0 below -745, overflows to +inf above 709.8
__device__ __forceinline__ double exp64(double x) {
    const DMathTable* T = dmath_table();
    if (x < -745.2) return 0.0;
    if (x > 709.79) return __builtin_huge_val();
    const double k = rint(x * T->log2e);
    const double r = fma(-k, T->ln2_lo, fma(-k, T->ln2_hi, x));
    double p = T->inv_fact[13];
#pragma unroll
    for (int n = 12; n >= 0; --n) p = fma(p, r, T->inv_fact[n]);
    return __builtin_amdgcn_ldexp(p, (int)k);
}

// natural log for x > 0 (normal or subnormal); log(0) = -inf, NaN for x < 0
__device__ __forceinline__ double log64(double x) {
    const DMathTable* T = dmath_table();
    if (!(x > 0.0)) return x == 0.0 ? -__builtin_huge_val() : __builtin_nan("");
    int e = __builtin_amdgcn_frexp_exp(x);          // x = m 2^e, m in [0.5, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    if (m < 0.70710678118654752440) {
        m = m + m;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double s2 = s * s;
    double p = T->inv_odd[11];
#pragma unroll
    for (int n = 10; n >= 0; --n) p = fma(p, s2, T->inv_odd[n]);
    const double de = (double)e;
    return fma(de, T->ln2_hi, fma(de, T->ln2_lo, 2.0 * s * p));
}

}  // namespace dev
}  // namespace pbe

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
// Coefficients are 1/n! and 1/(2n+1).  They sit in a __constant__ table read
// through a pointer in the constant address space that an empty asm makes
// opaque at every call: the reads are then scalar loads into SGPRs inside the
// caller's loop, instead of ~40 FP64 constants hoisted into vector registers
// for the whole time loop (gfx9 VOP3 instructions take no 64-bit literals).
#pragma once

#include <hip/hip_runtime.h>

namespace pbe {
namespace dev {

// [0..13] 1/n! for n = 13 .. 0; [14..25] 1/(2n+1) for n = 11 .. 0;
// [26] ln2_hi = ln 2 truncated to 32 significant bits (k*ln2_hi exact for |k| < 2^21),
// [27] ln2_lo = ln 2 - ln2_hi rounded, [28] 1/ln 2, [29] sqrt(1/2)
static __constant__ double g_dmath[32] = {
    1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0, 1.0 / 362880.0, 1.0 / 40320.0,
    1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0, 1.0,
    1.0 / 23.0, 1.0 / 21.0, 1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0,
    1.0 / 5.0, 1.0 / 3.0, 1.0,
    0.6931471803691238, 1.9082149292705877e-10, 1.4426950408889634, 0.70710678118654752440, 0.0, 0.0};

typedef const __attribute__((address_space(4))) double cdouble;

__device__ __forceinline__ const cdouble* dmath_table() {
    const cdouble* t = (const cdouble*)(g_dmath);
    asm volatile("" : "+s"(t));
    return t;
}

// p*r + c with the coefficient c in scalar registers, as one VOP3 v_fma_f64.
// Written out because instruction selection otherwise picks the two-address
// v_fmac_f64 and first copies c into a vector register pair (two extra VALU
// moves per Horner step).
__device__ __forceinline__ double fma_sc(double p, double r, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(p), "v"(r), "s"(c));
    return d;
}

// a/b for b in [2^-1000, 2^1000] in magnitude: hardware reciprocal, one
// Newton step on it, then one residual correction of the quotient (within
// about an ulp of the correctly rounded a/b).  Six VALU operations against
// eleven for the correctly rounded division with its scaling and fix-up.
__device__ __forceinline__ double div_near(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}
// a/b for any b: div_near inside its range, the exact division outside it
// (a wave-uniform b takes a scalar branch)
__device__ __forceinline__ double div_fast(double a, double b) {
    const double m = __builtin_fabs(b);
    if (m >= 0x1p-1000 && m <= 0x1p1000) return div_near(a, b);
    return a / b;
}

// e^x for finite x; underflows to 0 below -745, overflows to +inf above 709.8
__device__ __forceinline__ double exp64(double x) {
    if (x < -745.2) return 0.0;
    if (x > 709.79) return __builtin_huge_val();
    const cdouble* T = dmath_table();
    const double k = rint(x * T[28]);
    const double r = fma(-k, T[27], fma(-k, T[26], x));
    // Taylor series of e^r, Horner from 1/13! down to 1/0!
    double p = fma(T[0], r, T[1]);
#pragma unroll
    for (int n = 2; n < 14; ++n) p = fma_sc(p, r, T[n]);
    return __builtin_amdgcn_ldexp(p, (int)k);
}

// natural log for x > 0 (normal or subnormal); log(0) = -inf, NaN for x < 0
__device__ __forceinline__ double log64(double x) {
    if (!(x > 0.0)) return x == 0.0 ? -__builtin_huge_val() : __builtin_nan("");
    const cdouble* T = dmath_table();
    int e = __builtin_amdgcn_frexp_exp(x);          // x = m 2^e, m in [0.5, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    if (m < T[29]) {
        m = m + m;
        e -= 1;
    }
    const double s = div_near(m - 1.0, m + 1.0);   // m + 1 lies in [1.7, 2.5]
    const double s2 = s * s;
    // 2 atanh(s) = 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23), Horner in s^2
    double p = fma(T[14], s2, T[15]);
#pragma unroll
    for (int n = 16; n < 26; ++n) p = fma_sc(p, s2, T[n]);
    const double de = (double)e;
    return fma(de, T[26], fma(de, T[27], 2.0 * s * p));
}

}  // namespace dev
}  // namespace pbe

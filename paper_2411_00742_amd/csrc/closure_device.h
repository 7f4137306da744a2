// Learned rate closure on the device (gfx950): a 3-64-64-2 tanh network that
// maps (S, T, log10 mu_2) to (ln G0, ln B) in place of the empirical rate laws
// (the empirical hybrid model of Sec. 4.2, Fig. 5a).
//
// Two evaluation paths, both run by one 64-lane wavefront per call:
//   bf16  weights and activations in bfloat16 on the matrix cores
//         (v_mfma_f32_16x16x16_bf16 / 16x16x32_bf16, fp32 accumulation);
//   fp64  plain FP64 vector arithmetic, one hidden unit per lane.
// The bf16 path is written in transposed form, out^T = W * in^T: the weights
// are the A operand (16 output units per tile) and the network inputs are the
// B operand's columns.  Column 0 carries the network input; columns 1, 2 and 3
// optionally carry the forward tangents d/dz0, d/dz1 and d/dz2 used by the adjoint;
// in the batched backward kernel all 16 columns are different inputs.  The
// host packs every A operand so that the k index of a lane's elements matches
// where the previous layer's accumulator left the same unit in that lane, so
// activations never move between lanes (see pack_closure).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dmath.h"
#include "fvm1d_device.h"
#include "pbe_internal.h"

namespace pbe {

constexpr int kMlpH = 64;
constexpr int kMlpNW = 4546;     // weights in the blob
constexpr int kMlpNC = 18;       // constants after the weights
// blob offsets: W1[64][3] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 256, kOffB2 = 4352, kOffW3 = 4416, kOffB3 = 4544;
// constants: in_shift[3] in_scale[3] out_shift[2] out_scale[2] lo[3] hi[3] s_min lnG0_max
enum { kCInShift = 0, kCInScale = 3, kCOutShift = 6, kCOutScale = 8, kCLo = 10, kCHi = 13, kCSmin = 16,
       kCLnG0Max = 17 };

namespace dev {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest with ties to even: the gfx950
// conversion instruction (v_cvt_pk_bf16_f32, two values per instruction)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    return __builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_bits(x) << 16); }

// tanh in fp32 from the hardware base-2 exponential: tanh|x| = (1 - e)/(1 + e),
// e = exp(-2|x|), with the hardware reciprocal of 1 + e in [1, 2] (about an ulp;
// the result is rounded to bfloat16, 2^-9 relative, before it is used)
__device__ __forceinline__ float tanh32(float x) {
    const float e = __builtin_amdgcn_exp2f(-2.8853900817779268f * __builtin_fabsf(x));
    return __builtin_copysignf((1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e), x);
}
// tanh in fp64 from exp64 (absolute error ~1e-16)
__device__ __forceinline__ double tanh64(double x) {
    const double e = exp64(-2.0 * __builtin_fabs(x));
    return __builtin_copysign((1.0 - e) / (1.0 + e), x);
}

__device__ __forceinline__ f32x4 mfma16(uint2 a, s16x4 b, f32x4 c) {
    s16x4 av;
    av.x = (short)(a.x & 0xFFFFu); av.y = (short)(a.x >> 16); av.z = (short)(a.y & 0xFFFFu); av.w = (short)(a.y >> 16);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma32(uint4 a, s16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// B operand of a 32-deep k-step from two accumulator tiles: elements 0-3 from
// tile lo, 4-7 from tile hi (the host packs A with the same k order).
__device__ __forceinline__ s16x8 pack_b(const float (&lo)[4], const float (&hi)[4]) {
    s16x8 b;
    b[0] = (short)bf16_bits(lo[0]); b[1] = (short)bf16_bits(lo[1]);
    b[2] = (short)bf16_bits(lo[2]); b[3] = (short)bf16_bits(lo[3]);
    b[4] = (short)bf16_bits(hi[0]); b[5] = (short)bf16_bits(hi[1]);
    b[6] = (short)bf16_bits(hi[2]); b[7] = (short)bf16_bits(hi[3]);
    return b;
}

// value of v in lane 16*(lane/16), i.e. in column 0 of this lane's rows
__device__ __forceinline__ float from_column0(float v) {
    const int src = (int)(threadIdx.x & 48u);
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Hidden activation of one accumulator tile.  Column 0: t = tanh(pre);
// tangent columns 1..3 (TAN): pre * (1 - t0^2) with t0 the column-0 value of
// the same unit; other columns stay 0 (their pre-activation is 0).
template <bool TAN>
__device__ __forceinline__ void activate(f32x4 d, float (&h)[4], float (&t)[4]) {
    const int c = threadIdx.x & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float th = tanh32(d[e]);
        t[e] = th;
        if (TAN) {
            const float t0 = from_column0(th);
            h[e] = c == 0 ? th : d[e] * (1.0f - t0 * t0);
        } else {
            h[e] = th;
        }
    }
}

__device__ __forceinline__ f32x4 bias_tile(const float* b, int t, bool use) {
    const int g = threadIdx.x >> 4;
    const float4 v = *reinterpret_cast<const float4*>(b + 16 * t + 4 * g);
    f32x4 r;
    r[0] = use ? v.x : 0.0f; r[1] = use ? v.y : 0.0f; r[2] = use ? v.z : 0.0f; r[3] = use ? v.w : 0.0f;
    return r;
}

// bf16 network on one input (column 0).  With TAN, column 1 + i carries
// d/dz_i and dy[o][i] returns dy_o/dz_i (i = 0, 1, 2).
// All lanes must be active.  Results are wave-uniform.
template <bool TAN>
__device__ __forceinline__ void net_bf16(const ClosureDev& cd, double z0, double z1, double z2, double (&y)[2],
                                         double (&dy)[2][3]) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, g = lane >> 4;
    // layer-1 B operand (16 deep: element e of lane group g is input k = 4g + e)
    s16x4 b1 = {0, 0, 0, 0};
    const bool col0 = (c == 0) && (g == 0);
    b1.x = col0 ? (short)bf16_bits((float)z0) : (TAN && c == 1 && g == 0 ? (short)0x3F80 : (short)0);
    b1.y = col0 ? (short)bf16_bits((float)z1) : (TAN && c == 2 && g == 0 ? (short)0x3F80 : (short)0);
    b1.z = col0 ? (short)bf16_bits((float)z2) : (TAN && c == 3 && g == 0 ? (short)0x3F80 : (short)0);
    float h[4][4], tt[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const f32x4 d = mfma16(cd.a1[t * 64 + lane], b1, bias_tile(cd.bias, t, c == 0));
        activate<TAN>(d, h[t], tt);
    }
    s16x8 bk[2] = {pack_b(h[0], h[1]), pack_b(h[2], h[3])};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 d = bias_tile(cd.bias + kMlpH, t, c == 0);
        d = mfma32(cd.a2[(t * 2 + 0) * 64 + lane], bk[0], d);
        d = mfma32(cd.a2[(t * 2 + 1) * 64 + lane], bk[1], d);
        activate<TAN>(d, h[t], tt);
    }
    bk[0] = pack_b(h[0], h[1]);
    bk[1] = pack_b(h[2], h[3]);
    f32x4 o;
    o[0] = (c == 0 && g == 0) ? cd.bias[2 * kMlpH] : 0.0f;
    o[1] = (c == 0 && g == 0) ? cd.bias[2 * kMlpH + 1] : 0.0f;
    o[2] = 0.0f;
    o[3] = 0.0f;
    o = mfma32(cd.a3[lane], bk[0], o);
    o = mfma32(cd.a3[64 + lane], bk[1], o);
    y[0] = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(o[0]), 0));
    y[1] = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(o[1]), 0));
    if (TAN) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            dy[0][i] = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(o[0]), 1 + i));
            dy[1][i] = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(o[1]), 1 + i));
        }
    }
}

__device__ __forceinline__ double bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// fp64 network on one input, hidden unit j in lane j.  Same outputs as net_bf16.
template <bool TAN>
__device__ __forceinline__ void net_fp64(const ClosureDev& cd, double z0, double z1, double z2, double (&y)[2],
                                         double (&dy)[2][3]) {
#pragma clang fp contract(off)
    const int j = threadIdx.x & 63;
    const double* w = cd.w64;
    const double w10 = w[kOffW1 + 3 * j], w11 = w[kOffW1 + 3 * j + 1], w12 = w[kOffW1 + 3 * j + 2];
    double a1 = w[kOffB1 + j];
    a1 = a1 + w10 * z0;
    a1 = a1 + w11 * z1;
    a1 = a1 + w12 * z2;
    const double h1 = tanh64(a1);
    const double s1 = 1.0 - h1 * h1;
    const double t10 = w10 * s1, t11 = w11 * s1, t12 = w12 * s1;
    double a2 = w[kOffB2 + j], u0 = 0.0, u1 = 0.0, u2 = 0.0;
    for (int i = 0; i < kMlpH; ++i) {
        const double wij = w[kOffW2 + i * kMlpH + j];
        a2 = a2 + wij * bcast(h1, i);
        if (TAN) {
            u0 = u0 + wij * bcast(t10, i);
            u1 = u1 + wij * bcast(t11, i);
            u2 = u2 + wij * bcast(t12, i);
        }
    }
    const double h2 = tanh64(a2);
    const double s2 = 1.0 - h2 * h2;
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        const double w3 = w[kOffW3 + o * kMlpH + j];
        y[o] = w[kOffB3 + o] + wave_sum(w3 * h2);
        if (TAN) {
            dy[o][0] = wave_sum(w3 * (u0 * s2));
            dy[o][1] = wave_sum(w3 * (u1 * s2));
            dy[o][2] = wave_sum(w3 * (u2 * s2));
        }
    }
}

// Closure rates for one simulation step.  S = C/Csat - 1 (unclipped),
// x = (S, T, log10 mu2).  Inside the box the network gives G0 [um/s] and B;
// outside it the plain power law stands in (fallback).  The network's log
// growth rate is trusted up to lnG0_max and held there above it (clamped:
// no derivative through G0), which bounds the steps a CFL-limited solve
// takes.  With TAN also returns the normalised inputs and dy/dz for the adjoint.
struct ClosureRates {
    double G0, B, S;
    bool fallback, clamped;
    double z[3];
    double dy[2][3];
};

template <bool TAN, int PREC>
__device__ __forceinline__ ClosureRates closure_rates(const ClosureDev& cd, const Process& p, const SimParams& q,
                                                      double C, double t, double mu2) {
#pragma clang fp contract(off)
    ClosureRates r;
    const double T = temperature(q, t);
    const double* k = cd.c;
    r.S = uniform(div_fast(C, solubility(p, T)) - 1.0);
    const double x2 = mu2 > 0.0 ? log64(mu2) / 2.302585092994046 : 0.0;
    const double x[3] = {r.S, T, x2};
    bool inside = r.S > uniform(k[kCSmin]) && mu2 > 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) inside = inside && x[i] >= uniform(k[kCLo + i]) && x[i] <= uniform(k[kCHi + i]);
    r.fallback = uniform((int)!inside) != 0;
    r.clamped = false;
#pragma unroll
    for (int i = 0; i < 3; ++i) r.dy[0][i] = r.dy[1][i] = 0.0;
    if (r.fallback) {
        r.z[0] = r.z[1] = r.z[2] = 0.0;
        const Process pp{PBE_LAW_POWER, p.scheme, p.sol_law, p.cs0, p.cs1, p.alpha, p.cfl, p.dt_max, p.t_end};
        const Rates pr = rates_plain(pp, q, C, t);
        r.G0 = pr.G0;
        r.B = pr.B;
        return r;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) r.z[i] = uniform((x[i] - uniform(k[kCInShift + i])) * uniform(k[kCInScale + i]));
    double y[2];
    if (PREC == kClosureFp64)
        net_fp64<TAN>(cd, r.z[0], r.z[1], r.z[2], y, r.dy);
    else
        net_bf16<TAN>(cd, r.z[0], r.z[1], r.z[2], y, r.dy);
    const double lnG = uniform(uniform(k[kCOutShift]) + uniform(k[kCOutScale]) * uniform(y[0]));
    const double lnG_max = uniform(k[kCLnG0Max]);
    r.clamped = lnG > lnG_max;
    r.G0 = uniform(exp64(r.clamped ? lnG_max : lnG));
    r.B = uniform(exp64(uniform(k[kCOutShift + 1]) + uniform(k[kCOutScale + 1]) * uniform(y[1])));
    if (TAN) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            r.dy[0][i] = uniform(r.dy[0][i]);
            r.dy[1][i] = uniform(r.dy[1][i]);
        }
    }
    return r;
}

// In-the-loop correction (Sec. 4.2, Fig. 5b), after a growth step with
// Courant factor c = dt G0/dL > 0: each interior face i+1/2 (0 <= i <= N-2)
// carries Y = sigma nu (W2 . tanh(W1 x + b1) + b2) with x the four cells
// f_{i-1..i+2} over sigma = their largest magnitude (cells outside the domain,
// including the pad slots, read 0) and nu = c (1 + gamma L_face); then
// f_i += Y_{i-1/2} - Y_{i+1/2}.  The end faces carry nothing.  wl: the sim's
// PBE_CORR_NW weights W1[8][5] b1[8] W2[8] b2, staged in LDS (every read is
// a broadcast).  One wavefront per simulation.  The slots are evaluated one
// after the other (each slot's window is tied to the previous slot's result),
// which keeps the eight hidden units of one face live at a time.
template <int K>
__device__ __forceinline__ void correct_step(double (&u)[K], LaneGeom g, double c, int N, const double* wl) {
    constexpr int H = PBE_CORR_H;
    asm volatile("" : "+v"(g.xb));
    const double uL = shift_from_left(u[K - 1], 0.0);                        // cell left of slot 0
    const double uR = shift_from_right(u[0], 0.0);                           // cell right of slot K-1
    const double uR2 = shift_from_right(K >= 2 ? u[K >= 2 ? 1 : 0] : uR, 0.0);   // two right of slot K-1
    double Y[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double xc = g.xb + (double)k;   // cell index of slot k
        double fm1 = (xc - 1.0 >= 0.0) ? (k >= 1 ? u[k >= 1 ? k - 1 : 0] : uL) : 0.0;
        double f0 = u[k];
        double fp1 = k + 1 < K ? u[k + 1 < K ? k + 1 : 0] : uR;
        double fp2 = k + 2 < K ? u[k + 2 < K ? k + 2 : 0] : (k + 2 == K ? uR : uR2);
        if (k > 0) asm volatile("" : "+v"(fm1), "+v"(f0), "+v"(fp1), "+v"(fp2) : "v"(Y[k > 0 ? k - 1 : 0]));
        const double sigma = fmax(fmax(__builtin_fabs(fm1), __builtin_fabs(f0)),
                                  fmax(__builtin_fabs(fp1), __builtin_fabs(fp2)));
        const bool ok = xc >= 0.0 && xc <= (double)(N - 2) && sigma > 0.0;
        const double inv = ok ? 1.0 / sigma : 0.0;
        const double nu = c * fma(g.gdL, xc + 1.0, 1.0);
        const double x0 = fm1 * inv, x1 = f0 * inv, x2 = fp1 * inv, x3 = fp2 * inv;
        double y = wl[7 * H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            double a = wl[5 * H + h];
            a = fma(wl[h * 5 + 0], x0, a);
            a = fma(wl[h * 5 + 1], x1, a);
            a = fma(wl[h * 5 + 2], x2, a);
            a = fma(wl[h * 5 + 3], x3, a);
            a = fma(wl[h * 5 + 4], nu, a);
            y = fma(wl[6 * H + h], tanh64(a), y);
        }
        Y[k] = ok ? sigma * nu * y : 0.0;
    }
    const double Y_in = shift_from_left(Y[K - 1], 0.0);   // face left of slot 0
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] += (k == 0 ? Y_in : Y[k >= 1 ? k - 1 : 0]) - Y[k];
}

}  // namespace dev
}  // namespace pbe

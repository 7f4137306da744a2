// Learned-closure kernels: operand packing, a standalone forward (for tests),
// the batched weight gradient, its deterministic reduction and Adam.
//
// Weight gradient.  The adjoint sweep leaves one row per (simulation, step):
// the normalised network input z (3) and the cotangent ybar (2) of the
// network output at that step (zero where the plain law stood in).  The
// gradient of the loss with respect to the weights is sum_rows J_W(z)^T ybar,
// a contraction over all rows (about 1.5e7 for 4096 simulations x 3600 steps):
// each wavefront re-runs the forward pass on 16 rows at a time (the rows are
// the 16 columns of the B operand), back-propagates, and accumulates
// dW2 = delta2 h1^T and dW1 = delta1 z^T on the matrix cores with the row
// index as the contraction dimension.  Per-wave partial gradients are summed
// in a fixed order by a second kernel, so the result does not depend on
// scheduling.
#include <algorithm>
#include <cmath>

#include "closure_device.h"
#include "pbe_internal.h"

namespace pbe {
namespace {

using namespace dev;

__device__ __forceinline__ uint16_t bf16_of(float x) { return (uint16_t)bf16_bits(x); }

// k index of element e (0..7) of lane group g in k-step s of a 64-deep
// contraction: elements 0-3 and 4-7 come from accumulator tiles 2s and 2s+1,
// where a lane of group g holds units 4g..4g+3 of the tile.
__device__ __forceinline__ int kappa(int s, int g, int e) { return 16 * (2 * s + e / 4) + 4 * g + (e & 3); }

struct PackOut {
    double* w64;
    uint16_t* a1;
    uint16_t* a2;
    uint16_t* a3;
    uint16_t* a2t;
    float* bias;
    float* w3r;
    double* c;
};

__global__ void k_pack_closure(const float* __restrict__ blob, PackOut o) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    const float* W1 = blob + kOffW1;
    const float* W2 = blob + kOffW2;
    const float* W3 = blob + kOffW3;
    // fp64 copy with W2 transposed
    for (int i = tid; i < kMlpNW; i += nth) {
        double v;
        if (i >= kOffW2 && i < kOffB2) {
            const int q = i - kOffW2, a = q / kMlpH, b = q % kMlpH;   // W2T[a][b] = W2[b][a]
            v = (double)W2[b * kMlpH + a];
        } else {
            v = (double)blob[i];
        }
        o.w64[i] = v;
    }
    // layer 1: 4 tiles x 64 lanes x 4 elements, k = 4g + e
    for (int i = tid; i < 4 * 64 * 4; i += nth) {
        const int t = i / 256, l = (i / 4) % 64, e = i % 4;
        const int r = l % 16, g = l / 16, k = 4 * g + e;
        o.a1[i] = k < 3 ? bf16_of(W1[(16 * t + r) * 3 + k]) : (uint16_t)0;
    }
    // layer 2 and its transpose: [tile][k-step][lane][8]
    for (int i = tid; i < 4 * 2 * 64 * 8; i += nth) {
        const int t = i / 1024, s = (i / 512) % 2, l = (i / 8) % 64, e = i % 8;
        const int r = l % 16, g = l / 16, k = kappa(s, g, e);
        o.a2[i] = bf16_of(W2[(16 * t + r) * kMlpH + k]);
        o.a2t[i] = bf16_of(W2[k * kMlpH + 16 * t + r]);
    }
    // layer 3: rows 0 and 1 of a single tile
    for (int i = tid; i < 2 * 64 * 8; i += nth) {
        const int s = i / 512, l = (i / 8) % 64, e = i % 8;
        const int r = l % 16, g = l / 16, k = kappa(s, g, e);
        o.a3[i] = r < 2 ? bf16_of(W3[r * kMlpH + k]) : (uint16_t)0;
    }
    for (int i = tid; i < 2 * kMlpH + 4; i += nth)
        o.bias[i] = i < kMlpH ? blob[kOffB1 + i] : i < 2 * kMlpH ? blob[kOffB2 + i - kMlpH]
                  : i < 2 * kMlpH + 2 ? blob[kOffB3 + i - 2 * kMlpH] : 0.0f;
    for (int i = tid; i < 2 * kMlpH; i += nth) o.w3r[i] = bf16_round(W3[i]);
    for (int i = tid; i < kMlpNC; i += nth) o.c[i] = (double)blob[kMlpNW + i];
}

// Standalone forward on raw inputs x[n][3] (no box): y[n][2], dy[n][2][3] = dy_o/dz_i.
__global__ __launch_bounds__(64) void k_closure_forward(ClosureDev cd, int n, const double* __restrict__ x,
                                                         double* __restrict__ y, double* __restrict__ dy) {
    for (int r = blockIdx.x; r < n; r += gridDim.x) {
        double z[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) z[i] = uniform((uniform(x[3 * r + i]) - cd.c[kCInShift + i]) * cd.c[kCInScale + i]);
        double yy[2], dd[2][3];
        if (cd.precision == PBE_MLP_FP64)
            net_fp64<true>(cd, z[0], z[1], z[2], yy, dd);
        else
            net_bf16<true>(cd, z[0], z[1], z[2], yy, dd);
        if (threadIdx.x == 0) {
            y[2 * r] = yy[0];
            y[2 * r + 1] = yy[1];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                dy[6 * r + i] = dd[0][i];
                dy[6 * r + 3 + i] = dd[1][i];
            }
        }
    }
}

// rows[r] = (z0, z1, z2, ybar0, ybar1) for r < n, zero rows up to row_cap; *steps = n
__global__ void k_stage_rows(int n, int row_cap, const double* __restrict__ z, const double* __restrict__ ybar,
                             double* __restrict__ rows, int32_t* __restrict__ steps) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *steps = n;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < row_cap; r += gridDim.x * blockDim.x) {
        double* q = rows + (size_t)r * 5;
        const bool in = r < n;
        q[0] = in ? z[3 * r] : 0.0;
        q[1] = in ? z[3 * r + 1] : 0.0;
        q[2] = in ? z[3 * r + 2] : 0.0;
        q[3] = in ? ybar[2 * r] : 0.0;
        q[4] = in ? ybar[2 * r + 1] : 0.0;
    }
}

__device__ __forceinline__ f32x4 mfma16r(s16x4 a, s16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16x16 tile held in accumulator layout (lane (c, g) element e = row 4g+e,
// column c) -> operand layout (lane (r, g) element e = row r, column 4g+e),
// rounded to bfloat16.  One wavefront per block.
__device__ __forceinline__ s16x4 transpose_bf16(float (*T)[17], const float (&v)[4]) {
    const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) T[4 * g + e][c] = v[e];
    __syncthreads();
    s16x4 r;
    r.x = (short)bf16_bits(T[c][4 * g + 0]);
    r.y = (short)bf16_bits(T[c][4 * g + 1]);
    r.z = (short)bf16_bits(T[c][4 * g + 2]);
    r.w = (short)bf16_bits(T[c][4 * g + 3]);
    return r;
}

// sum over the 16 columns of a lane group (lanes 16g..16g+15)
__device__ __forceinline__ float sum16(float v) {
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__global__ __launch_bounds__(64) void k_closure_grad_bf16(ClosureDev cd, const double* __restrict__ rows,
                                                           const int32_t* __restrict__ steps, int n_sims, int row_cap,
                                                           double* __restrict__ partial) {
    __shared__ float T[16][17];
    const int lane = threadIdx.x, c = lane & 15, g = lane >> 4;
    const int tiles_per_sim = (row_cap + 15) / 16;
    const int n_tiles = n_sims * tiles_per_sim;
    f32x4 gw2[4][4], gw1[4];
    float gb1[4][4], gb2[4][4], gw3[2][4][4], gb3[2] = {0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gw1[a] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gw2[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            gb1[a][b] = 0.0f; gb2[a][b] = 0.0f; gw3[0][a][b] = 0.0f; gw3[1][a][b] = 0.0f;
        }
    }
    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int s = tile / tiles_per_sim;
        const int m0 = (tile % tiles_per_sim) * 16;
        const int ns = uniform(steps[s]);
        if (m0 >= ns) continue;
        const double* base = rows + ((size_t)s * row_cap + m0) * 5;
        const bool valid = m0 + c < ns;
        double z[3], yb[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) z[i] = valid ? base[c * 5 + i] : 0.0;
        yb[0] = valid ? base[c * 5 + 3] : 0.0;
        yb[1] = valid ? base[c * 5 + 4] : 0.0;
        // forward on the 16 rows (columns)
        s16x4 b1;
        b1.x = g == 0 ? (short)bf16_bits((float)z[0]) : (short)0;
        b1.y = g == 0 ? (short)bf16_bits((float)z[1]) : (short)0;
        b1.z = g == 0 ? (short)bf16_bits((float)z[2]) : (short)0;
        b1.w = 0;
        float h1[4][4], t1[4][4], h2[4][4], t2[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f32x4 d = mfma16(cd.a1[t * 64 + lane], b1, bias_tile(cd.bias, t, true));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                t1[t][e] = tanh32(d[e]);
                h1[t][e] = bf16_round(t1[t][e]);
            }
        }
        s16x8 bk0 = pack_b(h1[0], h1[1]), bk1 = pack_b(h1[2], h1[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 d = bias_tile(cd.bias + kMlpH, t, true);
            d = mfma32(cd.a2[(t * 2 + 0) * 64 + lane], bk0, d);
            d = mfma32(cd.a2[(t * 2 + 1) * 64 + lane], bk1, d);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                t2[t][e] = tanh32(d[e]);
                h2[t][e] = bf16_round(t2[t][e]);
            }
        }
        // backward: delta2 = (W3^T ybar) * (1 - t2^2)
        const float y0 = (float)yb[0], y1 = (float)yb[1];
        float d2[4][4], d1[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int u = 16 * t + 4 * g + e;
                d2[t][e] = (cd.w3r[u] * y0 + cd.w3r[kMlpH + u] * y1) * (1.0f - t2[t][e] * t2[t][e]);
                gw3[0][t][e] += y0 * h2[t][e];
                gw3[1][t][e] += y1 * h2[t][e];
                gb2[t][e] += d2[t][e];
            }
        gb3[0] += g == 0 ? y0 : 0.0f;
        gb3[1] += g == 0 ? y1 : 0.0f;
        // delta1 = (W2^T delta2) * (1 - t1^2)
        bk0 = pack_b(d2[0], d2[1]);
        bk1 = pack_b(d2[2], d2[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 d = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            d = mfma32(cd.a2t[(t * 2 + 0) * 64 + lane], bk0, d);
            d = mfma32(cd.a2t[(t * 2 + 1) * 64 + lane], bk1, d);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                d1[t][e] = d[e] * (1.0f - t1[t][e] * t1[t][e]);
                gb1[t][e] += d1[t][e];
            }
        }
        // dW2 += delta2 h1^T and dW1 += delta1 z^T, contracting over the 16 rows
        s16x4 hT[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) hT[t] = transpose_bf16(T, h1[t]);
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) {
            const s16x4 a = transpose_bf16(T, d2[jt]);
#pragma unroll
            for (int it = 0; it < 4; ++it) gw2[jt][it] = mfma16r(a, hT[it], gw2[jt][it]);
        }
        // B operand of dW1: rows 4g..4g+3 of this tile, input component c (< 3)
        s16x4 bz;
        {
            short zz[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 4 * g + e;
                const double v = (c < 3 && m < ns) ? base[(4 * g + e) * 5 + (c < 3 ? c : 0)] : 0.0;
                zz[e] = (short)bf16_bits((float)v);
            }
            bz.x = zz[0]; bz.y = zz[1]; bz.z = zz[2]; bz.w = zz[3];
        }
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) gw1[jt] = mfma16r(transpose_bf16(T, d1[jt]), bz, gw1[jt]);
    }

    // write this wave's partial gradient
    double* out = partial + (size_t)blockIdx.x * kMlpNW;
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 16 * jt + 4 * g + e;
#pragma unroll
            for (int it = 0; it < 4; ++it) out[kOffW2 + j * kMlpH + 16 * it + c] = (double)gw2[jt][it][e];
            if (c < 3) out[kOffW1 + j * 3 + c] = (double)gw1[jt][e];
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = 16 * t + 4 * g + e;
            const float s1 = sum16(gb1[t][e]), s2 = sum16(gb2[t][e]);
            const float w30 = sum16(gw3[0][t][e]), w31 = sum16(gw3[1][t][e]);
            if (c == 0) {
                out[kOffB1 + u] = (double)s1;
                out[kOffB2 + u] = (double)s2;
                out[kOffW3 + u] = (double)w30;
                out[kOffW3 + kMlpH + u] = (double)w31;
            }
        }
    const double s0 = wave_sum((double)gb3[0]), s1 = wave_sum((double)gb3[1]);
    if (lane == 0) {
        out[kOffB3] = s0;
        out[kOffB3 + 1] = s1;
    }
}

// fp64 weight gradient: one row at a time, hidden unit j in lane j; dW2 is
// accumulated in LDS as acc[i][j] = dW2[i][j], so lane j touches column j.
__global__ __launch_bounds__(64) void k_closure_grad_fp64(ClosureDev cd, const double* __restrict__ rows,
                                                           const int32_t* __restrict__ steps, int n_sims, int row_cap,
                                                           double* __restrict__ partial) {
#pragma clang fp contract(off)
    __shared__ double acc[kMlpH * kMlpH];
    const int j = threadIdx.x;
    const double* w = cd.w64;
    for (int i = 0; i < kMlpH; ++i) acc[i * kMlpH + j] = 0.0;
    double gw1[3] = {0.0, 0.0, 0.0}, gb1 = 0.0, gb2 = 0.0, gw3[2] = {0.0, 0.0}, gb3[2] = {0.0, 0.0};
    const double w10 = w[kOffW1 + 3 * j], w11 = w[kOffW1 + 3 * j + 1], w12 = w[kOffW1 + 3 * j + 2];
    const double w30 = w[kOffW3 + j], w31 = w[kOffW3 + kMlpH + j];
    const int64_t n_rows = (int64_t)n_sims * row_cap;
    for (int64_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
        const int s = (int)(r / row_cap), m = (int)(r % row_cap);
        if (m >= uniform(steps[s])) continue;
        const double* q = rows + r * 5;
        const double z0 = uniform(q[0]), z1 = uniform(q[1]), z2 = uniform(q[2]);
        const double y0 = uniform(q[3]), y1 = uniform(q[4]);
        if (y0 == 0.0 && y1 == 0.0) continue;
        double a1 = w[kOffB1 + j];
        a1 = a1 + w10 * z0;
        a1 = a1 + w11 * z1;
        a1 = a1 + w12 * z2;
        const double h1 = tanh64(a1);
        double a2 = w[kOffB2 + j];
        for (int i = 0; i < kMlpH; ++i) a2 = a2 + w[kOffW2 + i * kMlpH + j] * bcast(h1, i);
        const double h2 = tanh64(a2);
        double d2 = w30 * y0;
        d2 = d2 + w31 * y1;
        d2 = d2 * (1.0 - h2 * h2);
        gw3[0] = gw3[0] + y0 * h2;
        gw3[1] = gw3[1] + y1 * h2;
        gb3[0] = gb3[0] + y0;
        gb3[1] = gb3[1] + y1;
        gb2 = gb2 + d2;
        // delta1_j = sum_i W2[i][j] delta2_i, with W2[i][j] = W2T[j][i]
        double d1 = 0.0;
        for (int i = 0; i < kMlpH; ++i) {
            const double d2i = bcast(d2, i);
            d1 = d1 + w[kOffW2 + j * kMlpH + i] * d2i;
            // dW2[i][j] += delta2_i h1_j
            acc[i * kMlpH + j] = acc[i * kMlpH + j] + d2i * h1;
        }
        d1 = d1 * (1.0 - h1 * h1);
        gb1 = gb1 + d1;
        gw1[0] = gw1[0] + d1 * z0;
        gw1[1] = gw1[1] + d1 * z1;
        gw1[2] = gw1[2] + d1 * z2;
    }
    __syncthreads();
    double* out = partial + (size_t)blockIdx.x * kMlpNW;
    for (int i = 0; i < kMlpH; ++i) out[kOffW2 + i * kMlpH + j] = acc[i * kMlpH + j];
    out[kOffW1 + 3 * j] = gw1[0];
    out[kOffW1 + 3 * j + 1] = gw1[1];
    out[kOffW1 + 3 * j + 2] = gw1[2];
    out[kOffB1 + j] = gb1;
    out[kOffB2 + j] = gb2;
    out[kOffW3 + j] = gw3[0];
    out[kOffW3 + kMlpH + j] = gw3[1];
    if (j == 0) {
        out[kOffB3] = gb3[0];
        out[kOffB3 + 1] = gb3[1];
    }
}

// out[k] = sum over b of partial[b][k], b ascending
__global__ void k_reduce_partials(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpNW) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * kMlpNW + k];
    out[k] = s;
}

// Adam (Kingma and Ba), the optimiser of Sec. 4.1 / App. C, on fp32 weights
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const double* __restrict__ g, int n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = (float)g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (__builtin_sqrtf(vi / c2) + eps);
}

}  // namespace

// packed operands take about 58 KB
size_t closure_pack_bytes() { return 65536; }

// Carve the packed operands out of `mem` (closure_pack_bytes(), 256-byte aligned) and fill them from a
// device blob of kMlpNW + kMlpNC floats.
hipError_t pack_closure(const float* d_blob, void* mem, int precision, ClosureDev* cd, hipStream_t st) {
    char* p = static_cast<char*>(mem);
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 15) & ~size_t(15);
        return r;
    };
    PackOut o;
    o.w64 = reinterpret_cast<double*>(take(sizeof(double) * kMlpNW));
    o.a1 = reinterpret_cast<uint16_t*>(take(2 * 4 * 64 * 4));
    o.a2 = reinterpret_cast<uint16_t*>(take(2 * 4 * 2 * 64 * 8));
    o.a2t = reinterpret_cast<uint16_t*>(take(2 * 4 * 2 * 64 * 8));
    o.a3 = reinterpret_cast<uint16_t*>(take(2 * 2 * 64 * 8));
    o.bias = reinterpret_cast<float*>(take(sizeof(float) * (2 * kMlpH + 4)));
    o.w3r = reinterpret_cast<float*>(take(sizeof(float) * 2 * kMlpH));
    o.c = reinterpret_cast<double*>(take(sizeof(double) * kMlpNC));
    hipLaunchKernelGGL(k_pack_closure, dim3(8), dim3(256), 0, st, d_blob, o);
    cd->w64 = o.w64;
    cd->a1 = reinterpret_cast<const uint2*>(o.a1);
    cd->a2 = reinterpret_cast<const uint4*>(o.a2);
    cd->a2t = reinterpret_cast<const uint4*>(o.a2t);
    cd->a3 = reinterpret_cast<const uint4*>(o.a3);
    cd->bias = o.bias;
    cd->w3r = o.w3r;
    cd->c = o.c;
    cd->precision = precision;
    return hipGetLastError();
}

hipError_t launch_closure_forward(const ClosureDev& cd, int n, const double* x, double* y, double* dy,
                                  hipStream_t st) {
    const int blocks = n < 2048 ? (n > 0 ? n : 1) : 2048;
    hipLaunchKernelGGL(k_closure_forward, dim3(blocks), dim3(64), 0, st, cd, n, x, y, dy);
    return hipGetLastError();
}

hipError_t launch_closure_grad(const ClosureDev& cd, const double* rows, const int32_t* steps, int n_sims,
                               int row_cap, double* partial, int n_blocks, double* out, hipStream_t st) {
    if (cd.precision == PBE_MLP_FP64)
        hipLaunchKernelGGL(k_closure_grad_fp64, dim3(n_blocks), dim3(64), 0, st, cd, rows, steps, n_sims, row_cap,
                           partial);
    else
        hipLaunchKernelGGL(k_closure_grad_bf16, dim3(n_blocks), dim3(64), 0, st, cd, rows, steps, n_sims, row_cap,
                           partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_partials, dim3((kMlpNW + 255) / 256), dim3(256), 0, st, partial, n_blocks, out);
    return hipGetLastError();
}

hipError_t launch_stage_rows(int n, int row_cap, const double* z, const double* ybar, double* rows, int32_t* steps,
                             hipStream_t st) {
    const int blocks = std::max(1, std::min(1024, (row_cap + 255) / 256));
    hipLaunchKernelGGL(k_stage_rows, dim3(blocks), dim3(256), 0, st, n, row_cap, z, ybar, rows, steps);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const double* g, int n, int step, float lr, float b1, float b2,
                       float eps, hipStream_t st) {
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace pbe

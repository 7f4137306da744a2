// 2D size-and-shape PBE (length L1 x width L2), Godunov dimensional splitting
// (paper Sec. 2.1: the update of Eq. (8) applied along each length in turn),
// SSP-RK3 per sweep, FP64, many simulations per launch (gfx950).
//
// One global step = three launches (captured in a graph by the host):
//   k_rows2d  L1 sweep: one wavefront per row, the row in registers exactly as
//             the 1D kernel holds a simulation (same stage code), in place; the
//             row passes through LDS on its way in and out so that every
//             global access is a contiguous 512-byte wave access;
//   k_cols2d  L2 sweep: a wavefront owns 64 adjacent columns and a segment of
//             rows; each lane marches down its column with the three SSP-RK3
//             stages pipelined in registers (stage s lags s rows), so every
//             load and store is a coalesced 512-byte row segment and no lane
//             talks to another.  Segments start 6 rows early (the stencil halo
//             of three stages); the sweep reads one buffer and writes the other,
//             with eight row loads in flight per wave.
//             It also sums the moments of the swept state per block;
//   k_final2d one wavefront per simulation: reduces the block moments in a fixed
//             order, applies the solute balance (Eq. (9) with mu_{1,2}), records
//             samples, and computes the next step's rates, CFL step (SI Eq. (S3))
//             and the corner nucleation ghosts.
#include "fvm1d_device.h"
#include "pbe_internal.h"

namespace pbe {
namespace {

using namespace dev;

// The row moves between HBM and registers through LDS: the wave reads and
// writes the row as 64 consecutive doubles per instruction (element e = lane +
// 64 i of the right-aligned row), and each lane takes its K consecutive cells
// from LDS.  Element e sits at (e / K) * P + e % K with P = K rounded up to odd,
// so the K-strided per-lane reads fall in distinct banks.
template <int K>
__device__ __forceinline__ void row_sweep(const Fvm2dArgs& a, int parity, int s, int j, double* lds) {
    const int lane = threadIdx.x;
    const int n1 = uniform(a.n1[s]);
    const int pad = 64 * K - n1;
    LaneGeom g;
    g.xb = (double)(lane * K - pad);
    g.gdL = 0.0;   // size-independent growth along each axis
    g.npad = min(max(pad - lane * K, 0), K);
    const int64_t o = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
    double* row = a.buf[parity] + o + (int64_t)j * n1;
    // nucleation: row 0 receives half the corner source through its L1 = 0 face
    const double ghost = j == 0 ? uniform(a.gh1[s]) : 0.0;
    const double c = uniform(a.c1[s]);
    constexpr int P = K | 1;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = lane + 64 * i;
        const int cell = e - pad;   // < n1 always; < 0 in the pad
        lds[(e / K) * P + e % K] = cell >= 0 ? row[cell] : 0.0;
    }
    __syncthreads();
    double u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = lds[lane * P + k];
    (void)fvm_step<K, PBE_SCHEME_SSPRK3>(u, g, c, ghost);
#pragma unroll
    for (int k = 0; k < K; ++k) lds[lane * P + k] = u[k];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = lane + 64 * i;
        const int cell = e - pad;
        if (cell >= 0) row[cell] = lds[(e / K) * P + e % K];
    }
}

template <int KLO>
__global__ __launch_bounds__(64) void k_rows2d(Fvm2dArgs a, int parity, int begin) {
    __shared__ double lds[64 * ((KLO + 7) | 1)];
    const int r = begin + (int)blockIdx.x;
    const int s = uniform(a.row_sim[r]);
    if (!uniform(a.active[s])) return;
    const int j = uniform(a.row_j[r]);
    const int K = uniform((a.n1[s] + 63) >> 6);
    switch (K - KLO) {
        case 0: row_sweep<KLO + 0>(a, parity, s, j, lds); break;
        case 1: row_sweep<KLO + 1>(a, parity, s, j, lds); break;
        case 2: row_sweep<KLO + 2>(a, parity, s, j, lds); break;
        case 3: row_sweep<KLO + 3>(a, parity, s, j, lds); break;
        case 4: row_sweep<KLO + 4>(a, parity, s, j, lds); break;
        case 5: row_sweep<KLO + 5>(a, parity, s, j, lds); break;
        case 6: row_sweep<KLO + 6>(a, parity, s, j, lds); break;
        case 7: row_sweep<KLO + 7>(a, parity, s, j, lds); break;
        default: break;
    }
}

// One SSP-RK3 stage running down a column: holds the last two inputs and the
// face value below them; fed the input at row r+1 it emits the stage output at row r.
struct ColStage {
    double im1, i0, Fm1;
};
__device__ __forceinline__ double col_face(double a, double b, double x) {
    return b + half_limited_slope(b - a, x - b);
}
__device__ __forceinline__ double col_feed(ColStage& st, double x, double c, double u0r, double wa, double wb,
                                           bool first, int r, int n2, double ghost) {
    const double F = col_face(st.im1, st.i0, x);
    const double v = st.i0 + c * (st.Fm1 - F);
    double out = first ? v : wa * u0r + wb * v;
    out = r < 0 ? ghost : (r >= n2 ? 0.0 : out);   // ghost rows below L2 = 0, nothing past L2_max
    st.im1 = st.i0;
    st.i0 = x;
    st.Fm1 = F;
    return out;
}

constexpr int kColAhead = 8;   // row loads in flight per wave in the column sweep

__global__ __launch_bounds__(64) void k_cols2d(Fvm2dArgs a, int parity) {
    const int b = blockIdx.x;
    const int s = uniform(a.cb_sim[b]);
    if (!uniform(a.active[s])) return;
    const int lane = threadIdx.x;
    const int n1 = uniform(a.n1[s]), n2 = uniform(a.n2[s]);
    const int col0 = uniform(a.cb_col0[b]), row0 = uniform(a.cb_row0[b]);
    const int row1 = min(row0 + a.seg, n2);
    const int i = col0 + lane;
    const bool valid = i < n1;
    const int64_t o = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
    const double* src = a.buf[parity] + o + (valid ? i : 0);
    double* dst = a.buf[parity ^ 1] + o + (valid ? i : 0);
    const double c = uniform(a.c2[s]);
    // column 0 receives the other half of the corner source through its L2 = 0 face
    const double ghost = i == 0 ? uniform(a.gh2[s]) : 0.0;
    const double d1 = uniform(a.L1[s]) / n1, d2 = uniform(a.L2[s]) / n2;
    const double L1c = (i + 0.5) * d1;

    ColStage s1{0.0, 0.0, 0.0}, s2{0.0, 0.0, 0.0}, s3{0.0, 0.0, 0.0};
    double u0_1 = 0.0, u0_2 = 0.0, u0_3 = 0.0;   // f^n at rows R-1, R-2, R-3
    double m00 = 0.0, m10 = 0.0, m01 = 0.0, m12 = 0.0;
    // Input rows are loaded kColAhead rows ahead of their use into a ring, so
    // a wave keeps that many row loads in flight instead of waiting on each
    // one; rows outside [0, n2) read a clamped in-range row and are replaced
    // by the ghost (below L2 = 0) or 0 (past L2_max).
    const int R0 = row0 - 6, R1 = row1 + 2;
    // (the ring holds the raw loads; the substitution is applied when a row is
    // consumed, so nothing waits on a load before its turn)
    auto load_row = [&](int R) -> double { return src[(int64_t)min(max(R, 0), n2 - 1) * n1]; };
    double ring[kColAhead];
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) ring[j] = load_row(R0 + j);
    for (int Rb = R0; Rb <= R1; Rb += kColAhead) {
#pragma unroll
        for (int j = 0; j < kColAhead; ++j) {
            const int R = Rb + j;
            if (R > R1) break;
            const double x = R < 0 ? ghost : (R >= n2 || !valid ? 0.0 : ring[j]);
            ring[j] = load_row(R + kColAhead);
            const double v1 = col_feed(s1, x, c, 0.0, 0.0, 1.0, true, R - 1, n2, ghost);
            const double v2 = col_feed(s2, v1, c, u0_2, 0.75, 0.25, false, R - 2, n2, ghost);
            const double v3 = col_feed(s3, v2, c, u0_3, 1.0 / 3.0, 2.0 / 3.0, false, R - 3, n2, ghost);
            const int r = R - 3;
            if (r >= row0 && r < row1) {
                if (valid) dst[(int64_t)r * n1] = v3;
                const double f = valid ? v3 : 0.0;
                const double L2c = (r + 0.5) * d2;
                m00 += f;
                m10 = fma(L1c, f, m10);
                m01 = fma(L2c, f, m01);
                m12 = fma(L1c * L2c * L2c, f, m12);
            }
            u0_3 = u0_2;
            u0_2 = u0_1;
            u0_1 = x;
        }
    }
    const double dA = d1 * d2;
    m00 = wave_sum(m00) * dA;
    m10 = wave_sum(m10) * dA;
    m01 = wave_sum(m01) * dA;
    m12 = wave_sum(m12) * dA;
    if (lane == 0) {
        double* p = a.part + (int64_t)b * 4;
        p[0] = m00; p[1] = m10; p[2] = m01; p[3] = m12;
    }
}

// Per simulation: finish the step (init = 0) or start the solve (init = 1), then
// prepare the next step's rates, step size and ghosts.
__global__ __launch_bounds__(64) void k_final2d(Fvm2dArgs a, int init) {
    const int s = blockIdx.x;
    const int lane = threadIdx.x;
    const Process p{a.law, PBE_SCHEME_SSPRK3, a.sol_law, a.cs0, a.cs1, a.alpha, a.cfl, a.dt_max, a.t_end};
    const double* P = a.par + (size_t)s * PBE_NPAR;
    const SimParams q = load_params(P);
    const double kg2 = uniform(P[PBE_P_KG2]), g2 = uniform(P[PBE_P_G2]);
    const int n1 = uniform(a.n1[s]), n2 = uniform(a.n2[s]);
    const double d1 = uniform(a.L1[s]) / n1, d2 = uniform(a.L2[s]) / n2;
    const int ns = a.n_samples;
    double C, t;
    int step, next, status;
    if (init) {
        // volume moment of the initial state (midpoint rule, SI Eq. (S5))
        const int64_t o = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
        double m12 = 0.0;
        for (int j = 0; j < n2; ++j) {
            const double L2c = (j + 0.5) * d2;
            for (int i = lane; i < n1; i += 64) {
                const double L1c = (i + 0.5) * d1;
                m12 = fma(L1c * L2c * L2c, a.f0[o + (int64_t)j * n1 + i], m12);
            }
        }
        m12 = wave_sum(m12) * d1 * d2;
        C = uniform(a.C0[s]);
        t = 0.0;
        step = 0; next = 0; status = 0;
        if (lane == 0) a.mu12[s] = m12;
    } else {
        if (!uniform(a.active[s])) return;
        C = uniform(a.C[s]); t = uniform(a.t[s]);
        step = uniform(a.step[s]); next = uniform(a.next[s]); status = uniform(a.status[s]);
        // block moments of the new state, summed in block order
        double m[4] = {0.0, 0.0, 0.0, 0.0};
        const int b0 = uniform(a.cb_first[s]), b1 = uniform(a.cb_first[s + 1]);
        for (int bb = b0 + lane; bb < b1; bb += 64)
#pragma unroll
            for (int k = 0; k < 4; ++k) m[k] += a.part[(int64_t)bb * 4 + k];
#pragma unroll
        for (int k = 0; k < 4; ++k) m[k] = wave_sum(m[k]);
        // discrete solute balance, Eq. (9), with the volume moment mu_{1,2}
        C = uniform(C - p.alpha * (m[3] - uniform(a.mu12[s])));
        const bool hit = uniform(a.hit[s]) != 0;
        const double t_next = uniform(next < ns ? a.t_samples[min(next, ns - 1)] : p.t_end);
        t = uniform(hit ? t_next : t + uniform(a.dt[s]));
        ++step;
        if (!isfinite(C) || !isfinite(m[3])) status |= PBE_SIM_NONFINITE;
        if (hit) {
            while (next < ns && a.t_samples[next] <= t) {
                const int64_t oo = (int64_t)s * ns + next;
                if (lane == 0) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) a.mom_s[oo * 4 + k] = m[k];
                    a.C_s[oo] = C;
                    a.samp_step[oo] = step;
                }
                ++next;
            }
        }
        if (lane == 0) a.mu12[s] = m[3];
    }
    // next step
    int active = 1;
    double dt = 0.0, c1 = 0.0, c2 = 0.0, gh1 = 0.0, gh2 = 0.0;
    int hit = 0;
    if (!(t < p.t_end) || (status & PBE_SIM_NONFINITE)) {
        active = 0;
    } else if (step >= a.step_cap) {
        status |= PBE_SIM_STEPCAP;
        active = 0;
    } else {
        const Rates2 r = rates_2d(p, q, kg2, g2, C, t);
        const double t_next = uniform(next < ns ? a.t_samples[min(next, ns - 1)] : p.t_end);
        double lim = __builtin_huge_val();
        if (r.G1 > 0.0) lim = fmin(lim, d1 / r.G1);
        if (r.G2 > 0.0) lim = fmin(lim, d2 / r.G2);
        const double dd = fmin(p.cfl * lim, p.dt_max);
        const double rem = t_next - t;
        hit = dd >= rem - 1e-12 * p.t_end;
        dt = uniform(hit ? rem : dd);
        if (!(dt > 0.0) || !isfinite(dt)) {
            status |= PBE_SIM_NONFINITE;
            active = 0;
        }
        c1 = dt * r.G1 / d1;
        c2 = dt * r.G2 / d2;
        gh1 = r.G1 > 0.0 ? r.B / (2.0 * d2 * r.G1) : 0.0;
        gh2 = r.G2 > 0.0 ? r.B / (2.0 * d1 * r.G2) : 0.0;
    }
    if (lane == 0) {
        a.C[s] = C; a.t[s] = t; a.step[s] = step; a.next[s] = next; a.status[s] = status;
        a.active[s] = active; a.dt[s] = dt; a.hit[s] = hit;
        a.c1[s] = c1; a.c2[s] = c2; a.gh1[s] = gh1; a.gh2[s] = gh2;
    }
}

// final state of every sim (it sits in buf[steps % 2]) into a packed output
__global__ void k_out2d(Fvm2dArgs a, double* f_out) {
    const int s = blockIdx.y;
    const int64_t o = a.off[s], n = a.off[s + 1] - o;
    const double* src = a.buf[a.step[s] & 1] + o;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        f_out[o + i] = src[i];
}

}  // namespace

hipError_t launch_rows2d(int cls, const Fvm2dArgs& a, int parity, int begin, int count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    switch (cls) {
        case 0: hipLaunchKernelGGL(k_rows2d<1>, dim3(count), dim3(64), 0, st, a, parity, begin); break;
        case 1: hipLaunchKernelGGL(k_rows2d<9>, dim3(count), dim3(64), 0, st, a, parity, begin); break;
        case 2: hipLaunchKernelGGL(k_rows2d<17>, dim3(count), dim3(64), 0, st, a, parity, begin); break;
        default: hipLaunchKernelGGL(k_rows2d<25>, dim3(count), dim3(64), 0, st, a, parity, begin); break;
    }
    return hipGetLastError();
}

hipError_t launch_cols2d(const Fvm2dArgs& a, int parity, hipStream_t st) {
    hipLaunchKernelGGL(k_cols2d, dim3(a.n_cb), dim3(64), 0, st, a, parity);
    return hipGetLastError();
}

hipError_t launch_final2d(const Fvm2dArgs& a, int init, hipStream_t st) {
    hipLaunchKernelGGL(k_final2d, dim3(a.n_sims), dim3(64), 0, st, a, init);
    return hipGetLastError();
}

hipError_t launch_out2d(const Fvm2dArgs& a, double* f_out, hipStream_t st) {
    hipLaunchKernelGGL(k_out2d, dim3(64, a.n_sims), dim3(256), 0, st, a, f_out);
    return hipGetLastError();
}

}  // namespace pbe

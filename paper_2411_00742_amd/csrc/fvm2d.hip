// 2D size-and-shape PBE (length L1 x width L2), Godunov dimensional splitting
// (paper Sec. 2.1: the update of Eq. (8) applied along each length in turn,
// L1 first) or Strang splitting (L1 over dt/2, L2 over dt, L1 over dt/2: the
// second L1 sweep runs on each finished row inside the same pass), SSP-RK3 (or
// the one-step form of Eq. (8)) per sweep, FP64, many simulations per launch
// (gfx950).
//
// One global step = two launches (captured in a graph by the host):
//   k_step2d  both sweeps in one pass over the state.  A wavefront owns a tile
//             of TW columns x seg rows of one simulation and marches down its
//             rows: each input row is loaded once (64 consecutive doubles, a
//             coalesced 512-byte access), swept along L1 across the lanes (one
//             cell per lane, neighbours by DPP; the tile is widened by the
//             stencil halo of the three stages, 6 cells left and 3 right, whose
//             lanes are recomputed by the neighbouring tile), and the swept
//             value enters the lane's L2 pipeline: the three SSP-RK3 stages
//             along the column held in registers, stage s lagging s rows.  The
//             finished row (3 rows behind the input) goes to the other state
//             buffer.  So the state crosses HBM once per step (read f^n, write
//             f^{n+1}) instead of once per sweep.  Tiles start 6 rows early
//             and end 2 rows late (the L2 halo).  The tile also sums the
//             moments of the new state and the number that leaves through
//             L1_max and L2_max.
//   k_final2d one wavefront per simulation: reduces the tile partials in a
//             fixed order, applies the solute balance (Eq. (9) with mu_{1,2}),
//             records samples, and computes the next step's rates, CFL step
//             (SI Eq. (S3)) and the corner nucleation ghosts.  (Folding this
//             into the tile kernel with a last-tile ticket needs a device-scope
//             release per tile, which writes back the L2 of the tile's XCD:
//             three times slower in total.)
// At the start of a solve, k_init2d sums the initial state's volume moment
// per tile and k_final2d (init) adds those partials and prepares step 0.
#include <type_traits>

#include "fvm1d_device.h"
#include "pbe_internal.h"

namespace pbe {
namespace {

using namespace dev;

// Stencil halo of a sweep: an updated cell depends on 2 cells to its left and
// 1 to its right per stage.
template <int SCHEME>
struct Halo2d {
    static constexpr int stages = SCHEME == PBE_SCHEME_SSPRK3 ? 3 : 1;
    static constexpr int left = 2 * stages, right = stages;
    static constexpr int width = 64 - left - right;   // output columns of a tile
};

// Neighbour values across the wave with no fill: lanes without a source read
// 0 (DPP bound_ctrl).  Only halo lanes of a tile ever read that value.
__device__ __forceinline__ double from_left(double v) { return dpp_src<0x138>(v); }    // wave_shr:1
__device__ __forceinline__ double from_right(double v) { return dpp_src<0x130>(v); }   // wave_shl:1

// L1 sweep of one row across the wave, one cell per lane (stage inputs u,
// faces H = face value right of each lane's cell).  In tiles that reach past
// the domain (EXT), lanes left of it hold the row's inflow ghost and lanes
// past L1_max hold 0, and are put back to those values after every stage.
// Returns the new value; *hN receives the stage-weighted value of this lane's
// right face (the outflow face for the lane at n1 - 1).
template <int SCHEME, bool EXT>
__device__ __forceinline__ double row_sweep_tile(double u, double c, double ghost, bool left_ext, bool right_ext,
                                                 double* hN) {
    auto ext = [&](double v) { return EXT ? (left_ext ? ghost : (right_ext ? 0.0 : v)) : v; };
    if constexpr (SCHEME == PBE_SCHEME_LW_TVD) {
        const double H = face_value<SCHEME>(from_left(u), u, from_right(u), 1.0, c);
        const double v = u + c * (from_left(H) - H);
        *hN = H;
        return ext(v);
    } else {
        const double u0 = u;
        double h[3];
#pragma unroll
        for (int st = 0; st < 3; ++st) {
            const double H = face_value<SCHEME>(from_left(u), u, from_right(u), 1.0, c);
            const double v = u + c * (from_left(H) - H);
            u = st == 0 ? v : (st == 1 ? 0.75 * u0 + 0.25 * v : (1.0 / 3.0) * u0 + (2.0 / 3.0) * v);
            u = ext(u);
            h[st] = H;
        }
        *hN = fma(h[0] + h[1], 1.0 / 6.0, (2.0 / 3.0) * h[2]);
        return u;
    }
}

// One stage running down a column: holds the last two inputs and the face
// value below them; fed the input at row r+1 it emits the stage output at row
// r and *F the face value between rows r and r+1.  EDGE: r may lie outside
// [0, n2) (ghost rows below L2 = 0 hold the ghost, nothing past L2_max).
struct ColStage {
    double a, i0, Fm1;   // slope i0 - (row below i0), row i0, face value below i0
};
template <int SCHEME, bool EDGE>
__device__ __forceinline__ double col_feed(ColStage& st, double x, double c, double u0r, double wa, double wb,
                                           bool first, int r, int n2, double ghost, double* F_out) {
    const double b = x - st.i0;
    const double F = face_value_ab<SCHEME>(st.a, b, st.i0, 1.0, c);
    const double v = st.i0 + c * (st.Fm1 - F);
    double out = first ? v : wa * u0r + wb * v;
    if (EDGE) out = r < 0 ? ghost : (r >= n2 ? 0.0 : out);
    st.a = b;
    st.i0 = x;
    st.Fm1 = F;
    *F_out = F;
    return out;
}

constexpr int kColAhead = 8;   // row loads in flight per wave

// Block b -> tile: the hardware hands consecutive blocks to the 8 XCDs in
// turn, so blocks b, b + 8, b + 16, ... share an XCD (and its L2).  They get
// consecutive tiles, which read each other's halo rows and columns.
__device__ __forceinline__ int tile_of_block(int b, int n_blocks) {
    const int per_xcd = n_blocks >> 3;   // n_blocks is a multiple of 8
    return (b & 7) * per_xcd + (b >> 3);
}

// Per simulation: finish the step (init = 0) or start the solve (init = 1), then
// prepare the next step's rates, step size and ghosts.
__device__ void finalize_sim(const Fvm2dArgs& a, int s, int init) {
    const int lane = threadIdx.x;
    const Process p{a.law, a.scheme, a.sol_law, a.cs0, a.cs1, a.alpha, a.cfl, a.dt_max, a.t_end};
    const double* P = a.par + (size_t)s * PBE_NPAR;
    const SimParams q = load_params(P);
    const double kg2 = uniform(P[PBE_P_KG2]), g2 = uniform(P[PBE_P_G2]), Eg2 = uniform(P[PBE_P_EG2]);
    const int n1 = uniform(a.n1[s]), n2 = uniform(a.n2[s]);
    const double d1 = uniform(a.L1[s]) / n1, d2 = uniform(a.L2[s]) / n2;
    const int ns = a.n_samples;
    double C, t, out, mu0 = 0.0;
    int step, next, status;
    if (init) {
        // volume moment of the initial state (midpoint rule, SI Eq. (S5)):
        // the tile partials k_init2d left, summed in tile order
        double m12 = 0.0;
        const int b0 = uniform(a.cb_first[s]), b1 = uniform(a.cb_first[s + 1]);
        for (int bb = b0 + lane; bb < b1; bb += 64) m12 += a.part[(int64_t)bb * 5 + 3];
        m12 = wave_sum(m12);
        C = uniform(a.C0[s]);
        t = 0.0;
        out = 0.0;
        step = 0; next = 0; status = 0;
        if (lane == 0) a.mu12[s] = m12;
    } else {
        if (!uniform(a.active[s])) return;
        C = uniform(a.C[s]); t = uniform(a.t[s]); out = uniform(a.outflow[s]);
        step = uniform(a.step[s]); next = uniform(a.next[s]); status = uniform(a.status[s]);
        // tile moments of the new state and outflow, summed in tile order
        double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const int b0 = uniform(a.cb_first[s]), b1 = uniform(a.cb_first[s + 1]);
        for (int bb = b0 + lane; bb < b1; bb += 64)
#pragma unroll
            for (int k = 0; k < 5; ++k) m[k] += a.part[(int64_t)bb * 5 + k];
#pragma unroll
        for (int k = 0; k < 5; ++k) m[k] = wave_sum(m[k]);
        out = uniform(out + m[4]);
        mu0 = m[0];
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
        // crystals that left through L1_max or L2_max (counted, not returned to the solution)
        if (!init && out > 1e-12 * fmax(mu0, 1e-300)) status |= PBE_SIM_OUTFLOW;
    } else if (step >= a.step_cap) {
        status |= PBE_SIM_STEPCAP;
        active = 0;
    } else {
        const Rates2 r = rates_2d(p, q, kg2, g2, Eg2, C, t);
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
        a.C[s] = C; a.t[s] = t; a.step[s] = step; a.next[s] = next; a.status[s] = status; a.outflow[s] = out;
        a.active[s] = active; a.dt[s] = dt; a.hit[s] = hit;
        a.c1[s] = c1; a.c2[s] = c2; a.gh1[s] = gh1; a.gh2[s] = gh2;
    }
}

__global__ __launch_bounds__(64) void k_final2d(Fvm2dArgs a, int init) { finalize_sim(a, blockIdx.x, init); }

// Tile geometry: Godunov splitting sweeps L1 once, so a tile's first output
// lane is the L1 halo's width in; Strang splitting sweeps L1 again on the
// output rows, which takes a second halo on each side.
template <int SCHEME, bool STRANG>
struct Tile2d {
    using H = Halo2d<SCHEME>;
    static constexpr int lo = STRANG ? 2 * H::left : H::left;                   // first output lane
    static constexpr int width = STRANG ? 64 - 2 * (H::left + H::right) : H::width;
};

// (held to four waves per SIMD: left to itself the compiler gives the SSP-RK3
// tile 140 registers, three waves per SIMD)
template <int SCHEME, bool STRANG>
__global__ __launch_bounds__(64, 4) void k_step2d(Fvm2dArgs a, int parity) {
    using H = Halo2d<SCHEME>;
    using TL = Tile2d<SCHEME, STRANG>;
    constexpr bool RK = SCHEME == PBE_SCHEME_SSPRK3;
    const int b = tile_of_block((int)blockIdx.x, (int)gridDim.x);
    if (b >= a.n_cb) return;
    const int s = uniform(a.cb_sim[b]);
    if (!uniform(a.active[s])) return;
    const int lane = threadIdx.x;
    const int n1 = uniform(a.n1[s]), n2 = uniform(a.n2[s]);
    const int c0 = uniform(a.cb_col0[b]), r0 = uniform(a.cb_row0[b]);
    const int r1 = min(r0 + a.seg, n2);
    const int col = c0 - TL::lo + lane;
    const bool left_ext = col < 0, right_ext = col >= n1;
    // a tile whose lanes all lie inside the domain needs no exterior masks
    const bool interior = c0 - TL::lo >= 0 && c0 - TL::lo + 63 < n1;
    const bool out_lane = lane >= TL::lo && lane < TL::lo + TL::width && !right_ext;
    const int colc = min(max(col, 0), n1 - 1);
    const int64_t o = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
    const double* src = a.buf[parity] + o + colc;
    double* dst = a.buf[parity ^ 1] + o + colc;
    // Strang: each L1 sweep covers half the step (c1 * 0.5 = (dt/2) G1/dL1 exactly)
    const double c1 = STRANG ? 0.5 * uniform(a.c1[s]) : uniform(a.c1[s]);
    const double c2 = uniform(a.c2[s]);
    const double gh1 = uniform(a.gh1[s]);
    // column 0 receives half the corner source through its L2 = 0 face (the
    // L1 sweep's row 0 the other half, through its L1 = 0 face)
    const double ghost2 = col == 0 ? uniform(a.gh2[s]) : 0.0;
    const double d1 = uniform(a.L1[s]) / n1, d2 = uniform(a.L2[s]) / n2;
    const double L1c = (col + 0.5) * d1;

    ColStage s1{0.0, 0.0, 0.0}, s2{0.0, 0.0, 0.0}, s3{0.0, 0.0, 0.0};
    double u0_1 = 0.0, u0_2 = 0.0, u0_3 = 0.0;   // L2 stage inputs at rows R-1, R-2, R-3
    double m00 = 0.0, m01 = 0.0, m02 = 0.0;     // this column's sums of f, L2 f, L2^2 f
    double hL1 = 0.0, hL2 = 0.0;                 // stage-weighted outflow face values
    // input rows R0..R1: the tile's rows plus the L2 halo; the output row is R - stages
    const int R0 = r0 - 2 * H::stages, R1 = r1 + H::stages - 1;
    // a ring keeps kColAhead row loads in flight; rows outside [0, n2) read a
    // clamped in-range row whose value is not used
    auto load_row = [&](int R) -> double { return src[(int64_t)min(max(R, 0), n2 - 1) * n1]; };
    double ring[kColAhead];
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) ring[j] = load_row(R0 + j);

    // One input row R.  FAST: an interior tile and a row whose L2 stage rows
    // all lie inside [0, n2): no exterior masks, ghost rows or outflow faces.
    auto row = [&](auto fast, int R, double raw) {
        constexpr bool FAST = decltype(fast)::value;
        // L1 sweep of row R (rows outside the domain are the L2 ghost / zero)
        double x;
        if (!FAST && R < 0) {
            x = ghost2;
        } else if (!FAST && R >= n2) {
            x = 0.0;
        } else {
            double hN;
            if (FAST || interior) {
                x = row_sweep_tile<SCHEME, false>(raw, c1, 0.0, false, false, &hN);
            } else {
                const double g1 = R == 0 ? gh1 : 0.0;   // row 0's inflow ghost
                x = row_sweep_tile<SCHEME, true>(left_ext ? g1 : (right_ext ? 0.0 : raw), c1, g1, left_ext, right_ext,
                                                 &hN);
                if (col == n1 - 1 && R >= r0 && R < r1) hL1 += hN;
            }
        }
        // L2 sweep: the stages pipelined down the column
        double v, Fs[3];
        int r;
        if constexpr (RK) {
            const double v1 = col_feed<SCHEME, !FAST>(s1, x, c2, 0.0, 0.0, 1.0, true, R - 1, n2, ghost2, &Fs[0]);
            const double v2 = col_feed<SCHEME, !FAST>(s2, v1, c2, u0_2, 0.75, 0.25, false, R - 2, n2, ghost2, &Fs[1]);
            v = col_feed<SCHEME, !FAST>(s3, v2, c2, u0_3, 1.0 / 3.0, 2.0 / 3.0, false, R - 3, n2, ghost2, &Fs[2]);
            r = R - 3;
            u0_3 = u0_2;
            u0_2 = u0_1;
            u0_1 = x;
        } else {
            v = col_feed<SCHEME, !FAST>(s1, x, c2, 0.0, 0.0, 1.0, true, R - 1, n2, ghost2, &Fs[0]);
            r = R - 1;
        }
        // the face past L2_max of each stage is formed when that stage emits row
        // n2 - 1, i.e. while rows n2 .. n2 + stages - 1 are fed (only in the tile
        // that owns row n2 - 1)
        if (!FAST && R >= n2 && r1 == n2) {
            if constexpr (RK) {
                hL2 += R == n2 ? Fs[0] * (1.0 / 6.0) : (R == n2 + 1 ? Fs[1] * (1.0 / 6.0) : Fs[2] * (2.0 / 3.0));
            } else {
                hL2 += Fs[0];
            }
        }
        if (r >= r0 && r < r1) {
            if constexpr (STRANG) {
                // the second half-step L1 sweep, on the finished row r
                double hN;
                if (FAST || interior) {
                    v = row_sweep_tile<SCHEME, false>(v, c1, 0.0, false, false, &hN);
                } else {
                    const double g1 = r == 0 ? gh1 : 0.0;
                    v = row_sweep_tile<SCHEME, true>(left_ext ? g1 : (right_ext ? 0.0 : v), c1, g1, left_ext,
                                                     right_ext, &hN);
                    if (col == n1 - 1) hL1 += hN;
                }
            }
            if (out_lane) dst[(int64_t)r * n1] = v;
            const double f = out_lane ? v : 0.0;
            const double L2c = (r + 0.5) * d2;
            m00 += f;
            m01 = fma(L2c, f, m01);
            m02 = fma(L2c * L2c, f, m02);
        }
    };
    for (int Rb = R0; Rb <= R1; Rb += kColAhead) {
        if (interior && Rb >= H::stages && Rb + kColAhead - 1 <= min(R1, n2 - 1)) {
#pragma unroll
            for (int j = 0; j < kColAhead; ++j) {
                const double raw = ring[j];
                ring[j] = load_row(Rb + j + kColAhead);
                row(std::true_type{}, Rb + j, raw);
            }
        } else {
#pragma unroll
            for (int j = 0; j < kColAhead; ++j) {
                const int R = Rb + j;
                if (R > R1) break;
                const double raw = ring[j];
                ring[j] = load_row(R + kColAhead);
                row(std::false_type{}, R, raw);
            }
        }
    }
    const double dA = d1 * d2;
    const double m10 = wave_sum(L1c * m00) * dA;   // the column's L1 is constant
    const double m12 = wave_sum(L1c * m02) * dA;
    m00 = wave_sum(m00) * dA;
    m01 = wave_sum(m01) * dA;
    // number leaving through L1_max (rows of this tile) and L2_max (its columns):
    // dt G1 hN d2 per row and dt G2 hN d1 per column, with dt G = c dL
    const double outf = wave_sum(c1 * (out_lane ? hL1 : 0.0) + c2 * (out_lane ? hL2 : 0.0)) * dA;
    if (lane == 0) {
        double* p = a.part + (int64_t)b * 5;
        p[0] = m00; p[1] = m10; p[2] = m01; p[3] = m12; p[4] = outf;
    }
}

// Volume moment mu_{1,2} of the initial state, one partial per tile (the
// tiles of the step kernel: its owned columns x its rows), so that the start
// of a solve reads each simulation once across the whole chip instead of
// with one wavefront per simulation.
__global__ __launch_bounds__(64) void k_init2d(Fvm2dArgs a, int tile_width) {
    const int b = tile_of_block((int)blockIdx.x, (int)gridDim.x);
    if (b >= a.n_cb) return;
    const int s = uniform(a.cb_sim[b]);
    const int lane = threadIdx.x;
    const int n1 = uniform(a.n1[s]), n2 = uniform(a.n2[s]);
    const int c0 = uniform(a.cb_col0[b]), r0 = uniform(a.cb_row0[b]);
    const int r1 = min(r0 + a.seg, n2);
    const int col = c0 + lane;
    const bool own = lane < tile_width && col < n1;
    const int64_t o = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
    const double d1 = uniform(a.L1[s]) / n1, d2 = uniform(a.L2[s]) / n2;
    const double* src = a.f0 + o + min(col, n1 - 1);
    double m = 0.0;
    for (int r = r0; r < r1; ++r) {
        const double L2c = (r + 0.5) * d2;
        m = fma(L2c * L2c, src[(int64_t)r * n1], m);
    }
    const double m12 = wave_sum(own ? (col + 0.5) * d1 * m : 0.0) * d1 * d2;
    if (lane == 0) a.part[(int64_t)b * 5 + 3] = m12;
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

int step2d_tile_width(int scheme, int strang) {
    if (strang)
        return scheme == PBE_SCHEME_LW_TVD ? Tile2d<PBE_SCHEME_LW_TVD, true>::width
                                           : Tile2d<PBE_SCHEME_SSPRK3, true>::width;
    return scheme == PBE_SCHEME_LW_TVD ? Tile2d<PBE_SCHEME_LW_TVD, false>::width
                                       : Tile2d<PBE_SCHEME_SSPRK3, false>::width;
}

hipError_t launch_step2d(const Fvm2dArgs& a, int parity, hipStream_t st) {
    const int blocks = (a.n_cb + 7) / 8 * 8;   // a multiple of 8 (see tile_of_block)
    const dim3 g(blocks), w(64);
    if (a.scheme == PBE_SCHEME_LW_TVD) {
        if (a.strang) hipLaunchKernelGGL((k_step2d<PBE_SCHEME_LW_TVD, true>), g, w, 0, st, a, parity);
        else hipLaunchKernelGGL((k_step2d<PBE_SCHEME_LW_TVD, false>), g, w, 0, st, a, parity);
    } else {
        if (a.strang) hipLaunchKernelGGL((k_step2d<PBE_SCHEME_SSPRK3, true>), g, w, 0, st, a, parity);
        else hipLaunchKernelGGL((k_step2d<PBE_SCHEME_SSPRK3, false>), g, w, 0, st, a, parity);
    }
    return hipGetLastError();
}

hipError_t launch_final2d(const Fvm2dArgs& a, int init, hipStream_t st) {
    if (init) {   // the initial volume moment's tile partials first
        const int blocks = (a.n_cb + 7) / 8 * 8;
        hipLaunchKernelGGL(k_init2d, dim3(blocks), dim3(64), 0, st, a, step2d_tile_width(a.scheme, a.strang));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_final2d, dim3(a.n_sims), dim3(64), 0, st, a, init);
    return hipGetLastError();
}

hipError_t launch_out2d(const Fvm2dArgs& a, double* f_out, hipStream_t st) {
    hipLaunchKernelGGL(k_out2d, dim3(64, a.n_sims), dim3(256), 0, st, a, f_out);
    return hipGetLastError();
}

}  // namespace pbe

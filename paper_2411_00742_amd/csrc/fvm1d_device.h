// Device-side building blocks of the 1D finite-volume step (gfx950).
//
// Mapping: one wavefront owns one simulation for its whole time loop.  The
// N cells are held in registers, K = ceil(N/64) consecutive cells per lane,
// right-aligned: lane l, slot k holds cell i = l*K + k - pad with
// pad = 64*K - N.  Right alignment puts the last cell (and so the outflow face
// at L_max) at lane 63, slot K-1 for every N; the pad slots on the left hold
// the inflow ghost value, which makes the face at L = 0 carry exactly the
// nucleation flux.  Neighbour cells across lanes move with DPP wave shifts;
// nothing touches LDS or HBM inside the time loop.
//
// Numerics follow the paper (arXiv 2411.00742): flux-limited upwind fluxes
// with the van Leer limiter (Sec. 2.1 Eq. (8), SI Eqs. (S1)-(S2)), CFL step
// (SI Eq. (S3)), discrete solute balance (Eq. (9)), rates driven by the
// supersaturation (App. A).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dmath.h"
#include "pbe.h"

namespace pbe {
namespace dev {

// ---------------------------------------------------------------- wave helpers
// lane l receives v from lane l-1; lane 0 receives `fill` (DPP wave_shr:1)
__device__ __forceinline__ double shift_from_left(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x138, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// lane l receives v from lane l+1; lane 63 receives `fill` (DPP wave_shl:1)
__device__ __forceinline__ double shift_from_right(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), 0x130, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), 0x130, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// every lane reads v from its DPP source lane (0 where it has none); no
// previous-value operand, so no fill copy is needed
template <int CTRL>
__device__ __forceinline__ double dpp_src(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_value(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
// Wave-uniform copy of a value every lane already agrees on (first active
// lane, into scalar registers).  Used on the per-step scalars (t, C, rates,
// dt) so the compiler keeps the time loop's control flow scalar.
__device__ __forceinline__ double uniform(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum over the 64 lanes with DPP (pairs, quads, half rows, rows, then the
// row broadcasts); the total lands in lane 63 and is read back as a
// wave-uniform scalar, so everything computed from it stays scalar.  After
// the first four steps every lane holds its row's sum R_r; row_bcast:15 adds
// R_{r-1} to row r and row_bcast:31 adds row 1's value (R_0 + R_1) to rows 2
// and 3, so row 3 ends with R_0 + R_1 + R_2 + R_3.  Other lanes end with
// partial sums nobody reads, which lets every DPP move run on all rows.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_src<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_src<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_src<0x141>(v);   // row_half_mirror
    v += dpp_src<0x140>(v);   // row_mirror
    v += dpp_src<0x142>(v);   // row_bcast:15
    v += dpp_src<0x143>(v);   // row_bcast:31
    return lane_value(v, 63);
}

// ---------------------------------------------------------------- wave pairs
// Long simulations run on two wavefronts of one workgroup: wave w holds the
// global lanes 64w..64w+63 of the right-aligned layout.  The two values that
// cross the wave boundary in each stage, and the per-step sums, pass through
// a few LDS slots around a workgroup barrier.  Every branch of the time loop
// depends only on values both waves hold bitwise identically (t, C, step,
// status, and sums combined in the same order), so both waves always reach
// the same barriers.
struct Pair {
    double* x;   // workgroup LDS: two alternating sets of 6 slots, then a write sink of 128 doubles
    int w;       // this wave's index in the workgroup
    int ph;      // which slot set the next exchange uses (both waves flip it in step)
};
constexpr int kPairSlots = 12 + 128;

// lane `mine` stores v in slot k; every other lane writes its own sink slot (no branch)
__device__ __forceinline__ void publish(const Pair& pr, int slot, bool mine, double v) {
    pr.x[mine ? slot : 12 + (int)threadIdx.x] = v;
}

// Sum of a wave-uniform value over the simulation's waves, identical on all of
// them.  One barrier: the slot set alternates, so a wave can only overwrite a
// set after the other wave has passed the next barrier, i.e. has read it.
template <int W>
__device__ __forceinline__ double group_sum(double wave_total, Pair* pr) {
    if constexpr (W == 1) {
        return wave_total;
    } else {
        double* x = pr->x + 6 * pr->ph;
        pr->ph ^= 1;
        x[4 + pr->w] = wave_total;   // all lanes of the wave store the same value
        __syncthreads();
        return uniform(x[4] + x[5]);
    }
}

// ---------------------------------------------------------------- process
struct Process {
    int law, scheme, sol_law;
    double cs0, cs1, alpha, cfl, dt_max, t_end;
};

struct SimParams {
    double kg, g, kb, b, gamma, Eg, Eb, T0, T1, tr;
    double inv_tr;   // 1/tr (0 when tr = 0)
    double kd, d;    // dissolution: G0 = -1e6 kd (-S)^d where S < 0
};

// (each value is made explicitly wave-uniform: loaded through a vector load,
// it would otherwise occupy a VGPR pair per parameter for the whole solve)
__device__ __forceinline__ SimParams load_params(const double* P) {
    SimParams q;
    q.kg = uniform(P[PBE_P_KG]); q.g = uniform(P[PBE_P_G]); q.kb = uniform(P[PBE_P_KB]);
    q.b = uniform(P[PBE_P_B]); q.gamma = uniform(P[PBE_P_GAMMA]);
    q.Eg = uniform(P[PBE_P_EG]); q.Eb = uniform(P[PBE_P_EB]); q.T0 = uniform(P[PBE_P_T0]);
    q.T1 = uniform(P[PBE_P_T1]); q.tr = uniform(P[PBE_P_TRAMP]);
    q.inv_tr = q.tr > 0.0 ? 1.0 / q.tr : 0.0;
    q.kd = uniform(P[PBE_P_KD]); q.d = uniform(P[PBE_P_D]);
    return q;
}

// cooling ramp T0 -> T1 over tr seconds, then held
__device__ __forceinline__ double temperature(const SimParams& q, double t) {
    const double frac = q.tr > 0.0 ? fmin(t, q.tr) * q.inv_tr : 1.0;
    return q.T0 + (q.T1 - q.T0) * frac;
}
__device__ __forceinline__ double solubility(const Process& p, double T) {
    return p.sol_law == PBE_SOL_EXP ? p.cs0 * exp64(p.cs1 * T) : p.cs0 + p.cs1 * T;
}

// Rates at the current concentration.  S = C/Csat - 1; growth G0 (um/s, at
// L = 0) and nucleation B act only for S > 0.  S^g and S^b share one log.
// DIS: below saturation the crystals dissolve at G0 = -1e6 kd (-S)^d (no
// nucleation), the growth/dissolution rate of SI S1.1 in the form of the
// growth power law.
struct Rates {
    double G0, B, S, lnS, arrG, arrB;   // lnS and the Arrhenius factors are kept for the adjoint,
    double Sg, Sb;                      // and so are S^g and S^b
};
template <bool DIS = false>
__device__ __forceinline__ Rates rates_plain(const Process& p, const SimParams& q, double C, double t) {
    Rates r;
    const double T = temperature(q, t);
    r.S = div_fast(C, solubility(p, T)) - 1.0;
    r.G0 = 0.0; r.B = 0.0; r.lnS = 0.0; r.arrG = 1.0; r.arrB = 1.0; r.Sg = 0.0; r.Sb = 0.0;
    if (r.S > 0.0) {
        r.lnS = log64(r.S);
        if (p.law == PBE_LAW_ARRHENIUS) {
            const double iT = div_fast(1.0, T + 273.15);
            r.arrG = exp64(-q.Eg * iT);
            r.arrB = exp64(-q.Eb * iT);
        }
        r.Sg = exp64(q.g * r.lnS);
        r.Sb = exp64(q.b * r.lnS);
        r.G0 = 1e6 * q.kg * r.Sg * r.arrG;
        r.B = q.kb * r.Sb * r.arrB;
    } else if (DIS && r.S < 0.0 && q.kd > 0.0) {
        r.G0 = -1e6 * q.kd * exp64(q.d * log64(-r.S));
    }
    r.G0 = uniform(r.G0);
    r.B = uniform(r.B);
    r.S = uniform(r.S);
    return r;
}

// Rates of the polynomial growth law (Sec. 4.1, Eq. (poly_growth_rate)):
// G0 = a_1 S + ... + a_k S^k for S = C/Csat - 1 > 0 (the a_j in um/s), with
// nucleation kb S^b.  Lane l sums the terms of the exponents j = l + 1 + 64 m
// (Horner in S^64 over m) and the wave adds the lanes up, so k up to 1024
// costs at most 16 steps per lane.  DER: also dG0/dS, and the per-lane S^(l+1)
// and S^64 from which the adjoint forms each coefficient's derivative S^j.
struct PolyTerms {
    double dGdS, Sl, S64;
};
template <bool DER>
__device__ __forceinline__ Rates rates_poly(const Process& p, const SimParams& q, double C, double t,
                                            const double* a, int k, PolyTerms* pt) {
    Rates r;
    const double T = temperature(q, t);
    r.S = div_fast(C, solubility(p, T)) - 1.0;
    r.G0 = 0.0; r.B = 0.0; r.lnS = 0.0; r.arrG = 1.0; r.arrB = 1.0; r.Sg = 0.0; r.Sb = 0.0;
    double dG = 0.0, Sl = 0.0, S64 = 0.0;
    if (r.S > 0.0) {
        const int lane = threadIdx.x & 63;
        r.lnS = log64(r.S);
        Sl = exp64((double)(lane + 1) * r.lnS);
        S64 = uniform(exp64(64.0 * r.lnS));
        const int M = (k + 63) >> 6;
        double acc = 0.0, dacc = 0.0;
        for (int m = M - 1; m >= 0; --m) {
            const int j = lane + 64 * m;
            const double aj = a[min(j, k - 1)];
            const double am = j < k ? aj : 0.0;
            acc = fma(acc, S64, am);
            if (DER) dacc = fma(dacc, S64, (double)(j + 1) * am);
        }
        r.G0 = wave_sum(Sl * acc);
        if (DER) dG = div_fast(wave_sum(Sl * dacc), r.S);
        r.Sb = exp64(q.b * r.lnS);
        r.B = q.kb * r.Sb;
    }
    r.G0 = uniform(r.G0);
    r.B = uniform(r.B);
    r.S = uniform(r.S);
    if (DER) {
        pt->dGdS = uniform(dG);
        pt->Sl = Sl;
        pt->S64 = S64;
    }
    return r;
}

// Rates of the 2D model: growth along each axis (G1 with kg, g; G2 with kg2, g2)
// and nucleation, all driven by the same supersaturation.
struct Rates2 {
    double G1, G2, B, S;
};
__device__ __forceinline__ Rates2 rates_2d(const Process& p, const SimParams& q, double kg2, double g2, double Eg2,
                                           double C, double t) {
    Rates2 r;
    const double T = temperature(q, t);
    r.S = C / solubility(p, T) - 1.0;
    r.G1 = 0.0; r.G2 = 0.0; r.B = 0.0;
    if (r.S > 0.0) {
        const double lnS = log64(r.S);
        double aG = 1.0, aG2 = 1.0, aB = 1.0;
        if (p.law == PBE_LAW_ARRHENIUS) {
            aG = exp64(-q.Eg / (T + 273.15));
            aG2 = exp64(-Eg2 / (T + 273.15));
            aB = exp64(-q.Eb / (T + 273.15));
        }
        r.G1 = 1e6 * q.kg * exp64(q.g * lnS) * aG;
        r.G2 = 1e6 * kg2 * exp64(g2 * lnS) * aG2;
        r.B = q.kb * exp64(q.b * lnS) * aB;
    }
    r.G1 = uniform(r.G1);
    r.G2 = uniform(r.G2);
    r.B = uniform(r.B);
    r.S = uniform(r.S);
    return r;
}

// Step size: CFL limit nu*dL/max_face |G| (|G| grows with L, so the max is at
// L_max), capped by dt_max, landing exactly on the next sample time.
__device__ __forceinline__ bool choose_dt(const Process& p, double G0, double gamma, double Lmax, double dL, double t,
                                          double t_next, double* dt) {
    const double Gmax = __builtin_fabs(G0) * (1.0 + gamma * Lmax);
    const double lim = Gmax > 0.0 ? div_fast(p.cfl * dL, Gmax) : __builtin_huge_val();
    const double d = fmin(lim, p.dt_max);
    const double rem = t_next - t;
    const bool hit = d >= rem - 1e-12 * p.t_end;
    *dt = uniform(hit ? rem : d);
    return uniform((int)hit) != 0;
}

// nucleation enters as the inflow ghost B/G0 left of L = 0, so the flux
// through L = 0 is B
__device__ __forceinline__ double inflow_ghost(double B, double G0) {
    return G0 > 0.0 ? div_fast(B, G0) : 0.0;
}
// Courant factor c = dt G0 / dL of the stage update (1/dL fixed per simulation)
__device__ __forceinline__ double courant(double dt, double G0, double inv_dL) { return dt * G0 * inv_dL; }

// ---------------------------------------------------------------- flux
// van Leer limited slope psi = phi(a/b)*b = 2ab/(a+b) when a and b share a
// strict sign, else 0 (SI Eqs. (S1)-(S2) in division-safe form).
// 1/d for the limiter's denominator d = a + b with ab > 0 (so |d| >= 2 sqrt(ab)
// >= 4.4e-162, never subnormal, and 1/d stays finite): the hardware
// reciprocal (relative error around 2^-23) refined by one Newton step, which
// squares the error to ~1e-14 relative: three VALU operations instead of the
// eleven of the correctly rounded division.  The limiter is a smooth function
// of a and b away from the select, so a relative error of 1e-14 in psi moves
// the solution by far less than the 1e-10 it is checked to.
__device__ __forceinline__ double recip_limiter(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// Half the van Leer slope, psi/2 = ab/(a+b) when a and b share a strict sign,
// else 0.  Every face needs only psi/2, and p * (1/(a+b)) is exactly half of
// 2p * (1/(a+b)) (scaling by 2 does not change the rounding), so the doubling
// and the halving are both left out.  One select at the end: where the slopes
// disagree a + b may be 0 or tiny and the quotient garbage, but it is discarded.
__device__ __forceinline__ double half_limited_slope(double a, double b) {
    const double p = a * b;
    const bool same = p > 0.0;
    const double q = p * recip_limiter(a + b);
    return same ? q : 0.0;
}

// Face value H = w (f_i + kappa/2 psi) with w = G(L_face)/G0, from the slopes
// a = f_i - f_{i-1} and b = f_{i+1} - f_i; the face flux is G0*H.  kappa = 1
// (method of lines) or 1 - nu_face (one-step update, Eq. (8)).
template <int SCHEME>
__device__ __forceinline__ double face_value_ab(double a, double b, double ui, double w, double c) {
    const double h = half_limited_slope(a, b);
    if (SCHEME == PBE_SCHEME_LW_TVD) {
        const double kappa = 1.0 - c * w;
        return w * fma(kappa, h, ui);
    }
    return w * (ui + h);
}
template <int SCHEME>
__device__ __forceinline__ double face_value(double um1, double ui, double up1, double w, double c) {
    return face_value_ab<SCHEME>(ui - um1, up1 - ui, ui, w, c);
}

// Geometry of one lane's slots.
struct LaneGeom {
    double xb;      // cell index of slot 0 as a double (negative inside the pad)
    double gdL;     // gamma * dL
    int npad;       // pad slots in this lane (slots k < npad hold the ghost)
};

// face weight of the face right of slot k: 1 + gamma*max(L_face, 0)
__device__ __forceinline__ double face_weight(const LaneGeom& g, int k) {
    return fma(g.gdL, fmax(g.xb + (double)(k + 1), 0.0), 1.0);
}

// slots in flight in the stage loop (see the ordering barrier in fvm_stage)
template <int K>
constexpr int kStageLag = 1;

// One Runge-Kutta stage on the wavefront's cells:
//   v = u + c (H_{i-1/2} - H_{i+1/2}),   u <- first ? v : wa*u0 + wb*v
// with c = dt*G0/dL.  Returns this lane's last face value (lane 63: L_max).
template <int K, int SCHEME, int W = 1, int LAG = kStageLag<K>>
__device__ __forceinline__ double fvm_stage(double (&u)[K], const double (&u0)[K], LaneGeom g, double c,
                                            double ghost, double wa, double wb, bool first, Pair* pr = nullptr) {
    static_assert(W == 1 || K >= 2, "wave pairs hold at least two cells per lane");
    // recompute the face weights in every stage instead of keeping K of them live
    asm volatile("" : "+v"(g.xb));
    // values entering at the wave's ends: the inflow ghost on the left and 0
    // beyond L_max, or the neighbouring wave's boundary cells
    double fillL = ghost, fillR = 0.0;
    double b_um1 = 0.0, b_ui = 0.0, b_up1 = 0.0;
    if constexpr (W == 2) {
        const int lane = threadIdx.x & 63;
        const int set = 6 * pr->ph;   // alternate slot sets: see group_sum
        pr->ph ^= 1;
        publish(*pr, set + 0, pr->w == 0 && lane == 63, u[K - 1]);
        publish(*pr, set + 1, pr->w == 0 && lane == 63, u[K >= 2 ? K - 2 : 0]);
        publish(*pr, set + 2, pr->w == 1 && lane == 0, u[0]);
        __syncthreads();
        b_ui = pr->x[set + 0];
        b_um1 = pr->x[set + 1];
        b_up1 = pr->x[set + 2];
        fillL = pr->w == 1 ? b_ui : ghost;
        fillR = pr->w == 0 ? b_up1 : 0.0;
    }
    const double uL = shift_from_left(u[K - 1], fillL);
    const double uR = shift_from_right(u[0], fillR);
    const double Hlast = face_value<SCHEME>(K >= 2 ? u[K >= 2 ? K - 2 : 0] : uL, u[K - 1], uR,
                                            face_weight(g, K - 1), c);
    double fillH = ghost;
    if constexpr (W == 2) {
        // wave 1 forms the face between the waves from the same three cells, the
        // same face coordinate and the same code as lane 63 of wave 0, so both
        // waves hold that face value bitwise; no second exchange is needed
        const double xf = lane_value(g.xb, 0);   // slot-0 cell index of lane 0 = index of that face
        const double Hb = face_value<SCHEME>(b_um1, b_ui, b_up1, fma(g.gdL, fmax(xf, 0.0), 1.0), c);
        fillH = pr->w == 1 ? Hb : ghost;
    }
    const double HL = shift_from_left(Hlast, fillH);
    double Hprev = HL;
    double a = u[0] - uL;   // slope left of slot 0
    // unclamped face weight z = 1 + gamma dL x of the face right of slot k,
    // stepped by gamma dL per slot from the face left of slot 0; with
    // gamma >= 0, max(z, 1) = 1 + gamma max(L, 0).  (z is formed by an add
    // after the ordering barrier below, so the max needs no NaN canonicalise.)
    double zl = fma(g.gdL, g.xb, 1.0);
    double nv_prev = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double ui = u[k];
        const double up1 = (k + 1 < K) ? u[k + 1 < K ? k + 1 : 0] : uR;
        const double b = up1 - ui;
        const double z = zl + g.gdL;
        const double H = (k == K - 1) ? Hlast : face_value_ab<SCHEME>(a, b, ui, fmax(z, 1.0), c);
        const double v = ui + c * (Hprev - H);
        const double nv = first ? v : wa * u0[k] + wb * v;
        u[k] = nv;
        Hprev = H;
        a = b;
        zl = z;
        // Sliding-window order: the inputs of the next slot that are not yet
        // derived from this one (the carried slope, the face weight and the
        // cell two to the right) are made to depend on this slot's result, so
        // the scheduler cannot compute the faces of all K slots up front (that
        // keeps several arrays of K doubles live).  u[k + 2] is tied in place,
        // which costs no copy.  The last slot takes Hlast, computed up front,
        // and needs neither the slope nor the weight.
        // With LAG = 2 the next slot waits for the slot before this one
        // instead, so two slots are in flight: more registers, more overlap
        // of the dependent FP64 chains for the long grids that run alone on
        // a SIMD.
        if constexpr (LAG == 1) {
            if (k + 2 < K) asm volatile("" : "+v"(u[k + 2 < K ? k + 2 : 0]), "+v"(a), "+v"(zl) : "v"(nv));
        } else {
            if (k + 2 < K) asm volatile("" : "+v"(u[k + 2 < K ? k + 2 : 0]), "+v"(a), "+v"(zl) : "v"(nv_prev));
            nv_prev = nv;
        }
    }
    return Hlast;
}

// Full time step with frozen rates.  Returns the stage-weighted face value at
// L_max (meaningful on lane 63) so outflow = dt*G0*that.
template <int K, int SCHEME, int W = 1, int LAG = kStageLag<K>>
__device__ __forceinline__ double fvm_step(double (&u)[K], const LaneGeom& g, double c, double ghost,
                                           Pair* pr = nullptr) {
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = k < g.npad ? ghost : u[k];   // select, not a divergent branch
    if (SCHEME == PBE_SCHEME_LW_TVD) {
        double u0[K];
        return fvm_stage<K, SCHEME, W, LAG>(u, u0, g, c, ghost, 0.0, 1.0, true, pr);
    }
    double u0[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u0[k] = u[k];
    const double h0 = fvm_stage<K, SCHEME, W, LAG>(u, u0, g, c, ghost, 0.0, 1.0, true, pr);
    const double h1 = fvm_stage<K, SCHEME, W, LAG>(u, u0, g, c, ghost, 0.75, 0.25, false, pr);
    const double h2 = fvm_stage<K, SCHEME, W, LAG>(u, u0, g, c, ghost, 1.0 / 3.0, 2.0 / 3.0, false, pr);
    return fma(h0 + h1, 1.0 / 6.0, (2.0 / 3.0) * h2);
}

// ---------------------------------------------------------------- dissolution
// With G0 < 0 the crystals shrink and every face takes its upwind value from
// the cell on its right: the face right of cell i carries
//   H = w (f_{i+1} - kappa/2 psi(f_{i+1} - f_i, f_{i+2} - f_{i+1})),
// the mirror image of the growth face (psi is symmetric in its two slopes),
// with kappa = 1 or 1 - |c| w.  Cells left of L = 0 (the pad slots and the
// fill left of lane 0) are 0 in every stage: what crosses L = 0 has
// dissolved.  Beyond L_max the density is 0, so nothing enters there.
template <int SCHEME>
__device__ __forceinline__ double face_value_dis(double a, double b, double up1, double w, double c) {
    const double h = half_limited_slope(a, b);
    if (SCHEME == PBE_SCHEME_LW_TVD) {
        const double kappa = fma(c, w, 1.0);   // 1 - |c| w with c < 0
        return w * fma(-kappa, h, up1);
    }
    return w * (up1 - h);
}

// One stage v = u + c (H_{i-1/2} - H_{i+1/2}) with c = dt G0/dL < 0, then
// u <- first ? v : wa u0 + wb v, pad slots back to 0.  One wavefront per
// simulation.  The face left of slot 0 is formed by each lane; the face right
// of its last slot is the right neighbour's (0 past L_max).
template <int K, int SCHEME>
__device__ __forceinline__ void fvm_stage_dis(double (&u)[K], const double (&u0)[K], LaneGeom g, double c, double wa,
                                              double wb, bool first) {
    asm volatile("" : "+v"(g.xb));
    const double uL = shift_from_left(u[K - 1], 0.0);                  // cell left of slot 0
    const double uR = shift_from_right(u[0], 0.0);                     // cell right of slot K-1
    const double u1 = K >= 2 ? u[K >= 2 ? 1 : 0] : uR;
    const double Hfirst = face_value_dis<SCHEME>(u[0] - uL, u1 - u[0], u[0],
                                                 fma(g.gdL, fmax(g.xb, 0.0), 1.0), c);
    const double Hlast = shift_from_right(Hfirst, 0.0);
    double Hprev = Hfirst;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double ui = u[k];
        double H = Hlast;   // the last slot's right face is the right neighbour's first face
        if (k + 1 < K) {
            const double up1 = u[k + 1 < K ? k + 1 : 0];
            const double up2 = (k + 2 < K) ? u[k + 2 < K ? k + 2 : 0] : uR;
            H = face_value_dis<SCHEME>(up1 - ui, up2 - up1, up1, fma(g.gdL, fmax(g.xb + (double)(k + 1), 0.0), 1.0),
                                       c);
        }
        const double v = ui + c * (Hprev - H);
        const double nv = first ? v : wa * u0[k] + wb * v;
        u[k] = k < g.npad ? 0.0 : nv;
        Hprev = H;
        if (k + 2 < K) asm volatile("" : "+v"(u[k + 2 < K ? k + 2 : 0]) : "v"(nv));
    }
}

// Full dissolution step with frozen rates (SSP-RK3 or the one-step update).
template <int K, int SCHEME>
__device__ __forceinline__ void fvm_step_dis(double (&u)[K], const LaneGeom& g, double c) {
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = k < g.npad ? 0.0 : u[k];
    double u0[K];
    if (SCHEME == PBE_SCHEME_LW_TVD) {
        fvm_stage_dis<K, SCHEME>(u, u0, g, c, 0.0, 1.0, true);
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) u0[k] = u[k];
    fvm_stage_dis<K, SCHEME>(u, u0, g, c, 0.0, 1.0, true);
    fvm_stage_dis<K, SCHEME>(u, u0, g, c, 0.75, 0.25, false);
    fvm_stage_dis<K, SCHEME>(u, u0, g, c, 1.0 / 3.0, 2.0 / 3.0, false);
}

// Load / store this lane's K cells of one simulation's packed array `row`
// (cell 0 at row[0]).  Every per-cell device array carries a leading guard of
// kCellGuard doubles, so row + (cell index of slot 0) stays inside the
// allocation even for pad slots: loads are unconditional (pad slots then take
// `pad_value` by a select), which keeps the K-slot array out of divergent
// control flow (a per-slot guarded load makes the compiler copy the whole
// array through every branch).  Stores of pad slots are masked off.
template <int K>
__device__ __forceinline__ void load_cells(double (&u)[K], const double* row, int i0, int npad, double pad_value) {
    int j0 = i0;
    asm volatile("" : "+v"(j0));
    const double* lp = row + j0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = lp[k];
        u[k] = k < npad ? pad_value : x;
    }
}
template <int K>
__device__ __forceinline__ void store_cells(const double (&u)[K], double* row, int i0, int npad) {
    int j0 = i0;
    asm volatile("" : "+v"(j0));
    double* lp = row + j0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k >= npad) lp[k] = u[k];
}

// this lane's part of sum_i x_i^3 f_i, x_i = L_i/dL the cell centre in cell
// widths (pad slots weigh 0); mu_3 = dL^4 times the wave's sum
template <int K>
__device__ __forceinline__ double lane_moment3(const double (&u)[K], const LaneGeom& g) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = fmax(g.xb + ((double)k + 0.5), 0.0);
        s = fma(x * x * x, u[k], s);
    }
    return s;
}

// the same for x_i^2 f_i; mu_2 = dL^3 times the wave's sum
template <int K>
__device__ __forceinline__ double lane_moment2(const double (&u)[K], const LaneGeom& g) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = fmax(g.xb + ((double)k + 0.5), 0.0);
        s = fma(x * x, u[k], s);
    }
    return s;
}

template <int K>
__device__ __forceinline__ void lane_moments(const double (&u)[K], const LaneGeom& g, double dL, double m[4]) {
    m[0] = m[1] = m[2] = m[3] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double x = g.xb + ((double)k + 0.5);
        const double L = fmax(x, 0.0) * dL;
        const double f = x > 0.0 ? u[k] : 0.0;
        m[0] += f;
        m[1] = fma(L, f, m[1]);
        m[2] = fma(L * L, f, m[2]);
        m[3] = fma(L * L * L, f, m[3]);
    }
}

}  // namespace dev
}  // namespace pbe

// Discrete adjoint of the batched 1D solve (gfx950, FP64).
//
// Reverse-mode derivative of the recorded outputs (samples of f, mu_0..mu_3
// and C) with respect to each simulation's (kg, g, kb, b, gamma).  The paper
// obtains such gradients by reverse-mode AD with checkpointing through the
// whole time loop (Sec. 4.1, SI S2.1); here the adjoint of the time loop is
// written by hand.  The step size is differentiated in the branch each step
// takes: a CFL-limited step nu dL / (G0 (1 + gamma L_max)) (SI Eq. (S3))
// depends on the growth rate and gamma, a step that lands on a sample time
// depends on the time reached, and the time reached moves the temperature of
// the cooling ramp, hence the solubility and the rates; a step of dt_max is a
// constant.  The schedule itself (which branch, how many steps) is piecewise
// constant in the parameters and has no derivative.
//
// One wavefront per simulation, same register layout as the forward kernel.
// For each checkpoint segment (ckpt_every steps), last to first:
//   1. reload the checkpoint (f, C, t) and recompute the segment forward with
//      the forward kernel's step, writing the state at each step to a tape and
//      the step's scalars (rates, step size, ghost, Courant factor, solubility
//      terms) to a per-step record (the learned closure's rates come from the
//      record its forward solve kept of every step);
//   2. walk the segment backwards: for step m-1 -> m, recompute the three
//      SSP-RK3 stage states on-chip from the taped f^{m-1}, then apply the
//      transposed Jacobians of the stages, the solute balance (Eq. (9)) and
//      the rate laws (their values read from the record, one step ahead),
//      adding sample cotangents as their steps are reached.
// Derivative conventions: the limited slope psi = 2ab/(a+b) for ab > 0 has
// zero derivative where ab <= 0; max(S, 0) and S^p have zero derivative at S <= 0.
#include "closure_device.h"
#include "fvm1d_device.h"
#include "pbe_internal.h"

namespace pbe {
namespace {

using namespace dev;

// Adjoint of one stage v_i = u_i + c (H_{i-1/2} - H_{i+1/2}) taken at the stage
// input u.  On entry ub holds vbar (adjoint of v); on exit ub holds ubar.
// Accumulates per lane: cbar (adjoint of c), gbar (adjoint of the inflow
// ghost value, lane 0 only) and gam (adjoint of gamma through the face weights).
template <int K>
__device__ __forceinline__ void adj_stage(const double* __restrict__ us, double (&ub)[K], LaneGeom g, double c,
                                          double ghost, int lane, double& cbar, double& gbar, double& gam, double dL) {
    asm volatile("" : "+v"(g.xb));
    // us: this stage's input state in LDS, slot k of this lane at us[k * 64 + lane]
    const double uL = shift_from_left(us[(K - 1) * 64 + lane], ghost);
    const double uR = shift_from_right(us[lane], 0.0);
    const double vbR = shift_from_right(ub[0], 0.0);   // vbar of the cell right of this lane (none past L_max)
    const double vb0 = ub[0];
    // leftmost face of the wave (left of lane 0, slot 0) carries H = ghost
    if (lane == 0) {
        cbar = fma(ghost, vb0, cbar);
        gbar = fma(c, vb0, gbar);
    }
    double send_left = 0.0;   // -abar of slot 0: belongs to the left neighbour's last cell
    double carry = 0.0;       // bbar of slot k-1 to add to slot k
    double vbk = vb0;         // original vbar_k
    double uk = us[lane];
    double a = uk - uL;       // slope left of slot 0 (then carried from slot to slot)
    // stage inputs are read from LDS two slots ahead (the memory clobber on the
    // ordering barrier keeps each read in front of it), so no slot waits on LDS
    double pre = K >= 2 ? us[(K >= 2 ? 1 : 0) * 64 + lane] : uR;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double up1 = (k + 1 < K) ? pre : uR;
        if (k + 2 < K) pre = us[(k + 2 < K ? k + 2 : 0) * 64 + lane];
        const double vbk1 = (k + 1 < K) ? ub[k + 1 < K ? k + 1 : 0] : vbR;   // still original here
        const double b = up1 - uk;
        const double p = a * b;
        const bool same = p > 0.0;
        // the forward's reciprocal where the limiter is active (so psi/2 = p r
        // matches the forward bitwise) and 0 where it is not, which zeroes
        // psi/2 and both its derivatives with one select
        const double r = same ? recip_limiter(a + b) : 0.0;
        const double hpsi = p * r;
        // d(psi/2)/da = (b/(a+b))^2, d(psi/2)/db = (a/(a+b))^2: both ratios lie in
        // (0, 1] when ab > 0, so neither factor over- or underflows in the far tails of f
        const double br = b * r, ar = a * r;
        const double xf = fmax(g.xb + (double)(k + 1), 0.0);
        const double Lf = xf * dL;
        const double w = fma(g.gdL, xf, 1.0);
        const double face = uk + hpsi;
        const double H = w * face;
        const double dv = vbk1 - vbk;
        cbar = fma(H, dv, cbar);
        const double Hb = c * dv;
        gam = fma(Hb * face, Lf, gam);
        const double pb = Hb * w;   // adjoint of the face value f_k + psi_k/2 (times -1 for the right cell)
        const double ab = pb * (br * br);
        const double bb = pb * (ar * ar);
        // ubar_k = vbar_k (direct term) + face terms + what slot k-1 pushed right
        const double ubk = vbk + pb + ab - bb + carry;
        if (k == 0) {
            send_left = -ab;
        } else {
            ub[k >= 1 ? k - 1 : 0] -= ab;
        }
        ub[k] = ubk;
        carry = bb;
        vbk = vbk1;
        a = b;
        uk = up1;
        // sliding-window order (see fvm_stage): the next slot starts after this one
        asm volatile("" : "+v"(a) : "v"(ubk) : "memory");
    }
    // bbar of the last slot goes to the right neighbour's slot 0; -abar of
    // slot 0 to the left neighbour's last slot (lane 0: to the ghost)
    const double from_left = shift_from_left(carry, 0.0);
    const double from_right = shift_from_right(send_left, 0.0);
    ub[0] += from_left;
    ub[K - 1] += from_right;
    if (lane == 0) gbar += send_left;
}

template <int K>
__device__ __forceinline__ void set_pad(double (&u)[K], const LaneGeom& g, double v) {
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = k < g.npad ? v : u[k];
}

template <int K>
__device__ __forceinline__ void stage_fwd(double (&u)[K], const double (&u0)[K], const LaneGeom& g, double c,
                                          double ghost, double wa, double wb, bool first) {
    (void)fvm_stage<K, PBE_SCHEME_SSPRK3>(u, u0, g, c, ghost, wa, wb, first);
}

// number of sample times at or before t (the times ascend strictly): binary
// search, once per checkpoint segment; within a segment the count advances
// one sample at a time, as in the forward loop
__device__ __forceinline__ int samples_reached(const double* ts, int ns, double t) {
    int lo = 0, hi = ns;   // ts[0..lo) <= t < ts[hi..ns)
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (uniform(ts[mid]) <= t) lo = mid + 1;
        else hi = mid;
    }
    return uniform(lo);
}

// the learned closure (a network) as opposed to the plain or polynomial laws
constexpr bool is_net(int cl) { return cl == kClosureBf16 || cl == kClosureFp64; }

template <int K, int CL>
__device__ __forceinline__ void adjoint_sim(const Adj1dArgs& A, int s, double* __restrict__ lds) {
    const Fvm1dArgs& a = A.fw;
    const int lane = threadIdx.x;
    const int N = uniform(a.ncell[s]);
    const int64_t base = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
    const double Lmax = uniform(a.Lmax[s]);
    const double dL = Lmax / N;
    const double inv_dL = (double)N / Lmax;
    const double dL3 = dL * dL * dL, dL4 = dL3 * dL;   // moment scales in cell units
    const SimParams q = load_params(a.par + (size_t)s * PBE_NPAR);
    const Process p{a.law, a.scheme, a.sol_law, a.cs0, a.cs1, a.alpha, a.cfl, a.dt_max, a.t_end};
    const int ns = a.n_samples;
    const double* ts = a.t_samples;
    const int Kc = a.ckpt_every;

    const int pad = 64 * K - N;
    LaneGeom g;
    g.xb = (double)(lane * K - pad);
    g.gdL = q.gamma * dL;
    g.npad = min(max(pad - lane * K, 0), K);
    const int i0 = lane * K - pad;

    const int n_total = uniform(a.step[s]);
    if (uniform(a.status[s]) & (PBE_SIM_NONFINITE | PBE_SIM_STEPCAP)) {
        // the forward did not reach t_end: no derivative is defined
        if (lane == 0)
            for (int j = 0; j < PBE_NGRAD; ++j) A.gpar[(int64_t)s * PBE_NGRAD + j] = __builtin_nan("");
        return;
    }
    double lam[K];
#pragma unroll
    for (int k = 0; k < K; ++k) lam[k] = 0.0;
    if (A.gf && A.gf_is_final) load_cells(lam, A.gf + base, i0, g.npad, 0.0);
    double lamC = 0.0;
    double lamT = 0.0;   // adjoint of the time reached after the step being reversed
    double gk[4] = {0.0, 0.0, 0.0, 0.0};
    double gam = 0.0;    // per lane: gamma through the face weights
    double gams = 0.0;   // wave-uniform: gamma through the CFL step
    int qs = ns - 1;   // next sample (from the end) whose cotangent is still to be added
    // step index and cotangents of sample qs, and the bracket of sample times
    // around the reverse walk's current time (nx samples lie at or before it;
    // t_lo is the last of them, t_lo2 the one before, t_hi the next): carried
    // across steps and loaded one sample ahead of their use, so no step waits
    // on a memory round trip for them
    // (up to 8 cells per lane they stay as loaded until the step that consumes
    // them, lane j < 4 holding the cotangent of mu_j and lane 4 that of C, so no
    // step waits on them; the 9-16 class has no registers to spare for that)
    constexpr bool AHEAD = K <= 8;
    int qstep_v = -1;
    double q_v = 0.0, q_gc = 0.0, q_gm[4] = {0.0, 0.0, 0.0, 0.0};
    auto load_sample = [&](int qq) {
        const int64_t o = (int64_t)s * ns + qq;
        if constexpr (AHEAD) {
            qstep_v = a.samp_step[o];
            const int j = min(lane, 4);
            q_v = j < 4 ? (A.gmom ? A.gmom[o * 4 + j] : 0.0) : (A.gC ? A.gC[o] : 0.0);
        } else {
            qstep_v = uniform(a.samp_step[o]);
            q_gc = A.gC ? uniform(A.gC[o]) : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) q_gm[j] = A.gmom ? uniform(A.gmom[o * 4 + j]) : 0.0;
        }
    };
    if (qs >= 0) load_sample(qs);
    int nx = ns;
    double t_lo = ns > 0 ? uniform(ts[ns - 1]) : -__builtin_huge_val();
    double t_lo2 = ns > 1 ? uniform(ts[ns - 2]) : -__builtin_huge_val();
    double t_hi = p.t_end;

    double* tape = A.tape + base * Kc;
    double* tapeC = A.tape_C + (int64_t)s * Kc;
    double* tapeT = A.tape_t + (int64_t)s * Kc;
    // learned closure: the forward taped each step's closure quantities
    // (lane j < kClosureTape reads quantity j of a step)
    const double* tapeR = is_net(CL) ? a.ck_r + (int64_t)s * a.step_cap * kClosureTape : nullptr;
    const int rj = min(lane, kClosureTape - 1);
    double* tapeS = A.tape_s + (int64_t)s * Kc * kStepTape;
    double* rows = A.rows + (int64_t)s * A.row_cap * 5;
    // polynomial law: its coefficients, and d/da_j accumulated in LDS after the
    // stage buffers (lane l owns the exponents j = l + 1 + 64 m, slot m * 64 + l)
    const double* coef = a.poly + (int64_t)s * a.n_poly;
    double* ga = lds + 4 * K * 64;
    const int n_terms = CL == kClosurePoly ? (a.n_poly + 63) >> 6 : 0;
    for (int m = 0; m < n_terms; ++m) ga[m * 64 + lane] = 0.0;

    // learned closure checkpointed at every step: the forward kept every state
    // and every step's scalars, so the whole trajectory is one segment with
    // nothing to recompute
    const bool every = is_net(CL) && a.ck_s != nullptr && Kc == 1;
    const int n_seg = every ? 1 : (n_total + Kc - 1) / Kc;
    // the recompute pass tapes a record of the step's scalars for the reverse step
    constexpr bool REC = CL == kClosureNone || CL == kClosurePoly || is_net(CL);
    // learned closure: the network's input and output scales, loaded once (a
    // load inside the step would wait, through the in-order memory counter,
    // for the record prefetches issued before it)
    double cs_out0 = 0.0, cs_out1 = 0.0, cs_in0 = 0.0, cs_in1 = 0.0, cs_in2 = 0.0;
    if constexpr (is_net(CL)) {
        const double* kc = a.cd.c;
        cs_out0 = uniform(kc[kCOutScale]);
        cs_out1 = uniform(kc[kCOutScale + 1]);
        cs_in0 = uniform(kc[kCInScale]);
        cs_in1 = uniform(kc[kCInScale + 1]);
        cs_in2 = uniform(kc[kCInScale + 2]);
    }
    for (int seg = n_seg - 1; seg >= 0; --seg) {
        const int m0 = every ? 0 : seg * Kc;
        const int m1 = every ? n_total : min(m0 + Kc, n_total);
        // the segment's states and step records: the forward's own with `every`
        const double* tp = every ? a.ck_f + base * a.n_ckpt : tape;
        const double* tsp = every ? a.ck_s + (int64_t)s * a.step_cap * kStepTape : tapeS;
        if (!every) {
        // ---- recompute the segment forward, taping the state at each step
        double u[K];
        load_cells(u, a.ck_f + base * a.n_ckpt + (int64_t)seg * N, i0, g.npad, 0.0);
        double C = uniform(a.ck_C[(int64_t)s * a.n_ckpt + seg]);
        double t = uniform(a.ck_t[(int64_t)s * a.n_ckpt + seg]);
        int next = samples_reached(ts, ns, t);
        double t_next = uniform(next < ns ? ts[min(next, ns - 1)] : p.t_end);
        // up to 8 cells per lane: the sample time after t_next, loaded ahead and
        // kept as loaded until a step lands on t_next (a load there would wait
        // behind the tape stores)
        double t_nn = AHEAD && next + 1 < ns ? ts[next + 1] : p.t_end;
        LaneGeom gm = g;
        asm volatile("" : "+v"(gm.xb));
        double mu3_old = wave_sum(lane_moment3(u, gm)) * dL4;
        double crn = is_net(CL) ? tapeR[(int64_t)m0 * kClosureTape + rj] : 0.0;   // one step ahead
        for (int m = m0; m < m1; ++m) {
            Rates r;
            [[maybe_unused]] PolyTerms ptr{0.0, 0.0, 0.0};
            if constexpr (CL == kClosureNone) {
                r = rates_plain(p, q, C, t);
            } else if constexpr (CL == kClosurePoly) {
                r = rates_poly<true>(p, q, C, t, coef, a.n_poly, &ptr);
            } else {
                // learned closure: the rates the forward took at this step (the
                // plain power law where the network's box excluded the state)
                const double cr = crn;
                if (m + 1 < m1) crn = tapeR[(int64_t)(m + 1) * kClosureTape + rj];
                if ((int)bcast(cr, 0) & 1) {
                    const Process pp{PBE_LAW_POWER, p.scheme, p.sol_law, p.cs0, p.cs1, p.alpha, p.cfl, p.dt_max,
                                     p.t_end};
                    r = rates_plain(pp, q, C, t);
                } else {
                    r.G0 = bcast(cr, 1);
                    r.B = bcast(cr, 2);
                    r.S = 0.0; r.lnS = 0.0; r.arrG = 1.0; r.arrB = 1.0; r.Sg = 0.0; r.Sb = 0.0;
                }
            }
            double dt;
            const bool hit = choose_dt(p, r.G0, q.gamma, Lmax, dL, t, t_next, &dt);
            const double ghost = inflow_ghost(r.B, r.G0);
            const double cf = courant(dt, r.G0, inv_dL);
            if constexpr (REC) {
                // the step's scalars as the reverse step uses them, so that it
                // reads them (one step ahead) instead of forming them again
                const double Tm = temperature(q, t);
                const double Csat = solubility(p, Tm);
                const double dCsat = p.sol_law == PBE_SOL_EXP ? p.cs1 * Csat : p.cs1;
                const double iT = 1.0 / (Tm + 273.15);
                // (polynomial law: dG0/dS in place of the Arrhenius growth
                // factor and S^64 in place of 1/(T + 273.15)^2, which it has no use for)
                const bool PL = CL == kClosurePoly;
                const double v[kStepTape] = {r.G0, r.B, r.S, r.lnS, PL ? ptr.dGdS : r.arrG, r.arrB, r.Sg, r.Sb, dt,
                                             hit ? 1.0 : 0.0, ghost, cf, Csat, -(C / Csat) * dCsat / Csat,
                                             (q.tr > 0.0 && t < q.tr) ? (q.T1 - q.T0) * q.inv_tr : 0.0,
                                             PL ? ptr.S64 : iT * iT};
                if (lane == 0) {
                    double* ts_ = tapeS + (int64_t)(m - m0) * kStepTape;
#pragma unroll
                    for (int j = 0; j < kStepTape; ++j) ts_[j] = v[j];
                }
            }
            // the state the step starts from, taped after the rates so that their
            // loads do not wait for these stores
            store_cells(u, tape + (int64_t)(m - m0) * N, i0, g.npad);
            if (lane == 0) {
                tapeC[m - m0] = C;
                tapeT[m - m0] = t;
            }
            (void)fvm_step<K, PBE_SCHEME_SSPRK3>(u, g, cf, ghost);
            LaneGeom g2 = g;
            asm volatile("" : "+v"(g2.xb));
            const double mu3 = wave_sum(lane_moment3(u, g2)) * dL4;
            C = uniform(C - p.alpha * (mu3 - mu3_old));
            mu3_old = mu3;
            t = uniform(hit ? t_next : t + dt);
            if constexpr (AHEAD) {
                if (hit && next < ns) {
                    // landed on sample time ts[next] = t; later samples at the same time are skipped too
                    ++next;
                    double tn = uniform(t_nn);
                    while (next < ns && tn <= t) {
                        ++next;
                        tn = uniform(next < ns ? ts[next] : p.t_end);
                    }
                    t_next = next < ns ? tn : p.t_end;
                    t_nn = next + 1 < ns ? ts[next + 1] : p.t_end;
                }
            } else if (hit) {
                while (next < ns && uniform(ts[next]) <= t) ++next;
                t_next = uniform(next < ns ? ts[min(next, ns - 1)] : p.t_end);
            }
        }
        // (each lane reads back only the tape addresses it wrote itself)
        }

        // ---- reverse walk over the segment
        // taped scalars of the first reverse step; each step prefetches the
        // next one's.  With a record (plain laws, learned closure) the step
        // reads everything from it (lane j < kStepTape holds scalar j, kept as
        // loaded until the step reads it, so no step waits on a load it has
        // just issued: with the wait counter in order, that wait would also
        // cover the state load above it) and needs neither C nor t.
        double Cn = REC ? 0.0 : uniform(tapeC[m1 - 1 - m0]);
        double tn = REC ? 0.0 : uniform(tapeT[m1 - 1 - m0]);
        double recn = REC ? tsp[(int64_t)(m1 - 1 - m0) * kStepTape + (lane & (kStepTape - 1))] : 0.0;
        // learned closure: the step's taped closure quantities, also one step ahead
        double crecn = is_net(CL) ? tapeR[(int64_t)(m1 - 1) * kClosureTape + rj] : 0.0;
        for (int m = m1; m > m0; --m) {
            // state at m-1 from the tape: issued first, consumed after the rates
            double u0[K];
            load_cells(u0, tp + (int64_t)(m - 1 - m0) * N, i0, g.npad, 0.0);
            const double Cm = Cn;
            const double tm = tn;
            const double rec = recn;
            const double crec = crecn;
            if (m - 1 > m0) {
                if constexpr (REC) {
                    recn = tsp[(int64_t)(m - 2 - m0) * kStepTape + (lane & (kStepTape - 1))];
                    if constexpr (is_net(CL)) crecn = tapeR[(int64_t)(m - 2) * kClosureTape + rj];
                } else {
                    Cn = uniform(tapeC[m - 2 - m0]);
                    tn = uniform(tapeT[m - 2 - m0]);
                }
            }
            // cotangents of the samples taken at state m
            while (qs >= 0 && uniform(qstep_v) == m) {
                lamC += AHEAD ? bcast(q_v, 4) : q_gc;
                const double gm4[4] = {AHEAD ? bcast(q_v, 0) : q_gm[0], AHEAD ? bcast(q_v, 1) : q_gm[1],
                                       AHEAD ? bcast(q_v, 2) : q_gm[2], AHEAD ? bcast(q_v, 3) : q_gm[3]};
                LaneGeom g3 = g;
                asm volatile("" : "+v"(g3.xb));
                double gcell[K];
                if (A.gf && !A.gf_is_final)
                    load_cells(gcell, A.gf + base * ns + (int64_t)qs * N, i0, g.npad, 0.0);
                else
#pragma unroll
                    for (int k = 0; k < K; ++k) gcell[k] = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double x = g3.xb + ((double)k + 0.5);
                    const double L = fmax(x, 0.0) * dL;
                    const double add = ((gm4[3] * L + gm4[2]) * L + gm4[1]) * L * dL + gm4[0] * dL + gcell[k];
                    lam[k] += x > 0.0 ? add : 0.0;
                }
                --qs;
                if (qs >= 0) load_sample(qs);
                else qstep_v = -1;
            }

            // samples reached at tm (the forward's sample index at step m-1)
            if constexpr (!REC) {
                while (nx > 0 && t_lo > tm) {
                    --nx;
                    t_hi = t_lo;
                    t_lo = t_lo2;
                    t_lo2 = nx > 1 ? uniform(ts[nx - 2]) : -__builtin_huge_val();
                }
            }
            Rates r;
            bool fb = true;        // plain power law at this step
            bool clamped = false;  // closure: ln G0 held at its bound (no derivative through G0)
            double cz[3] = {0.0, 0.0, 0.0}, cj[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, cmu2 = 0.0;
            PolyTerms pt{0.0, 0.0, 0.0};
            if constexpr (CL == kClosureNone) {
                r.G0 = bcast(rec, 0); r.B = bcast(rec, 1); r.S = bcast(rec, 2); r.lnS = bcast(rec, 3);
                r.arrG = bcast(rec, 4); r.arrB = bcast(rec, 5); r.Sg = bcast(rec, 6); r.Sb = bcast(rec, 7);
            } else if constexpr (CL == kClosurePoly) {
                r.G0 = bcast(rec, 0); r.B = bcast(rec, 1); r.S = bcast(rec, 2); r.lnS = bcast(rec, 3);
                r.arrG = 1.0; r.arrB = bcast(rec, 5); r.Sg = bcast(rec, 6); r.Sb = bcast(rec, 7);
                pt.dGdS = bcast(rec, 4);
                pt.S64 = bcast(rec, 15);
                pt.Sl = r.S > 0.0 ? exp64((double)(lane + 1) * r.lnS) : 0.0;
            } else {
                // the rates from the record (the power law's where the network fell back)
                const int flags = (int)bcast(crec, 0);
                fb = (flags & 1) != 0;
                clamped = (flags & 2) != 0;
                r.G0 = bcast(rec, 0); r.B = bcast(rec, 1); r.S = bcast(rec, 2); r.lnS = bcast(rec, 3);
                r.arrG = bcast(rec, 4); r.arrB = bcast(rec, 5); r.Sg = bcast(rec, 6); r.Sb = bcast(rec, 7);
                if (!fb) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) cz[i] = bcast(crec, 3 + i);
#pragma unroll
                    for (int i = 0; i < 6; ++i) cj[i] = bcast(crec, 6 + i);
                    cmu2 = bcast(crec, 12);
                }
            }
            double dt, ghost, c;
            bool hit;
            if constexpr (REC) {
                dt = bcast(rec, 8);
                hit = bcast(rec, 9) != 0.0;
                ghost = bcast(rec, 10);
                c = bcast(rec, 11);
            } else {
                hit = choose_dt(p, r.G0, q.gamma, Lmax, dL, tm, t_hi, &dt);
                ghost = inflow_ghost(r.B, r.G0);
                c = courant(dt, r.G0, inv_dL);
            }

            // stage input states u0, u1, u2 into this wave's LDS
            set_pad(u0, g, ghost);
            {
                double u[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    u[k] = u0[k];
                    lds[(0 * K + k) * 64 + lane] = u0[k];
                }
                stage_fwd(u, u0, g, c, ghost, 0.0, 1.0, true);
#pragma unroll
                for (int k = 0; k < K; ++k) lds[(1 * K + k) * 64 + lane] = u[k];
                stage_fwd(u, u0, g, c, ghost, 0.75, 0.25, false);
#pragma unroll
                for (int k = 0; k < K; ++k) lds[(2 * K + k) * 64 + lane] = u[k];
            }

            // solute balance: Phi's output f^m also feeds C^m = C^{m-1} - alpha (mu3(f^m) - mu3(f^{m-1}))
            // ub in registers; the direct (identity) part of the step's adjoint,
            // l0, waits in LDS (slot k of this lane at l0s[k * 64 + lane]) while
            // the three stage adjoints run, which keeps their registers free
            double ub[K];
            double* l0s = lds + 3 * K * 64;
            {
                LaneGeom g4 = g;
                asm volatile("" : "+v"(g4.xb));
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double L = fmax(g4.xb + ((double)k + 0.5), 0.0) * dL;
                    const double lp = lam[k] - p.alpha * lamC * (L * L * L * dL);
                    ub[k] = (2.0 / 3.0) * lp;   // vbar of stage 3
                    l0s[k * 64 + lane] = (1.0 / 3.0) * lp;
                }
            }
            double cbar = 0.0, gbar = 0.0;
            adj_stage<K>(lds + 2 * K * 64, ub, g, c, ghost, lane, cbar, gbar, gam, dL);   // ub = adjoint of u2
#pragma unroll
            for (int k = 0; k < K; ++k) {
                l0s[k * 64 + lane] = fma(0.75, ub[k], l0s[k * 64 + lane]);
                ub[k] = 0.25 * ub[k];
            }
            adj_stage<K>(lds + 1 * K * 64, ub, g, c, ghost, lane, cbar, gbar, gam, dL);   // ub = adjoint of u1
            adj_stage<K>(lds, ub, g, c, ghost, lane, cbar, gbar, gam, dL);   // ub = adjoint of u0 via stage 1
            {
                LaneGeom g5 = g;
                asm volatile("" : "+v"(g5.xb));
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double l = l0s[k * 64 + lane] + ub[k];
                    const bool padk = k < g5.npad;   // pad slots were set to the ghost at the step start
                    const double L = fmax(g5.xb + ((double)k + 0.5), 0.0) * dL;
                    gbar += padk ? l : 0.0;
                    lam[k] = padk ? 0.0 : fma(p.alpha * lamC, L * L * L * dL, l);
                }
            }
            // rates and step: c = dt G0/dL, ghost = B/G0; t^m = t^{m-1} + dt, or
            // the sample time the step lands on (a constant)
            const double cb = wave_sum(cbar);
            const double gb = wave_sum(gbar);
            double dtb = (hit ? 0.0 : lamT) + cb * r.G0 * inv_dL;   // adjoint of dt
            double lamT_prev = hit ? 0.0 : lamT;                    // adjoint of t^{m-1}
            double G0b = cb * dt * inv_dL, Bb = 0.0;
            if (r.G0 > 0.0) {
                Bb = gb / r.G0;
                G0b -= gb * ghost / r.G0;
            }
            if (hit) {
                lamT_prev -= dtb;   // dt = t_next - t^{m-1}
            } else if (dt < p.dt_max) {
                // CFL-limited: dt = nu dL / (G0 (1 + gamma L_max))
                const double wmax = fma(q.gamma, Lmax, 1.0);
                G0b -= dtb * dt / r.G0;
                gams -= dtb * dt * Lmax / wmax;
            }
            // temperature of the ramp at t^{m-1}, the solubility and its slope,
            // dS/dT = -(C/Csat) Csat'(T) / Csat (plain laws: from the record)
            double Csat, dTdt, dSdT, iT2;
            if constexpr (REC) {
                Csat = bcast(rec, 12);
                dSdT = bcast(rec, 13);
                dTdt = bcast(rec, 14);
                iT2 = bcast(rec, 15);
            } else {
                const double Tm = temperature(q, tm);
                Csat = solubility(p, Tm);
                const double dCsat = p.sol_law == PBE_SOL_EXP ? p.cs1 * Csat : p.cs1;
                dTdt = (q.tr > 0.0 && tm < q.tr) ? (q.T1 - q.T0) * q.inv_tr : 0.0;
                dSdT = -(Cm / Csat) * dCsat / Csat;
                const double iT = 1.0 / (Tm + 273.15);
                iT2 = iT * iT;
            }
            double Tb = 0.0;
            if (!fb) {
                // closure: ln G0 = a0 + s0 y0 (held at its bound when clamped),
                // ln B = a1 + s1 y1 with y = net(z), z0 = (S - h0) k0,
                // z1 = (T - h1) k1, z2 = (log10 mu2 - h2) k2
                const double yb0 = clamped ? 0.0 : G0b * r.G0 * cs_out0;
                const double yb1 = Bb * r.B * cs_out1;
                const double Sbar = (yb0 * cj[0] + yb1 * cj[1]) * cs_in0;
                lamC += Sbar / Csat;
                Tb = (yb0 * cj[2] + yb1 * cj[3]) * cs_in1 + Sbar * dSdT;
                const double mbar = (yb0 * cj[4] + yb1 * cj[5]) * cs_in2 / (cmu2 * 2.302585092994046);
                LaneGeom g6 = g;
                asm volatile("" : "+v"(g6.xb));
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const double x = g6.xb + ((double)k + 0.5);
                    const double L = fmax(x, 0.0) * dL;
                    lam[k] += x > 0.0 ? mbar * (L * L * dL) : 0.0;
                }
                if (lane == 0) {
                    double* rw = rows + (int64_t)(m - 1) * 5;
                    rw[0] = cz[0]; rw[1] = cz[1]; rw[2] = cz[2]; rw[3] = yb0; rw[4] = yb1;
                }
            } else if (r.S > 0.0) {
                const double dGdS = CL == kClosurePoly ? pt.dGdS : q.g * r.G0 / r.S;
                const double dBdS = q.b * r.B / r.S;
                const double Sbar = G0b * dGdS + Bb * dBdS;
                lamC += Sbar / Csat;
                Tb = Sbar * dSdT;
                if (CL == kClosureNone && p.law == PBE_LAW_ARRHENIUS) {
                    // exp(-E/(T + 273.15)) factors
                    Tb += (G0b * r.G0 * q.Eg + Bb * r.B * q.Eb) * iT2;
                }
                if constexpr (CL == kClosurePoly) {
                    // dG0/da_j = S^j
                    double pw = pt.Sl;
                    for (int mm = 0; mm < n_terms; ++mm) {
                        ga[mm * 64 + lane] = fma(G0b, pw, ga[mm * 64 + lane]);
                        pw *= pt.S64;
                    }
                } else {
                    gk[0] += G0b * 1e6 * r.Sg * r.arrG;
                    gk[1] += G0b * r.G0 * r.lnS;
                }
                gk[2] += Bb * r.Sb * r.arrB;
                gk[3] += Bb * r.B * r.lnS;
            }
            if (is_net(CL) && fb && lane == 0) {
                double* rw = rows + (int64_t)(m - 1) * 5;
                rw[0] = 0.0; rw[1] = 0.0; rw[2] = 0.0; rw[3] = 0.0; rw[4] = 0.0;
            }
            lamT = uniform(fma(Tb, dTdt, lamT_prev));
            lamC = uniform(lamC);
        }
    }
    const double gg = wave_sum(gam) + gams;
    if (lane == 0) {
        double* o = A.gpar + (int64_t)s * PBE_NGRAD;
        o[0] = gk[0]; o[1] = gk[1]; o[2] = gk[2]; o[3] = gk[3]; o[4] = gg;
    }
    if constexpr (CL == kClosurePoly) {
        for (int m = 0; m < n_terms; ++m) {
            const int j = m * 64 + lane;
            if (j < a.n_poly) A.gpoly[(int64_t)s * a.n_poly + j] = ga[m * 64 + lane];
        }
    }
}

// Adjoint classes: cells per lane 1-8 and 9-16 (grids up to 1024 cells).
// waves per SIMD each adjoint class is held to: two for the 1-8 class of the
// plain and polynomial laws (what it spills lies outside the step loops; a
// second wave per SIMD hides more latency), one for the 9-16 class and for the
// learned closure, whose 1-8 class at two waves spills the step record's
// prefetch inside the reverse loop (each spill waits for the loads before it)
constexpr int adj_waves_per_simd(int klo, int cl) {
    return klo == 1 && cl != kClosureBf16 && cl != kClosureFp64 ? 2 : 1;
}

template <int KLO, int CL>
__global__ __launch_bounds__(64, adj_waves_per_simd(KLO, CL)) void k_adj1d(Adj1dArgs A, int cls_begin, int cls_count, int32_t* queue) {
    // the three SSP-RK3 stage input states of the step being reversed and the
    // direct part of its adjoint (each lane owns its column)
    __shared__ double lds[4 * (KLO + 7) * 64 + (CL == kClosurePoly ? kMaxPoly : 0)];
    for (;;) {
        const int ticket = atomicAdd(queue, threadIdx.x == 0 ? 1 : 0);
        const int idx = __builtin_amdgcn_readfirstlane(ticket);
        if (idx >= cls_count) break;
        const int s = uniform(A.fw.order[cls_begin + idx]);
        const int K = uniform((A.fw.ncell[s] + 63) >> 6);
        switch (K - KLO) {
            case 0: adjoint_sim<KLO + 0, CL>(A, s, lds); break;
            case 1: adjoint_sim<KLO + 1, CL>(A, s, lds); break;
            case 2: adjoint_sim<KLO + 2, CL>(A, s, lds); break;
            case 3: adjoint_sim<KLO + 3, CL>(A, s, lds); break;
            case 4: adjoint_sim<KLO + 4, CL>(A, s, lds); break;
            case 5: adjoint_sim<KLO + 5, CL>(A, s, lds); break;
            case 6: adjoint_sim<KLO + 6, CL>(A, s, lds); break;
            case 7: adjoint_sim<KLO + 7, CL>(A, s, lds); break;
            default: break;
        }
    }
}

}  // namespace

template <int CL>
static hipError_t launch_cl(int cls, const Adj1dArgs& A, int n_blocks, int begin, int count, int32_t* queue,
                            hipStream_t st) {
    if (cls == 0)
        hipLaunchKernelGGL((k_adj1d<1, CL>), dim3(n_blocks), dim3(64), 0, st, A, begin, count, queue);
    else if (cls == 1)
        hipLaunchKernelGGL((k_adj1d<9, CL>), dim3(n_blocks), dim3(64), 0, st, A, begin, count, queue);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_adj1d_class(int cls, const Adj1dArgs& A, int n_blocks, int begin, int count, int32_t* queue,
                              hipStream_t st) {
    if (A.fw.closure == kClosurePoly) return launch_cl<kClosurePoly>(cls, A, n_blocks, begin, count, queue, st);
    if (A.fw.closure == kClosureBf16) return launch_cl<kClosureBf16>(cls, A, n_blocks, begin, count, queue, st);
    if (A.fw.closure == kClosureFp64) return launch_cl<kClosureFp64>(cls, A, n_blocks, begin, count, queue, st);
    return launch_cl<kClosureNone>(cls, A, n_blocks, begin, count, queue, st);
}

template <int CL>
static hipError_t adj_occupancy(int cls, int* per_cu) {
    return cls == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_adj1d<1, CL>, 64, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_adj1d<9, CL>, 64, 0);
}

int adj1d_class_resident_blocks(int cls, int closure) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = closure == kClosureBf16   ? adj_occupancy<kClosureBf16>(cls, &per_cu)
                         : closure == kClosureFp64 ? adj_occupancy<kClosureFp64>(cls, &per_cu)
                         : closure == kClosurePoly ? adj_occupancy<kClosurePoly>(cls, &per_cu)
                                                   : adj_occupancy<kClosureNone>(cls, &per_cu);
    if (e != hipSuccess) return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

}  // namespace pbe

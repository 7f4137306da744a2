// Batched persistent 1D solver kernel (gfx950, FP64).
//
// One launch runs every simulation of a handle: each 64-lane workgroup pulls
// simulation indices from an atomic queue (sims pre-sorted longest first) and
// runs that simulation's whole time loop with the density in registers (see
// fvm1d_device.h for the lane mapping).  Per step: rates from the current
// concentration, step size, three fused SSP-RK3 stages (or the one-step
// update), volume moment by wave reduction, solute balance, sampling.
#include "closure_device.h"
#include "fvm1d_device.h"
#include "pbe_internal.h"

namespace pbe {
namespace {

using namespace dev;

// polynomial law: the running simulation's coefficients (one array for every
// instantiation of run_sim, so a kernel holds 8 KB of LDS, not 8 KB per lane count)
__shared__ double poly_lds[kMaxPoly];

// W = 1: one wavefront per simulation; W = 2: a wave pair (see Pair), with
// `lane` the global lane 0..127 of the right-aligned layout.
// TAPE (learned closure, a solve that will be differentiated): also evaluate the
// network's input Jacobian and tape the step for the adjoint; its own kernel
// instantiation, so that the solves without it keep their registers.
template <int K, int SCHEME, int CL, int W, bool TAPE = false>
__device__ __forceinline__ void run_sim(const Fvm1dArgs& a, int s, Pair* pr) {
    static_assert(W == 1 || CL == kClosureNone, "the closure and dissolution kernels run one wavefront per simulation");
    const int lane = W == 2 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
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

    const int pad = 64 * W * K - N;
    LaneGeom g;
    g.xb = (double)(lane * K - pad);
    g.gdL = q.gamma * dL;
    g.npad = min(max(pad - lane * K, 0), K);
    const int i0 = lane * K - pad;   // cell index of slot 0

    // in-the-loop correction: the sim's weights, staged in LDS once per simulation
    [[maybe_unused]] const double* corr_w = nullptr;
    if constexpr (CL == kCorrect) {
        __shared__ double wsh[PBE_CORR_NW];
        __syncthreads();   // the previous simulation's reads are done
        if (lane < PBE_CORR_NW) wsh[lane] = a.corr[(int64_t)s * PBE_CORR_NW + lane];
        __syncthreads();
        corr_w = wsh;
    }

    // polynomial law: the sim's coefficients, staged in LDS once per simulation
    // (read every step; a global load there would wait, through the in-order
    // memory counter, for the sample stores of the step before)
    [[maybe_unused]] const double* coef = nullptr;
    if constexpr (CL == kClosurePoly) {
        __syncthreads();   // the previous simulation's reads are done
        for (int j = lane; j < a.n_poly; j += 64) poly_lds[j] = a.poly[(int64_t)s * a.n_poly + j];
        __syncthreads();
        coef = poly_lds;
    }

    double u[K];
    load_cells(u, (a.from_initial ? a.f0 : a.f) + base, i0, g.npad, 0.0);

    double C, t, mu3_old, out;
    int step, next, status;
    if (a.from_initial) {
        C = uniform(a.C0[s]);
        t = 0.0;
        mu3_old = group_sum<W>(wave_sum(lane_moment3(u, g)), pr) * dL4;
        out = 0.0;
        step = 0; next = 0; status = 0;
    } else {
        C = a.C[s]; t = a.t[s]; mu3_old = a.mu3[s]; out = a.outflow[s];
        step = a.step[s]; next = a.next[s]; status = a.status[s];
    }
    C = uniform(C); t = uniform(t); mu3_old = uniform(mu3_old);
    step = uniform(step); next = uniform(next); status = uniform(status);
    // next sample time (reloaded only when a sample is taken) and the next
    // checkpoint (index and step), so no step pays a load or a division for them
    double t_next = uniform(next < ns ? ts[min(next, ns - 1)] : p.t_end);
    int ck_c = a.ckpt_every > 0 ? (step + a.ckpt_every - 1) / a.ckpt_every : 0;
    int ck_at = a.ckpt_every > 0 ? ck_c * a.ckpt_every : -1;

    for (int it = 0; it < a.max_steps; ++it) {
        if (!(t < p.t_end) || (status & PBE_SIM_NONFINITE)) break;
        // keep per-cell geometry from being hoisted out of the time loop into registers
        asm volatile("" : "+v"(g.xb));
        if (step >= a.step_cap) { status |= PBE_SIM_STEPCAP; break; }
        Rates r;
        [[maybe_unused]] bool net_fallback = false;
        if constexpr (CL == kClosureNone) {
            r = rates_plain(p, q, C, t);
        } else if constexpr (CL == kDissolve) {
            r = rates_plain<true>(p, q, C, t);
        } else if constexpr (CL == kCorrect) {
            r = rates_plain(p, q, C, t);
        } else if constexpr (CL == kClosurePoly) {
            r = rates_poly<false>(p, q, C, t, coef, a.n_poly, nullptr);
        } else {
            // learned closure: inputs S, T and mu_2 of the current state
            LaneGeom g2 = g;
            asm volatile("" : "+v"(g2.xb));
            const double mu2 = wave_sum(lane_moment2(u, g2)) * dL3;
            ClosureRates cr;
            if constexpr (TAPE) {
                // a solve that will be differentiated: also the network's input
                // Jacobian (the tangent columns of the same matrix products),
                // taped with the step's inputs and rates for the adjoint
                cr = closure_rates<true, CL>(a.cd, p, q, C, t, mu2);
                if (lane == 0) {
                    double* tr = a.ck_r + ((int64_t)s * a.step_cap + step) * kClosureTape;
                    tr[0] = (cr.fallback ? 1.0 : 0.0) + (cr.clamped ? 2.0 : 0.0);
                    tr[1] = cr.G0; tr[2] = cr.B;
                    tr[3] = cr.z[0]; tr[4] = cr.z[1]; tr[5] = cr.z[2];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        tr[6 + 2 * i] = cr.dy[0][i];
                        tr[7 + 2 * i] = cr.dy[1][i];
                    }
                    tr[12] = mu2;
                }
            } else {
                cr = closure_rates<false, CL>(a.cd, p, q, C, t, mu2);
            }
            r.G0 = cr.G0;
            r.B = cr.B;
            r.S = cr.S;
            net_fallback = cr.fallback;
            if (cr.fallback) status |= PBE_SIM_FALLBACK;
        }
        double dt;
        const bool hit = choose_dt(p, r.G0, q.gamma, Lmax, dL, t, t_next, &dt);
        if (!(dt > 0.0) || !isfinite(dt)) {   // rates overflowed: stop this sim
            status |= PBE_SIM_NONFINITE;
            break;
        }
        // nucleation: ghost cells at L < 0 hold B/G0 so the flux through L = 0 is B
        const double ghost = inflow_ghost(r.B, r.G0);
        if (a.rate_log && lane == 0) {   // opt-in record of the step size and rates (step < step_cap here)
            double* rl = a.rate_log + ((int64_t)s * a.step_cap + step) * 3;
            rl[0] = dt; rl[1] = r.G0; rl[2] = r.B;
        }

        if (step == ck_at) {
            const int c = ck_c++;
            ck_at += a.ckpt_every;
            if (c < a.n_ckpt) {
                store_cells(u, a.ck_f + base * a.n_ckpt + (int64_t)c * N, i0, g.npad);
                if (lane == 0) {
                    a.ck_C[(int64_t)s * a.n_ckpt + c] = C;
                    a.ck_t[(int64_t)s * a.n_ckpt + c] = t;
                }
            }
        }

        const double cour = courant(dt, r.G0, inv_dL);
        if constexpr (TAPE) {
            if (a.ck_s) {
                // checkpointed at every step: also the scalars the adjoint's
                // reverse step reads (the rates of the plain power law where the
                // network fell back, the step size, ghost, Courant factor and
                // solubility terms), formed as the adjoint's recompute would
                Rates rr;
                if (net_fallback) {
                    const Process pp{PBE_LAW_POWER, p.scheme, p.sol_law, p.cs0, p.cs1, p.alpha, p.cfl, p.dt_max,
                                     p.t_end};
                    rr = rates_plain(pp, q, C, t);
                } else {
                    rr.G0 = r.G0; rr.B = r.B;
                    rr.S = 0.0; rr.lnS = 0.0; rr.arrG = 1.0; rr.arrB = 1.0; rr.Sg = 0.0; rr.Sb = 0.0;
                }
                const double Tm = temperature(q, t);
                const double Csat = solubility(p, Tm);
                const double dCsat = p.sol_law == PBE_SOL_EXP ? p.cs1 * Csat : p.cs1;
                const double iT = 1.0 / (Tm + 273.15);
                const double v[kStepTape] = {rr.G0, rr.B, rr.S, rr.lnS, rr.arrG, rr.arrB, rr.Sg, rr.Sb, dt,
                                             hit ? 1.0 : 0.0, ghost, cour, Csat, -(C / Csat) * dCsat / Csat,
                                             (q.tr > 0.0 && t < q.tr) ? (q.T1 - q.T0) * q.inv_tr : 0.0, iT * iT};
                if (lane == 0) {
                    double* rec = a.ck_s + ((int64_t)s * a.step_cap + step) * kStepTape;
#pragma unroll
                    for (int j = 0; j < kStepTape; ++j) rec[j] = v[j];
                }
            }
        }
        double hN;
        if constexpr (CL == kDissolve) {
            if (cour < 0.0) {   // dissolving: nothing crosses L_max
                fvm_step_dis<K, SCHEME>(u, g, cour);
                hN = 0.0;
            } else {
                hN = fvm_step<K, SCHEME, W>(u, g, cour, ghost, pr);
            }
        } else {
            hN = fvm_step<K, SCHEME, W>(u, g, cour, ghost, pr);
            if constexpr (CL == kCorrect) {
                if (cour > 0.0) correct_step<K>(u, g, cour, N, corr_w);
            }
        }
        out = fma(dt * r.G0, hN, out);

        // discrete solute balance, Eq. (9): C^{n+1} = C^n - alpha (mu3^{n+1} - mu3^n)
        LaneGeom gm = g;
        asm volatile("" : "+v"(gm.xb));
        const double mu3 = group_sum<W>(wave_sum(lane_moment3(u, gm)), pr) * dL4;
        C = uniform(C - p.alpha * (mu3 - mu3_old));
        mu3_old = mu3;
        t = uniform(hit ? t_next : t + dt);
        ++step;
        if (!isfinite(C) || !isfinite(mu3)) {
            status |= PBE_SIM_NONFINITE;
            break;
        }
        if (hit) {
            while (next < ns && ts[next] <= t) {
                double m[4];
                LaneGeom gm = g;
                asm volatile("" : "+v"(gm.xb));
                lane_moments(u, gm, dL, m);
                const int64_t o = (int64_t)s * ns + next;
#pragma unroll
                for (int j = 0; j < 4; ++j) m[j] = group_sum<W>(wave_sum(m[j]), pr) * dL;
                if (lane == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) a.mom_s[o * 4 + j] = m[j];
                    a.C_s[o] = C;
                    a.samp_step[o] = step;
                }
                if (a.record_f) store_cells(u, a.f_s + base * ns + (int64_t)next * N, i0, g.npad);
                ++next;
            }
            t_next = uniform(next < ns ? ts[min(next, ns - 1)] : p.t_end);
        }
    }

    // save the running state
    store_cells(u, a.f + base, i0, g.npad);
    // the outflow face belongs to lane 63 of the last wave, which writes the per-sim scalars
    const double out63 = lane_value(out, 63);
    if (!(t < p.t_end) || (status & PBE_SIM_NONFINITE)) {
        double m[4];
        lane_moments(u, g, dL, m);
        const double mu0 = group_sum<W>(wave_sum(m[0]), pr) * dL;
        if (out63 > 1e-12 * fmax(mu0, 1e-300)) status |= PBE_SIM_OUTFLOW;
    }
    if (lane == 64 * (W - 1)) {
        a.C[s] = C; a.t[s] = t; a.mu3[s] = mu3_old; a.outflow[s] = out63;
        a.step[s] = step; a.next[s] = next; a.status[s] = status;
    }
}

// One kernel per class of cells-per-lane K (1-8, 9-16; longer grids use the
// wave-pair kernel below): each class gets the register budget of its largest
// K instead of the global maximum.  The classes run concurrently, each over
// its own work queue.
// waves per SIMD each class is held to (the register budget follows: 4 -> 128,
// 3 -> 168, 2 -> 256 VGPRs); the 25-32 class needs the whole budget; the
// closure kernels hold the 1-8 class at 4 (a few spills, but one wave per
// simulation of a 4096-simulation batch fits the device at once) and the
// 9-16 class at 2
constexpr int fvm_waves_per_simd(int klo, int cl) {   // (kDissolve: as the plain laws)
    if (cl == kCorrect) return 2;   // the correction network's eight hidden units need the registers
    return (cl == kClosureBf16 || cl == kClosureFp64) ? (klo == 1 ? 4 : 2)
                                                      : klo == 1 ? 4 : klo == 9 ? 3 : klo == 17 ? 2 : 1;
}

// run simulation s with its K (uniform) in [KA, KHI]: a chain of scalar branches
template <int KA, int KHI, int SCHEME, int CL, bool TAPE = false>
__device__ __forceinline__ void run_k(const Fvm1dArgs& a, int s, int K) {
    if constexpr (KA <= KHI) {
        if (K == KA)
            run_sim<KA, SCHEME, CL, 1, TAPE>(a, s, nullptr);
        else
            run_k<KA + 1, KHI, SCHEME, CL, TAPE>(a, s, K);
    }
}

template <int SCHEME, int KLO, int KHI, int CL, bool TAPE = false>
__global__ __launch_bounds__(64, fvm_waves_per_simd(KLO, CL)) void k_fvm1d(Fvm1dArgs a, int cls_begin, int cls_count,
                                                                        int32_t* queue) {
    // Longer grids get higher issue priority where waves of different classes
    // share a SIMD: the simulations with the most cells per lane set the
    // makespan, the short ones fill the gaps.
    if constexpr (KLO >= 25) __builtin_amdgcn_s_setprio(3);
    else if constexpr (KLO >= 17) __builtin_amdgcn_s_setprio(2);
    else if constexpr (KLO >= 9) __builtin_amdgcn_s_setprio(1);
    for (;;) {
        // Every lane executes the atomic (only lane 0 adds 1) and the ticket
        // is lane 0's return value.  Popping inside `if (lane == 0)` instead
        // puts a divergent region in front of the broadcast: the loop is then
        // structurized so that lanes 1-63 re-enter without lane 0 and read a
        // stale index from it forever.
        const int ticket = atomicAdd(queue, threadIdx.x == 0 ? 1 : 0);
        const int idx = __builtin_amdgcn_readfirstlane(ticket);
        if (idx >= cls_count) break;
        const int s = uniform(a.order[cls_begin + idx]);
        const int K = uniform((a.ncell[s] + 63) >> 6);
        run_k<KLO, KHI, SCHEME, CL, TAPE>(a, s, K);
    }
}

// Grids of more than 1024 cells on a wave pair: K = ceil(N/128) = 9..16 cells
// per lane, so a long simulation gets the register budget (and occupancy) of
// the 513-1024-cell class and half the serial work per wave, at the price of
// the per-step scalar work done twice and a barrier per stage.  This wins when
// there are too few simulations to fill the device; with thousands of
// simulations one wave per simulation is faster.  The autotuner chooses.
template <int SCHEME>
__global__ __launch_bounds__(128) void k_fvm1d_pair(Fvm1dArgs a, int cls_begin, int cls_count, int32_t* queue) {
    __shared__ double xs[kPairSlots];
    __shared__ int ticket_slot;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    Pair pr{xs, w, 0};
    for (;;) {
        // wave 0 takes the ticket (branch-free within the wave, as in k_fvm1d)
        if (w == 0) {
            const int ticket = atomicAdd(queue, threadIdx.x == 0 ? 1 : 0);
            ticket_slot = __builtin_amdgcn_readfirstlane(ticket);
        }
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(ticket_slot);
        __syncthreads();   // the slot is rewritten only after both waves have read it
        if (idx >= cls_count) break;
        const int s = uniform(a.order[cls_begin + idx]);
        const int K = uniform((a.ncell[s] + 127) >> 7);
        switch (K - 9) {
            case 0: run_sim<9, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 1: run_sim<10, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 2: run_sim<11, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 3: run_sim<12, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 4: run_sim<13, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 5: run_sim<14, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 6: run_sim<15, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            case 7: run_sim<16, SCHEME, kClosureNone, 2>(a, s, &pr); break;
            default: break;
        }
    }
}

__global__ void k_reset_counter(int32_t* c, int n) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n) c[threadIdx.x] = 0;
}

}  // namespace

template <int SCHEME, int N>
static hipError_t launch_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* q,
                               hipStream_t st) {
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_fvm1d<SCHEME, 1, 8, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        case 1: hipLaunchKernelGGL((k_fvm1d<SCHEME, 9, 16, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        case 2:
            if (N == kClosureNone && a.pair_long)
                hipLaunchKernelGGL((k_fvm1d_pair<SCHEME>), dim3(n_blocks), dim3(128), 0, st, a, begin, count, q);
            else
                hipLaunchKernelGGL((k_fvm1d<SCHEME, 17, 24, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q);
            break;
        default: hipLaunchKernelGGL((k_fvm1d<SCHEME, 25, 32, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
    }
    return hipGetLastError();
}

// the closure kernels cover SSP-RK3 on grids up to 1024 cells (classes 0 and 1)
template <int CL>
static hipError_t launch_closure_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* q,
                                       hipStream_t st) {
    constexpr int R = PBE_SCHEME_SSPRK3;
    switch (cls) {
        case 0:
            if constexpr (CL == kClosureBf16 || CL == kClosureFp64) {
                if (a.ck_r) {   // a solve that will be differentiated
                    hipLaunchKernelGGL((k_fvm1d<R, 1, 8, CL, true>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q);
                    break;
                }
            }
            hipLaunchKernelGGL((k_fvm1d<R, 1, 8, CL>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q);
            break;
        case 1:
            if constexpr (CL == kClosureBf16 || CL == kClosureFp64) {
                if (a.ck_r) {
                    hipLaunchKernelGGL((k_fvm1d<R, 9, 16, CL, true>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q);
                    break;
                }
            }
            hipLaunchKernelGGL((k_fvm1d<R, 9, 16, CL>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fvm1d_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* queue,
                              hipStream_t st) {
    if (a.closure == kClosurePoly) return launch_closure_class<kClosurePoly>(cls, a, n_blocks, begin, count, queue, st);
    if (a.closure == kClosureBf16) return launch_closure_class<kClosureBf16>(cls, a, n_blocks, begin, count, queue, st);
    if (a.closure == kClosureFp64) return launch_closure_class<kClosureFp64>(cls, a, n_blocks, begin, count, queue, st);
    if (a.closure == kCorrect) {   // grids of up to 512 cells (the coarse grids it is meant for)
        if (cls != 0) return hipErrorInvalidValue;
        if (a.scheme == PBE_SCHEME_LW_TVD)
            hipLaunchKernelGGL((k_fvm1d<PBE_SCHEME_LW_TVD, 1, 8, kCorrect>), dim3(n_blocks), dim3(64), 0, st, a,
                               begin, count, queue);
        else
            hipLaunchKernelGGL((k_fvm1d<PBE_SCHEME_SSPRK3, 1, 8, kCorrect>), dim3(n_blocks), dim3(64), 0, st, a,
                               begin, count, queue);
        return hipGetLastError();
    }
    if (a.closure == kDissolve) {
        if (a.scheme == PBE_SCHEME_LW_TVD)
            return launch_class<PBE_SCHEME_LW_TVD, kDissolve>(cls, a, n_blocks, begin, count, queue, st);
        return launch_class<PBE_SCHEME_SSPRK3, kDissolve>(cls, a, n_blocks, begin, count, queue, st);
    }
    if (a.scheme == PBE_SCHEME_LW_TVD)
        return launch_class<PBE_SCHEME_LW_TVD, kClosureNone>(cls, a, n_blocks, begin, count, queue, st);
    return launch_class<PBE_SCHEME_SSPRK3, kClosureNone>(cls, a, n_blocks, begin, count, queue, st);
}

hipError_t launch_reset_counter(int32_t* counter, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter, n);
    return hipGetLastError();
}

template <int CL>
static hipError_t occupancy(int cls, int pairs, int* per_cu) {
    constexpr int R = PBE_SCHEME_SSPRK3;
    switch (cls) {
        case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fvm1d<R, 1, 8, CL>, 64, 0);
        case 1:   // (the correction runs the first class only)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                per_cu, k_fvm1d<R, 9, 16, CL == kCorrect ? kClosureNone : CL>, 64, 0);
        case 2:
            if (pairs) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fvm1d_pair<R>, 128, 0);
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                per_cu, k_fvm1d<R, 17, 24, CL == kDissolve ? kDissolve : kClosureNone>, 64, 0);
        default:
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(
                per_cu, k_fvm1d<R, 25, 32, CL == kDissolve ? kDissolve : kClosureNone>, 64, 0);
    }
}

int fvm1d_class_resident_blocks(int cls, int closure, int pairs) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = closure == kClosureBf16   ? occupancy<kClosureBf16>(cls, pairs, &per_cu)
                         : closure == kClosureFp64 ? occupancy<kClosureFp64>(cls, pairs, &per_cu)
                         : closure == kClosurePoly ? occupancy<kClosurePoly>(cls, pairs, &per_cu)
                         : closure == kDissolve    ? occupancy<kDissolve>(cls, pairs, &per_cu)
                         : closure == kCorrect     ? occupancy<kCorrect>(cls, pairs, &per_cu)
                                                   : occupancy<kClosureNone>(cls, pairs, &per_cu);
    if (e != hipSuccess) return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

}  // namespace pbe

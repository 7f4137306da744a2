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

template <int K, int SCHEME, int CL>
__device__ __forceinline__ void run_sim(const Fvm1dArgs& a, int s) {
    const int lane = threadIdx.x;
    const int N = uniform(a.ncell[s]);
    const int64_t base = (int64_t)uniform((int)a.off[s]) | ((int64_t)uniform((int)(a.off[s] >> 32)) << 32);
    const double Lmax = uniform(a.Lmax[s]);
    const double dL = Lmax / N;
    const SimParams q = load_params(a.par + (size_t)s * PBE_NPAR);
    const Process p{a.law, a.scheme, a.sol_law, a.cs0, a.cs1, a.alpha, a.cfl, a.dt_max, a.t_end};
    const int ns = a.n_samples;
    const double* ts = a.t_samples;

    const int pad = 64 * K - N;
    LaneGeom g;
    g.xb = (double)(lane * K - pad);
    g.gdL = q.gamma * dL;
    g.npad = min(max(pad - lane * K, 0), K);
    const int i0 = lane * K - pad;   // cell index of slot 0

    double u[K];
    load_cells(u, (a.from_initial ? a.f0 : a.f) + base, i0, g.npad, 0.0);

    double C, t, mu3_old, out;
    int step, next, status;
    if (a.from_initial) {
        C = uniform(a.C0[s]);
        t = 0.0;
        mu3_old = wave_sum(lane_moment3(u, g, dL)) * dL;
        out = 0.0;
        step = 0; next = 0; status = 0;
    } else {
        C = a.C[s]; t = a.t[s]; mu3_old = a.mu3[s]; out = a.outflow[s];
        step = a.step[s]; next = a.next[s]; status = a.status[s];
    }
    C = uniform(C); t = uniform(t); mu3_old = uniform(mu3_old);
    step = uniform(step); next = uniform(next); status = uniform(status);

    for (int it = 0; it < a.max_steps; ++it) {
        if (!(t < p.t_end) || (status & PBE_SIM_NONFINITE)) break;
        // keep per-cell geometry from being hoisted out of the time loop into registers
        asm volatile("" : "+v"(g.xb));
        if (step >= a.step_cap) { status |= PBE_SIM_STEPCAP; break; }
        Rates r;
        if constexpr (CL == kClosureNone) {
            r = rates_plain(p, q, C, t);
        } else {
            // learned closure: inputs S, T and mu_2 of the current state
            LaneGeom g2 = g;
            asm volatile("" : "+v"(g2.xb));
            const double mu2 = wave_sum(lane_moment2(u, g2, dL)) * dL;
            const ClosureRates cr = closure_rates<false, CL>(a.cd, p, q, C, t, mu2);
            r.G0 = cr.G0;
            r.B = cr.B;
            r.S = cr.S;
            if (cr.fallback) status |= PBE_SIM_FALLBACK;
        }
        const double t_next = uniform(next < ns ? ts[min(next, ns - 1)] : p.t_end);
        double dt;
        const bool hit = choose_dt(p, r.G0, q.gamma, Lmax, dL, t, t_next, &dt);
        if (!(dt > 0.0) || !isfinite(dt)) {   // rates overflowed: stop this sim
            status |= PBE_SIM_NONFINITE;
            break;
        }
        // nucleation: ghost cells at L < 0 hold B/G0 so the flux through L = 0 is B
        const double ghost = r.G0 > 0.0 ? r.B / r.G0 : 0.0;

        if (a.ckpt_every > 0 && step % a.ckpt_every == 0) {
            const int c = step / a.ckpt_every;
            if (c < a.n_ckpt) {
                store_cells(u, a.ck_f + base * a.n_ckpt + (int64_t)c * N, i0, g.npad);
                if (lane == 0) {
                    a.ck_C[(int64_t)s * a.n_ckpt + c] = C;
                    a.ck_t[(int64_t)s * a.n_ckpt + c] = t;
                }
            }
        }

        const double cour = dt * r.G0 / dL;
        const double hN = fvm_step<K, SCHEME>(u, g, cour, ghost);
        out = fma(dt * r.G0, hN, out);

        // discrete solute balance, Eq. (9): C^{n+1} = C^n - alpha (mu3^{n+1} - mu3^n)
        LaneGeom gm = g;
        asm volatile("" : "+v"(gm.xb));
        const double mu3 = wave_sum(lane_moment3(u, gm, dL)) * dL;
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
                for (int j = 0; j < 4; ++j) m[j] = wave_sum(m[j]) * dL;
                if (lane == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) a.mom_s[o * 4 + j] = m[j];
                    a.C_s[o] = C;
                    a.samp_step[o] = step;
                }
                if (a.record_f) store_cells(u, a.f_s + base * ns + (int64_t)next * N, i0, g.npad);
                ++next;
            }
        }
    }

    // save the running state
    store_cells(u, a.f + base, i0, g.npad);
    const double out63 = lane_value(out, 63);
    if (!(t < p.t_end) || (status & PBE_SIM_NONFINITE)) {
        double m[4];
        lane_moments(u, g, dL, m);
        const double mu0 = wave_sum(m[0]) * dL;
        if (out63 > 1e-12 * fmax(mu0, 1e-300)) status |= PBE_SIM_OUTFLOW;
    }
    if (lane == 0) {
        a.C[s] = C; a.t[s] = t; a.mu3[s] = mu3_old; a.outflow[s] = out63;
        a.step[s] = step; a.next[s] = next; a.status[s] = status;
    }
}

// One kernel per class of cells-per-lane K (1-8, 9-16, 17-24, 25-32): each
// class gets the register budget of its largest K instead of the global
// maximum.  The classes run concurrently, each over its own work queue.
template <int SCHEME, int KLO, int CL>
__global__ __launch_bounds__(64) void k_fvm1d(Fvm1dArgs a, int cls_begin, int cls_count, int32_t* queue) {
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
        switch (K - KLO) {
            case 0: run_sim<KLO + 0, SCHEME, CL>(a, s); break;
            case 1: run_sim<KLO + 1, SCHEME, CL>(a, s); break;
            case 2: run_sim<KLO + 2, SCHEME, CL>(a, s); break;
            case 3: run_sim<KLO + 3, SCHEME, CL>(a, s); break;
            case 4: run_sim<KLO + 4, SCHEME, CL>(a, s); break;
            case 5: run_sim<KLO + 5, SCHEME, CL>(a, s); break;
            case 6: run_sim<KLO + 6, SCHEME, CL>(a, s); break;
            case 7: run_sim<KLO + 7, SCHEME, CL>(a, s); break;
            default: break;
        }
    }
}

__global__ void k_reset_counter(int32_t* c, int n) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n) c[threadIdx.x] = 0;
}

}  // namespace

template <int SCHEME>
static hipError_t launch_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* q,
                               hipStream_t st) {
    constexpr int N = kClosureNone;
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_fvm1d<SCHEME, 1, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        case 1: hipLaunchKernelGGL((k_fvm1d<SCHEME, 9, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        case 2: hipLaunchKernelGGL((k_fvm1d<SCHEME, 17, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        default: hipLaunchKernelGGL((k_fvm1d<SCHEME, 25, N>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
    }
    return hipGetLastError();
}

// the closure kernels cover SSP-RK3 on grids up to 1024 cells (classes 0 and 1)
template <int CL>
static hipError_t launch_closure_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* q,
                                       hipStream_t st) {
    constexpr int R = PBE_SCHEME_SSPRK3;
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_fvm1d<R, 1, CL>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        case 1: hipLaunchKernelGGL((k_fvm1d<R, 9, CL>), dim3(n_blocks), dim3(64), 0, st, a, begin, count, q); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fvm1d_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* queue,
                              hipStream_t st) {
    if (a.closure == kClosureBf16) return launch_closure_class<kClosureBf16>(cls, a, n_blocks, begin, count, queue, st);
    if (a.closure == kClosureFp64) return launch_closure_class<kClosureFp64>(cls, a, n_blocks, begin, count, queue, st);
    if (a.scheme == PBE_SCHEME_LW_TVD) return launch_class<PBE_SCHEME_LW_TVD>(cls, a, n_blocks, begin, count, queue, st);
    return launch_class<PBE_SCHEME_SSPRK3>(cls, a, n_blocks, begin, count, queue, st);
}

hipError_t launch_reset_counter(int32_t* counter, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter, n);
    return hipGetLastError();
}

template <int CL>
static hipError_t occupancy(int cls, int* per_cu) {
    constexpr int R = PBE_SCHEME_SSPRK3;
    switch (cls) {
        case 0: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fvm1d<R, 1, CL>, 64, 0);
        case 1: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fvm1d<R, 9, CL>, 64, 0);
        case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fvm1d<R, 17, kClosureNone>, 64, 0);
        default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_fvm1d<R, 25, kClosureNone>, 64, 0);
    }
}

int fvm1d_class_resident_blocks(int cls, int closure) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = closure == kClosureBf16   ? occupancy<kClosureBf16>(cls, &per_cu)
                         : closure == kClosureFp64 ? occupancy<kClosureFp64>(cls, &per_cu)
                                                   : occupancy<kClosureNone>(cls, &per_cu);
    if (e != hipSuccess) return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

}  // namespace pbe

// Internal kernel argument blocks and launchers shared by the host library
// (pbe_api.cpp) and the HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbe.h"

namespace pbe {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxCellsPerLane = 32;  // 1D grids up to 64*32 = 2048 cells per wavefront
// leading guard (in doubles) of every per-cell device array: a lane's slot-0
// pointer may sit up to 64*K - N < 2048 cells before a simulation's first cell
constexpr int kCellGuard = 2048;

// Learned closure operands on the device (packed by pack_closure from the
// weight blob; layout described in closure_device.h).
struct ClosureDev {
    const double* w64;       // fp64 pack: W1[64][3] b1[64] W2T[64][64] (W2T[i][j] = W2[j][i]) b2[64] W3[2][64] b3[2]
    const uint2* a1;         // layer 1 A operands [4 tiles][64 lanes], 4 bf16 each
    const uint4* a2;         // layer 2 A operands [4 tiles][2 k-steps][64 lanes], 8 bf16 each
    const uint4* a3;         // layer 3 A operands [2 k-steps][64 lanes]
    const uint4* a2t;        // W2 transposed, for the backward [4][2][64]
    const float* bias;       // b1[64] b2[64] b3[2] pad[2]
    const float* w3r;        // W3 rounded to bfloat16, as float [2][64]
    const double* c;         // the 18 constants (normalisation, output scaling, box, s_min, lnG0_max)
    int32_t precision;       // PBE_MLP_BF16 or PBE_MLP_FP64
    int32_t pad_;
};

// rate-law variants of the 1D kernels: the plain laws, the learned closure
// (bf16 or fp64 network) and the polynomial growth law
// rate path of the kernels: the plain laws (growth only), the learned closure
// (bf16 / fp64), the polynomial growth law, the plain laws with dissolution
// below saturation, or the plain laws with the in-the-loop correction
enum { kClosureNone = 0, kClosureBf16 = 1, kClosureFp64 = 2, kClosurePoly = 3, kDissolve = 4, kCorrect = 5 };
constexpr int kMaxPoly = 1024;   // polynomial coefficients per simulation

// per step of a learned-closure solve: flags (1 = fallback, 2 = ln G0 clamped),
// G0, B, z0, z1, z2, dy0/dz_i and dy1/dz_i for i = 0, 1, 2 (pairs), mu2
constexpr int kClosureTape = 13;

// per taped step, as the forward formed them: G0, B, S,
// ln S, the two Arrhenius factors, S^g, S^b, dt, landed-on-a-sample flag,
// inflow ghost, Courant factor, Csat(T), dS/dT, dT/dt, 1/(T + 273.15)^2
constexpr int kStepTape = 16;

// Everything the 1D forward kernel reads or writes.  Device pointers only.
struct Fvm1dArgs {
    int32_t n_sims, n_samples;
    int32_t law, scheme, sol_law, record_f;
    double cs0, cs1, alpha, cfl, dt_max, t_end;
    const double* t_samples;   // [n_samples]
    const int32_t* order;      // [S] sims in launch order (longest first)
    int32_t* queue;            // work counter, zeroed before each launch
    const int64_t* off;        // [S+1] packed cell offsets
    const int32_t* ncell;      // [S]
    const double* Lmax;        // [S]
    const double* par;         // [S*PBE_NPAR]
    const double* C0;          // [S]
    const double* f0;          // [sum N] initial densities
    // running state (resumable between launches)
    double* f;                 // [sum N]
    double* C;                 // [S]
    double* t;                 // [S]
    double* mu3;               // [S] volume moment of the current state
    double* outflow;           // [S] number that left through L_max
    int32_t* step;             // [S]
    int32_t* next;             // [S] index of the next sample time
    int32_t* status;           // [S] PBE_SIM_* bits
    // recorded samples
    double* mom_s;             // [S][n_samples][4]
    double* C_s;               // [S][n_samples]
    double* f_s;               // [sum N * n_samples] (record_f) sim-major
    int32_t* samp_step;        // [S][n_samples] step index at which each sample was taken
    // checkpoints of (f, C, t) every ckpt_every steps
    double* ck_f;              // [sum N * n_ckpt]
    double* ck_C;              // [S * n_ckpt]
    double* ck_t;              // [S * n_ckpt]
    int32_t ckpt_every, n_ckpt;
    int32_t max_steps;         // steps allowed in this launch
    int32_t from_initial;      // 1: start from (f0, C0, t = 0)
    int32_t step_cap;          // absolute per-sim step limit (PBE_SIM_STEPCAP when hit)
    int32_t pair_long;         // 1: class 2 runs grids > 1024 cells on wave pairs
    int32_t closure;           // kClosure*: which rate law the kernels run
    ClosureDev cd;             // closure == kClosureBf16 / kClosureFp64
    double* rate_log;          // [S][step_cap][3] (dt, G0, B) of every step, or null
    const double* poly;        // closure == kClosurePoly: [S][n_poly] growth coefficients a_1..a_k
    const double* corr;        // closure == kCorrect: [S][PBE_CORR_NW] in-the-loop correction weights
    int32_t n_poly, pad1_;
    // learned closure with checkpoints: [S][step_cap][kClosureTape] the closure
    // quantities of every step, taped by the forward for the adjoint; else null
    double* ck_r;
    // learned closure checkpointed at every step: [S][step_cap][kStepTape] the
    // step scalars of every step, so the adjoint recomputes nothing; else null
    double* ck_s;
};

// Adjoint of the 1D solve (reverse sweep over checkpointed segments).
struct Adj1dArgs {
    Fvm1dArgs fw;              // forward description (state buffers are read-only here)
    const double* gf;          // cotangent of the recorded f (or final f), may be null
    const double* gmom;        // [S][n_samples][4], may be null
    const double* gC;          // [S][n_samples], may be null
    double* gpar;              // [S][PBE_NGRAD] output
    double* tape;              // [sum N * ckpt_every] per-sim segment tape of states
    double* tape_C;            // [S * ckpt_every]
    double* tape_t;            // [S * ckpt_every]
    double* tape_s;            // [S * ckpt_every * kStepTape] per-step scalars of the plain laws
    double* rows;              // [S * row_cap * 5] per-step (z0, z1, z2, ybar0, ybar1) for the weight gradient
    int32_t row_cap;           // rows per simulation (>= step_cap, multiple of 16)
    int32_t gf_is_final;       // 1: gf is the cotangent of the final state (no RECORD_F)
    double* gpoly;             // polynomial law: [S][n_poly] d/d(a_1..a_k) output
};

// 2D Godunov-split solver: per global step one pass over tiles that sweeps
// L1 and then L2 (double buffered) with moment partials, and a per-sim finalize.
struct Fvm2dArgs {
    int32_t n_sims, n_samples;
    int32_t law, sol_law, scheme, strang;   // strang: Strang splitting (else Godunov, L1 then L2)
    double cs0, cs1, alpha, cfl, dt_max, t_end;
    const double* t_samples;
    const int64_t* off;        // [S+1] cell offsets (sim s stored [n2][n1])
    const int32_t* n1;         // [S]
    const int32_t* n2;         // [S]
    const double* L1;          // [S]
    const double* L2;          // [S]
    const double* par;         // [S*PBE_NPAR]
    const double* C0;          // [S]
    const double* f0;          // [sum n1*n2]
    double* buf[2];            // state buffers: before global step g the state is in buf[g % 2]
    // per-sim scalars
    double* C;                 // [S]
    double* t;                 // [S]
    double* mu12;              // [S] volume moment of the current state
    double* outflow;           // [S] number that left through L1_max and L2_max
    int32_t* step;             // [S]
    int32_t* next;             // [S]
    int32_t* status;           // [S]
    int32_t* active;           // [S] 1 while the sim still steps
    int32_t* n_active;         // [1] number of active sims after the last finalize
    double* c1;                // [S] Courant factors dt*G/dL of the current step
    double* c2;
    double* gh1;               // [S] inflow ghost of row 0 (L1 sweep) and column 0 (L2 sweep)
    double* gh2;
    double* dt;                // [S]
    int32_t* hit;              // [S] step lands on the next sample time
    // tiles (step2d_tile_width(scheme) columns x seg rows), sim by sim
    const int32_t* cb_sim;     // [n_cb]
    const int32_t* cb_col0;
    const int32_t* cb_row0;
    const int32_t* cb_first;   // [S+1] first tile of each sim
    int32_t n_cb, seg;
    double* part;              // [n_cb][5] moments mu_00, mu_10, mu_01, mu_12 of the new state and outflow
    double* mom_s;             // [S][n_samples][4]: mu_00, mu_10, mu_01, mu_12
    double* C_s;               // [S][n_samples]
    int32_t* samp_step;        // [S][n_samples]
    int32_t step_cap;
    int32_t pad_;
};

// Launchers (defined in the .hip files).  Return hipSuccess or the launch error.
// 1D solve kernel classes by cells per lane K = ceil(N/64): class c covers
// kSolveKlo[c] <= K < kSolveKlo[c + 1].  The last class holds the grids that
// need the whole register file (one wave per SIMD).
constexpr int kFvmClasses = 4;
constexpr int kSolveKlo[kFvmClasses + 1] = {1, 9, 17, 25, 33};
inline int fvm1d_class_of(int n_cells) {
    const int K = (n_cells + 63) / 64;
    return K < kSolveKlo[1] ? 0 : K < kSolveKlo[2] ? 1 : K < kSolveKlo[3] ? 2 : 3;
}
// 1D solves: one wavefront per simulation in the four classes above, or
// (pairs) grids of more than 1024 cells on a wave pair with K = ceil(N/128) =
// 9..16 in class 2 and class 3 empty.  Classes 0 and 1 are the same either way.
inline int solve1d_class_of(int n_cells, bool pairs) {
    return pairs ? (n_cells <= 512 ? 0 : n_cells <= 1024 ? 1 : 2) : fvm1d_class_of(n_cells);
}
hipError_t launch_fvm1d_class(int cls, const Fvm1dArgs& a, int n_blocks, int begin, int count, int32_t* queue,
                              hipStream_t st);
hipError_t launch_reset_counter(int32_t* counter, int n, hipStream_t st);
int fvm1d_class_resident_blocks(int cls, int closure, int pairs);
constexpr int kAdjClasses = 2;   // adjoint classes: cells per lane 1-8, 9-16 (grids up to 1024 cells)
hipError_t launch_adj1d_class(int cls, const Adj1dArgs& A, int n_blocks, int begin, int count, int32_t* queue,
                              hipStream_t st);
int adj1d_class_resident_blocks(int cls, int closure);
int step2d_tile_width(int scheme, int strang);   // output columns of one 2D tile
hipError_t launch_step2d(const Fvm2dArgs& a, int parity, hipStream_t st);
hipError_t launch_final2d(const Fvm2dArgs& a, int init, hipStream_t st);
hipError_t launch_out2d(const Fvm2dArgs& a, double* f_out, hipStream_t st);
// learned closure (closure.hip)
constexpr int kMlpWeights = 4546, kMlpConsts = 18;
size_t closure_pack_bytes();
hipError_t pack_closure(const float* d_blob, void* mem, int precision, ClosureDev* cd, hipStream_t st);
hipError_t launch_closure_forward(const ClosureDev& cd, int n, const double* x, double* y, double* dy, hipStream_t st);
hipError_t launch_closure_grad(const ClosureDev& cd, const double* rows, const int32_t* steps, int n_sims,
                               int row_cap, double* partial, int n_blocks, double* out, hipStream_t st);
hipError_t launch_stage_rows(int n, int row_cap, const double* z, const double* ybar, double* rows, int32_t* steps,
                             hipStream_t st);
hipError_t launch_adam(float* w, float* m, float* v, const double* g, int n, int step, float lr, float b1, float b2,
                       float eps, hipStream_t st);

}  // namespace pbe

// extra per-sim status bit used internally and reported through status_out
#define PBE_SIM_STEPCAP 8

/*
 * pbe.h - C ABI of the MI355X (gfx950) crystallization population-balance solver.
 *
 * The library advances many independent batch-crystallizer simulations on one
 * GPU.  Each simulation solves the growth population balance (paper Sec. 2.1,
 * Eq. (1), in one size coordinate or in two with Godunov splitting) with the
 * high-resolution finite-volume flux and van Leer limiter (Eq. (8), SI
 * Eqs. (S1)-(S2)), a CFL-limited step (SI Eq. (S3)), nucleation entering as a
 * flux at L = 0, and the discrete solute balance (Eq. (9)) that sets the
 * supersaturation driving the rate laws (App. A).  pbe_grad returns exact
 * derivatives of recorded outputs (the paper's reverse-mode use, Sec. 4.1,
 * Eq. (10)) through a hand-written discrete adjoint with checkpointing.
 *
 * Conventions (all entry points):
 *   - Every call returns a pbe_status code; nothing throws across the ABI.
 *     Argument errors are detected on the host before any device work.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Units: L um, t s, T degC, f #/(m^3 um^ndim), G um/s, B #/(m^3 s),
 *     C g solute / g solvent.  The rate constant kg is given in m/s.
 *   - Layouts: 1D sims are packed back to back, sim s occupying
 *     [off_s, off_s + N_s) with off_0 = 0, off_{s+1} = off_s + N_s.
 *     2D sims occupy n1_s*n2_s cells stored [n2][n1] (L1 contiguous).
 *   - Per-sim parameter row par[s*PBE_NPAR + k], k = PBE_P_*.
 */
#ifndef PBE_H
#define PBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbe_handle pbe_handle;

typedef enum {
    PBE_OK = 0,
    PBE_EINVAL = -1,        /* invalid argument (checked on the host, nothing launched) */
    PBE_ENOMEM = -2,        /* device allocation failed; nothing leaked */
    PBE_EDEVICE = -3,       /* HIP runtime error */
    PBE_ENONFINITE = -4,    /* reserved: per-sim non-finite states are reported in status_out */
    PBE_ESTATE = -5,        /* call not valid in the handle's current state */
    PBE_EUNSUPPORTED = -6   /* combination of options not implemented */
} pbe_status;

enum { PBE_SCHEME_SSPRK3 = 0,   /* method of lines, Shu-Osher SSP-RK3, kappa = 1 flux */
       PBE_SCHEME_LW_TVD = 1 }; /* the paper's one-step limited update, Eq. (8) */
enum { PBE_LAW_POWER = 0,       /* G = kg S^g (1 + gamma L), B = kb S^b, S = C/Csat - 1 */
       PBE_LAW_ARRHENIUS = 1,   /* power law times exp(-Eg/(T+273.15)), exp(-Eb/(T+273.15)) (App. A, Eq. A.2) */
       PBE_LAW_MLP = 2,         /* learned closure for (G0, B); see pbe_problem.mlp */
       PBE_LAW_POLY = 3 };      /* G0 = a_1 S + ... + a_k S^k (um/s), B = kb S^b: the polynomial
                                   growth law of Sec. 4.1, Eq. (poly_growth_rate); see pbe_problem.poly */
enum { PBE_SOL_LINEAR = 0,      /* Csat = cs0 + cs1 T */
       PBE_SOL_EXP = 1 };       /* Csat = cs0 exp(cs1 T) (App. A, Eq. A.1) */
/* per-sim status bits written to status_out */
enum { PBE_SIM_OK = 0, PBE_SIM_NONFINITE = 1, PBE_SIM_OUTFLOW = 2, PBE_SIM_FALLBACK = 4 };
/* pbe_problem.flags */
enum { PBE_FLAG_DEVICE_PTRS = 1,  /* output/cotangent pointers are device memory, stream-ordered */
       PBE_FLAG_RECORD_F = 2,     /* record the number density at every sample time */
       PBE_FLAG_AUTOTUNE = 4,     /* 2D: pick the launch shape with pbe_tune at create (cached per
                                     process); 1D: PBE_EUNSUPPORTED (see pbe_tune) */
       PBE_FLAG_RECORD_RATES = 8,    /* 1D: record (dt, G0, B) of every step, read with pbe_rate_log */
       PBE_FLAG_STRANG = 16 };       /* 2D: Strang splitting, L1 over dt/2, L2 over dt, L1 over dt/2,
                                        instead of Godunov's L1 then L2 (Sec. 2.1); 1D: PBE_EUNSUPPORTED */

/* per-sim parameter row */
/* kg [m/s], g, kb [#/(m^3 s)], b, gamma [1/um], kg2, g2 (2D second axis), Eg, Eb [K] (Arrhenius
 * law), T0, T1 [degC], t_ramp [s], Eg2 [K] (2D second axis, Arrhenius law: App. A Eq. (A.2) takes
 * one activation temperature per axis), kd [m/s], d: dissolution.  In an undersaturated solution
 * (C < Csat) the power and Arrhenius laws of a 1D simulation shrink the crystals at
 * G0 = -1e6 kd (1 - C/Csat)^d um/s (the growth/dissolution rate of SI S1.1; this law mirrors the
 * growth power law) with no nucleation; the upwind side of every face flips, crystals leave through
 * L = 0 and nothing enters through L_max.  kd = 0 (the default) leaves them unchanged there.
 * kd > 0 is refused (PBE_EUNSUPPORTED) by the 2D path, the other laws, and pbe_grad. */
enum { PBE_P_KG = 0, PBE_P_G, PBE_P_KB, PBE_P_B, PBE_P_GAMMA, PBE_P_KG2, PBE_P_G2, PBE_P_EG, PBE_P_EB,
       PBE_P_T0, PBE_P_T1, PBE_P_TRAMP, PBE_P_EG2, PBE_P_KD, PBE_P_D, PBE_NPAR };
#define PBE_NGRAD 5   /* pbe_grad returns d/d(kg, g, kb, b, gamma) per sim */

/* Learned closure (law PBE_LAW_MLP): the empirical hybrid model of Sec. 4.2,
 * Fig. 5a, in which a network replaces the growth/nucleation rate laws.
 * Blob of PBE_MLP_NW weights then PBE_MLP_NC constants (float):
 *   W1[64][3] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]
 *   in_shift[3] in_scale[3] out_shift[2] out_scale[2] lo[3] hi[3] s_min lnG0_max
 * Inputs x = (S, T [degC], log10 mu_2) with S = C/Csat - 1 and mu_2 of the
 * current state; z = (x - in_shift) * in_scale; h1 = tanh(W1 z + b1),
 * h2 = tanh(W2 h1 + b2), y = W3 h2 + b3; ln G0 = min(out_shift0 + out_scale0 y0,
 * lnG0_max) (G0 in um/s; held at the bound, with zero derivative, above it, which
 * bounds the number of CFL-limited steps) and ln B = out_shift1 + out_scale1 y1.
 * Where S <= s_min,
 * mu_2 <= 0 or x leaves [lo, hi], the power law with the sim's (kg, g, kb, b)
 * is used and PBE_SIM_FALLBACK is set.  PBE_MLP_BF16: bfloat16 weights and
 * activations on the matrix cores with fp32 accumulation; PBE_MLP_FP64: fp64.
 * The closure runs the SSP-RK3 scheme on grids of up to 1024 cells. */
#define PBE_MLP_NW 4546
#define PBE_MLP_NC 18
enum { PBE_MLP_BF16 = 0, PBE_MLP_FP64 = 1 };

typedef struct {
    int32_t ndim;               /* 1 or 2 */
    int32_t n_sims;             /* S >= 1 */
    const int32_t *n_cells;     /* host [S*ndim]; 1D: N_s in [4, 2048]; 2D: (n1_s, n2_s) in [4, 4096] */
    const double *L_max;        /* host [S*ndim] domain lengths, um */
    const double *f0;           /* host, packed initial densities (see layouts) */
    const double *C0;           /* host [S] initial concentration */
    const double *par;          /* host [S*PBE_NPAR] kinetics and the cooling ramp
                                   T(t) = T0 + (T1 - T0) min(t, t_ramp)/t_ramp */
    const float *mlp;           /* host, law == PBE_LAW_MLP only: closure blob of PBE_MLP_NW + PBE_MLP_NC
                                   floats (layout below); copied at create */
    int32_t law, scheme, sol_law;
    int32_t n_samples;          /* >= 1 */
    double cs0, cs1;            /* solubility coefficients */
    double alpha;               /* rho_c k_v / rho_solvent: C drop per unit volume moment */
    double cfl;                 /* Courant number nu in (0, 1] */
    double dt_max;              /* cap on the step size, s */
    double t_end;               /* end time, s */
    const double *t_samples;    /* host [n_samples], strictly ascending in (0, t_end] */
    int32_t ckpt_every;         /* 0: no gradients; K > 0: checkpoint every K steps for pbe_grad (1D) */
    int32_t max_steps;          /* per-sim step budget (0: derived from t_end, dt_max and the CFL bound) */
    int32_t flags;              /* PBE_FLAG_* */
    int32_t mlp_precision;      /* law == PBE_LAW_MLP: PBE_MLP_BF16 or PBE_MLP_FP64 */
    int32_t n_poly;             /* law == PBE_LAW_POLY: coefficients per sim, k in [1, PBE_MAX_POLY] */
    const double *poly;         /* law == PBE_LAW_POLY: host [S][n_poly] a_1..a_k, finite and >= 0 (the
                                   paper's constraint); grids of up to 1024 cells, SSP-RK3 */
    const double *corr;         /* NULL, or host [S][PBE_CORR_NW]: weights of the in-the-loop correction
                                   (below), per sim; 1D grids of up to 512 cells (the coarse grids it
                                   stands in for fine ones on), power or Arrhenius law without
                                   dissolution, forward only (ckpt_every = 0) */
} pbe_problem;
#define PBE_MAX_POLY 1024

/* In-the-loop correction (Sec. 4.2, Fig. 5b: a network inside the time loop
 * that offsets the discretisation error of each step, so a coarse grid can
 * stand in for a fine one).  After every growth step (G0 > 0) each interior
 * face i+1/2 (0 <= i <= N-2) of a simulation gets the correction flux
 *   Y = sigma nu (W2 . tanh(W1 x + b1) + b2),  x = (f_{i-1}, f_i, f_{i+1}, f_{i+2}) / sigma, nu,
 * sigma = max |f_{i-1..i+2}| (Y = 0 where sigma = 0; cells outside the domain
 * read 0), nu = dt G0 (1 + gamma L_face) / dL the face's Courant number; then
 * f_i += Y_{i-1/2} - Y_{i+1/2}.  The faces at L = 0 and L_max are left alone,
 * so the number balance and every boundary flux are the solver's.  Weights
 * (FP64): W1[8][5] b1[8] W2[8] b2. */
#define PBE_CORR_H 8
#define PBE_CORR_NW 57

/* Create a handle: validates `p`, deep-copies every input to device memory
 * (the caller may free its buffers on return), orders the sims for the
 * persistent launch and records the launch graph.  `hip_stream` is the HIP
 * stream all work is ordered on (NULL = default stream).  The state starts at
 * the initial condition of Sec. 2.1 Eqs. (3)-(7): the seed f0 and c0, at t = 0.
 * Errors: PBE_EINVAL (any field out of range), PBE_ENOMEM, PBE_EDEVICE. */
int pbe_create(const pbe_problem *p, void *hip_stream, pbe_handle **out);

/* Advance every unfinished simulation by at most n_steps time steps from its
 * current state (the initial condition after create/reset): n_steps turns of
 * the loop of Sec. 2.2 Fig. 1 (rates, step size, PSSD update, moments, solute
 * balance).  Samples falling inside are recorded.  If n_active_out != NULL the
 * call waits and stores the number of sims that have not reached t_end. */
int pbe_step(pbe_handle *h, int32_t n_steps, int32_t *n_active_out);

/* Restart from the initial condition (Sec. 2.1 Eqs. (3)-(7)). */
int pbe_reset(pbe_handle *h);

/* Solve every simulation from the initial condition to t_end (one graph launch)
 * and write:
 *   f_out      RECORD_F: densities at each sample, sim-major [s][sample][cells_s];
 *              otherwise the final densities, packed [sum cells].
 *   mom_out    [S][n_samples][4]: 1D mu_0..mu_3 (SI Eq. (S5), midpoint rule);
 *              2D mu_00, mu_10, mu_01, mu_12.
 *   C_out      [S][n_samples] concentration at the samples.
 *   steps_out  [S] steps taken;  status_out [S] PBE_SIM_* bits.
 * Any output may be NULL.  With PBE_FLAG_DEVICE_PTRS outputs are device
 * pointers written stream-ordered and the call returns without waiting;
 * otherwise they are host pointers and the call blocks.
 * With ckpt_every > 0 the forward pass also stores checkpoints for pbe_grad;
 * under law == MLP it also evaluates the network's input Jacobian at every step
 * and keeps it with the step's network inputs and rates (104 B per sim-step,
 * sized by the step cap), so that pbe_grad does not evaluate the network again;
 * with ckpt_every == 1 it keeps every step's state and step scalars (8 B per
 * cell and 128 B per sim per step, sized by the step cap) and pbe_grad
 * recomputes nothing. */
int pbe_solve(pbe_handle *h, double *f_out, double *mom_out, double *C_out,
              int32_t *steps_out, int32_t *status_out);

/* Copy the current state (after pbe_step) and the samples recorded so far
 * into the same outputs as pbe_solve (f_out is the current density unless
 * RECORD_F).  Samples not yet reached read as 0. */
int pbe_fetch(pbe_handle *h, double *f_out, double *mom_out, double *C_out,
              int32_t *steps_out, int32_t *status_out);

/* Vector-Jacobian product of the outputs of the last pbe_solve (1D only),
 * the reverse-mode derivative of the paper's Sec. 4.1 (Eq. (10)) / SI S2.1:
 * given cotangents gf (shape of f_out), gmom (shape of mom_out), gC (shape
 * of C_out) - each may be NULL for zero - write
 *   gpar_out  [S][PBE_NGRAD] = d<cot, outputs>/d(kg, g, kb, b, gamma) per sim,
 *   gmlp_out  law == MLP: [PBE_MLP_NW] d<cot, outputs>/d(closure weights), summed over sims
 *             (double, not float: the sum runs over every (sim, step) row, ~1e7 of them)
 *             (may be NULL); ignored for other laws.
 * Every step size is differentiated in the branch the forward solve took: a
 * CFL-limited step (SI Eq. (S3)) through G0 and gamma, a step landing on a
 * sample time through the time reached, the time through the temperature of
 * the cooling ramp; steps of dt_max are constants.  Which branch each step
 * takes, and so the step count, is piecewise constant and not differentiated.
 * A sim that did not reach t_end (PBE_SIM_NONFINITE or the step cap) gets NaN.
 * Requires ckpt_every > 0 and a completed pbe_solve (PBE_ESTATE otherwise). */
int pbe_grad(pbe_handle *h, const double *gf, const double *gmom, const double *gC,
             double *gpar_out, double *gmlp_out);

/* Replace every sim's polynomial growth coefficients (law == PBE_LAW_POLY) with
 * poly[S][n_poly] (host, or device with PBE_FLAG_DEVICE_PTRS; host values are
 * checked to be finite and >= 0) and restart from the initial condition.
 * Waits for the handle's queued work.  PBE_ESTATE for other laws, or (host
 * pointers, derived step budget) when the new law's step bound exceeds the
 * budget sized at create. */
int pbe_set_poly(pbe_handle *h, const double *poly);

/* Replace every sim's correction weights (a handle created with pbe_problem.corr)
 * with corr[S][PBE_CORR_NW] (host, or device with PBE_FLAG_DEVICE_PTRS; host
 * values are checked to be finite) and restart from the initial condition.
 * Waits for the handle's queued work.  PBE_ESTATE for a handle without the
 * correction.  Training loops perturb the weights of many copies of a
 * simulation in one call (batched forward differences). */
int pbe_set_corr(pbe_handle *h, const double *corr);

/* pbe_grad for the polynomial growth law (Sec. 4.1: the gradient of the
 * estimation loss with respect to the law's coefficients): the same
 * vector-Jacobian product of the last solve's outputs, written as
 *   gpar_out   [S][PBE_NGRAD] as in pbe_grad (kg and g do not enter: 0), may be NULL,
 *   gpoly_out  [S][n_poly] d<cot, outputs>/d(a_1..a_k) per sim.
 * Same conditions as pbe_grad; PBE_ESTATE for other laws. */
int pbe_grad_poly(pbe_handle *h, const double *gf, const double *gmom, const double *gC, double *gpar_out,
                  double *gpoly_out);

/* Replace the closure weights (law == MLP) with w[PBE_MLP_NW] (host pointer,
 * or device pointer with PBE_FLAG_DEVICE_PTRS; the blob's constants are kept)
 * and restart from the initial condition.  Ordered on the handle's stream
 * after its queued work; non-finite weights give PBE_EINVAL (host pointers only
 * are checked).  PBE_ESTATE for other laws. */
int pbe_set_mlp(pbe_handle *h, const float *w);

/* The closure network alone (no box, no rates): for raw inputs
 * x[n][3] = (S, T, log10 mu_2) writes y[n][2] (the two network outputs) and
 * dy[n][2][3] = dy_o/dz_i of the normalised inputs.  x, y, dy are device
 * pointers ordered on hip_stream; blob is a host closure blob.  Blocks until
 * done (it copies the blob in and frees its scratch). */
int pbe_mlp_forward(const float *blob, int32_t precision, int32_t n, const double *x, double *y, double *dy,
                    void *hip_stream);

/* Weight gradient of the closure network alone: gw[PBE_MLP_NW] =
 * sum_r (dy/dW at z_r)^T ybar_r over n rows of normalised inputs z[n][3] and
 * output cotangents ybar[n][2] - the contraction pbe_grad performs over the
 * rows its adjoint sweep leaves (the closure of Sec. 4.2, Fig. 5a, trained
 * through the solver).  bf16 precision: the same bfloat16 forward and
 * backward on the matrix cores (fp32 accumulation); fp64: plain FP64.  z,
 * ybar, gw are device pointers ordered on hip_stream; blob is a host closure
 * blob.  Blocks until done (it copies the blob in and frees its scratch). */
int pbe_mlp_vjp(const float *blob, int32_t precision, int32_t n, const double *z, const double *ybar, double *gw,
                void *hip_stream);

/* pbe_mlp_vjp for callers that cannot allocate device memory (code under HIP
 * graph capture, tight training loops, harnesses that forbid hipMalloc): the
 * same result, bitwise, for n <= PBE_MLP_VJP_NOALLOC_MAX_ROWS rows (PBE_EINVAL
 * beyond), with no hipMalloc, hipFree or other allocation.  Its scratch is a
 * fixed device array of the library (about 9.6 MB: blob copy, packed
 * operands, staged rows, one partial gradient per 16-row tile), one per GPU,
 * held until the process ends.  Every call on a GPU uses that GPU's array, so
 * calls that overlap on one GPU (other host threads, or streams that are not
 * ordered) race; each call blocks until its result is in gw.  z, ybar, gw are
 * device pointers on the current device ordered on hip_stream; blob is host. */
#define PBE_MLP_VJP_NOALLOC_MAX_ROWS 4096
int pbe_mlp_vjp_noalloc(const float *blob, int32_t precision, int32_t n, const double *z, const double *ybar,
                        double *gw, void *hip_stream);

/* One Adam step (Kingma and Ba; the optimiser of Sec. 4.1 / App. C) on device
 * arrays of n floats: w -= lr * mhat / (sqrt(vhat) + eps) with the moment
 * estimates m, v updated from the gradient g (device, double) and bias
 * correction for step >= 1.  Ordered on hip_stream, does not wait. */
int pbe_adam(float *w, float *m, float *v, const double *g, int32_t n, int32_t step, float lr, float beta1,
             float beta2, float eps, void *hip_stream);

/* Replace every sim's parameter row (host pointer [S*PBE_NPAR], same checks
 * as pbe_create) without rebuilding the handle, e.g. between optimizer
 * iterations; the handle restarts from the initial condition.  Waits for the
 * handle's queued work first.  1D with a derived step budget (max_steps = 0 at
 * create): PBE_ESTATE, nothing changed, if a sim's step bound under the new
 * kinetics exceeds the budget sized at create (the checkpoints and gradient
 * rows are sized from it); create the handle with a larger max_steps instead. */
int pbe_set_par(pbe_handle *h, const double *par);

/* Launch shape chosen by pbe_tune. */
typedef struct {
    int32_t blocks[4];          /* 1D: persistent workgroups per kernel class (cells per lane 1-8,
                                   9-16, 17-24, 25-32; 0 for an empty class) */
    int32_t seg_2d;             /* 2D: rows per column block of the L2 sweep */
    int32_t pair_long;          /* 1D: grids over 1024 cells run on wave pairs (class 2) instead of
                                   one wavefront with 17-32 cells per lane (classes 2, 3) */
    int32_t n_candidates;       /* configurations timed; 0 when taken from the process cache */
    float best_ms;              /* trial time of the chosen configuration */
    float default_ms;           /* trial time of the default configuration */
} pbe_tuning;

/* Autotuner: time candidate launch shapes on this handle's own problem and
 * keep the fastest (2D: column-block length 32, 64, 128 or 256 rows; a
 * candidate replaces the default of 64 only when its trial is at least 3%
 * faster, smaller differences being timing noise).  Each candidate runs the
 * solve from the initial condition, limited to trial_steps steps per
 * simulation (0: to t_end), timed with HIP events from the first step on.  2D results agree
 * to rounding (the moment partial sums are grouped by column block).  The
 * choice is cached per process under the problem's shape (dimension, sizes,
 * closure variant); with use_cache != 0 a cached choice is applied without
 * timing.  Waits for the handle's queued work first, then blocks; the handle
 * restarts from the initial condition.  out may be NULL.  pbe_create runs this
 * with use_cache = 1 when flags has PBE_FLAG_AUTOTUNE.
 * 1D handles: PBE_EUNSUPPORTED (timing 1D candidates is switched off; apply a
 * 1D launch shape with pbe_set_launch). */
int pbe_tune(pbe_handle *h, int32_t trial_steps, int32_t use_cache, pbe_tuning *out);

/* Apply a launch shape without timing (e.g. one pbe_tune chose before): the
 * fields of pbe_tuning that describe the shape are used (blocks and
 * pair_long for 1D, seg_2d for 2D; seg_2d in [16, 4096]); counts are clipped to
 * each class's size.  pair_long requires the plain rate laws.  The handle
 * restarts from the initial condition.  PBE_EINVAL on a NULL or out-of-range
 * argument. */
int pbe_set_launch(pbe_handle *h, const pbe_tuning *t);

/* Step sizes and rates the last pbe_solve used (1D, created with
 * PBE_FLAG_RECORD_RATES): out[s][k][0..2] = (dt, G0 [um/s], B [#/(m^3 s)]) of
 * step k of sim s (the rates of Sec. 2.1 / App. A, or of the learned closure,
 * and the step of SI Eq. (S3)) for k < min(steps_s, n_steps), 0 beyond.
 * n_steps in [1, step budget] (the step budget is max_steps, or the one
 * derived at create).  out is [S][n_steps][3] doubles, a device pointer
 * (stream-ordered, returns at once) with PBE_FLAG_DEVICE_PTRS, else host
 * memory (blocks).  PBE_ESTATE without the flag or before a solve;
 * PBE_EUNSUPPORTED for 2D handles; PBE_EINVAL for n_steps out of range. */
int pbe_rate_log(pbe_handle *h, int32_t n_steps, double *out);

/* Release all device memory of the handle.  NULL is a no-op.  (Resource
 * management only; no passage of the paper corresponds.) */
void pbe_destroy(pbe_handle *h);

/* Static message for a pbe_status code. */
const char *pbe_strerror(int code);

/* Elapsed device time (ms) of the last pbe_solve / pbe_grad kernel work,
 * measured with HIP events on the handle's stream around the launch. */
int pbe_last_kernel_ms(pbe_handle *h, float *solve_ms, float *grad_ms);

#ifdef __cplusplus
}
#endif
#endif /* PBE_H */

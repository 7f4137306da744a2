/*
 * FP64 CPU oracle for the crystallization population-balance solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only the test suite, the package smoke
 * check and the CPU-baseline leg of the benchmark may load it; the solver
 * library never links, calls or falls back to it.  It shares no code, header,
 * table or helper with the GPU path.
 *
 * What it computes (paper: "Modern, Efficient, and Differentiable Transport
 * Equation Models using JAX", arXiv 2411.00742):
 *   - the growth PBE, Sec. 2.1 Eq. (1), reduced to one size coordinate or
 *     kept in two with Godunov dimensional splitting (Sec. 2.1);
 *   - the high-resolution finite-volume flux with the van Leer limiter,
 *     Sec. 2.1 Eq. (8) and SI S1.1 Eqs. (S1)-(S2), in the flux form
 *     F = G (f_i + kappa/2 * psi), psi = phi(theta) * (f_{i+1} - f_i);
 *     kappa = 1 - G dt/dL is the paper's one-step update, kappa = 1 the
 *     method-of-lines form advanced by Shu-Osher SSP-RK3;
 *   - the CFL time step, SI S1.1 Eq. (S3);
 *   - the discrete solute mass balance, Sec. 2.1 Eq. (9);
 *   - moments, SI S1.2 Eq. (S5), and the method-of-moments ODEs, Eq. (S4);
 *   - forward-mode derivatives (dual numbers), SI S2.1-S2.2, used as the
 *     reference gradient, with the step sizes differentiated in the branch
 *     the primal run takes (or, on request, held at the primal run's values).
 *
 * Units: L um, t s, T degC, f #/(m^3 um^d), G um/s, B #/(m^3 s), C g/g.
 * Kinetic parameter kg is in m/s and is scaled by 1e6 to um/s.
 *
 * Per-simulation parameter row (REF_NPAR doubles):
 *   0 kg, 1 g, 2 kb, 3 b, 4 gamma [1/um], 5 kg2, 6 g2, 7 Eg [K], 8 Eb [K],
 *   9 T0, 10 T1, 11 t_ramp, 12 Eg2 [K] (the second axis' growth activation
 *   temperature of the Arrhenius law; App. A Eq. (A.2) has one per axis),
 *   13 kd [m/s], 14 d: dissolution.  Where the solution is undersaturated
 *   (C < Csat) the power and Arrhenius laws of a 1D simulation let crystals
 *   shrink at G0 = -1e6 kd (1 - C/Csat)^d (um/s) with no nucleation; kd = 0
 *   keeps them unchanged there.  With G0 < 0 the upwind cell of a face is the
 *   one on its right: F = G (f_{i+1} - kappa/2 psi(f_{i+1} - f_i, f_{i+2} - f_{i+1})),
 *   kappa = 1 or 1 - |G| dt/dL; crystals leave through L = 0 (a ghost of 0
 *   left of it) and nothing enters through L_max (ghosts of 0 beyond it).
 */
#ifndef PBE_ORACLE_H
#define PBE_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REF_NPAR 15
#define REF_NTAN 5          /* tangent directions: kg, g, kb, b, gamma */

enum { REF_SCHEME_SSPRK3 = 0, REF_SCHEME_LW_TVD = 1 };
/* REF_LAW_POLY: growth G0 = a_1 S + a_2 S^2 + ... + a_k S^k with S = C/Csat - 1 > 0 (the
 * polynomial growth law of Sec. 4.1, Eq. (poly_growth_rate), in um per time unit; the sim's
 * poly[] holds a_1..a_k), nucleation by the power law kb S^b. */
enum { REF_LAW_POWER = 0, REF_LAW_ARRHENIUS = 1, REF_LAW_MLP = 2, REF_LAW_POLY = 3 };
enum { REF_SOL_LINEAR = 0, REF_SOL_EXP = 1 };
enum { REF_SIM_OK = 0, REF_SIM_NONFINITE = 1, REF_SIM_OUTFLOW = 2, REF_SIM_FALLBACK = 4 };

/* Learned closure (Sec. 4.2, Fig. 5a: a network replaces the advection-rate
 * computation of the loop in Fig. 1).  Blob of REF_MLP_NBLOB floats:
 *   W1[64][3] b1[64] W2[64][64] b2[64] W3[2][64] b3[2]        (REF_MLP_NW weights)
 *   in_shift[3] in_scale[3] out_shift[2] out_scale[2] lo[3] hi[3] s_min lnG0_max
 * Inputs x = (S, T [degC], log10 mu_2) with S = C/Csat - 1, normalised as
 * z_k = (x_k - in_shift_k) * in_scale_k;  h1 = tanh(W1 z + b1),
 * h2 = tanh(W2 h1 + b2), y = W3 h2 + b3;  ln G0 = min(out_shift_0 + out_scale_0 y_0,
 * lnG0_max) (G0 in um/s) and ln B = out_shift_1 + out_scale_1 y_1.  Where S <= s_min,
 * mu_2 <= 0 or some x_k lies outside [lo_k, hi_k], the plain power law with the
 * simulation's (kg, g, kb, b) is used instead and REF_SIM_FALLBACK is set.
 * Precision REF_MLP_FP64: all in double.  REF_MLP_BF16: z, the weights and the
 * hidden activations are rounded to bfloat16 (round to nearest even, z going
 * through float first), each pre-activation is the exact sum plus the float
 * bias rounded once to float, tanh is rounded to float before the bfloat16
 * rounding, and y is rounded to float.  Derivatives pass through the roundings
 * unchanged, with tanh' = 1 - t^2 at the float value t. */
#define REF_MLP_H 64
#define REF_MLP_NW 4546
#define REF_MLP_NC 18
#define REF_MLP_NBLOB (REF_MLP_NW + REF_MLP_NC)
enum { REF_MLP_BF16 = 0, REF_MLP_FP64 = 1 };

/* Dimensional splitting of the 2D step (Sec. 2.1): Godunov (Lie), a full L1
 * sweep then a full L2 sweep; or Strang, an L1 sweep over half the step, the
 * L2 sweep over the whole step, and another L1 sweep over the second half. */
enum { REF_SPLIT_LIE = 0, REF_SPLIT_STRANG = 1 };

typedef struct {
    int32_t law, scheme, sol_law, mlp_precision;
    double cs0, cs1;          /* Csat = cs0 + cs1*T (linear) or cs0*exp(cs1*T) */
    double alpha;             /* rho_c * k_v / rho_solvent, g/g per (um^3/m^3) */
    double cfl, dt_max, t_end;
    const float *mlp;         /* law == REF_LAW_MLP: closure blob [REF_MLP_NBLOB] */
    int32_t splitting;        /* 2D: REF_SPLIT_LIE or REF_SPLIT_STRANG */
} ref_process;

/* One 1D simulation.  Inputs first, then optional outputs (NULL = skip). */
typedef struct {
    int32_t n;                /* cells on [0, L_max] */
    int32_t n_samples;
    int32_t max_steps;        /* stop after this many steps (state is then "current") */
    int32_t n_replay;         /* >0: use dt_replay[0..n_replay) as the step sizes */
    int32_t n_rates_replay;   /* >0: use G0_replay, B_replay[0..n_rates_replay) instead of the rate law */
    double L_max;
    double C0;
    const double *f0;         /* [n] */
    const double *par;        /* [REF_NPAR] */
    const double *t_samples;  /* [n_samples] ascending in (0, t_end] */
    const double *dt_replay;
    const double *G0_replay, *B_replay;
    int32_t n_poly;           /* law == REF_LAW_POLY: number of coefficients k */
    const double *poly;       /* law == REF_LAW_POLY: [n_poly] a_1..a_k */
    /* outputs */
    double *f_samples;        /* [n_samples][n] */
    double *mom;              /* [n_samples][4]  mu_0..mu_3 */
    double *C;                /* [n_samples] */
    double *f_final;          /* [n] state when the loop stops */
    double *dt_log;           /* [max_steps] step sizes taken */
    double *G0_log, *B_log;   /* [max_steps] rates used in each step */
    int32_t *steps, *status;
    double *C_final, *t_final, *outflow;
    const double *corr;       /* NULL, or the in-the-loop correction's REF_CORR_NW weights (below) */
} ref_sim1d;

/* In-the-loop correction (Sec. 4.2, Fig. 5b: a network in the time loop that
 * offsets the discretisation error of each step).  After every growth step
 * (G0 > 0) each interior face i+1/2 (0 <= i <= n-2) gets a correction flux
 *   Y = sigma nu (W2 . tanh(W1 x + b1) + b2),
 *   x = (f_{i-1}, f_i, f_{i+1}, f_{i+2}) / sigma and nu,
 * with sigma = max |f_{i-1..i+2}| (Y = 0 where sigma = 0), cells outside the
 * domain read as 0, and nu = dt G0 (1 + gamma L_face) / dL the face's Courant
 * number; then f_i += Y_{i-1/2} - Y_{i+1/2}.  The faces at L = 0 and L_max are
 * not corrected, so the number balance and every boundary flux stay those of
 * the solver.  Weights: W1[8][5] b1[8] W2[8] b2, REF_CORR_NW doubles. */
#define REF_CORR_H 8
#define REF_CORR_NW 57

/* One 2D simulation, f stored [n2][n1] with L1 contiguous. */
typedef struct {
    int32_t n1, n2, n_samples, max_steps;
    double L1_max, L2_max, C0;
    const double *f0, *par, *t_samples;
    double *mom;              /* [n_samples][4]: mu_00, mu_10, mu_01, mu_12 */
    double *C;                /* [n_samples] */
    double *f_final;          /* [n2][n1] */
    double *dt_log;
    int32_t *steps, *status;
    double *C_final, *t_final, *outflow;
} ref_sim2d;

/* van Leer limiter phi(theta), SI Eq. (S2). */
double ref_phi_vanleer(double theta);
/* Limited slope psi(a, b) = phi(a/b) * b in division-safe form; 0 where a*b <= 0. */
double ref_limited_slope(double a, double b);

int ref_solve1d(const ref_process *p, ref_sim1d *s);
/* Independent sims over a pool of n_threads std::threads (<=0: hardware concurrency).
 * Returns the number of threads used. */
int ref_solve1d_batch(const ref_process *p, ref_sim1d *sims, int32_t n_sims, int32_t n_threads);

/* Step sizes in the derivatives: REF_DT_DIFF differentiates each step in the
 * branch its values select (a CFL-limited step nu*dL/(G0 (1 + gamma L_max))
 * depends on the rates and gamma, a step that lands on a sample time on the
 * time reached; the time, the cooling ramp's temperature and so the rates
 * carry that dependence); the step count and the branches are those of the
 * primal run.  REF_DT_FROZEN replays the primal run's step sizes as constants. */
enum { REF_DT_DIFF = 0, REF_DT_FROZEN = 1 };

/* Forward-mode derivatives of the recorded samples w.r.t. (kg, g, kb, b, gamma).
 * dF [n_samples][n][5], dM [n_samples][4][5], dC [n_samples][5] (each may be NULL). */
int ref_tangent1d(const ref_process *p, ref_sim1d *s, int32_t dt_mode, double *dF, double *dM, double *dC);

/* (double)(bfloat16)(float)x with round-to-nearest-even at both steps. */
double ref_bf16(double x);
/* Closure network alone on n inputs x[n][3] = (S, T, log10 mu_2), ignoring the
 * box: y[n][2]; dy[n][2][3] = dy/dz (may be NULL). */
int ref_mlp_forward(const float *blob, int32_t precision, int32_t n, const double *x, double *y, double *dy);
/* Weight gradient of sum_r ybar[r] . y(z[r]) over n rows of normalised inputs
 * z[n][3]: gw[REF_MLP_NW], same order as the blob's weights. */
int ref_mlp_vjp(const float *blob, int32_t precision, int32_t n, const double *z, const double *ybar, double *gw);
/* Learned-closure solve: forward-mode derivatives along the weight direction
 * v[REF_MLP_NW] (tangent 0) and along gamma (tangent 1), steps as dt_mode says.
 * dF [n_samples][n][2], dM [n_samples][4][2], dC [n_samples][2]. */
int ref_tangent1d_mlp(const ref_process *p, ref_sim1d *s, int32_t dt_mode, const double *v, double *dF, double *dM,
                      double *dC);
/* Polynomial growth law: forward-mode derivatives along the coefficient
 * direction v[n_poly] (tangent 0) and along gamma (tangent 1), steps as
 * dt_mode says.  dF [n_samples][n][2], dM [n_samples][4][2], dC [n_samples][2]. */
int ref_tangent1d_poly(const ref_process *p, ref_sim1d *s, int32_t dt_mode, const double *v, double *dF, double *dM,
                       double *dC);

/* Solve with the in-the-loop correction (s->corr set): forward-mode derivatives
 * along the weight direction v[REF_CORR_NW] (tangent 0) and along gamma
 * (tangent 1), steps as dt_mode says.  dF [n_samples][n][2], dM [n_samples][4][2], dC [n_samples][2]. */
int ref_tangent1d_corr(const ref_process *p, ref_sim1d *s, int32_t dt_mode, const double *v, double *dF, double *dM,
                       double *dC);

int ref_solve2d(const ref_process *p, ref_sim2d *s);
int ref_solve2d_batch(const ref_process *p, ref_sim2d *sims, int32_t n_sims, int32_t n_threads);

/* Method of moments (SI S1.2 Eq. (S4) reduced to one size coordinate, with
 * G = G0 (1 + gamma L) and nucleation at L = 0) coupled to the solute balance,
 * integrated with Dormand-Prince 5(4).  mu_init[4]; outputs [n_samples][4], [n_samples]. */
int ref_mom1d(const ref_process *p, const double *par, double C0, const double *mu_init,
              int32_t n_samples, const double *t_samples, double rtol, double atol,
              double *mu_out, double *C_out);
/* 2D cross moments mu_00, mu_10, mu_01, mu_11, mu_02, mu_12 (size-independent G1, G2). */
int ref_mom2d(const ref_process *p, const double *par, double C0, const double *mu_init,
              int32_t n_samples, const double *t_samples, double rtol, double atol,
              double *mu_out, double *C_out);

/* The worked forward-mode example of SI S2.2: y1 = sin x1/(x1+x2), y2 = (x1+x2) e^x2.
 * out = [y1, y2, dy1/dx1, dy1/dx2, dy2/dx1, dy2/dx2]. */
void ref_dual_example(double x1, double x2, double *out);

#ifdef __cplusplus
}
#endif
#endif

// FP64 CPU oracle for the crystallization PBE solver.
//
// TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
// CPU-baseline leg of the benchmark; never by the solver library.
//
// Everything here is written to be read against the paper (arXiv 2411.00742)
// rather than to be fast: one simulation at a time, plain loops over an array
// padded with ghost cells, no fusion.  The scalar type is a template parameter
// only so that the same loop can run on dual numbers for forward-mode
// derivatives (SI S2.1).
#include "pbe_oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Dual numbers (forward mode, SI S2.1): value plus ND tangent components.
// ---------------------------------------------------------------------------
template <int ND>
struct Dual {
    double v;
    double d[ND];
    Dual() : v(0.0) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
    Dual(double x) : v(x) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }  // NOLINT: implicit on purpose
};

template <int ND> Dual<ND> operator+(const Dual<ND>& a, const Dual<ND>& b) {
    Dual<ND> r(a.v + b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
}
template <int ND> Dual<ND> operator-(const Dual<ND>& a, const Dual<ND>& b) {
    Dual<ND> r(a.v - b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
}
template <int ND> Dual<ND> operator-(const Dual<ND>& a) {
    Dual<ND> r(-a.v); for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k]; return r;
}
template <int ND> Dual<ND> operator*(const Dual<ND>& a, const Dual<ND>& b) {
    Dual<ND> r(a.v * b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r;
}
template <int ND> Dual<ND> operator/(const Dual<ND>& a, const Dual<ND>& b) {
    // d(a/b) = (da - (a/b) db) / b, written without b*b so tiny b does not underflow
    Dual<ND> r(a.v / b.v);
    for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
template <int ND> Dual<ND> operator+(const Dual<ND>& a, double b) { return a + Dual<ND>(b); }
template <int ND> Dual<ND> operator+(double a, const Dual<ND>& b) { return Dual<ND>(a) + b; }
template <int ND> Dual<ND> operator-(const Dual<ND>& a, double b) { return a - Dual<ND>(b); }
template <int ND> Dual<ND> operator-(double a, const Dual<ND>& b) { return Dual<ND>(a) - b; }
template <int ND> Dual<ND> operator*(const Dual<ND>& a, double b) { return a * Dual<ND>(b); }
template <int ND> Dual<ND> operator*(double a, const Dual<ND>& b) { return Dual<ND>(a) * b; }
template <int ND> Dual<ND> operator/(const Dual<ND>& a, double b) { return a / Dual<ND>(b); }
template <int ND> Dual<ND> operator/(double a, const Dual<ND>& b) { return Dual<ND>(a) / b; }

template <int ND> Dual<ND> exp(const Dual<ND>& a) {
    Dual<ND> r(std::exp(a.v)); for (int k = 0; k < ND; ++k) r.d[k] = r.v * a.d[k]; return r;
}
template <int ND> Dual<ND> log(const Dual<ND>& a) {
    Dual<ND> r(std::log(a.v)); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / a.v; return r;
}
template <int ND> Dual<ND> sin(const Dual<ND>& a) {
    Dual<ND> r(std::sin(a.v)); for (int k = 0; k < ND; ++k) r.d[k] = std::cos(a.v) * a.d[k]; return r;
}
template <int ND> Dual<ND> tanh(const Dual<ND>& a) {
    Dual<ND> r(std::tanh(a.v)); for (int k = 0; k < ND; ++k) r.d[k] = (1.0 - r.v * r.v) * a.d[k]; return r;
}
// |x| with derivative sign(x), and 0 at x == 0.
template <int ND> Dual<ND> fabs(const Dual<ND>& a) {
    if (a.v > 0) return a;
    if (a.v < 0) return -a;
    return Dual<ND>(0.0);
}

inline double val(double x) { return x; }
template <int ND> double val(const Dual<ND>& x) { return x.v; }
inline void set_tangent(double&, int, double) {}
template <int ND> void set_tangent(Dual<ND>& x, int k, double v) { if (k >= 0 && k < ND) x.d[k] = v; }
inline void scale_tangent(double&, double) {}
template <int ND> void scale_tangent(Dual<ND>& x, double s) { for (int k = 0; k < ND; ++k) x.d[k] *= s; }
inline double fabs(double x) { return std::fabs(x); }
inline double exp(double x) { return std::exp(x); }
inline double log(double x) { return std::log(x); }
inline double tanh(double x) { return std::tanh(x); }
// replace the value of x, keeping its derivative (rounding steps are passed through)
inline double with_value(double, double v) { return v; }
template <int ND> Dual<ND> with_value(const Dual<ND>& x, double v) { Dual<ND> r = x; r.v = v; return r; }

// x^p for x >= 0 with p > 0: 0 (and zero derivative) at x == 0.
inline double power(double x, double p) { return x > 0.0 ? std::pow(x, p) : 0.0; }
template <int ND> Dual<ND> power(const Dual<ND>& x, const Dual<ND>& p) {
    if (!(x.v > 0.0)) return Dual<ND>(0.0);
    Dual<ND> r(std::pow(x.v, p.v));
    const double lx = std::log(x.v);
    for (int k = 0; k < ND; ++k) r.d[k] = r.v * (p.d[k] * lx + p.v * x.d[k] / x.v);
    return r;
}

// ---------------------------------------------------------------------------
// Process and kinetics.
// ---------------------------------------------------------------------------
enum { K_KG, K_G, K_KB, K_B, K_GAMMA, K_KG2, K_G2, K_EG, K_EB, K_T0, K_T1, K_TRAMP, K_EG2, K_KD, K_D };

template <class R>
struct Kinetics {
    R kg, g, kb, b, gamma, kg2, g2;
    double Eg, Eb, Eg2;
    double kd, d;           // dissolution (S < 0): G0 = -1e6 kd (-S)^d
    std::vector<R> poly;   // a_1..a_k of the polynomial growth law
    std::vector<R> corr;   // in-the-loop correction weights (empty: none)
};

template <class R>
Kinetics<R> load_kinetics(const double* par) {
    Kinetics<R> k;
    k.kg = R(par[K_KG]); k.g = R(par[K_G]); k.kb = R(par[K_KB]); k.b = R(par[K_B]);
    k.gamma = R(par[K_GAMMA]); k.kg2 = R(par[K_KG2]); k.g2 = R(par[K_G2]);
    k.Eg = par[K_EG]; k.Eb = par[K_EB]; k.Eg2 = par[K_EG2];
    k.kd = par[K_KD]; k.d = par[K_D];
    return k;
}

// The kinetics of one 1D simulation: its parameter row and, for the polynomial
// law, its coefficients (tangent direction: coefficient j moves along v[j]).
template <class R>
Kinetics<R> load_kinetics_sim(const ref_sim1d* s, const double* v = nullptr, int dir = -1,
                              const double* vc = nullptr) {
    Kinetics<R> k = load_kinetics<R>(s->par);
    if (s->poly && s->n_poly > 0) {
        k.poly.resize(s->n_poly);
        for (int j = 0; j < s->n_poly; ++j) {
            k.poly[j] = R(s->poly[j]);
            if (v && dir >= 0) set_tangent(k.poly[j], dir, v[j]);
        }
    }
    if (s->corr) {   // correction weights (tangent 0 moves them along vc)
        k.corr.resize(REF_CORR_NW);
        for (int j = 0; j < REF_CORR_NW; ++j) {
            k.corr[j] = R(s->corr[j]);
            if (vc) set_tangent(k.corr[j], 0, vc[j]);
        }
    }
    return k;
}

// Linear cooling from T0 to T1 over t_ramp seconds, then held at T1.  The
// time may carry derivatives (the step size, and so the time reached, depends
// on the parameters wherever the CFL limit sets the step).
template <class R>
R temperature(const double* par, const R& t) {
    const double tr = par[K_TRAMP];
    const R frac = (tr > 0.0 && val(t) < tr) ? t / tr : R(1.0);
    return par[K_T0] + (par[K_T1] - par[K_T0]) * frac;
}
double temperature(const double* par, double t) { return temperature<double>(par, t); }

// Solubility: linear, or the exponential form of App. A Eq. (A.1).
template <class R>
R solubility(const ref_process* p, const R& T) {
    return p->sol_law == REF_SOL_EXP ? p->cs0 * exp(p->cs1 * T) : p->cs0 + p->cs1 * T;
}
double solubility(const ref_process* p, double T) { return solubility<double>(p, T); }

// Relative supersaturation S = C/Csat - 1, and its positive part: the growth
// and nucleation laws act only while the solution is supersaturated
// (App. A, the condition stated under Eq. (A.2)).
template <class R, class Q>
R supersaturation_pos(R C, const Q& Csat) {
    R S = C / Csat - 1.0;
    if (val(S) > 0.0) return S;
    return R(0.0);
}

// Growth rate G0 [um/s] at L = 0 along axis 1, the second axis rate G2, and
// the nucleation rate B [#/(m^3 s)].  Power law, or the power law times the
// Arrhenius temperature factor of App. A Eq. (A.2).
template <class R, class Q>
void rate_laws(int law, const Kinetics<R>& k, const Q& T, R Sp, R& G0, R& G2, R& B) {
    G0 = 1e6 * k.kg * power(Sp, k.g);
    G2 = 1e6 * k.kg2 * power(Sp, k.g2);
    B = k.kb * power(Sp, k.b);
    if (law == REF_LAW_ARRHENIUS) {
        G0 = G0 * exp(-k.Eg / (T + 273.15));
        G2 = G2 * exp(-k.Eg2 / (T + 273.15));
        B = B * exp(-k.Eb / (T + 273.15));
    }
    if (law == REF_LAW_POLY) {
        // Eq. (poly_growth_rate): sum of a_j S^j over j = 1..k
        G0 = R(0.0);
        R Sj = Sp;
        for (size_t j = 0; j < k.poly.size(); ++j) {
            G0 = G0 + k.poly[j] * Sj;
            Sj = Sj * Sp;
        }
        G2 = R(0.0);
    }
}

// Dissolution: in an undersaturated solution (C < Csat) the crystals of the
// power and Arrhenius laws shrink at G0 = -1e6 kd (1 - C/Csat)^d um/s; the
// paper names the growth/dissolution rate of each axis without a law for the
// latter, so this one mirrors the growth power law.  Zero when kd = 0 or
// C >= Csat.
template <class R, class Q>
R dissolution_rate(const Kinetics<R>& k, const R& C, const Q& Csat) {
    const R under = 1.0 - C / Csat;
    if (!(val(under) > 0.0) || !(k.kd > 0.0)) return R(0.0);
    return -1e6 * k.kd * power(under, R(k.d));
}

// ---------------------------------------------------------------------------
// Learned closure (Sec. 4.2, Fig. 5a): a network in place of the rate laws.
// Layout of the blob and the precision rules are stated in pbe_oracle.h.
// ---------------------------------------------------------------------------
constexpr int MH = REF_MLP_H;
constexpr int OFF_W1 = 0, OFF_B1 = 3 * MH, OFF_W2 = 4 * MH, OFF_B2 = 4 * MH + MH * MH, OFF_W3 = 5 * MH + MH * MH,
              OFF_B3 = 7 * MH + MH * MH;
static_assert(OFF_B3 + 2 == REF_MLP_NW, "closure weight count");
enum { C_IN_SHIFT = 0, C_IN_SCALE = 3, C_OUT_SHIFT = 6, C_OUT_SCALE = 8, C_LO = 10, C_HI = 13, C_SMIN = 16,
       C_LNG0_MAX = 17 };

// float -> bfloat16 -> float, round to nearest with ties to even on the 16
// discarded bits of the IEEE single pattern (finite inputs)
float round_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    float r;
    std::memcpy(&r, &u, 4);
    return r;
}
double bf16_of_double(double x) { return (double)round_bf16((float)x); }

template <class R>
struct Net {
    int precision = REF_MLP_FP64;
    std::vector<R> w;        // REF_MLP_NW weights as used (bf16-rounded weight values in BF16 mode)
    double c[REF_MLP_NC];    // normalisation constants and box
};

// Weights from the blob; in BF16 mode the matrices (not the biases) are
// rounded to bfloat16.  dir (may be null) seeds tangent 0 with a direction.
template <class R>
Net<R> load_net(const float* blob, int precision, const double* dir, int dir_slot) {
    Net<R> n;
    n.precision = precision;
    n.w.resize(REF_MLP_NW);
    for (int i = 0; i < REF_MLP_NW; ++i) {
        const bool is_bias = (i >= OFF_B1 && i < OFF_W2) || (i >= OFF_B2 && i < OFF_W3) || i >= OFF_B3;
        double v = (double)blob[i];
        if (precision == REF_MLP_BF16 && !is_bias) v = (double)round_bf16(blob[i]);
        n.w[i] = R(v);
        if (dir) set_tangent(n.w[i], dir_slot, dir[i]);
    }
    for (int k = 0; k < REF_MLP_NC; ++k) n.c[k] = (double)blob[REF_MLP_NW + k];
    return n;
}

// One hidden unit's activation from its pre-activation (exact sum + bias).
template <class R>
R activate(const Net<R>& n, const R& pre) {
    if (n.precision == REF_MLP_FP64) return tanh(pre);
    const float pf = (float)val(pre);
    const float t = (float)std::tanh((double)pf);
    R h = with_value(pre, (double)round_bf16(t));
    // derivative of tanh at the rounded pre-activation, through the roundings
    scale_tangent(h, 1.0 - (double)t * (double)t);
    return h;
}

// y = W3 tanh(W2 tanh(W1 z + b1) + b2) + b3 on normalised inputs z.
template <class R>
void net_forward(const Net<R>& n, const R z[3], R y[2]) {
    const std::vector<R>& w = n.w;
    R zi[3];
    for (int k = 0; k < 3; ++k)
        zi[k] = n.precision == REF_MLP_BF16 ? with_value(z[k], bf16_of_double((double)(float)val(z[k]))) : z[k];
    R h1[MH], h2[MH];
    for (int j = 0; j < MH; ++j) {
        R a = w[OFF_B1 + j];
        for (int k = 0; k < 3; ++k) a = a + w[OFF_W1 + j * 3 + k] * zi[k];
        h1[j] = activate(n, a);
    }
    for (int j = 0; j < MH; ++j) {
        R a = w[OFF_B2 + j];
        for (int i = 0; i < MH; ++i) a = a + w[OFF_W2 + j * MH + i] * h1[i];
        h2[j] = activate(n, a);
    }
    for (int o = 0; o < 2; ++o) {
        R a = w[OFF_B3 + o];
        for (int j = 0; j < MH; ++j) a = a + w[OFF_W3 + o * MH + j] * h2[j];
        y[o] = n.precision == REF_MLP_BF16 ? with_value(a, (double)(float)val(a)) : a;
    }
}

// Closure rates at supersaturation S (not clipped), temperature T and second
// moment mu2.  Returns true when the plain power law was used instead.
template <class R>
bool closure_rates(const Net<R>& n, const Kinetics<R>& k, const R& S, const R& T, const R& mu2, R& G0, R& B) {
    const double* c = n.c;
    bool inside = val(S) > c[C_SMIN] && val(mu2) > 0.0;
    R x[3] = {S, T, R(0.0)};
    if (inside) x[2] = log(mu2) / std::log(10.0);
    for (int q = 0; q < 3 && inside; ++q) inside = val(x[q]) >= c[C_LO + q] && val(x[q]) <= c[C_HI + q];
    if (!inside) {
        const R Sp = val(S) > 0.0 ? S : R(0.0);
        G0 = 1e6 * k.kg * power(Sp, k.g);
        B = k.kb * power(Sp, k.b);
        return true;
    }
    R z[3], y[2];
    for (int q = 0; q < 3; ++q) z[q] = (x[q] - c[C_IN_SHIFT + q]) * c[C_IN_SCALE + q];
    net_forward(n, z, y);
    // the network's growth rate is trusted up to exp(lnG0_max): beyond it the
    // log-rate is held at that bound (zero derivative), which also bounds the
    // number of CFL-limited steps a solve can take
    R lnG = c[C_OUT_SHIFT] + c[C_OUT_SCALE] * y[0];
    if (val(lnG) > c[C_LNG0_MAX]) lnG = R(c[C_LNG0_MAX]);
    G0 = exp(lnG);
    B = exp(c[C_OUT_SHIFT + 1] + c[C_OUT_SCALE + 1] * y[1]);
    return false;
}

// ---------------------------------------------------------------------------
// Limiter (SI S1.1).
// ---------------------------------------------------------------------------
double phi_vanleer(double theta) { return (theta + std::fabs(theta)) / (1.0 + std::fabs(theta)); }

// psi(a, b) = phi(a/b) * b, where a is the upwind difference and b the
// difference across the face.  Multiplying numerator and denominator of phi by
// |b| gives (a|b| + |a|b) / (|a| + |b|), which is defined everywhere; it is
// zero unless a and b have the same strict sign (the limiter's flat/extremum
// case, including the 0/0 and x/0 ratios of Eq. (S1)).
template <class R>
R limited_slope(const R& a, const R& b) {
    const bool same_sign = (val(a) > 0.0 && val(b) > 0.0) || (val(a) < 0.0 && val(b) < 0.0);
    if (!same_sign) return R(0.0);
    return (a * fabs(b) + fabs(a) * b) / (fabs(a) + fabs(b));
}

// ---------------------------------------------------------------------------
// One-dimensional finite-volume building blocks.
// ---------------------------------------------------------------------------
// Face fluxes F[j], j = 0..n, where face j separates cells j-1 and j and sits
// at L = j*dL.  Growth (G0 > 0) moves crystals to larger sizes, so the upwind
// cell of face j is i = j-1.  Ghost cells: i = -1 and i = -2 hold `inflow` (set
// so that G(0)*inflow is the nucleation flux at L = 0), i = n holds 0 (f -> 0
// for large L, Sec. 2.1 Eqs. (4)-(6)).
//   F[j] = vel_j * (f_i + kappa_j/2 * psi(f_i - f_{i-1}, f_{i+1} - f_i))
// with vel_j = G0 (1 + gamma L_j); kappa = 1 for the method-of-lines form and
// kappa = 1 - |vel_j| dt/dL for the one-step update of Eq. (8).
// Dissolution (G0 < 0) moves crystals to smaller sizes: the upwind cell of
// face j is i = j, its slope pair is taken on that side, and the ghosts are 0
// at i = -1 (what crosses L = 0 has dissolved) and at i = n, n+1 (nothing
// enters through L_max):
//   F[j] = vel_j * (f_j - kappa_j/2 * psi(f_j - f_{j-1}, f_{j+1} - f_j)).
template <class R>
void face_fluxes(const std::vector<R>& u, int n, double dL, const R& G0, const R& gamma, const R& inflow,
                 int scheme, const R& dt, std::vector<R>& F) {
    std::vector<R> e(n + 4);           // e[i + 2] is cell i, i = -2..n+1
    const bool shrink = val(G0) < 0.0;
    e[0] = shrink ? R(0.0) : inflow;
    e[1] = shrink ? R(0.0) : inflow;
    for (int i = 0; i < n; ++i) e[i + 2] = u[i];
    e[n + 2] = R(0.0);
    e[n + 3] = R(0.0);
    for (int j = 0; j <= n; ++j) {
        const R vel = G0 * (1.0 + gamma * (j * dL));
        R kappa(1.0);
        if (scheme == REF_SCHEME_LW_TVD) kappa = 1.0 - fabs(vel) * (dt / dL);
        if (!shrink) {
            const int i = j - 1;
            const R fi = e[i + 2];
            const R psi = limited_slope(fi - e[i + 1], e[i + 3] - fi);
            F[j] = vel * (fi + 0.5 * kappa * psi);
        } else {
            const R fj = e[j + 2];
            const R psi = limited_slope(fj - e[j + 1], e[j + 3] - fj);
            F[j] = vel * (fj - 0.5 * kappa * psi);
        }
    }
}

// Conservative right-hand side R_i = -(F_{i+1/2} - F_{i-1/2}) / dL.
template <class R>
void flux_divergence(const std::vector<R>& F, int n, double dL, std::vector<R>& rhs) {
    for (int i = 0; i < n; ++i) rhs[i] = -(F[i + 1] - F[i]) / dL;
}

// One time step of one line of cells with frozen G0, gamma, inflow and dt.
// SSP-RK3 in Shu-Osher form, or the single stage of Eq. (8).
// `out` accumulates dt * (stage-weighted flux through the last face).
template <class R>
void advance_line(std::vector<R>& f, int n, double dL, const R& G0, const R& gamma, const R& inflow,
                  int scheme, const R& dt, R& out) {
    std::vector<R> F(n + 1), rhs(n);
    if (scheme == REF_SCHEME_LW_TVD) {
        face_fluxes(f, n, dL, G0, gamma, inflow, scheme, dt, F);
        flux_divergence(F, n, dL, rhs);
        for (int i = 0; i < n; ++i) f[i] = f[i] + dt * rhs[i];
        out = out + dt * F[n];
        return;
    }
    std::vector<R> u1(n), u2(n);
    face_fluxes(f, n, dL, G0, gamma, inflow, scheme, dt, F);
    flux_divergence(F, n, dL, rhs);
    const R F0 = F[n];
    for (int i = 0; i < n; ++i) u1[i] = f[i] + dt * rhs[i];

    face_fluxes(u1, n, dL, G0, gamma, inflow, scheme, dt, F);
    flux_divergence(F, n, dL, rhs);
    const R F1 = F[n];
    for (int i = 0; i < n; ++i) u2[i] = 0.75 * f[i] + 0.25 * (u1[i] + dt * rhs[i]);

    face_fluxes(u2, n, dL, G0, gamma, inflow, scheme, dt, F);
    flux_divergence(F, n, dL, rhs);
    const R F2 = F[n];
    for (int i = 0; i < n; ++i) f[i] = (1.0 / 3.0) * f[i] + (2.0 / 3.0) * (u2[i] + dt * rhs[i]);

    out = out + dt * (F0 / 6.0 + F1 / 6.0 + (2.0 / 3.0) * F2);
}

// In-the-loop correction (Sec. 4.2, Fig. 5b), applied after a growth step: a
// small network reads the four cells around each interior face, scaled by
// their largest magnitude, and the face's Courant number, and returns a
// correction flux; the corrected state is f_i + Y_{i-1/2} - Y_{i+1/2}.  The
// layout of the weights and the exact form are stated in pbe_oracle.h.
template <class R>
void correct_line(std::vector<R>& f, int n, double dL, const R& G0, const R& gamma, const R& dt,
                  const std::vector<R>& w) {
    const int H = REF_CORR_H;
    const int oW1 = 0, oB1 = 5 * H, oW2 = 6 * H, oB2 = 7 * H;
    auto cell = [&](int i) { return (i < 0 || i >= n) ? R(0.0) : f[i]; };
    std::vector<R> Y(n + 1, R(0.0));   // Y[j]: face between cells j-1 and j; j = 0 and j = n stay 0
    for (int j = 1; j < n; ++j) {
        const int i = j - 1;
        R x[4] = {cell(i - 1), cell(i), cell(i + 1), cell(i + 2)};
        R sigma(0.0);
        for (int q = 0; q < 4; ++q) {
            const R a = fabs(x[q]);
            if (val(a) > val(sigma)) sigma = a;
        }
        if (!(val(sigma) > 0.0)) continue;
        const R nu = dt * G0 * (1.0 + gamma * (j * dL)) / dL;
        R in[5];
        for (int q = 0; q < 4; ++q) in[q] = x[q] / sigma;
        in[4] = nu;
        R y = w[oB2];
        for (int h = 0; h < H; ++h) {
            R a = w[oB1 + h];
            for (int q = 0; q < 5; ++q) a = a + w[oW1 + h * 5 + q] * in[q];
            y = y + w[oW2 + h] * tanh(a);
        }
        Y[j] = sigma * nu * y;
    }
    for (int i = 0; i < n; ++i) f[i] = f[i] + (Y[i] - Y[i + 1]);
}

// Moment mu_k = sum_i L_i^k f_i dL with L_i the cell centre (SI Eq. (S5),
// midpoint quadrature).
template <class R>
R moment1d(const std::vector<R>& f, int n, double dL, int k) {
    R m(0.0);
    for (int i = 0; i < n; ++i) {
        const double L = (i + 0.5) * dL;
        double w = 1.0;
        for (int q = 0; q < k; ++q) w *= L;
        m = m + w * f[i] * dL;
    }
    return m;
}

bool finite(double x) { return std::isfinite(x); }

// Which limit sets a step: the CFL bound of SI Eq. (S3), the cap dt_max, or
// the clamp that lands the step on the next sample time (or t_end).
enum { DT_CFL = 0, DT_CAP = 1, DT_LAND = 2 };

// Step size: CFL limit nu*dL/max G (SI Eq. (S3)), capped at dt_max, clamped so
// that the step lands exactly on the next sample time (or t_end).  A replayed
// step size counts as a constant (the cap).  Returns which limit applies.
int choose_dt(double cfl_limit, double dt_max, double t, double t_next, double t_end, const double* replay,
              int n_replay, int step, double* dt) {
    double d;
    int kind;
    if (replay && step < n_replay) {
        d = replay[step];
        kind = DT_CAP;
    } else if (cfl_limit < dt_max) {
        d = cfl_limit;
        kind = DT_CFL;
    } else {
        d = dt_max;
        kind = DT_CAP;
    }
    const double rem = t_next - t;
    if (d >= rem - 1e-12 * t_end) {
        *dt = rem;
        return DT_LAND;
    }
    *dt = d;
    return kind;
}

// ---------------------------------------------------------------------------
// 1D solve (the loop of the paper's flowchart, Fig. 1): rates from the current
// concentration, step size, PSSD update, moments, mass balance, sampling.
// ---------------------------------------------------------------------------
template <class R>
struct Tangents {
    std::vector<R>* f_samples = nullptr;  // [n_samples * n]
    std::vector<R>* mom = nullptr;        // [n_samples * 4]
    std::vector<R>* C = nullptr;          // [n_samples]
};

template <class R>
int solve1d_impl(const ref_process* p, ref_sim1d* s, const Kinetics<R>& k, Tangents<R>* tan_out,
                 const Net<R>* net = nullptr) {
    const int n = s->n;
    const double dL = s->L_max / n;
    std::vector<R> f(n);
    for (int i = 0; i < n; ++i) f[i] = R(s->f0[i]);
    R C(s->C0);
    // Time carries derivatives: a CFL-limited step (SI Eq. (S3)) depends on
    // the growth rate, so the time reached after it, the temperature of the
    // cooling ramp and the length of a step that lands on a sample time all
    // depend on the parameters.  With a replayed schedule every step is a
    // constant and so is the time.
    R t(0.0);
    R mu3_old = moment1d(f, n, dL, 3);
    R out(0.0);
    int step = 0, next = 0, status = REF_SIM_OK;
    const int max_steps = s->max_steps > 0 ? s->max_steps : std::numeric_limits<int>::max();

    auto record = [&](int q) {
        if (s->f_samples) for (int i = 0; i < n; ++i) s->f_samples[(size_t)q * n + i] = val(f[i]);
        for (int m = 0; m < 4; ++m) {
            const R mu = moment1d(f, n, dL, m);
            if (s->mom) s->mom[q * 4 + m] = val(mu);
            if (tan_out && tan_out->mom) (*tan_out->mom)[q * 4 + m] = mu;
        }
        if (s->C) s->C[q] = val(C);
        if (tan_out && tan_out->C) (*tan_out->C)[q] = C;
        if (tan_out && tan_out->f_samples)
            for (int i = 0; i < n; ++i) (*tan_out->f_samples)[(size_t)q * n + i] = f[i];
    };

    while (val(t) < p->t_end && step < max_steps) {
        const R T = temperature<R>(s->par, t);
        const R Csat = solubility<R>(p, T);
        const R Sp = supersaturation_pos(C, Csat);
        R G0, G2, B;
        if (p->law == REF_LAW_MLP) {
            // closure inputs: supersaturation, temperature and mu_2 of the current state
            if (closure_rates(*net, k, C / Csat - 1.0, T, moment1d(f, n, dL, 2), G0, B)) status |= REF_SIM_FALLBACK;
        } else {
            rate_laws(p->law, k, T, Sp, G0, G2, B);
            if (p->law == REF_LAW_POWER || p->law == REF_LAW_ARRHENIUS) {
                const R Gd = dissolution_rate(k, C, Csat);
                if (val(Gd) < 0.0) G0 = Gd;
            }
        }
        // rates handed in from elsewhere (checks the finite-volume part on its own)
        if (s->G0_replay && s->B_replay && step < s->n_rates_replay) {
            G0 = R(s->G0_replay[step]);
            B = R(s->B_replay[step]);
        }

        const double t_next = next < s->n_samples ? s->t_samples[next] : p->t_end;
        // the fastest face moves at |G0| (1 + gamma L_max), growing or dissolving
        const double Gmax = std::fabs(val(G0)) * (1.0 + val(k.gamma) * s->L_max);
        const double cfl_limit = Gmax > 0.0 ? p->cfl * dL / Gmax : std::numeric_limits<double>::infinity();
        double dtv;
        const int kind = choose_dt(cfl_limit, p->dt_max, val(t), t_next, p->t_end, s->dt_replay, s->n_replay, step,
                                   &dtv);
        const bool hit = kind == DT_LAND;
        // the step as a function of the state and parameters, in the branch the values select
        R dt(dtv);
        if (kind == DT_CFL) dt = with_value(p->cfl * dL / (fabs(G0) * (1.0 + k.gamma * s->L_max)), dtv);
        if (kind == DT_LAND) dt = with_value(t_next - t, dtv);
        if (s->dt_log) s->dt_log[step] = dtv;
        if (s->G0_log) s->G0_log[step] = val(G0);
        if (s->B_log) s->B_log[step] = val(B);

        // Nucleation enters through the face at L = 0 as the flux B: the two
        // inflow ghost cells hold B/G0, so that G0 * ghost = B.
        const R inflow = val(G0) > 0.0 ? B / G0 : R(0.0);
        advance_line(f, n, dL, G0, k.gamma, inflow, p->scheme, dt, out);
        if (!k.corr.empty() && val(G0) > 0.0) correct_line(f, n, dL, G0, k.gamma, dt, k.corr);

        // Discrete mass balance, Eq. (9), with the 1D volume moment mu_3.
        const R mu3 = moment1d(f, n, dL, 3);
        C = C - p->alpha * (mu3 - mu3_old);
        mu3_old = mu3;

        t = hit ? R(t_next) : t + dt;
        ++step;
        if (!finite(val(C)) || !finite(val(mu3))) {
            status |= REF_SIM_NONFINITE;
            break;
        }
        if (hit) {
            while (next < s->n_samples && s->t_samples[next] <= val(t)) record(next++);
        }
    }
    const double mu0 = val(moment1d(f, n, dL, 0));
    if (val(out) > 1e-12 * std::max(mu0, 1e-300)) status |= REF_SIM_OUTFLOW;
    if (s->f_final) for (int i = 0; i < n; ++i) s->f_final[i] = val(f[i]);
    if (s->steps) *s->steps = step;
    if (s->status) *s->status = status;
    if (s->C_final) *s->C_final = val(C);
    if (s->t_final) *s->t_final = val(t);
    if (s->outflow) *s->outflow = val(out);
    return 0;
}

// ---------------------------------------------------------------------------
// 2D solve: Godunov (Lie) splitting, a full L1 sweep over every row followed
// by a full L2 sweep over every column, each one SSP-RK3 step (Sec. 2.1); or
// Strang splitting, L1 over dt/2, L2 over dt, L1 over dt/2.  Nucleation at the
// corner L1 = L2 = 0 is split equally between the two axes' inflow faces of
// the corner cell (under Strang the L1 share enters in two halves).
// ---------------------------------------------------------------------------
double moment2d(const std::vector<double>& f, int n1, int n2, double d1, double d2, int p, int q) {
    double m = 0.0;
    for (int j = 0; j < n2; ++j) {
        const double L2 = (j + 0.5) * d2;
        double w2 = 1.0;
        for (int r = 0; r < q; ++r) w2 *= L2;
        for (int i = 0; i < n1; ++i) {
            const double L1 = (i + 0.5) * d1;
            double w1 = 1.0;
            for (int r = 0; r < p; ++r) w1 *= L1;
            m += w1 * w2 * f[(size_t)j * n1 + i] * d1 * d2;
        }
    }
    return m;
}

int solve2d_impl(const ref_process* p, ref_sim2d* s) {
    const int n1 = s->n1, n2 = s->n2;
    const double d1 = s->L1_max / n1, d2 = s->L2_max / n2;
    const Kinetics<double> k = load_kinetics<double>(s->par);
    std::vector<double> f(s->f0, s->f0 + (size_t)n1 * n2);
    std::vector<double> line;
    double C = s->C0, t = 0.0, out = 0.0;
    double mu12_old = moment2d(f, n1, n2, d1, d2, 1, 2);
    int step = 0, next = 0, status = REF_SIM_OK;
    const int max_steps = s->max_steps > 0 ? s->max_steps : std::numeric_limits<int>::max();
    auto record = [&](int q) {
        if (s->mom) {
            s->mom[q * 4 + 0] = moment2d(f, n1, n2, d1, d2, 0, 0);
            s->mom[q * 4 + 1] = moment2d(f, n1, n2, d1, d2, 1, 0);
            s->mom[q * 4 + 2] = moment2d(f, n1, n2, d1, d2, 0, 1);
            s->mom[q * 4 + 3] = moment2d(f, n1, n2, d1, d2, 1, 2);
        }
        if (s->C) s->C[q] = C;
    };
    while (t < p->t_end && step < max_steps) {
        const double T = temperature(s->par, t);
        const double Sp = supersaturation_pos(C, solubility(p, T));
        double G1, G2, B;
        rate_laws(p->law, k, T, Sp, G1, G2, B);
        const double t_next = next < s->n_samples ? s->t_samples[next] : p->t_end;
        // SI Eq. (S3): dt = nu * min(dL1/G1, dL2/G2)
        double lim = std::numeric_limits<double>::infinity();
        if (G1 > 0.0) lim = std::min(lim, d1 / G1);
        if (G2 > 0.0) lim = std::min(lim, d2 / G2);
        double dt;
        const bool hit = choose_dt(p->cfl * lim, p->dt_max, t, t_next, p->t_end, nullptr, 0, step, &dt) == DT_LAND;
        if (s->dt_log) s->dt_log[step] = dt;

        // sweep along L1 over a time h: every row j is a 1D line of n1 cells
        auto sweep_rows = [&](double h) {
            line.resize(n1);
            for (int j = 0; j < n2; ++j) {
                for (int i = 0; i < n1; ++i) line[i] = f[(size_t)j * n1 + i];
                const double inflow = (j == 0 && G1 > 0.0) ? B / (2.0 * d2 * G1) : 0.0;
                double o = 0.0;
                advance_line(line, n1, d1, G1, 0.0, inflow, p->scheme, h, o);
                out += o * d2;
                for (int i = 0; i < n1; ++i) f[(size_t)j * n1 + i] = line[i];
            }
        };
        // sweep along L2 over a time h: every column i is a 1D line of n2 cells
        auto sweep_cols = [&](double h) {
            line.resize(n2);
            for (int i = 0; i < n1; ++i) {
                for (int j = 0; j < n2; ++j) line[j] = f[(size_t)j * n1 + i];
                const double inflow = (i == 0 && G2 > 0.0) ? B / (2.0 * d1 * G2) : 0.0;
                double o = 0.0;
                advance_line(line, n2, d2, G2, 0.0, inflow, p->scheme, h, o);
                out += o * d1;
                for (int j = 0; j < n2; ++j) f[(size_t)j * n1 + i] = line[j];
            }
        };
        if (p->splitting == REF_SPLIT_STRANG) {
            sweep_rows(0.5 * dt);
            sweep_cols(dt);
            sweep_rows(0.5 * dt);
        } else {
            sweep_rows(dt);
            sweep_cols(dt);
        }
        // Eq. (9) with the volume moment mu_{1,2} = int L1 L2^2 f
        const double mu12 = moment2d(f, n1, n2, d1, d2, 1, 2);
        C = C - p->alpha * (mu12 - mu12_old);
        mu12_old = mu12;
        t = hit ? t_next : t + dt;
        ++step;
        if (!finite(C) || !finite(mu12)) { status |= REF_SIM_NONFINITE; break; }
        if (hit) while (next < s->n_samples && s->t_samples[next] <= t) record(next++);
    }
    const double mu0 = moment2d(f, n1, n2, d1, d2, 0, 0);
    if (out > 1e-12 * std::max(mu0, 1e-300)) status |= REF_SIM_OUTFLOW;
    if (s->f_final) std::copy(f.begin(), f.end(), s->f_final);
    if (s->steps) *s->steps = step;
    if (s->status) *s->status = status;
    if (s->C_final) *s->C_final = C;
    if (s->t_final) *s->t_final = t;
    if (s->outflow) *s->outflow = out;
    return 0;
}

template <class Fn>
int run_pool(int n_items, int n_threads, Fn fn) {
    if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    n_threads = std::max(1, std::min(n_threads, std::max(1, n_items)));
    std::atomic<int> nextw(0);
    std::vector<std::thread> pool;
    for (int w = 0; w < n_threads; ++w)
        pool.emplace_back([&]() {
            for (int i = nextw++; i < n_items; i = nextw++) fn(i);
        });
    for (auto& th : pool) th.join();
    return n_threads;
}

// ---------------------------------------------------------------------------
// Method of moments, Dormand-Prince 5(4) with step-size control.
// ---------------------------------------------------------------------------
struct MomSystem {
    const ref_process* p;
    const double* par;
    int dim;  // 1 or 2
};

// y = (mu..., C).  1D: mu_0..mu_3.  2D: mu_00, mu_10, mu_01, mu_11, mu_02, mu_12.
void mom_rhs(const MomSystem& sys, double t, const double* y, double* dy) {
    const Kinetics<double> k = load_kinetics<double>(sys.par);
    const double T = temperature(sys.par, t);
    if (sys.dim == 1) {
        const double Sp = supersaturation_pos(y[4], solubility(sys.p, T));
        double G0, G2, B;
        rate_laws(sys.p->law, k, T, Sp, G0, G2, B);
        const double Gd = dissolution_rate(k, y[4], solubility(sys.p, T));
        if (Gd < 0.0) G0 = Gd;
        // d/dt int L^k f = k int L^(k-1) G f (+ B for k = 0), G = G0 (1 + gamma L);
        // under dissolution this holds for k >= 1 (what leaves through L = 0 has
        // zero size) and for mu_0 while no crystal reaches L = 0
        dy[0] = B;
        for (int m = 1; m <= 3; ++m) dy[m] = m * G0 * (y[m - 1] + k.gamma * y[m]);
        dy[4] = -sys.p->alpha * dy[3];
    } else {
        const double Sp = supersaturation_pos(y[6], solubility(sys.p, T));
        double G1, G2, B;
        rate_laws(sys.p->law, k, T, Sp, G1, G2, B);
        // Eq. (S4): d mu_pq/dt = p G1 mu_{p-1,q} + q G2 mu_{p,q-1} (+ B at p = q = 0)
        dy[0] = B;                                   // mu_00
        dy[1] = G1 * y[0];                           // mu_10
        dy[2] = G2 * y[0];                           // mu_01
        dy[3] = G1 * y[2] + G2 * y[1];               // mu_11
        dy[4] = 2.0 * G2 * y[2];                     // mu_02
        dy[5] = G1 * y[4] + 2.0 * G2 * y[3];         // mu_12
        dy[6] = -sys.p->alpha * dy[5];
    }
}

int dopri5(const MomSystem& sys, int ny, double* y, int n_samples, const double* t_samples, double rtol, double atol,
           double* y_out) {
    static const double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
    static const double a21 = 1.0 / 5;
    static const double a31 = 3.0 / 40, a32 = 9.0 / 40;
    static const double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
    static const double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561, a54 = -212.0 / 729;
    static const double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                        a65 = -5103.0 / 18656;
    static const double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784, b6 = 11.0 / 84;
    static const double e1 = 35.0 / 384 - 5179.0 / 57600, e3 = 500.0 / 1113 - 7571.0 / 16695,
                        e4 = 125.0 / 192 - 393.0 / 640, e5 = -2187.0 / 6784 + 92097.0 / 339200,
                        e6 = 11.0 / 84 - 187.0 / 2100, e7 = -1.0 / 40;
    std::vector<double> k1(ny), k2(ny), k3(ny), k4(ny), k5(ny), k6(ny), k7(ny), yt(ny), yn(ny);
    double t = 0.0, h = 1e-3;
    long guard = 0;
    for (int q = 0; q < n_samples; ++q) {
        const double tq = t_samples[q];
        while (t < tq) {
            if (++guard > 50000000L) return -1;
            bool last = false;
            if (t + h >= tq) { h = tq - t; last = true; }
            mom_rhs(sys, t, y, k1.data());
            for (int i = 0; i < ny; ++i) yt[i] = y[i] + h * a21 * k1[i];
            mom_rhs(sys, t + c2 * h, yt.data(), k2.data());
            for (int i = 0; i < ny; ++i) yt[i] = y[i] + h * (a31 * k1[i] + a32 * k2[i]);
            mom_rhs(sys, t + c3 * h, yt.data(), k3.data());
            for (int i = 0; i < ny; ++i) yt[i] = y[i] + h * (a41 * k1[i] + a42 * k2[i] + a43 * k3[i]);
            mom_rhs(sys, t + c4 * h, yt.data(), k4.data());
            for (int i = 0; i < ny; ++i) yt[i] = y[i] + h * (a51 * k1[i] + a52 * k2[i] + a53 * k3[i] + a54 * k4[i]);
            mom_rhs(sys, t + c5 * h, yt.data(), k5.data());
            for (int i = 0; i < ny; ++i)
                yt[i] = y[i] + h * (a61 * k1[i] + a62 * k2[i] + a63 * k3[i] + a64 * k4[i] + a65 * k5[i]);
            mom_rhs(sys, t + h, yt.data(), k6.data());
            for (int i = 0; i < ny; ++i)
                yn[i] = y[i] + h * (b1 * k1[i] + b3 * k3[i] + b4 * k4[i] + b5 * k5[i] + b6 * k6[i]);
            mom_rhs(sys, t + h, yn.data(), k7.data());
            double err = 0.0;
            for (int i = 0; i < ny; ++i) {
                const double ei = h * (e1 * k1[i] + e3 * k3[i] + e4 * k4[i] + e5 * k5[i] + e6 * k6[i] + e7 * k7[i]);
                const double sc = atol + rtol * std::max(std::fabs(y[i]), std::fabs(yn[i]));
                err += (ei / sc) * (ei / sc);
            }
            err = std::sqrt(err / ny);
            if (err <= 1.0) {
                t = last ? tq : t + h;
                for (int i = 0; i < ny; ++i) y[i] = yn[i];
            }
            const double fac = err > 0.0 ? 0.9 * std::pow(err, -0.2) : 5.0;
            h = h * std::min(5.0, std::max(0.2, fac));
            if (h < 1e-12) h = 1e-12;
        }
        for (int i = 0; i < ny; ++i) y_out[(size_t)q * ny + i] = y[i];
    }
    return 0;
}

}  // namespace

extern "C" {

double ref_phi_vanleer(double theta) { return phi_vanleer(theta); }
double ref_limited_slope(double a, double b) { return limited_slope<double>(a, b); }

int ref_solve1d(const ref_process* p, ref_sim1d* s) {
    if (!p || !s || s->n < 1 || !s->f0 || !s->par) return -1;
    if (p->law == REF_LAW_MLP) {
        if (!p->mlp) return -1;
        const Net<double> net = load_net<double>(p->mlp, p->mlp_precision, nullptr, -1);
        return solve1d_impl<double>(p, s, load_kinetics_sim<double>(s), nullptr, &net);
    }
    if (p->law == REF_LAW_POLY && (!s->poly || s->n_poly < 1)) return -1;
    return solve1d_impl<double>(p, s, load_kinetics_sim<double>(s), nullptr);
}

int ref_solve1d_batch(const ref_process* p, ref_sim1d* sims, int32_t n_sims, int32_t n_threads) {
    return run_pool(n_sims, n_threads, [&](int i) { ref_solve1d(p, &sims[i]); });
}

// Primal run of one simulation that records its step sizes (for a replay).
static std::vector<double> primal_schedule(const ref_process* p, const ref_sim1d* s, const Net<double>* net) {
    const int cap = s->max_steps > 0 ? std::min(s->max_steps, 2000000) : 2000000;
    std::vector<double> dts(cap);
    int steps = 0;
    ref_sim1d s0 = *s;
    s0.f_samples = nullptr; s0.mom = nullptr; s0.C = nullptr; s0.f_final = nullptr;
    s0.G0_log = nullptr; s0.B_log = nullptr; s0.outflow = nullptr;
    s0.C_final = nullptr; s0.t_final = nullptr; s0.status = nullptr;
    s0.dt_log = dts.data();
    s0.steps = &steps;
    s0.max_steps = cap;
    solve1d_impl<double>(p, &s0, load_kinetics_sim<double>(&s0), nullptr, net);
    dts.resize(steps);
    return dts;
}

int ref_tangent1d(const ref_process* p, ref_sim1d* s, int32_t dt_mode, double* dF, double* dM, double* dC) {
    typedef Dual<REF_NTAN> D;
    if (!p || !s || s->n < 1 || p->law == REF_LAW_MLP) return -1;
    if (dt_mode != REF_DT_DIFF && dt_mode != REF_DT_FROZEN) return -1;
    Kinetics<D> k = load_kinetics_sim<D>(s);
    k.kg.d[0] = 1.0; k.g.d[1] = 1.0; k.kb.d[2] = 1.0; k.b.d[3] = 1.0; k.gamma.d[4] = 1.0;
    std::vector<D> tf((size_t)s->n_samples * s->n), tm((size_t)s->n_samples * 4), tc(s->n_samples);
    Tangents<D> tan;
    tan.f_samples = dF ? &tf : nullptr;
    tan.mom = &tm;
    tan.C = &tc;
    ref_sim1d s1 = *s;
    std::vector<double> dts;
    if (dt_mode == REF_DT_FROZEN) {
        // the step-size schedule of the primal run, replayed as constants
        dts = primal_schedule(p, s, nullptr);
        s1.dt_replay = dts.data();
        s1.n_replay = (int)dts.size();
        s1.max_steps = (int)dts.size();
    }
    solve1d_impl<D>(p, &s1, k, &tan);
    for (int q = 0; q < s->n_samples; ++q) {
        for (int d = 0; d < REF_NTAN; ++d) {
            if (dC) dC[q * REF_NTAN + d] = tc[q].d[d];
            for (int m = 0; m < 4; ++m)
                if (dM) dM[(q * 4 + m) * REF_NTAN + d] = tm[q * 4 + m].d[d];
            if (dF)
                for (int i = 0; i < s->n; ++i) dF[((size_t)q * s->n + i) * REF_NTAN + d] = tf[(size_t)q * s->n + i].d[d];
        }
    }
    return 0;
}

double ref_bf16(double x) { return bf16_of_double(x); }

int ref_mlp_forward(const float* blob, int32_t precision, int32_t n, const double* x, double* y, double* dy) {
    typedef Dual<3> D;
    if (!blob || n < 0 || !x || !y) return -1;
    const Net<D> net = load_net<D>(blob, precision, nullptr, -1);
    for (int r = 0; r < n; ++r) {
        D z[3], o[2];
        for (int q = 0; q < 3; ++q) {
            z[q] = D((x[r * 3 + q] - net.c[C_IN_SHIFT + q]) * net.c[C_IN_SCALE + q]);
            z[q].d[q] = 1.0;
        }
        net_forward(net, z, o);
        for (int j = 0; j < 2; ++j) {
            y[r * 2 + j] = o[j].v;
            if (dy)
                for (int q = 0; q < 3; ++q) dy[(r * 2 + j) * 3 + q] = o[j].d[q];
        }
    }
    return 0;
}

// Reverse pass of the network written out layer by layer (the transposed
// products of the forward pass); the roundings of BF16 mode act on values only.
int ref_mlp_vjp(const float* blob, int32_t precision, int32_t n, const double* z, const double* ybar, double* gw) {
    if (!blob || n < 0 || !z || !ybar || !gw) return -1;
    const Net<double> net = load_net<double>(blob, precision, nullptr, -1);
    const std::vector<double>& w = net.w;
    const bool bf = precision == REF_MLP_BF16;
    for (int i = 0; i < REF_MLP_NW; ++i) gw[i] = 0.0;
    for (int r = 0; r < n; ++r) {
        double zi[3], a1[MH], h1[MH], t1[MH], a2[MH], h2[MH], t2[MH];
        for (int k = 0; k < 3; ++k) zi[k] = bf ? bf16_of_double((double)(float)z[r * 3 + k]) : z[r * 3 + k];
        for (int j = 0; j < MH; ++j) {
            double a = w[OFF_B1 + j];
            for (int k = 0; k < 3; ++k) a += w[OFF_W1 + j * 3 + k] * zi[k];
            a1[j] = a;
            t1[j] = bf ? (double)(float)std::tanh((double)(float)a) : std::tanh(a);
            h1[j] = bf ? (double)round_bf16((float)t1[j]) : t1[j];
        }
        for (int j = 0; j < MH; ++j) {
            double a = w[OFF_B2 + j];
            for (int i = 0; i < MH; ++i) a += w[OFF_W2 + j * MH + i] * h1[i];
            a2[j] = a;
            t2[j] = bf ? (double)(float)std::tanh((double)(float)a) : std::tanh(a);
            h2[j] = bf ? (double)round_bf16((float)t2[j]) : t2[j];
        }
        (void)a1; (void)a2;
        const double yb[2] = {ybar[r * 2], ybar[r * 2 + 1]};
        double d2[MH], d1[MH];
        for (int o = 0; o < 2; ++o) {
            gw[OFF_B3 + o] += yb[o];
            for (int j = 0; j < MH; ++j) gw[OFF_W3 + o * MH + j] += yb[o] * h2[j];
        }
        for (int j = 0; j < MH; ++j) {
            double g = 0.0;
            for (int o = 0; o < 2; ++o) g += w[OFF_W3 + o * MH + j] * yb[o];
            d2[j] = g * (1.0 - t2[j] * t2[j]);
        }
        for (int j = 0; j < MH; ++j) {
            gw[OFF_B2 + j] += d2[j];
            for (int i = 0; i < MH; ++i) gw[OFF_W2 + j * MH + i] += d2[j] * h1[i];
        }
        for (int i = 0; i < MH; ++i) {
            double g = 0.0;
            for (int j = 0; j < MH; ++j) g += w[OFF_W2 + j * MH + i] * d2[j];
            d1[i] = g * (1.0 - t1[i] * t1[i]);
        }
        for (int j = 0; j < MH; ++j) {
            gw[OFF_B1 + j] += d1[j];
            for (int k = 0; k < 3; ++k) gw[OFF_W1 + j * 3 + k] += d1[j] * zi[k];
        }
    }
    return 0;
}

int ref_tangent1d_mlp(const ref_process* p, ref_sim1d* s, int32_t dt_mode, const double* v, double* dF, double* dM,
                      double* dC) {
    typedef Dual<2> D;
    if (!p || !s || s->n < 1 || p->law != REF_LAW_MLP || !p->mlp || !v) return -1;
    if (dt_mode != REF_DT_DIFF && dt_mode != REF_DT_FROZEN) return -1;
    const Net<D> net = load_net<D>(p->mlp, p->mlp_precision, v, 0);
    Kinetics<D> k = load_kinetics<D>(s->par);
    k.gamma.d[1] = 1.0;
    std::vector<D> tf((size_t)s->n_samples * s->n), tm((size_t)s->n_samples * 4), tc(s->n_samples);
    Tangents<D> tan;
    tan.f_samples = dF ? &tf : nullptr;
    tan.mom = &tm;
    tan.C = &tc;
    ref_sim1d s1 = *s;
    std::vector<double> dts;
    if (dt_mode == REF_DT_FROZEN) {
        const Net<double> net0 = load_net<double>(p->mlp, p->mlp_precision, nullptr, -1);
        dts = primal_schedule(p, s, &net0);
        s1.dt_replay = dts.data();
        s1.n_replay = (int)dts.size();
        s1.max_steps = (int)dts.size();
    }
    solve1d_impl<D>(p, &s1, k, &tan, &net);
    for (int q = 0; q < s->n_samples; ++q)
        for (int d = 0; d < 2; ++d) {
            if (dC) dC[q * 2 + d] = tc[q].d[d];
            for (int m = 0; m < 4; ++m)
                if (dM) dM[(q * 4 + m) * 2 + d] = tm[q * 4 + m].d[d];
            if (dF)
                for (int i = 0; i < s->n; ++i) dF[((size_t)q * s->n + i) * 2 + d] = tf[(size_t)q * s->n + i].d[d];
        }
    return 0;
}

int ref_tangent1d_poly(const ref_process* p, ref_sim1d* s, int32_t dt_mode, const double* v, double* dF, double* dM,
                       double* dC) {
    typedef Dual<2> D;
    if (!p || !s || s->n < 1 || p->law != REF_LAW_POLY || !s->poly || s->n_poly < 1 || !v) return -1;
    if (dt_mode != REF_DT_DIFF && dt_mode != REF_DT_FROZEN) return -1;
    Kinetics<D> k = load_kinetics_sim<D>(s, v, 0);
    k.gamma.d[1] = 1.0;
    std::vector<D> tf((size_t)s->n_samples * s->n), tm((size_t)s->n_samples * 4), tc(s->n_samples);
    Tangents<D> tan;
    tan.f_samples = dF ? &tf : nullptr;
    tan.mom = &tm;
    tan.C = &tc;
    ref_sim1d s1 = *s;
    std::vector<double> dts;
    if (dt_mode == REF_DT_FROZEN) {
        dts = primal_schedule(p, s, nullptr);
        s1.dt_replay = dts.data();
        s1.n_replay = (int)dts.size();
        s1.max_steps = (int)dts.size();
    }
    solve1d_impl<D>(p, &s1, k, &tan);
    for (int q = 0; q < s->n_samples; ++q)
        for (int d = 0; d < 2; ++d) {
            if (dC) dC[q * 2 + d] = tc[q].d[d];
            for (int m = 0; m < 4; ++m)
                if (dM) dM[(q * 4 + m) * 2 + d] = tm[q * 4 + m].d[d];
            if (dF)
                for (int i = 0; i < s->n; ++i) dF[((size_t)q * s->n + i) * 2 + d] = tf[(size_t)q * s->n + i].d[d];
        }
    return 0;
}

int ref_tangent1d_corr(const ref_process* p, ref_sim1d* s, int32_t dt_mode, const double* v, double* dF, double* dM,
                       double* dC) {
    typedef Dual<2> D;
    if (!p || !s || s->n < 1 || !s->corr || !v || p->law == REF_LAW_MLP) return -1;
    if (dt_mode != REF_DT_DIFF && dt_mode != REF_DT_FROZEN) return -1;
    Kinetics<D> k = load_kinetics_sim<D>(s, nullptr, -1, v);
    k.gamma.d[1] = 1.0;
    std::vector<D> tf((size_t)s->n_samples * s->n), tm((size_t)s->n_samples * 4), tc(s->n_samples);
    Tangents<D> tan;
    tan.f_samples = dF ? &tf : nullptr;
    tan.mom = &tm;
    tan.C = &tc;
    ref_sim1d s1 = *s;
    std::vector<double> dts;
    if (dt_mode == REF_DT_FROZEN) {
        dts = primal_schedule(p, s, nullptr);
        s1.dt_replay = dts.data();
        s1.n_replay = (int)dts.size();
        s1.max_steps = (int)dts.size();
    }
    solve1d_impl<D>(p, &s1, k, &tan);
    for (int q = 0; q < s->n_samples; ++q)
        for (int d = 0; d < 2; ++d) {
            if (dC) dC[q * 2 + d] = tc[q].d[d];
            for (int m = 0; m < 4; ++m)
                if (dM) dM[(q * 4 + m) * 2 + d] = tm[q * 4 + m].d[d];
            if (dF)
                for (int i = 0; i < s->n; ++i) dF[((size_t)q * s->n + i) * 2 + d] = tf[(size_t)q * s->n + i].d[d];
        }
    return 0;
}

int ref_solve2d(const ref_process* p, ref_sim2d* s) {
    if (!p || !s || s->n1 < 1 || s->n2 < 1 || !s->f0 || !s->par) return -1;
    if (p->law == REF_LAW_MLP || p->law == REF_LAW_POLY) return -2;
    return solve2d_impl(p, s);
}

int ref_solve2d_batch(const ref_process* p, ref_sim2d* sims, int32_t n_sims, int32_t n_threads) {
    return run_pool(n_sims, n_threads, [&](int i) { ref_solve2d(p, &sims[i]); });
}

int ref_mom1d(const ref_process* p, const double* par, double C0, const double* mu_init, int32_t n_samples,
              const double* t_samples, double rtol, double atol, double* mu_out, double* C_out) {
    if (p->law == REF_LAW_MLP || p->law == REF_LAW_POLY) return -2;
    MomSystem sys{p, par, 1};
    double y[5] = {mu_init[0], mu_init[1], mu_init[2], mu_init[3], C0};
    std::vector<double> yo((size_t)n_samples * 5);
    const int rc = dopri5(sys, 5, y, n_samples, t_samples, rtol, atol, yo.data());
    for (int q = 0; q < n_samples; ++q) {
        for (int m = 0; m < 4; ++m) mu_out[q * 4 + m] = yo[q * 5 + m];
        C_out[q] = yo[q * 5 + 4];
    }
    return rc;
}

int ref_mom2d(const ref_process* p, const double* par, double C0, const double* mu_init, int32_t n_samples,
              const double* t_samples, double rtol, double atol, double* mu_out, double* C_out) {
    MomSystem sys{p, par, 2};
    double y[7];
    for (int m = 0; m < 6; ++m) y[m] = mu_init[m];
    y[6] = C0;
    std::vector<double> yo((size_t)n_samples * 7);
    const int rc = dopri5(sys, 7, y, n_samples, t_samples, rtol, atol, yo.data());
    for (int q = 0; q < n_samples; ++q) {
        for (int m = 0; m < 6; ++m) mu_out[q * 6 + m] = yo[q * 7 + m];
        C_out[q] = yo[q * 7 + 6];
    }
    return rc;
}

void ref_dual_example(double x1, double x2, double* out) {
    typedef Dual<2> D;
    D a(x1), b(x2);
    a.d[0] = 1.0;
    b.d[1] = 1.0;
    const D s = a + b;
    const D y1 = sin(a) / s;
    const D y2 = s * exp(b);
    out[0] = y1.v; out[1] = y2.v;
    out[2] = y1.d[0]; out[3] = y1.d[1];
    out[4] = y2.d[0]; out[5] = y2.d[1];
}

}  // extern "C"

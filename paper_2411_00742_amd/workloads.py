"""Seeded synthetic inputs for the crystallization PBE solver.

This module only draws inputs: random kinetics, grid sizes, operating
conditions and seed distributions.  It holds none of the solver's arithmetic
(no fluxes, limiters, rates, moments or mass balance), so both the HIP path and
the FP64 CPU oracle can be fed from it without sharing any of the method.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), written out here from that
published definition.  Uniforms take the top 53 bits; normals use Box-Muller.

Units used throughout: L in micrometres, t in seconds, T in degrees Celsius,
number density f in #/(m^3 um^d) for a d-dimensional grid, G in um/s,
B in #/(m^3 s), concentration C in g solute per g solvent.

The workload shapes follow the paper's batch cooling crystallizer (Sec. 2.1,
Table 1: Gaussian seeds, cylinder shape factor, crystal density) with the
sizes of the batched / 2D / gradient / closure studies this solver targets.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy.special import erf

MASK64 = (1 << 64) - 1

# ---- integer codes shared by the C ABI, the oracle wrapper and this module --
SCHEME_SSPRK3 = 0      # method of lines + Shu-Osher SSP-RK3, limited upwind flux
SCHEME_LW_TVD = 1      # the paper's one-step limited Lax-Wendroff update (Eq. 8)
LAW_POWER = 0          # G = kg*S^g (1 + gamma*L), B = kb*S^b
LAW_ARRHENIUS = 1      # as above times exp(-E/(T+273.15)) (App. A, Eq. A.2 form)
LAW_MLP = 2            # learned closure
LAW_POLY = 3           # growth a_1 S + ... + a_k S^k (the polynomial law of Sec. 4.1)
CORR_H, CORR_NW = 8, 57   # in-the-loop correction network: W1[8][5] b1[8] W2[8] b2
SPLIT_LIE = 0          # 2D: Godunov splitting, L1 sweep then L2 sweep (Sec. 2.1)
SPLIT_STRANG = 1       # 2D: Strang splitting, L1 over dt/2, L2 over dt, L1 over dt/2
SOL_LINEAR = 0         # Csat = cs0 + cs1*T
SOL_EXP = 1            # Csat = cs0*exp(cs1*T)   (App. A, Eq. A.1)

# per-simulation parameter row (NPAR doubles)
P_KG, P_G, P_KB, P_B, P_GAMMA, P_KG2, P_G2, P_EG, P_EB, P_T0, P_T1, P_TRAMP, P_EG2, P_KD, P_D = range(15)
NPAR = 15

RHO_C_G_PER_UM3 = 1.11e-12          # crystal density, Table 1
K_V = math.pi / 4.0                  # cylinder shape factor, Table 1
RHO_SOLVENT_G_PER_M3 = 1.0e6         # 1000 kg/m^3 (not given by the paper)
ALPHA = RHO_C_G_PER_UM3 * K_V / RHO_SOLVENT_G_PER_M3   # g/g per (um^3/m^3)

CS0, CS1 = 0.1, 0.002                # linear solubility g/g and g/g/degC
T_HOT, T_COLD, T_RAMP, T_END = 40.0, 20.0, 3600.0, 3600.0


class SplitMix64:
    """SplitMix64 generator (Steele, Lea, Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform on [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_range(self, lo: float, hi: float) -> float:
        return lo + (hi - lo) * self.uniform()

    def log_uniform(self, lo: float, hi: float) -> float:
        return math.exp(self.uniform_range(math.log(lo), math.log(hi)))

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on {lo, ..., hi}."""
        return lo + min(int(self.uniform() * (hi - lo + 1)), hi - lo)

    def normal(self) -> float:
        """Standard normal by Box-Muller (one of the pair)."""
        u1 = self.uniform()
        u2 = self.uniform()
        u1 = max(u1, 1e-300)
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def csat_linear(T: float) -> float:
    """Solubility used by the workloads (an input choice, g/g)."""
    return CS0 + CS1 * T


def gaussian_seed_1d(n: int, L_max: float, mean: float, sd: float, total: float) -> np.ndarray:
    """Cell averages of a Gaussian number density on n uniform cells of [0, L_max].

    Cell averages come from differences of the normal CDF; the result is
    rescaled so that sum(f)*dL equals `total` exactly (up to rounding).
    """
    edges = np.linspace(0.0, L_max, n + 1)
    cdf = 0.5 * (1.0 + erf((edges - mean) / (sd * math.sqrt(2.0))))
    dL = L_max / n
    f = np.diff(cdf) / dL
    f = np.maximum(f, 0.0)
    f *= total / (f.sum() * dL)
    return f.astype(np.float64)


def gaussian_seed_2d(n1: int, n2: int, L1_max: float, L2_max: float,
                     mean: tuple, sd: tuple, rho: float, total: float) -> np.ndarray:
    """Bivariate normal density sampled at cell centres, shape [n2][n1] (L1 fastest).

    Rescaled so that sum(f)*dL1*dL2 equals `total`.
    """
    d1, d2 = L1_max / n1, L2_max / n2
    x = (np.arange(n1) + 0.5) * d1
    y = (np.arange(n2) + 0.5) * d2
    z1 = (x[None, :] - mean[0]) / sd[0]
    z2 = (y[:, None] - mean[1]) / sd[1]
    q = (z1 * z1 - 2.0 * rho * z1 * z2 + z2 * z2) / (1.0 - rho * rho)
    f = np.exp(-0.5 * q)
    f *= total / (f.sum() * d1 * d2)
    return np.ascontiguousarray(f, dtype=np.float64)


# ---- seed distributions of SI S1.3: a sample PSSD from a normal or log-normal
# distribution given its mean and (co)variance, scaled up to the crystallizer by
# the seed mass: beta = m_seed / (rho_c k_v * mass moment of the sample)

def lognormal_params(mean: float, sd: float):
    """(mu, sigma) of ln L for a log-normal L with the given mean and standard deviation."""
    s2 = math.log1p((sd / mean) ** 2)
    return math.log(mean) - 0.5 * s2, math.sqrt(s2)


def seed_sample_1d(kind: str, n: int, L_max: float, mean: float, sd: float) -> np.ndarray:
    """Sample PSSD on n uniform cells of [0, L_max]: cell averages of a normal or log-normal
    probability density with the given mean and standard deviation (CDF differences)."""
    edges = np.linspace(0.0, L_max, n + 1)
    if kind == "normal":
        cdf = 0.5 * (1.0 + erf((edges - mean) / (sd * math.sqrt(2.0))))
    elif kind == "lognormal":
        mu, sig = lognormal_params(mean, sd)
        with np.errstate(divide="ignore"):
            z = (np.log(edges) - mu) / (sig * math.sqrt(2.0))
        cdf = 0.5 * (1.0 + erf(z))
    else:
        raise ValueError(f"seed kind {kind!r}: 'normal' or 'lognormal'")
    return np.maximum(np.diff(cdf) / (L_max / n), 0.0)


def seed_sample_2d(kind: str, n1: int, n2: int, L1_max: float, L2_max: float, mean, cov) -> np.ndarray:
    """Sample PSSD [n2][n1] (L1 fastest): a bivariate normal or log-normal probability density
    at cell centres with mean vector `mean` and covariance matrix `cov` of (L1, L2)."""
    m = np.asarray(mean, dtype=np.float64)
    c = np.asarray(cov, dtype=np.float64)
    d1, d2 = L1_max / n1, L2_max / n2
    x = (np.arange(n1) + 0.5) * d1
    y = (np.arange(n2) + 0.5) * d2
    X, Y = np.meshgrid(x, y)
    if kind == "normal":
        mu, S, u, v, jac = m, c, X, Y, 1.0
    elif kind == "lognormal":
        # (ln L1, ln L2) is bivariate normal with Cov_ij = ln(1 + cov_ij / (m_i m_j))
        S = np.log1p(c / np.outer(m, m))
        mu = np.log(m) - 0.5 * np.diag(S)
        u, v, jac = np.log(X), np.log(Y), 1.0 / (X * Y)
    else:
        raise ValueError(f"seed kind {kind!r}: 'normal' or 'lognormal'")
    det = S[0, 0] * S[1, 1] - S[0, 1] * S[1, 0]
    du, dv = u - mu[0], v - mu[1]
    q = (S[1, 1] * du * du - 2.0 * S[0, 1] * du * dv + S[0, 0] * dv * dv) / det
    f = np.exp(-0.5 * q) / (2.0 * math.pi * math.sqrt(det)) * jac
    return np.ascontiguousarray(f, dtype=np.float64)


def scale_to_seed_mass(f_sample: np.ndarray, m_seed: float, rho_kv: float, L_max, n_cells) -> np.ndarray:
    """f0 = beta f_sample with beta = m_seed / (rho_c k_v * integral of the mass moment of the
    sample): L^3 in one size coordinate (equant crystals), L1 L2^2 in two (SI S1.3); midpoint
    rule at cell centres, as for the solver's moments."""
    if np.ndim(L_max) == 0:
        n = int(n_cells)
        dL = float(L_max) / n
        L = (np.arange(n) + 0.5) * dL
        mass = float((L ** 3 * f_sample).sum() * dL)
    else:
        n1, n2 = int(n_cells[0]), int(n_cells[1])
        d1, d2 = float(L_max[0]) / n1, float(L_max[1]) / n2
        x = (np.arange(n1) + 0.5) * d1
        y = (np.arange(n2) + 0.5) * d2
        mass = float((x[None, :] * (y ** 2)[:, None] * f_sample.reshape(n2, n1)).sum() * d1 * d2)
    return f_sample * (m_seed / (rho_kv * mass))


@dataclass
class Problem:
    """A batch of independent simulations plus the process settings they share.

    ndim == 1: n_cells[S], L_max[S], f0 packed [sum N_s].
    ndim == 2: n_cells[S, 2] = (n1, n2), L_max[S, 2], f0 packed [sum n1*n2],
               each sim stored [n2][n1] with L1 contiguous.
    par[S, NPAR]: kinetics and operating conditions (see the P_* indices).
    """
    ndim: int
    n_cells: np.ndarray
    L_max: np.ndarray
    f0: np.ndarray
    C0: np.ndarray
    par: np.ndarray
    t_samples: np.ndarray
    law: int = LAW_POWER
    scheme: int = SCHEME_SSPRK3
    sol_law: int = SOL_LINEAR
    cs0: float = CS0
    cs1: float = CS1
    alpha: float = ALPHA
    cfl: float = 0.5
    dt_max: float = 1.0
    t_end: float = T_END
    name: str = ""
    extra: dict = field(default_factory=dict)
    mlp: np.ndarray | None = None      # law == LAW_MLP: float32 closure blob [MLP_NBLOB]
    mlp_precision: int = 0             # MLP_BF16 or MLP_FP64
    poly: np.ndarray | None = None     # law == LAW_POLY: growth coefficients a_1..a_k per sim [S, k]
    splitting: int = SPLIT_LIE         # 2D: SPLIT_LIE or SPLIT_STRANG
    corr: np.ndarray | None = None     # 1D: in-the-loop correction weights per sim [S, CORR_NW]

    @property
    def n_sims(self) -> int:
        return int(self.C0.shape[0])

    def cells_per_sim(self) -> np.ndarray:
        if self.ndim == 1:
            return self.n_cells.astype(np.int64)
        return (self.n_cells[:, 0].astype(np.int64) * self.n_cells[:, 1].astype(np.int64))

    def offsets(self) -> np.ndarray:
        c = self.cells_per_sim()
        off = np.zeros(c.shape[0] + 1, dtype=np.int64)
        np.cumsum(c, out=off[1:])
        return off

    def f0_of(self, s: int) -> np.ndarray:
        off = self.offsets()
        f = self.f0[off[s]:off[s + 1]]
        if self.ndim == 2:
            n1, n2 = int(self.n_cells[s, 0]), int(self.n_cells[s, 1])
            return f.reshape(n2, n1)
        return f

    def subset(self, idx) -> "Problem":
        """The same problem restricted to the simulations in `idx` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        off = self.offsets()
        f0 = np.concatenate([self.f0[off[s]:off[s + 1]] for s in idx]) if len(idx) else np.zeros(0)
        return Problem(ndim=self.ndim, n_cells=self.n_cells[idx].copy(), L_max=self.L_max[idx].copy(),
                       f0=f0, C0=self.C0[idx].copy(), par=self.par[idx].copy(),
                       t_samples=self.t_samples.copy(), law=self.law, scheme=self.scheme,
                       sol_law=self.sol_law, cs0=self.cs0, cs1=self.cs1, alpha=self.alpha,
                       cfl=self.cfl, dt_max=self.dt_max, t_end=self.t_end,
                       name=self.name + "[subset]", extra=dict(self.extra),
                       mlp=None if self.mlp is None else self.mlp.copy(), mlp_precision=self.mlp_precision,
                       poly=None if self.poly is None else self.poly[idx].copy(), splitting=self.splitting,
                       corr=None if self.corr is None else self.corr[idx].copy())

    def with_(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


def _par_row(kg, g, kb, b, gamma=0.0, kg2=0.0, g2=0.0, Eg=0.0, Eb=0.0,
             T0=T_HOT, T1=T_COLD, t_ramp=T_RAMP, Eg2=None, kd=0.0, d=1.0) -> np.ndarray:
    r = np.zeros(NPAR)
    r[P_KG], r[P_G], r[P_KB], r[P_B], r[P_GAMMA] = kg, g, kb, b, gamma
    r[P_KG2], r[P_G2], r[P_EG], r[P_EB] = kg2, g2, Eg, Eb
    r[P_T0], r[P_T1], r[P_TRAMP] = T0, T1, t_ramp
    r[P_EG2] = Eg if Eg2 is None else Eg2
    r[P_KD], r[P_D] = kd, d
    return r


def draw_kinetics(rng: SplitMix64, with_gamma: bool):
    """Draw (kg, g, kb, b, gamma) in the ranges of the single-simulation workload."""
    kg = rng.log_uniform(1e-7, 1e-6)
    g = rng.uniform_range(1.0, 2.0)
    kb = rng.log_uniform(1e8, 1e10)
    b = rng.uniform_range(1.0, 3.0)
    gamma = rng.uniform_range(0.0, 2e-3) if with_gamma else 0.0
    return kg, g, kb, b, gamma


def uniform_samples(n: int, t_end: float = T_END) -> np.ndarray:
    return np.array([t_end * (k + 1) / n for k in range(n)], dtype=np.float64)


SEED_BASE = 241100742


def single_sim(variant: str = "drawn", n: int = 200, t_end: float = T_END,
               n_samples: int = 20) -> Problem:
    """One 1D simulation: 200 cells on [0, 1000] um, Gaussian seed 200 +- 30 um, 1e9 #/m^3.

    variant "drawn": kinetics drawn from the seeded generator;
    variant "mid":   kg = 3e-7 m/s, g = 1.5, kb = 1e9 #/m^3/s, b = 2.
    """
    rng = SplitMix64(SEED_BASE + 0)
    if variant == "mid":
        kg, g, kb, b, gamma = 3e-7, 1.5, 1e9, 2.0, 0.0
    else:
        kg, g, kb, b, gamma = draw_kinetics(rng, with_gamma=False)
    L_max = 1000.0
    f0 = gaussian_seed_1d(n, L_max, 200.0, 30.0, 1e9)
    return Problem(ndim=1, n_cells=np.array([n], dtype=np.int32), L_max=np.array([L_max]),
                   f0=f0, C0=np.array([csat_linear(T_HOT)]),
                   par=_par_row(kg, g, kb, b, gamma, t_ramp=T_RAMP)[None, :],
                   t_samples=uniform_samples(n_samples, t_end), t_end=t_end,
                   name=f"single-{variant}-N{n}")


def batched(n_sims: int = 4096, n_lo: int = 200, n_hi: int = 2000, t_end: float = T_END,
            n_samples: int = 20, seed_offset: int = 1) -> Problem:
    """Many independent 1D simulations with uneven grids and per-sim kinetics.

    N ~ U{n_lo..n_hi} on [0, 1000] um; kinetics as the single simulation plus
    size-dependent growth gamma ~ U[0, 2e-3] 1/um; Gaussian seed 200 +- 30 um.
    """
    rng = SplitMix64(SEED_BASE + seed_offset)
    ns, pars, seeds = [], [], []
    for _ in range(n_sims):
        kg, g, kb, b, gamma = draw_kinetics(rng, with_gamma=True)
        n = rng.randint(n_lo, n_hi)
        ns.append(n)
        pars.append(_par_row(kg, g, kb, b, gamma))
        seeds.append(gaussian_seed_1d(n, 1000.0, 200.0, 30.0, 1e9))
    return Problem(ndim=1, n_cells=np.array(ns, dtype=np.int32), L_max=np.full(n_sims, 1000.0),
                   f0=np.concatenate(seeds), C0=np.full(n_sims, csat_linear(T_HOT)),
                   par=np.array(pars), t_samples=uniform_samples(n_samples, t_end), t_end=t_end,
                   name=f"batched-{n_sims}x[{n_lo},{n_hi}]")


def shape_2d(n_sims: int = 64, n_lo: int = 256, n_hi: int = 1024, t_end: float = T_END,
             n_samples: int = 20, seed_offset: int = 2, square: bool = True) -> Problem:
    """2D length x width simulations on [0,1200] x [0,600] um (Table 1 domain and seed).

    n ~ U{n_lo..n_hi}; grids n x n (or independent n1, n2 when square=False);
    bivariate Gaussian seed (400, 250) +- (30, 30) um, correlation ~ U[0, 0.5],
    total 1e9 #/m^3; per-axis (kg_m, g_m) and (kb, b) from the 1D ranges.
    """
    rng = SplitMix64(SEED_BASE + seed_offset)
    ncs, pars, seeds = [], [], []
    for _ in range(n_sims):
        kg1 = rng.log_uniform(1e-7, 1e-6)
        g1 = rng.uniform_range(1.0, 2.0)
        kg2 = rng.log_uniform(1e-7, 1e-6)
        g2 = rng.uniform_range(1.0, 2.0)
        kb = rng.log_uniform(1e8, 1e10)
        b = rng.uniform_range(1.0, 3.0)
        rho = rng.uniform_range(0.0, 0.5)
        n1 = rng.randint(n_lo, n_hi)
        n2 = n1 if square else rng.randint(n_lo, n_hi)
        ncs.append((n1, n2))
        pars.append(_par_row(kg1, g1, kb, b, 0.0, kg2, g2))
        seeds.append(gaussian_seed_2d(n1, n2, 1200.0, 600.0, (400.0, 250.0), (30.0, 30.0), rho, 1e9).ravel())
    return Problem(ndim=2, n_cells=np.array(ncs, dtype=np.int32), L_max=np.tile([1200.0, 600.0], (n_sims, 1)),
                   f0=np.concatenate(seeds), C0=np.full(n_sims, csat_linear(T_HOT)), par=np.array(pars),
                   t_samples=uniform_samples(n_samples, t_end), t_end=t_end,
                   name=f"shape2d-{n_sims}x[{n_lo},{n_hi}]^2")


def estimation(n_sims: int = 1024, n: int = 1000, t_end: float = T_END, n_samples: int = 20,
               seed_offset: int = 3, spread: float = 0.3):
    """Parameter-estimation workload: truth kinetics and perturbed starting guesses.

    Returns (problem_at_guess, truth_par, noise) where noise[S, n_samples, 5]
    are standard normals for 2% multiplicative measurement noise on the four
    moments and C, and the guesses are truth * exp(spread*u), u ~ U[-1, 1].
    """
    rng = SplitMix64(SEED_BASE + seed_offset)
    truth, guess = [], []
    for _ in range(n_sims):
        kg, g, kb, b, _ = draw_kinetics(rng, with_gamma=False)
        truth.append(_par_row(kg, g, kb, b))
        u = [rng.uniform_range(-1.0, 1.0) for _ in range(4)]
        guess.append(_par_row(kg * math.exp(spread * u[0]), g * math.exp(spread * u[1]),
                              kb * math.exp(spread * u[2]), b * math.exp(spread * u[3])))
    noise = np.array([[[rng.normal() for _ in range(5)] for _ in range(n_samples)] for _ in range(n_sims)])
    f0 = gaussian_seed_1d(n, 1000.0, 200.0, 30.0, 1e9)
    prob = Problem(ndim=1, n_cells=np.full(n_sims, n, dtype=np.int32), L_max=np.full(n_sims, 1000.0),
                   f0=np.tile(f0, n_sims), C0=np.full(n_sims, csat_linear(T_HOT)), par=np.array(guess),
                   t_samples=uniform_samples(n_samples, t_end), t_end=t_end,
                   name=f"estimation-{n_sims}xN{n}")
    return prob, np.array(truth), noise


# closure network blob: W1[64][3] b1[64] W2[64][64] b2[64] W3[2][64] b3[2], then
# in_shift[3] in_scale[3] out_shift[2] out_scale[2] lo[3] hi[3] s_min lnG0_max
MLP_H = 64
MLP_NW = 4546
MLP_NC = 18
MLP_C_LNG0_MAX = MLP_NW + 17
MLP_NBLOB = MLP_NW + MLP_NC
MLP_BF16, MLP_FP64 = 0, 1
MLP_OFF = dict(W1=0, b1=192, W2=256, b2=4352, W3=4416, b3=4544)


def closure_consts(in_shift=(0.1, 30.0, 14.0), in_scale=(10.0, 0.1, 1.0), out_shift=(-4.0, 17.0),
                   out_scale=(2.0, 2.0), lo=(0.0, -10.0, 6.0), hi=(2.0, 80.0, 22.0), s_min=1e-8,
                   lnG0_max=-0.7) -> np.ndarray:
    """Normalisation and validity box of the closure inputs (S, T degC, log10 mu_2), and the
    largest growth rate the network may return (ln G0 is held at lnG0_max above it).

    Defaults fit the closure workload: S up to ~0.3, T in 15..40 degC, mu_2 of
    the seed ~4e13 um^2/m^3 growing to ~1e15; ln G0 ~ -4 (G0 ~ 0.02 um/s, capped
    at ~0.5 um/s) and ln B ~ 17 (B ~ 2e7 #/(m^3 s)).
    """
    return np.array(list(in_shift) + list(in_scale) + list(out_shift) + list(out_scale) + list(lo) + list(hi)
                    + [s_min, lnG0_max], dtype=np.float32)


def closure_net(seed_offset: int = 5, out_gain: float = 0.1, consts=None) -> np.ndarray:
    """Initial closure weights: Glorot-uniform matrices from the seeded generator
    (the output layer scaled by out_gain), zero biases, then the constants."""
    rng = SplitMix64(SEED_BASE + seed_offset)
    w = np.zeros(MLP_NBLOB, dtype=np.float32)

    def glorot(n_out, n_in, gain=1.0):
        a = gain * math.sqrt(6.0 / (n_in + n_out))
        return np.array([rng.uniform_range(-a, a) for _ in range(n_out * n_in)], dtype=np.float32)

    o = MLP_OFF
    w[o["W1"]:o["W1"] + 192] = glorot(64, 3)
    w[o["W2"]:o["W2"] + 4096] = glorot(64, 64)
    w[o["W3"]:o["W3"] + 128] = glorot(2, 64, out_gain)
    w[MLP_NW:] = closure_consts() if consts is None else consts
    return w


def closure(n_sims: int = 4096, n: int = 500, t_end: float = T_END, n_samples: int = 20,
            seed_offset: int = 4):
    """Learned-closure workload: one shared ground-truth law, varied operating conditions.

    Ground truth: power law times an Arrhenius temperature factor (the form of
    App. A, Eq. A.2), which the plain four-parameter power law cannot express.
    Per sim: C0 = Csat(40)*(1 + U[0, 0.1]), final temperature T1 ~ U[15, 25],
    seed mean ~ U[150, 250] um.  Returns (problem_with_truth_law, split) where
    split[s] is True for training sims (80%) and False for held-out ones.
    """
    rng = SplitMix64(SEED_BASE + seed_offset)
    Eg, Eb = 4000.0, 6000.0
    Tref = 30.0 + 273.15
    kg = 4e-7 * math.exp(Eg / Tref)
    kb = 2e9 * math.exp(Eb / Tref)
    pars, seeds, C0, split = [], [], [], []
    for _ in range(n_sims):
        c_rel = rng.uniform_range(0.0, 0.1)
        T1 = rng.uniform_range(15.0, 25.0)
        mean = rng.uniform_range(150.0, 250.0)
        split.append(rng.uniform() < 0.8)
        pars.append(_par_row(kg, 1.5, kb, 2.0, 0.0, Eg=Eg, Eb=Eb, T1=T1))
        seeds.append(gaussian_seed_1d(n, 1000.0, mean, 30.0, 1e9))
        C0.append(csat_linear(T_HOT) * (1.0 + c_rel))
    prob = Problem(ndim=1, n_cells=np.full(n_sims, n, dtype=np.int32), L_max=np.full(n_sims, 1000.0),
                   f0=np.concatenate(seeds), C0=np.array(C0), par=np.array(pars),
                   t_samples=uniform_samples(n_samples, t_end), t_end=t_end, law=LAW_ARRHENIUS,
                   name=f"closure-{n_sims}xN{n}")
    return prob, np.array(split)


def random_tiny(seed: int, n: int, t_end: float = 50.0, n_samples: int = 5, gamma: bool = True) -> Problem:
    """A small randomized single simulation for brute-force style checks."""
    rng = SplitMix64(SEED_BASE + 1000 + seed)
    kg, g, kb, b, gm = draw_kinetics(rng, with_gamma=gamma)
    mean = rng.uniform_range(0.3, 0.6) * 1000.0
    f0 = gaussian_seed_1d(n, 1000.0, mean, 60.0, 1e9)
    C0 = csat_linear(T_HOT) * (1.0 + rng.uniform_range(0.02, 0.1))
    return Problem(ndim=1, n_cells=np.array([n], dtype=np.int32), L_max=np.array([1000.0]), f0=f0,
                   C0=np.array([C0]), par=_par_row(kg, g, kb, b, gm)[None, :],
                   t_samples=uniform_samples(n_samples, t_end), t_end=t_end, name=f"tiny-{seed}-N{n}")


def cfl_limited(n_sims: int = 24, n_lo: int = 4, n_hi: int = 2048, t_end: float = 600.0, n_samples: int = 5,
                seed_offset: int = 6, dt_max: float = 60.0, sizes=None) -> Problem:
    """Simulations whose steps are set by the CFL bound rather than by dt_max.

    High initial supersaturation (C0 = Csat(40)*(1 + U[0.15, 0.3])), fast growth
    (kg ~ log-U[3e-7, 1e-6] m/s), size-dependent growth gamma ~ U[0, 2e-3] 1/um, a
    large step cap dt_max and a cooling ramp of U[0.3, 1.0]*t_end, so that the
    step size, and with it the time reached and the temperature, depend on the
    rates.  Sample times are irregular (uniform draws, sorted, the last at t_end)
    so they are not multiples of any step.  Grid sizes N ~ U{n_lo..n_hi} unless
    `sizes` is given.
    """
    rng = SplitMix64(SEED_BASE + seed_offset)
    ns_, pars, seeds, C0 = [], [], [], []
    for i in range(n_sims):
        kg = rng.log_uniform(3e-7, 1e-6)
        g = rng.uniform_range(1.0, 2.0)
        kb = rng.log_uniform(1e8, 1e10)
        b = rng.uniform_range(1.0, 3.0)
        gamma = rng.uniform_range(0.0, 2e-3)
        n = rng.randint(n_lo, n_hi) if sizes is None else int(sizes[i])
        c_rel = rng.uniform_range(0.15, 0.3)
        t_ramp = rng.uniform_range(0.3, 1.0) * t_end
        ns_.append(n)
        pars.append(_par_row(kg, g, kb, b, gamma, t_ramp=t_ramp))
        seeds.append(gaussian_seed_1d(n, 1000.0, 200.0, 30.0, 1e9))
        C0.append(csat_linear(T_HOT) * (1.0 + c_rel))
    ts = sorted(rng.uniform_range(0.05, 0.95) * t_end for _ in range(n_samples - 1)) + [t_end]
    return Problem(ndim=1, n_cells=np.array(ns_, dtype=np.int32), L_max=np.full(n_sims, 1000.0),
                   f0=np.concatenate(seeds), C0=np.array(C0), par=np.array(pars),
                   t_samples=np.array(ts, dtype=np.float64), t_end=t_end, dt_max=dt_max,
                   name=f"cfl-limited-{n_sims}x[{n_lo},{n_hi}]")


def dissolution(n_sims: int = 32, n_lo: int = 4, n_hi: int = 2048, t_end: float = 3000.0, n_samples: int = 6,
                seed_offset: int = 8, dt_max: float = 20.0, sizes=None, seed_kind: str = "lognormal") -> Problem:
    """Heating runs that grow and then dissolve: a slightly supersaturated start at 20 degC
    (C0 = Csat(20)(1 + U[0.02, 0.1])), heating to T1 ~ U[30, 45] degC over U[0.2, 0.6] t_end,
    growth kg ~ log-U[1e-7, 5e-7] m/s with nucleation, dissolution kd ~ log-U[5e-7, 5e-6] m/s
    with d ~ U[1, 1.5], gamma ~ U[0, 1e-3] 1/um.  Seeds (SI S1.3): `seed_kind` sample PSSDs with
    mean U[80, 300] um and sd U[15, 60] um scaled to a seed mass alpha mu_3 = U[1e-3, 8e-3] g/g,
    so that some runs dissolve every crystal and some only part.  Irregular sample times."""
    rng = SplitMix64(SEED_BASE + seed_offset)
    ns_, pars, seeds, C0 = [], [], [], []
    for i in range(n_sims):
        kg = rng.log_uniform(1e-7, 5e-7)
        g = rng.uniform_range(1.0, 2.0)
        kb = rng.log_uniform(1e8, 1e10)
        b = rng.uniform_range(1.0, 3.0)
        gamma = rng.uniform_range(0.0, 1e-3)
        kd = rng.log_uniform(5e-7, 5e-6)
        d = rng.uniform_range(1.0, 1.5)
        T1 = rng.uniform_range(30.0, 45.0)
        t_ramp = rng.uniform_range(0.2, 0.6) * t_end
        n = rng.randint(n_lo, n_hi) if sizes is None else int(sizes[i])
        mean = rng.uniform_range(80.0, 300.0)
        sd = rng.uniform_range(15.0, 60.0)
        m_seed = rng.uniform_range(1e-3, 8e-3)
        c_rel = rng.uniform_range(0.02, 0.1)
        ns_.append(n)
        pars.append(_par_row(kg, g, kb, b, gamma, T0=20.0, T1=T1, t_ramp=t_ramp, kd=kd, d=d))
        sample = seed_sample_1d(seed_kind, n, 1000.0, mean, sd)
        seeds.append(scale_to_seed_mass(sample, m_seed, ALPHA, 1000.0, n))
        C0.append(csat_linear(20.0) * (1.0 + c_rel))
    ts = sorted(rng.uniform_range(0.05, 0.95) * t_end for _ in range(n_samples - 1)) + [t_end]
    return Problem(ndim=1, n_cells=np.array(ns_, dtype=np.int32), L_max=np.full(n_sims, 1000.0),
                   f0=np.concatenate(seeds), C0=np.array(C0), par=np.array(pars),
                   t_samples=np.array(ts, dtype=np.float64), t_end=t_end, dt_max=dt_max,
                   name=f"dissolution-{n_sims}x[{n_lo},{n_hi}]")


def inloop(n_sims: int = 64, n_coarse: int = 50, refine: int = 16, t_end: float = 1800.0, n_samples: int = 8,
           seed_offset: int = 9, dt: float = 1800.0):
    """Coarse / fine pairs for the in-the-loop correction (Sec. 4.2, Fig. 5b): the same simulations
    on n_coarse cells and on refine * n_coarse cells of [0, 1000] um.  Each grid takes its own
    CFL-limited steps (nu = 0.5; dt, the cap, is the whole horizon by default), so the fine solve
    takes about `refine` times as many steps as the coarse one, as in the paper's coarse / fine
    comparison; with a small dt both grids share one step size and the coarse grid's error is the
    spatial discretisation error alone.  Growth kg ~ log-U[4e-7, 1.5e-6]
    m/s, g ~ U[1, 2], nucleation kb ~ log-U[1e7, 1e9], gamma ~ U[0, 1e-3] 1/um, cooling 40 -> 20 degC
    over U[0.5, 1] t_end, seeds of mean U[100, 250] um and sd U[15, 40] um (normal or log-normal)
    scaled to alpha mu_3 = U[2e-3, 1e-2] g/g.  Returns (coarse, fine)."""
    rng = SplitMix64(SEED_BASE + seed_offset)
    nf = n_coarse * refine
    pars, fc, ff, C0 = [], [], [], []
    for i in range(n_sims):
        kg = rng.log_uniform(4e-7, 1.5e-6)
        g = rng.uniform_range(1.0, 2.0)
        kb = rng.log_uniform(1e7, 1e9)
        b = rng.uniform_range(1.0, 3.0)
        gamma = rng.uniform_range(0.0, 1e-3)
        t_ramp = rng.uniform_range(0.5, 1.0) * t_end
        mean, sd = rng.uniform_range(100.0, 250.0), rng.uniform_range(15.0, 40.0)
        kind = "lognormal" if rng.uniform() < 0.5 else "normal"
        m_seed = rng.uniform_range(2e-3, 1e-2)
        pars.append(_par_row(kg, g, kb, b, gamma, t_ramp=t_ramp))
        fine = scale_to_seed_mass(seed_sample_1d(kind, nf, 1000.0, mean, sd), m_seed, ALPHA, 1000.0, nf)
        ff.append(fine)
        fc.append(fine.reshape(n_coarse, refine).mean(axis=1))    # the same seed, cell-averaged
        C0.append(csat_linear(T_HOT) * 1.02)
    ts = uniform_samples(n_samples, t_end)
    common = dict(ndim=1, L_max=np.full(n_sims, 1000.0), C0=np.array(C0), par=np.array(pars), t_samples=ts,
                  t_end=t_end, dt_max=dt)
    coarse = Problem(n_cells=np.full(n_sims, n_coarse, dtype=np.int32), f0=np.concatenate(fc),
                     name=f"inloop-coarse-{n_sims}x{n_coarse}", **common)
    fine_p = Problem(n_cells=np.full(n_sims, nf, dtype=np.int32), f0=np.concatenate(ff),
                     name=f"inloop-fine-{n_sims}x{nf}", **common)
    return coarse, fine_p


# ---- the paper's own 2D case (Table 1 and App. A, Table A.1)
PAPER_RHO_C = 1.11e-12               # g/um^3, Table 1
PAPER_KV = math.pi / 4.0             # cylinder, Table 1


def paper_2d(n1: int = 1200, n2: int = 600, t_end: float = 1000.0, n_samples: int = 4) -> Problem:
    """The paper's seeded batch crystallization in length x width (Table 1, App. A).

    Growth only (no nucleation), constant temperature 15 degC, exponential
    solubility c* = 3.37 exp(0.036 T) g/kg, per-axis Arrhenius growth
    G_m = k_m1 exp(-k_m2/(T + 273.15)) (S - 1)^k_m3 with Table A.1's constants
    (k_11 = 8.86e6 um/min, k_12 = 2450 K, k_13 = 3.7; k_21 = 4.088e5 um/min,
    k_22 = 2400 K, k_23 = 2.5), c0 = 8 g/kg, a Gaussian seed (400, 250) +- (30, 30)
    um scaled to a seed mass of 1 g, domain 1200 x 600 um on n1 x n2 bins, the
    one-step limited scheme of Eq. (8) at Courant number 0.9 and no cap on the
    step.  Units of this problem: time in minutes (the rates are in um/min),
    concentration in g per kg of solvent, number density per um^2 and kg of
    solvent, so alpha = rho_c k_v.  The printed simulation time "1000 [hour]"
    is garbled; it is read as 1000 minutes (t_end).
    """
    L1, L2 = 1200.0, 600.0
    f = gaussian_seed_2d(n1, n2, L1, L2, (400.0, 250.0), (30.0, 30.0), 0.0, 1.0)
    d1, d2 = L1 / n1, L2 / n2
    x = (np.arange(n1) + 0.5) * d1
    y = (np.arange(n2) + 0.5) * d2
    mu12 = float((x[None, :] * (y ** 2)[:, None] * f).sum() * d1 * d2)
    f = f * (1.0 / (PAPER_RHO_C * PAPER_KV * mu12))   # seed mass rho_c k_v mu_12 = 1 g
    # kg in the solver's units (1e6 kg is the rate constant in um per time unit)
    par = _par_row(8.86e6 / 1e6, 3.7, 0.0, 1.0, 0.0, kg2=4.088e5 / 1e6, g2=2.5, Eg=2.45e3, Eb=0.0,
                   T0=15.0, T1=15.0, t_ramp=0.0, Eg2=2.4e3)
    return Problem(ndim=2, n_cells=np.array([[n1, n2]], dtype=np.int32), L_max=np.array([[L1, L2]]),
                   f0=np.ascontiguousarray(f.ravel()), C0=np.array([8.0]), par=par[None, :],
                   t_samples=uniform_samples(n_samples, t_end), t_end=t_end, law=LAW_ARRHENIUS, sol_law=SOL_EXP,
                   cs0=3.37, cs1=0.036, alpha=PAPER_RHO_C * PAPER_KV, scheme=SCHEME_LW_TVD, cfl=0.9, dt_max=t_end,
                   name=f"paper2d-{n1}x{n2}")

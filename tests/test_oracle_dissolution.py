"""Pins of the oracle's dissolution (S < 0: crystals shrink, the paper's growth/dissolution
rates of SI S1.1; the law mirrors the growth power law, G0 = -1e6 kd (1 - C/Csat)^d).

- the first step's rate is the law evaluated from the inputs by hand;
- mirror identity: dissolution at speed -G on f is bitwise growth at speed +G on the
  reversed array (gamma = 0, no nucleation; van Leer's psi is symmetric and odd);
- one step of the one-step scheme equals the mirror image of Eq. (8), derived here from
  the Lax-Wendroff flux for a negative speed, in exact rationals;
- constant dissolution converges to the seed shifted towards L = 0 at second order;
- a solution heated out of saturation dissolves every crystal: mu_0 -> 0 and the
  concentration gains back alpha mu_3(0) (Eq. (9) telescopes);
- the CFL step is nu dL / (|G0| (1 + gamma L_max)) while dissolving;
- with the seed away from L = 0 the FVM converges to the moment ODEs with dissolution.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W

TINY_F = [0.0, 1.0, 3.0, 7.0, 6.0, 2.0, 4.0, 5.0, 0.5, 0.0]


def dissolving_problem(n=200, L_max=1000.0, mean=500.0, sd=40.0, kd=1e-7, d=1.0, gamma=0.0, under=0.3,
                       t_end=4000.0, n_samples=4, dt_max=1e9, cfl=0.5, scheme=W.SCHEME_SSPRK3, alpha=0.0,
                       T0=20.0, T1=20.0, t_ramp=1.0, C0=None):
    """Isothermal undersaturated run; alpha = 0 keeps C (and so G0) constant."""
    par = W._par_row(1e-7, 1.0, 1e9, 2.0, gamma, T0=T0, T1=T1, t_ramp=t_ramp, kd=kd, d=d)
    f0 = W.gaussian_seed_1d(n, L_max, mean, sd, 1e9)
    C0 = W.csat_linear(T0) * (1.0 - under) if C0 is None else C0
    return W.Problem(ndim=1, n_cells=np.array([n], dtype=np.int32), L_max=np.array([L_max]), f0=f0,
                     C0=np.array([C0]), par=par[None, :], t_samples=W.uniform_samples(n_samples, t_end),
                     t_end=t_end, dt_max=dt_max, cfl=cfl, scheme=scheme, alpha=alpha)


def test_rate_law_of_the_first_step(oracle):
    for d in (1.0, 1.7):
        p = dissolving_problem(kd=3e-7, d=d, under=0.2, n=50, t_end=10.0, n_samples=1)
        r = oracle.solve1d(p, 0, max_steps=1)
        Csat = W.csat_linear(20.0)
        under = 1.0 - p.C0[0] / Csat
        assert abs(r["G0"][0] - (-1e6 * 3e-7 * under ** d)) <= 1e-14 * abs(r["G0"][0])
        assert r["B"][0] == 0.0
    # kd = 0: nothing happens in an undersaturated solution
    p = dissolving_problem(kd=0.0, n=50, t_end=10.0, n_samples=1)
    r = oracle.solve1d(p, 0)
    assert np.all(r["G0"][: r["steps"]] == 0.0)
    np.testing.assert_allclose(r["f_final"], p.f0, rtol=1e-15)   # only the stage combination's rounding


@pytest.mark.parametrize("scheme", [W.SCHEME_SSPRK3, W.SCHEME_LW_TVD])
def test_mirror_of_growth_is_bitwise(oracle, scheme):
    n, steps = 64, 40
    rng = np.random.default_rng(3)
    f0 = np.abs(rng.normal(size=n)) * (rng.uniform(size=n) > 0.2)
    dt = np.full(steps, 0.7)
    G = 0.9 * np.linspace(0.5, 1.0, steps)                     # dt G / dL <= 0.63 with dL = 1
    base = dissolving_problem(n=n, L_max=float(n), mean=n / 2, sd=n / 8, n_samples=1, t_end=1e6, scheme=scheme)
    shrink = base.with_(f0=f0.copy())
    grow = base.with_(f0=f0[::-1].copy())
    rs = oracle.solve1d(shrink, 0, max_steps=steps, dt_replay=dt, rates_replay=(-G, np.zeros(steps)))
    rg = oracle.solve1d(grow, 0, max_steps=steps, dt_replay=dt, rates_replay=(G, np.zeros(steps)))
    assert rs["steps"] == rg["steps"] == steps
    np.testing.assert_array_equal(rs["f_final"], rg["f_final"][::-1])
    assert rs["outflow"] == 0.0 and rg["outflow"] > 0.0       # growth loses at L_max what dissolution loses at 0


def mirrored_correction(fi, fp1, fp2):
    """phi(theta_{i+1/2}) * (f_{i+1} - f_i) with the smoothness taken on the upwind (right) side,
    theta = (f_{i+2} - f_{i+1}) / (f_{i+1} - f_i) (SI Eqs. (S1)-(S2) for a negative speed)."""
    den = fp1 - fi
    if den == 0:
        return Fr(0)
    th = (fp2 - fp1) / den
    return (th + abs(th)) / (1 + abs(th)) * den


@pytest.mark.parametrize("steps", [1, 3])
def test_one_step_scheme_mirrors_eq8_exact(oracle, steps):
    """For a speed a < 0 the Lax-Wendroff flux is a f_{i+1} - (a/2)(1 - nu)(f_{i+1} - f_i) with
    nu = |a| dt/dL; limiting the correction gives
    f_i' = f_i + nu (f_{i+1} - f_i) - nu (1 - nu)/2 [phi_{i+1/2} D_{i+1/2} - phi_{i-1/2} D_{i-1/2}]."""
    n = len(TINY_F)
    p = dissolving_problem(n=n, L_max=float(n), mean=n / 2, sd=n / 8, kd=4e-7, under=0.5, t_end=50.0, n_samples=1,
                           dt_max=1.0, cfl=0.45, scheme=W.SCHEME_LW_TVD)
    p.f0 = np.array(TINY_F)
    r = oracle.solve1d(p, 0, max_steps=steps)
    assert np.all(r["G0"][:steps] < 0.0)
    f = [Fr(x) for x in p.f0]
    for k in range(steps):
        nu = -Fr(r["G0"][k]) * Fr(r["dt"][k])
        assert 0 < nu <= Fr(1, 2)
        ext = lambda i: Fr(0) if (i < 0 or i >= n) else f[i]
        new = []
        for i in range(n):
            cp = mirrored_correction(ext(i), ext(i + 1), ext(i + 2))     # face i+1/2
            cm = mirrored_correction(ext(i - 1), ext(i), ext(i + 1))     # face i-1/2
            new.append(ext(i) + nu * (ext(i + 1) - ext(i)) - Fr(1, 2) * nu * (1 - nu) * (cp - cm))
        f = new
    scale = max(abs(x) for x in f)
    for i in range(n):
        assert abs(Fr(r["f_final"][i]) - f[i]) <= scale * Fr(1, 2 ** 48), i


def test_constant_dissolution_converges_to_shifted_seed(oracle):
    """f(L, t) = f0(L + |G| t): the L1 error falls at second order on a smooth seed."""
    errs = []
    for n in (100, 200, 400, 800):
        p = dissolving_problem(n=n, mean=600.0, t_end=3000.0)
        r = oracle.solve1d(p, 0)
        shift = r["G0"][0] * p.t_end
        assert shift < -80.0
        exact = W.gaussian_seed_1d(n, 1000.0, 600.0 + shift, 40.0, 1e9)
        errs.append(np.abs(r["f_final"] - exact).sum() / np.abs(exact).sum())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] >= 1.5, (errs, orders)


def test_heating_dissolves_everything_and_returns_the_mass(oracle):
    """Heated 20 -> 40 degC: growth stops, the crystals dissolve through L = 0, mu_0 -> 0, and
    C ends at C0 + alpha mu_3(0) with C + alpha mu_3 constant all along (Eq. (9))."""
    n, L_max = 400, 400.0
    f0 = W.gaussian_seed_1d(n, L_max, 120.0, 20.0, 1e9)     # alpha mu_3 = 1.5e-3 g/g: all of it fits in solution
    par = W._par_row(2e-8, 1.0, 0.0, 2.0, 0.0, T0=20.0, T1=40.0, t_ramp=600.0, kd=2e-6, d=1.0)
    C0 = W.csat_linear(20.0) * 1.01
    p = W.Problem(ndim=1, n_cells=np.array([n], dtype=np.int32), L_max=np.array([L_max]), f0=f0,
                  C0=np.array([C0]), par=par[None, :], t_samples=np.array([300.0, 1500.0, 6000.0]), t_end=6000.0,
                  dt_max=5.0, cfl=0.5)
    r = oracle.solve1d(p, 0, record_f=True, log_steps=5000)
    dL = L_max / n
    L = (np.arange(n) + 0.5) * dL
    mu3_0 = (L ** 3 * f0).sum() * dL
    assert np.any(r["G0"][: r["steps"]] > 0.0) and np.any(r["G0"][: r["steps"]] < 0.0)
    mass = r["C"] + W.ALPHA * r["mom"][:, 3]
    np.testing.assert_allclose(mass, C0 + W.ALPHA * mu3_0, rtol=1e-13)
    assert r["mom"][-1, 0] < 1e-9 * f0.sum() * dL
    assert abs(r["C"][-1] - (C0 + W.ALPHA * mu3_0)) < 1e-9 * r["C"][-1]


def test_cfl_step_while_dissolving(oracle):
    nu, gamma, n, L_max = 0.45, 1.5e-3, 100, 1000.0
    p = dissolving_problem(n=n, L_max=L_max, kd=5e-7, gamma=gamma, cfl=nu, t_end=800.0, n_samples=2)
    r = oracle.solve1d(p, 0)
    G0 = r["G0"][0]
    assert G0 < 0.0 and np.all(r["G0"][: r["steps"]] == G0)
    dL = L_max / n
    vmax = max(abs(G0) * (1.0 + gamma * j * dL) for j in range(n + 1))
    dts = r["dt"][: r["steps"]]
    cfl = dts[np.abs(dts * vmax / dL - nu) < 1e-12]
    assert cfl.size >= r["steps"] - 2
    np.testing.assert_allclose(cfl, nu * dL / vmax, rtol=1e-15)


def test_fvm_converges_to_moment_odes_under_dissolution(oracle):
    """Partial dissolution by heating, seed far from L = 0: mu_1..mu_3 and C of the FVM approach
    the method-of-moments solution (SI Eq. (S4) with G0 < 0) as dL and dt shrink together."""
    errs = []
    for n in (100, 200, 400):
        f0 = W.gaussian_seed_1d(n, 1000.0, 500.0, 40.0, 1e9)
        par = W._par_row(1e-7, 1.0, 0.0, 2.0, 1e-3, T0=20.0, T1=35.0, t_ramp=1800.0, kd=1e-7, d=1.3)
        p = W.Problem(ndim=1, n_cells=np.array([n], dtype=np.int32), L_max=np.array([1000.0]), f0=f0,
                      C0=np.array([W.csat_linear(20.0) * 1.02]), par=par[None, :],
                      t_samples=np.array([900.0, 1800.0, 3600.0]), t_end=3600.0, dt_max=400.0 / n, cfl=0.5)
        r = oracle.solve1d(p, 0)
        dL = 1000.0 / n
        L = (np.arange(n) + 0.5) * dL
        mu_init = np.array([(L ** k * f0).sum() * dL for k in range(4)])
        mu, C = oracle.mom1d(p, 0, mu_init)
        assert C[-1] > p.C0[0]                        # the solute was given back
        errs.append(max(np.max(np.abs(r["mom"][:, 1:] - mu[:, 1:]) / np.abs(mu[:, 1:])),
                        np.max(np.abs(r["C"] - C) / C)))
    assert errs[-1] < 1e-4
    assert math.log2(errs[-2] / errs[-1]) >= 0.8, errs

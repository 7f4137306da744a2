"""Pins of the oracle's polynomial growth law (Sec. 4.1, Eq. (poly_growth_rate)):
G0 = a_1 S + ... + a_k S^k with S = C/Csat - 1.

- a law with a single non-zero coefficient a_j is the power law with exponent j
  and kg = a_j / 1e6 (the power law's kg is in m/s, the coefficients in um/s);
- the forward-mode tangent along a coefficient direction agrees with central
  differences of the solve, also where the CFL limit sets the step;
- forward mode is linear in the direction: the tangent along v1 + v2 is the sum
  of the tangents (to rounding).
"""
import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W


def poly_problem(coeffs, n=160, t_end=600.0, n_samples=4, dt_max=1.0, C0_rel=1.15):
    p = W.single_sim("mid", n=n, t_end=t_end, n_samples=n_samples)
    p = p.with_(law=W.LAW_POLY, poly=np.array([coeffs], dtype=np.float64), dt_max=dt_max, C0=p.C0.copy(),
                par=p.par.copy())
    p.C0[:] = W.csat_linear(40.0) * C0_rel
    return p


@pytest.mark.parametrize("j", [1, 2, 3])
def test_single_term_is_the_power_law(oracle, j):
    a = 0.4 * 10.0 ** (j - 1)
    coeffs = [0.0] * (j - 1) + [a]
    p = poly_problem(coeffs)
    q = p.with_(law=W.LAW_POWER, poly=None, par=p.par.copy())
    q.par[0, W.P_KG] = a / 1e6
    q.par[0, W.P_G] = float(j)
    rp, rq = oracle.solve1d(p, 0), oracle.solve1d(q, 0)
    assert rp["steps"] == rq["steps"]
    np.testing.assert_allclose(rp["mom"], rq["mom"], rtol=1e-12)
    np.testing.assert_allclose(rp["C"], rq["C"], rtol=1e-13)
    assert np.max(np.abs(rp["f_final"] - rq["f_final"])) <= 1e-12 * np.max(np.abs(rq["f_final"]))


@pytest.mark.parametrize("cfl_limited", [False, True])
def test_tangent_matches_central_differences(oracle, cfl_limited):
    coeffs = [0.3, 0.8, 1.5, 2.0]
    if cfl_limited:
        p = poly_problem(coeffs, n=200, dt_max=40.0, C0_rel=1.3)
    else:
        p = poly_problem(coeffs)
    base = oracle.solve1d(p, 0, record_f=True)
    if cfl_limited:
        assert np.sum(base["dt"] < p.dt_max * (1 - 1e-12)) > 0.8 * base["steps"]
    rng = np.random.default_rng(4)
    v = rng.normal(size=len(coeffs))
    tan = oracle.tangent1d_poly(p, 0, v)
    h = 1e-6
    outs = []
    for sg in (1, -1):
        q = p.with_(poly=p.poly + sg * h * v[None, :])
        o = oracle.solve1d(q, 0, record_f=True)
        assert o["steps"] == base["steps"]
        outs.append(o)
    eps = np.finfo(float).eps
    for key, tkey in [("mom", "dM"), ("C", "dC"), ("f_samples", "dF")]:
        want = (outs[0][key] - outs[1][key]) / (2 * h)
        noise = 1e3 * eps * np.max(np.abs(base[key])) / h
        tol = 1e-5 * np.max(np.abs(want)) + noise
        got = tan[tkey][..., 0]
        assert np.max(np.abs(got - want)) <= tol, (key, np.max(np.abs(got - want)), tol)


def test_tangent_is_linear_in_the_direction(oracle):
    p = poly_problem([0.3, 0.8, 1.5], dt_max=40.0, C0_rel=1.3, n=120)
    rng = np.random.default_rng(7)
    v1, v2 = rng.normal(size=3), rng.normal(size=3)
    t1, t2, t12 = (oracle.tangent1d_poly(p, 0, v)["dM"][..., 0] for v in (v1, v2, v1 + v2))
    np.testing.assert_allclose(t12, t1 + t2, rtol=1e-9, atol=1e-12 * np.max(np.abs(t12)))

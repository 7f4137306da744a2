"""Pins of the oracle's Strang splitting of the 2D step (Sec. 2.1 names Godunov's dimensional
splitting; Strang's symmetric form is the second-order variant): L1 over dt/2, L2 over dt,
L1 over dt/2.

- one step equals that composition of exact-rational SSP-RK3 line sweeps (each rounded to
  double before the next), and differs from the Godunov (L1 then L2) step;
- the corner source still adds exactly B dt to mu_00 per step (its L1 share enters in two
  halves) and C + alpha mu_{1,2} is constant;
- the solution converges to the 2D method of moments (SI Eq. (S4)) as dL and dt shrink;
- the Strang and Godunov solutions agree to first order in dt on a fixed grid.
"""
import math
from fractions import Fraction as Fr

import numpy as np

from paper_2411_00742_amd import workloads as W
from test_oracle_pins import exact_ssprk3_line, shape_problem


def test_strang_step_is_half_rows_cols_half_rows_exact(oracle):
    n1, n2 = 5, 4
    T, S = 20.0, 0.25
    kg1, g1, kg2, g2, kb, b = 3e-7, 1.0, 2e-7, 1.0, 4e8, 2.0
    par = W._par_row(kg1, g1, kb, b, 0.0, kg2, g2, T0=T, T1=T, t_ramp=1.0)
    f0 = np.array([[0, 1, 3, 2, 0], [1, 4, 6, 3, 1], [0, 2, 5, 4, 2], [0, 0, 1, 2, 1]], dtype=np.float64)
    p = W.Problem(ndim=2, n_cells=np.array([[n1, n2]], dtype=np.int32), L_max=np.array([[5.0, 4.0]]),
                  f0=f0.ravel(), C0=np.array([W.csat_linear(T) * (1 + S)]), par=par[None, :],
                  t_samples=np.array([50.0]), t_end=50.0, alpha=0.0, dt_max=1.0, cfl=0.45,
                  splitting=W.SPLIT_STRANG)
    r = oracle.solve2d(p, 0, max_steps=1)
    Sx = p.C0[0] / W.csat_linear(T) - 1.0
    G1, G2, B = Fr(1e6 * kg1 * Sx ** g1), Fr(1e6 * kg2 * Sx ** g2), Fr(kb * Sx ** b)
    dt = Fr(r["dt"][0])

    # each sweep is exact; its result is rounded to the nearest double before the next one
    # (exact rationals through three sweeps grow too long to evaluate in reasonable time), so
    # the composition is held to a few ulps per sweep
    rnd = lambda x: Fr(float(x))

    def rows(f, h):
        return [[rnd(x) for x in exact_ssprk3_line(f[j], G1, 0.0, B / (2 * G1) if j == 0 else Fr(0), h)[0]]
                for j in range(n2)]

    def cols(f, h):
        c = [exact_ssprk3_line([f[j][i] for j in range(n2)], G2, 0.0, B / (2 * G2) if i == 0 else Fr(0), h)[0]
             for i in range(n1)]
        return [[rnd(c[i][j]) for i in range(n1)] for j in range(n2)]

    f = [[Fr(x) for x in row] for row in f0]
    want = rows(cols(rows(f, dt / 2), dt), dt / 2)
    lie = cols(rows(f, dt), dt)
    got = r["f_final"]
    scale = max(abs(x) for row in want for x in row)
    err = max(abs(Fr(got[j, i]) - want[j][i]) for j in range(n2) for i in range(n1))
    assert err <= scale * Fr(1, 2 ** 44), float(err / scale)
    diff = max(abs(lie[j][i] - want[j][i]) for j in range(n2) for i in range(n1))
    assert diff > scale * Fr(1, 10 ** 6), float(diff / scale)


def test_strang_number_and_mass_balances(oracle):
    p = shape_problem(40, 40, 3e-7, 2e-7, kb=6e8, t_end=900.0).with_(splitting=W.SPLIT_STRANG)
    r = oracle.solve2d(p, 0)
    dA = (1200.0 / 40) * (600.0 / 40)
    B = 6e8 * (p.C0[0] / W.csat_linear(20.0) - 1.0) ** 2.0
    np.testing.assert_allclose(r["mom"][:, 0], p.f0.sum() * dA + B * p.t_samples, rtol=1e-11)
    q = W.shape_2d(n_sims=1, n_lo=60, n_hi=60, t_end=1200.0, n_samples=4).with_(splitting=W.SPLIT_STRANG)
    rq = oracle.solve2d(q, 0)
    f0 = q.f0_of(0)
    d1, d2 = 1200.0 / 60, 600.0 / 60
    L1 = (np.arange(60) + 0.5) * d1
    L2 = (np.arange(60) + 0.5) * d2
    mu12_0 = (L1[None, :] * (L2 ** 2)[:, None] * f0).sum() * d1 * d2
    np.testing.assert_allclose(rq["C"] + q.alpha * rq["mom"][:, 3], q.C0[0] + q.alpha * mu12_0, rtol=1e-12)


def test_strang_converges_to_mom(oracle):
    errs = []
    for n in (32, 64, 128):
        p = shape_problem(n, n, 3e-7, 2e-7, kb=2e8, alpha=W.ALPHA, T=25.0, S=0.3, t_end=1500.0, n_samples=3)
        p = p.with_(dt_max=40.0 / n, splitting=W.SPLIT_STRANG)
        r = oracle.solve2d(p, 0)
        f0 = p.f0_of(0)
        d1, d2 = 1200.0 / n, 600.0 / n
        L1 = (np.arange(n) + 0.5) * d1
        L2 = (np.arange(n) + 0.5) * d2
        mom = lambda a, b: ((L1 ** a)[None, :] * (L2 ** b)[:, None] * f0).sum() * d1 * d2
        mu_i = np.array([mom(0, 0), mom(1, 0), mom(0, 1), mom(1, 1), mom(0, 2), mom(1, 2)])
        mu, Cq = oracle.mom2d(p, 0, mu_i)
        errs.append(max(np.max(np.abs(r["mom"][:, 3] - mu[:, 5]) / mu[:, 5]),
                        np.max(np.abs(r["C"] - Cq) / Cq) * 10))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 0.8, (errs, orders)


def test_strang_and_godunov_agree_to_first_order_in_dt(oracle):
    diffs = []
    for dt_max in (8.0, 4.0, 2.0):
        p = shape_problem(48, 48, 4e-7, 3e-7, kb=3e8, t_end=400.0, S=0.5).with_(dt_max=dt_max, cfl=0.9)
        a = oracle.solve2d(p, 0)["f_final"]
        b = oracle.solve2d(p.with_(splitting=W.SPLIT_STRANG), 0)["f_final"]
        diffs.append(np.max(np.abs(a - b)) / np.max(np.abs(a)))
    assert diffs[-1] > 0.0
    assert all(math.log2(diffs[i] / diffs[i + 1]) >= 0.8 for i in range(2)), diffs

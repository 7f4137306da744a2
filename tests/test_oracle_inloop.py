"""Pins of the oracle's in-the-loop correction (Sec. 4.2, Fig. 5b): after each growth step a
small network adds a correction flux Y at every interior face, f_i += Y_{i-1/2} - Y_{i+1/2}.

- a zero output layer leaves the solver's result bitwise unchanged;
- one corrected step differs from the plain step by exactly the flux difference of the
  network evaluated with torch's float64 linear and tanh layers on the windows of the plain
  step's result (cells outside the domain read 0, boundary faces uncorrected);
- the correction moves nothing across the domain's ends: mu_0 stays constant without
  nucleation or outflow, for any weights;
- the corrected solver is homogeneous of degree one in f when the rates do not depend on it
  and nothing is born (alpha = 0, kb = 0): doubling the seed doubles every output bitwise
  (sigma carries the scale);
- the forward-mode tangent along a weight direction equals central differences.
"""
import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W


def corr_problem(n=40, seed=0, scale=0.3, t_end=200.0, alpha=None, kb=None):
    c, _ = W.inloop(n_sims=1, n_coarse=n, refine=2, t_end=t_end, n_samples=4, seed_offset=40 + seed)
    rng = np.random.default_rng(seed)
    w = rng.normal(scale=scale, size=(1, W.CORR_NW))
    kw = dict(corr=w)
    if alpha is not None:
        kw["alpha"] = alpha
    if kb is not None:
        par = c.par.copy()
        par[:, W.P_KB] = kb
        kw["par"] = par
    return c.with_(**kw)


def torch_correction(f, nu_face, w):
    """Correction of one state by the network built from torch float64 layers."""
    import torch
    H = W.CORR_H
    l1 = torch.nn.Linear(5, H, dtype=torch.float64)
    l2 = torch.nn.Linear(H, 1, dtype=torch.float64)
    with torch.no_grad():
        l1.weight.copy_(torch.tensor(w[:5 * H].reshape(H, 5)))
        l1.bias.copy_(torch.tensor(w[5 * H:6 * H]))
        l2.weight.copy_(torch.tensor(w[6 * H:7 * H].reshape(1, H)))
        l2.bias.copy_(torch.tensor(w[7 * H:7 * H + 1]))
    n = len(f)
    ext = np.concatenate([[0.0], f, [0.0, 0.0]])          # ext[i + 1] = f_i, zeros outside
    Y = np.zeros(n + 1)
    for j in range(1, n):
        x = ext[j - 1:j + 3]                              # f_{j-2}, f_{j-1}, f_j, f_{j+1}
        sig = np.max(np.abs(x))
        if sig == 0:
            continue
        inp = torch.tensor(np.append(x / sig, nu_face[j]))[None, :]
        with torch.no_grad():
            y = l2(torch.tanh(l1(inp)))[0, 0].item()
        Y[j] = sig * nu_face[j] * y
    return Y[:-1] - Y[1:]


def test_zero_output_layer_is_the_plain_solver(oracle):
    p = corr_problem()
    w = p.corr.copy()
    w[0, 6 * W.CORR_H:] = 0.0
    a = oracle.solve1d(p.with_(corr=w), 0)
    b = oracle.solve1d(p.with_(corr=None), 0)
    np.testing.assert_array_equal(a["f_final"], b["f_final"])
    np.testing.assert_array_equal(a["mom"], b["mom"])


@pytest.mark.parametrize("scheme", [W.SCHEME_SSPRK3, W.SCHEME_LW_TVD])
def test_one_corrected_step_equals_torch_network(oracle, scheme):
    p = corr_problem(n=30, scale=0.5).with_(scheme=scheme, t_end=10.0)
    plain = oracle.solve1d(p.with_(corr=None), 0, max_steps=1)
    corr = oracle.solve1d(p, 0, max_steps=1)
    G0, dt = plain["G0"][0], plain["dt"][0]
    assert G0 > 0
    n = int(p.n_cells[0])
    dL = 1000.0 / n
    gamma = p.par[0, W.P_GAMMA]
    nu = dt * G0 * (1.0 + gamma * np.arange(n + 1) * dL) / dL
    want = plain["f_final"] + torch_correction(plain["f_final"], nu, p.corr[0])
    scale = np.max(np.abs(want))
    assert np.max(np.abs(corr["f_final"] - want)) <= 1e-13 * scale
    assert np.max(np.abs(corr["f_final"] - plain["f_final"])) > 1e-6 * scale   # the correction is visible


def test_correction_keeps_the_number(oracle):
    p = corr_problem(scale=0.8, kb=0.0, t_end=600.0)
    r = oracle.solve1d(p, 0)
    dL = 1000.0 / int(p.n_cells[0])
    mu0 = p.f0.sum() * dL
    assert r["outflow"] < 1e-20 * mu0                     # (the seed's far tail only)
    np.testing.assert_allclose(r["mom"][:, 0], mu0, rtol=1e-13)
    plain = oracle.solve1d(p.with_(corr=None), 0)
    assert np.max(np.abs(r["f_final"] - plain["f_final"])) > 1e-3 * np.max(plain["f_final"])


def test_homogeneous_in_the_density(oracle):
    p = corr_problem(scale=0.6, alpha=0.0, kb=0.0, t_end=400.0)
    a = oracle.solve1d(p, 0)
    b = oracle.solve1d(p.with_(f0=2.0 * p.f0), 0)
    assert a["steps"] == b["steps"]
    np.testing.assert_array_equal(b["f_final"], 2.0 * a["f_final"])


def test_tangent_along_weights_matches_central_differences(oracle):
    p = corr_problem(scale=0.4, t_end=300.0)
    rng = np.random.default_rng(7)
    v = rng.normal(size=W.CORR_NW)
    tan = oracle.tangent1d_corr(p, 0, v)
    h = 1e-6
    rp = oracle.solve1d(p.with_(corr=p.corr + h * v[None, :]), 0)
    rm = oracle.solve1d(p.with_(corr=p.corr - h * v[None, :]), 0)
    assert rp["steps"] == rm["steps"]
    for key, tkey in (("mom", "dM"), ("C", "dC")):
        want = (rp[key] - rm[key]) / (2 * h)
        got = tan[tkey][..., 0]
        assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want)) + 1e-12, key
        assert np.max(np.abs(want)) > 0

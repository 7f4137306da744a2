"""Pins of the oracle's learned closure (Sec. 4.2, Fig. 5a) against things other
than itself: torch's float32 -> bfloat16 conversion, torch's float64 linear
layers and autograd, reductions of the closure to the plain power law, and
central differences of the oracle solve.
"""
import math

import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W

H = W.MLP_H
SIM_FALLBACK = 4   # status bit: the plain law stood in for the closure
O = W.MLP_OFF


def unpack(blob):
    b = np.asarray(blob, dtype=np.float64)
    return (b[O["W1"]:O["W1"] + 3 * H].reshape(H, 3), b[O["b1"]:O["b1"] + H],
            b[O["W2"]:O["W2"] + H * H].reshape(H, H), b[O["b2"]:O["b2"] + H],
            b[O["W3"]:O["W3"] + 2 * H].reshape(2, H), b[O["b3"]:O["b3"] + 2])


def normalise(blob, x):
    c = np.asarray(blob[W.MLP_NW:], dtype=np.float64)
    return (x - c[0:3]) * c[3:6]


def inputs(n, seed=0):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.0, 0.3, n), rng.uniform(15.0, 40.0, n), rng.uniform(13.0, 15.0, n)], axis=1)


def test_bf16_rounding_matches_torch(oracle):
    import torch
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, 2000),
                         # exact ties between two bfloat16 neighbours, both parities
                         [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.5 + 2.0 ** -9, 3.0 + 2.0 ** -7]])
    ref = torch.tensor(xs, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle.bf16(x) for x in xs])
    assert np.array_equal(got, ref)


def test_fp64_network_matches_torch_layers(oracle):
    import torch
    import torch.nn.functional as F
    blob = W.closure_net(seed_offset=7, out_gain=1.0)
    blob[O["b1"]:O["b1"] + H] = np.linspace(-0.3, 0.2, H)
    blob[O["b2"]:O["b2"] + H] = np.linspace(0.1, -0.25, H)
    blob[O["b3"]:O["b3"] + 2] = [0.3, -0.7]
    x = inputs(50)
    y, dy = oracle.mlp_forward(blob, W.MLP_FP64, x, with_jac=True)
    W1, b1, W2, b2, W3, b3 = (torch.tensor(a) for a in unpack(blob))
    z = torch.tensor(normalise(blob, x), requires_grad=True)
    yt = F.linear(torch.tanh(F.linear(torch.tanh(F.linear(z, W1, b1)), W2, b2)), W3, b3)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-15)
    for o in range(2):
        (g,) = torch.autograd.grad(yt[:, o].sum(), z, retain_graph=True)
        np.testing.assert_allclose(dy[:, o, :], g.numpy(), rtol=1e-12, atol=1e-15)


def test_fp64_weight_gradient_matches_torch_autograd(oracle):
    import torch
    import torch.nn.functional as F
    blob = W.closure_net(seed_offset=8, out_gain=1.0)
    blob[O["b2"]:O["b2"] + H] = np.linspace(-0.2, 0.2, H)
    z = normalise(blob, inputs(40, seed=1))
    ybar = np.random.default_rng(2).normal(size=(40, 2))
    g = oracle.mlp_vjp(blob, W.MLP_FP64, z, ybar)
    params = [torch.tensor(a, requires_grad=True) for a in unpack(blob)]
    W1, b1, W2, b2, W3, b3 = params
    yt = F.linear(torch.tanh(F.linear(torch.tanh(F.linear(torch.tensor(z), W1, b1)), W2, b2)), W3, b3)
    (yt * torch.tensor(ybar)).sum().backward()
    ref = np.concatenate([p.grad.numpy().reshape(-1) for p in params])
    np.testing.assert_allclose(g, ref, rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_bf16_network_follows_its_rounding_rules(oracle):
    """BF16 emulation rebuilt from torch's bfloat16 casts: same values to float32 rounding."""
    import torch
    blob = W.closure_net(seed_offset=9, out_gain=1.0)
    blob[O["b1"]:O["b1"] + H] = np.linspace(-0.1, 0.1, H)
    x = inputs(64, seed=4)
    y = oracle.mlp_forward(blob, W.MLP_BF16, x)

    def bf(a):
        return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()

    def f32(a):
        return np.asarray(a, dtype=np.float32).astype(np.float64)

    W1, b1, W2, b2, W3, b3 = unpack(blob)
    z = bf(f32(normalise(blob, x)))
    h1 = bf(f32(np.tanh(f32(z @ bf(W1).T + b1))))
    h2 = bf(f32(np.tanh(f32(h1 @ bf(W2).T + b2))))
    ref = f32(h2 @ bf(W3).T + b3)
    # float32 rounding of sums formed in a different order may move an
    # activation across a bfloat16 boundary: allow a few such flips
    err = np.abs(y - ref)
    assert np.quantile(err, 0.9) <= 1e-6 * np.abs(ref).max()
    assert err.max() <= 2.0 ** -7


def closure_problem(n_sims=3, n=200, t_end=400.0, precision=W.MLP_FP64, blob=None):
    prob, _ = W.closure(n_sims=n_sims, n=n, t_end=t_end, n_samples=4)
    return prob.with_(law=W.LAW_MLP, mlp=W.closure_net() if blob is None else blob, mlp_precision=precision)


def test_constant_closure_equals_constant_power_law(oracle):
    """Zero weight matrices: the network returns its output bias, i.e. constant G0 and B,
    which is the power law with exponents g = b = 0 whenever S > 0."""
    blob = W.closure_net()
    blob[:W.MLP_NW] = 0.0
    blob[O["b3"]:O["b3"] + 2] = [0.4, -0.3]
    c = blob[W.MLP_NW:].astype(np.float64)
    G0 = math.exp(c[6] + c[8] * float(np.float32(0.4)))
    B = math.exp(c[7] + c[9] * float(np.float32(-0.3)))
    for prec in (W.MLP_FP64, W.MLP_BF16):
        prob = closure_problem(precision=prec, blob=blob)
        plain = prob.with_(law=W.LAW_POWER, mlp=None)
        plain.par = prob.par.copy()
        plain.par[:, W.P_KG] = G0 / 1e6
        plain.par[:, W.P_G] = 0.0
        plain.par[:, W.P_KB] = B
        plain.par[:, W.P_B] = 0.0
        for s in range(prob.n_sims):
            a, b = oracle.solve1d(prob, s), oracle.solve1d(plain, s)
            assert a["status"] == b["status"] == 0 and a["steps"] == b["steps"]
            np.testing.assert_allclose(a["mom"], b["mom"], rtol=1e-12)
            np.testing.assert_allclose(a["C"], b["C"], rtol=1e-14)


def test_fallback_outside_the_box_is_the_plain_power_law(oracle):
    blob = W.closure_net()
    blob[W.MLP_NW + 16] = 10.0          # s_min above any supersaturation: always outside
    prob = closure_problem(blob=blob)
    plain = prob.with_(law=W.LAW_POWER, mlp=None)
    for s in range(prob.n_sims):
        a, b = oracle.solve1d(prob, s), oracle.solve1d(plain, s)
        assert a["status"] & SIM_FALLBACK and not b["status"] & SIM_FALLBACK
        assert np.array_equal(a["mom"], b["mom"]) and np.array_equal(a["f_final"], b["f_final"])


def exact_direction(blob, seed):
    """Weight direction with entries in {-1, 0, 1}: w +- 2^-20 v is exact in float32."""
    v = np.random.default_rng(seed).integers(-1, 2, W.MLP_NW).astype(np.float64)
    assert np.all(np.abs(blob[:W.MLP_NW]) < 4.0)
    return v


def test_closure_tangent_matches_central_differences(oracle):
    prob = closure_problem(n_sims=2, n=150, t_end=300.0)
    h = 2.0 ** -20
    for s in range(prob.n_sims):
        v = exact_direction(prob.mlp, 10 + s)
        tan = oracle.tangent1d_mlp(prob, s, v)
        r0 = oracle.solve1d(prob, s)
        vals = []
        for sg in (1.0, -1.0):
            blob = prob.mlp.copy()
            blob[:W.MLP_NW] = (blob[:W.MLP_NW].astype(np.float64) + sg * h * v).astype(np.float32)
            assert np.array_equal(blob[:W.MLP_NW].astype(np.float64), prob.mlp[:W.MLP_NW] + sg * h * v)
            r = oracle.solve1d(prob.with_(mlp=blob), s)
            assert r["steps"] == r0["steps"]
            vals.append(r)
        for key, tk in (("mom", "dM"), ("C", "dC")):
            fd = (vals[0][key] - vals[1][key]) / (2 * h)
            ad = tan[tk][..., 0]
            np.testing.assert_allclose(ad, fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max())
        # gamma direction
        hg = 1e-7
        pp, pm = prob.par.copy(), prob.par.copy()
        pp[s, W.P_GAMMA] += hg
        pm[s, W.P_GAMMA] -= hg
        rp, rm = oracle.solve1d(prob.with_(par=pp), s), oracle.solve1d(prob.with_(par=pm), s)
        fd = (rp["mom"] - rm["mom"]) / (2 * hg)
        np.testing.assert_allclose(tan["dM"][..., 1], fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max())


def test_growth_rate_clamp_is_a_constant_power_law(oracle):
    """Output bias above the clamp: ln G0 is held at lnG0_max, so the closure is the constant power
    law G0 = exp(lnG0_max) (g = 0), and a weight direction that only moves the G0 output has zero
    derivative while the clamp holds."""
    blob = W.closure_net()
    blob[:W.MLP_NW] = 0.0
    blob[O["b3"]:O["b3"] + 2] = [1.0, -0.3]          # ln G0 = -4 + 2*1 = -2 > lnG0_max
    blob[W.MLP_C_LNG0_MAX] = -2.8
    c = blob[W.MLP_NW:].astype(np.float64)
    assert c[6] + c[8] * 1.0 > c[17]
    G0 = math.exp(c[17])
    B = math.exp(c[7] + c[9] * float(np.float32(-0.3)))
    prob = closure_problem(blob=blob)
    plain = prob.with_(law=W.LAW_POWER, mlp=None, par=prob.par.copy())
    plain.par[:, W.P_KG] = G0 / 1e6
    plain.par[:, W.P_G] = 0.0
    plain.par[:, W.P_KB] = B
    plain.par[:, W.P_B] = 0.0
    v = np.zeros(W.MLP_NW)
    v[O["b3"]] = 1.0
    for s in range(prob.n_sims):
        a, b = oracle.solve1d(prob, s), oracle.solve1d(plain, s)
        assert a["status"] == b["status"] == 0 and a["steps"] == b["steps"]
        np.testing.assert_allclose(a["mom"], b["mom"], rtol=1e-12)
        tan = oracle.tangent1d_mlp(prob, s, v, with_f=False)
        assert np.all(tan["dM"][..., 0] == 0.0) and np.all(tan["dC"][..., 0] == 0.0)


def test_closure_tangent_through_the_cfl_step(oracle):
    """CFL-limited steps under the closure: derivatives along a weight direction (which moves the
    network's growth rate, hence the step, the time reached, the ramp temperature and the network's
    temperature input) agree with central differences of the free-running solve."""
    consts = W.closure_consts(lnG0_max=3.0)
    blob = W.closure_net(out_gain=0.5, consts=consts)
    blob[O["b3"]] = 1.2                       # G0 ~ 0.2 um/s: CFL-limited (dt ~ 6 s) below dt_max = 60 s
    prob = closure_problem(n_sims=2, n=400, t_end=200.0, blob=blob)
    prob = prob.with_(dt_max=60.0, par=prob.par.copy(), t_samples=W.uniform_samples(2, 200.0))
    prob.par[:, W.P_TRAMP] = 500.0
    h = 2.0 ** -18
    for s in range(prob.n_sims):
        r0 = oracle.solve1d(prob, s)
        assert r0["status"] == 0
        n_cfl = int(np.sum(r0["dt"] < prob.dt_max * (1 - 1e-12)))
        assert n_cfl >= 0.9 * r0["steps"], (n_cfl, r0["steps"])
        v = exact_direction(prob.mlp, 20 + s)
        tan = oracle.tangent1d_mlp(prob, s, v)
        frozen = oracle.tangent1d_mlp(prob, s, v, frozen_dt=True)
        vals = []
        for sg in (1.0, -1.0):
            b = prob.mlp.copy()
            b[:W.MLP_NW] = (b[:W.MLP_NW].astype(np.float64) + sg * h * v).astype(np.float32)
            r = oracle.solve1d(prob.with_(mlp=b), s)
            assert r["steps"] == r0["steps"]
            vals.append(r)
        for key, tk in (("mom", "dM"), ("C", "dC")):
            fd = (vals[0][key] - vals[1][key]) / (2 * h)
            np.testing.assert_allclose(tan[tk][..., 0], fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())
            # holding the schedule fixed misses the dependence through the step (5x the tolerance above)
            assert np.abs(frozen[tk][..., 0] - fd).max() > 5e-4 * np.abs(fd).max()

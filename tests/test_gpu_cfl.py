"""GPU parity where the CFL bound sets the step (SI Eq. (S3)), not dt_max.

Every workload here is built so that the oracle's own step log shows most steps
CFL-limited: high supersaturation, fast and size-dependent growth, a large
dt_max and sample times that are not multiples of any step.  Then the
data-dependent schedule must come out the same on both sides (equal step counts,
step sizes to rounding), and every output within the FP64 tolerance:
  - 1D SSP-RK3 and the one-step scheme of Eq. (8) at nu = 0.9, grids 4..2048;
  - the fp64 learned closure (including steps where ln G0 is clamped), and the
    bf16 closure checked in replay mode (the oracle's finite-volume part driven
    by the GPU's recorded (G0, B));
  - the 2D split solver (min-form CFL over both axes);
  - the adjoint, whose step sizes are differentiated in the branch each step
    takes, against the oracle's tangent of the free-running solve and against
    central differences of the GPU forward.
"""
import numpy as np
import pytest

from _helpers import TOL, rel_each, rel_inf, split_packed
from paper_2411_00742_amd import workloads as W

pytestmark = pytest.mark.gpu


def cfl_steps(prob, dt):
    """Number of CFL-limited steps in a step log: shorter than dt_max and not landing on a
    sample time (or t_end)."""
    t = np.cumsum(dt)
    marks = np.append(prob.t_samples, prob.t_end)
    lands = np.min(np.abs(t[:, None] - marks[None, :]), axis=1) <= 1e-9 * prob.t_end
    return int(np.sum((dt < prob.dt_max * (1 - 1e-12)) & ~lands))


def cfl_fraction(prob, ref):
    """Fraction of a sim's steps that are CFL-limited in the oracle's log."""
    return cfl_steps(prob, ref["dt"]) / max(len(ref["dt"]), 1)


def gpu_solve(prob, **kw):
    import paper_2411_00742_amd as pbe
    s = pbe.Solver(prob, record_rates=True, **kw)
    o = {k: v.cpu().numpy() for k, v in s.solve().items()}
    o["rates"] = s.rate_log(int(o["steps"].max())).cpu().numpy()
    s.close()
    return o


def compare_1d(prob, o, oracle, min_cfl=0.9, rates_replay=False):
    sizes = prob.cells_per_sim()
    fs = split_packed(o["f"], sizes)
    total, limited = 0, 0.0
    for s in range(prob.n_sims):
        st = int(o["steps"][s])
        if rates_replay:
            r = oracle.solve1d(prob, s, rates_replay=(o["rates"][s, :st, 1], o["rates"][s, :st, 2]))
        else:
            r = oracle.solve1d(prob, s)
            assert int(o["status"][s]) == r["status"], (s, o["status"][s], r["status"])
        assert st == r["steps"], (s, st, r["steps"])
        # a step that lands on a sample time is the difference of two times, which carry
        # rounding of the order of 1e-16 t_end from the steps before it
        np.testing.assert_allclose(o["rates"][s, :st, 0], r["dt"], rtol=1e-11, atol=1e-13 * prob.t_end,
                                   err_msg=f"dt of sim {s}")
        e_f = rel_inf(fs[s], r["f_final"])
        e_m = rel_each(o["mom"][s], r["mom"])
        e_c = rel_each(o["C"][s], r["C"])
        assert e_f <= TOL and e_m <= TOL and e_c <= TOL, (s, int(sizes[s]), e_f, e_m, e_c)
        total += r["steps"]
        limited += cfl_fraction(prob, r) * r["steps"]
    assert limited >= min_cfl * total, (limited, total)


@pytest.mark.parametrize("scheme,nu", [(W.SCHEME_SSPRK3, 0.5), (W.SCHEME_LW_TVD, 0.9)])
def test_cfl_limited_1d_ragged(torch_cuda, oracle, scheme, nu):
    sizes = [4, 5, 63, 64, 65, 129, 200, 511, 513, 700, 1023, 1025, 1536, 1999, 2047, 2048]
    prob = W.cfl_limited(len(sizes), sizes=sizes).with_(scheme=scheme, cfl=nu)
    o = gpu_solve(prob)
    compare_1d(prob, o, oracle)


def test_cfl_limited_1d_batch(torch_cuda, oracle):
    """48 sims of 4..2048 cells drawn at random, each checked against the oracle."""
    prob = W.cfl_limited(48, 4, 2048, seed_offset=16)
    o = gpu_solve(prob)
    compare_1d(prob, o, oracle)


def cfl_closure(prec, sizes=(64, 100, 129, 300, 512, 513, 1000, 1024), t_end=300.0, n_samples=4):
    """Closure solves whose steps are CFL-limited; ln G0 sits near its clamp so that some steps
    are clamped and some are not."""
    from test_gpu_closure import blob_with_biases, closure_problem
    blob = blob_with_biases()
    blob[W.MLP_NW:] = W.closure_consts(out_shift=(-2.0, 17.0), lnG0_max=-1.36)
    prob = closure_problem(list(sizes), t_end=t_end, prec=prec, blob=blob, n_samples=n_samples)
    prob = prob.with_(dt_max=30.0, C0=np.full(len(sizes), W.csat_linear(40.0) * 1.2))
    return prob


def test_cfl_limited_fp64_closure(torch_cuda, oracle):
    prob = cfl_closure(W.MLP_FP64)
    o = gpu_solve(prob)
    compare_1d(prob, o, oracle)
    G = np.concatenate([o["rates"][s, :int(o["steps"][s]), 1] for s in range(prob.n_sims)])
    Gmax = np.exp(np.float64(np.float32(-1.36)))
    clamped = np.sum(np.abs(G - Gmax) <= 1e-14 * Gmax)
    assert 10 <= clamped <= 0.9 * len(G), (clamped, len(G))


def test_cfl_limited_bf16_closure_replay(torch_cuda, oracle):
    """bf16 network on the matrix cores: the finite-volume solve, the CFL step and the solute
    balance are held to the FP64 tolerance by driving the oracle with the GPU's own (G0, B)."""
    prob = cfl_closure(W.MLP_BF16)
    o = gpu_solve(prob)
    compare_1d(prob, o, oracle, rates_replay=True)


def test_bf16_closure_replay_default_workload(torch_cuda, oracle):
    """The same replay check on the closure test workload (dt_max-limited steps)."""
    from test_gpu_closure import closure_problem
    prob = closure_problem([64, 100, 129, 300, 512, 513, 1000, 1024], prec=W.MLP_BF16)
    o = gpu_solve(prob)
    compare_1d(prob, o, oracle, min_cfl=0.0, rates_replay=True)


def test_cfl_limited_2d(torch_cuda, oracle):
    from test_gpu_fvm2d import problem2d
    p = problem2d([(300, 200), (700, 150), (1100, 90), (150, 600), (64, 257)], t_end=200.0, S_boost=1.3)
    p = p.with_(dt_max=40.0)
    import paper_2411_00742_amd as pbe
    s = pbe.Solver(p)
    g = {k: v.cpu().numpy() for k, v in s.solve().items()}
    s.close()
    fs = split_packed(g["f"], p.cells_per_sim())
    total, limited = 0, 0
    for i in range(p.n_sims):
        r = oracle.solve2d(p, i)
        assert int(g["steps"][i]) == r["steps"], (i, g["steps"][i], r["steps"])
        assert rel_inf(fs[i], r["f_final"].ravel()) <= TOL
        assert rel_each(g["mom"][i], r["mom"]) <= TOL and rel_each(g["C"][i], r["C"]) <= TOL
        total += r["steps"]
        limited += cfl_steps(p, r["dt"])
    assert limited >= 0.8 * total, (limited, total)


# --------------------------------------------------------------------------- adjoint
NG = 5


def assert_close(got, ref, s, tol=TOL):
    floor = 1e-6 * np.max(np.abs(ref))
    err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
    assert np.all(err <= tol), (s, got, ref, err)


def vjp_from_tangent(prob, s, tan, gf, gmom, gC, record_f):
    off = prob.offsets()
    n, ns = int(prob.n_cells[s]), len(prob.t_samples)
    v = np.einsum("qk,qkd->d", gmom[s], tan["dM"]) + np.einsum("q,qd->d", gC[s], tan["dC"])
    if record_f:
        v += np.einsum("qi,qid->d", gf[off[s] * ns:off[s + 1] * ns].reshape(ns, n), tan["dF"])
    else:
        v += np.einsum("i,id->d", gf[off[s]:off[s + 1]], tan["dF"][-1])
    return v


@pytest.mark.parametrize("record_f", [True, False])
def test_cfl_limited_adjoint_matches_oracle_tangent(torch_cuda, oracle, record_f):
    """The adjoint differentiates the CFL-limited step sizes, the landing steps and the ramp
    temperature; the oracle's tangent of the free-running solve is the reference, and the
    tangent with the schedule frozen is shown to be a different (wrong) answer here."""
    import torch
    import paper_2411_00742_amd as pbe
    sizes = [64, 100, 129, 300, 511, 512, 700, 1000, 1024]
    prob = W.cfl_limited(len(sizes), sizes=sizes, t_end=400.0, n_samples=4, seed_offset=26)
    s = pbe.Solver(prob, ckpt_every=16, record_f=record_f)
    o = {k: v.cpu().numpy() for k, v in s.solve().items()}
    rng = np.random.default_rng(11)
    ns = len(prob.t_samples)
    nf = int(prob.cells_per_sim().sum()) * (ns if record_f else 1)
    gf = rng.normal(size=nf) / np.max(np.abs(o["f"]))
    gmom = rng.normal(size=o["mom"].shape) / np.abs(o["mom"])
    gC = rng.normal(size=o["C"].shape) / np.abs(o["C"])
    g = s.grad(torch.tensor(gf), torch.tensor(gmom), torch.tensor(gC)).cpu().numpy()
    s.close()
    assert np.all(o["status"] == 0)
    far = 0
    for i in range(prob.n_sims):
        ref = vjp_from_tangent(prob, i, oracle.tangent1d(prob, i, with_f=True), gf, gmom, gC, record_f)
        assert_close(g[i], ref, i)
        frozen = vjp_from_tangent(prob, i, oracle.tangent1d(prob, i, with_f=True, frozen_dt=True), gf, gmom, gC,
                                  record_f)
        far += int(np.max(np.abs(frozen - ref) / np.maximum(np.abs(ref), 1e-6 * np.abs(ref).max())) > 1e-3)
    assert far >= prob.n_sims // 2, far


def test_cfl_limited_adjoint_matches_central_differences_of_gpu_forward(torch_cuda):
    import torch
    import paper_2411_00742_amd as pbe
    prob = W.cfl_limited(6, sizes=[120, 250, 400, 640, 800, 1000], t_end=400.0, n_samples=4, seed_offset=36)
    prob.par[:, W.P_GAMMA] = np.maximum(prob.par[:, W.P_GAMMA], 2e-4)   # gamma - h stays >= 0
    s = pbe.Solver(prob, ckpt_every=16)
    o = {k: v.cpu().numpy() for k, v in s.solve().items()}
    tm, tc = o["mom"] * 1.03, o["C"] * 0.999

    def loss(mom, C):
        return (((mom - tm) / tm) ** 2).sum(axis=(1, 2)) + (((C - tc) / tc) ** 2).sum(axis=1)

    gmom = 2 * (o["mom"] - tm) / tm ** 2
    gC = 2 * (o["C"] - tc) / tc ** 2
    g = s.grad(None, torch.tensor(gmom), torch.tensor(gC)).cpu().numpy()
    checked = 0
    for d, idx in enumerate([W.P_KG, W.P_G, W.P_KB, W.P_B, W.P_GAMMA]):
        h = 1e-6 * np.abs(prob.par[:, idx])
        vals, same = [], np.ones(prob.n_sims, dtype=bool)
        for sg in (1, -1):
            par = prob.par.copy()
            par[:, idx] += sg * h
            s.set_par(par)
            oo = {k: v.cpu().numpy() for k, v in s.solve().items()}
            same &= oo["steps"] == o["steps"]
            vals.append(loss(oo["mom"], oo["C"]))
        fd = (vals[0] - vals[1]) / (2 * h)
        scale = np.max(np.abs(fd))
        for i in np.nonzero(same)[0]:
            assert abs(g[i, d] - fd[i]) <= 1e-4 * abs(fd[i]) + 1e-7 * scale, (d, i, g[i, d], fd[i])
            checked += 1
    s.close()
    assert checked >= 0.8 * NG * prob.n_sims, checked


def test_cfl_limited_closure_adjoint_fp64(torch_cuda, oracle):
    """fp64 closure in the CFL-limited regime (with clamped steps): weight-direction and gamma
    derivatives against the oracle's tangent of the free-running solve."""
    import torch
    import paper_2411_00742_amd as pbe
    prob = cfl_closure(W.MLP_FP64, sizes=(100, 257, 640), t_end=200.0)
    prob.par[:, W.P_GAMMA] = [0.0, 5e-4, 1.2e-3]
    s = pbe.Solver(prob, ckpt_every=16)
    o = {k: v.cpu().numpy() for k, v in s.solve().items()}
    rng = np.random.default_rng(3)
    gmom = rng.normal(size=o["mom"].shape) / np.abs(o["mom"])
    gC = rng.normal(size=o["C"].shape) / np.abs(o["C"])
    gpar, gw = s.grad(None, torch.tensor(gmom), torch.tensor(gC), with_mlp=True)
    gpar, gw = gpar.cpu().numpy(), gw.cpu().numpy()
    s.close()
    vs = [rng.normal(size=W.MLP_NW) for _ in range(2)]
    ref_w = np.zeros(len(vs))
    for sidx in range(prob.n_sims):
        for i, v in enumerate(vs):
            tan = oracle.tangent1d_mlp(prob, sidx, v, with_f=False)
            ref_w[i] += np.einsum("qk,qk->", gmom[sidx], tan["dM"][..., 0]) + np.einsum("q,q->", gC[sidx],
                                                                                        tan["dC"][..., 0])
            if i == 0:
                dg = np.einsum("qk,qk->", gmom[sidx], tan["dM"][..., 1]) + np.einsum("q,q->", gC[sidx],
                                                                                     tan["dC"][..., 1])
                assert abs(gpar[sidx, 4] - dg) <= 1e-9 * max(abs(dg), 1e-300), (sidx, gpar[sidx, 4], dg)
    got = np.array([gw @ v for v in vs])
    np.testing.assert_allclose(got, ref_w, rtol=1e-9, atol=1e-12 * np.abs(ref_w).max())


def test_set_par_beyond_the_step_budget_is_refused(torch_cuda):
    """The step budget (and the checkpoints sized from it) is derived at create; kinetics whose
    CFL-limited step bound exceeds it are refused instead of truncating the solve."""
    import paper_2411_00742_amd as pbe
    prob = W.cfl_limited(4, sizes=[200, 400, 800, 1000], t_end=300.0, n_samples=3)
    s = pbe.Solver(prob, ckpt_every=16)
    s.solve()
    par = prob.par.copy()
    par[:, W.P_KG] *= 1.001
    s.set_par(par)                       # inside the headroom
    par[:, W.P_KG] *= 10.0
    with pytest.raises(pbe.PBEError) as e:
        s.set_par(par)
    assert e.value.code == pbe.PBE_ESTATE
    o = {k: v.cpu().numpy() for k, v in s.solve().items()}   # the handle kept the previous kinetics
    assert np.all(o["status"] == 0)
    s.close()

"""GPU parity of the in-the-loop correction (Sec. 4.2, Fig. 5b) and its training.

- corrected coarse solves with random weights on grids of 4..512 cells (ragged tails, pad
  slots), both schemes: step counts, densities at every sample, moments and C within the FP64
  tolerance of the oracle;
- a zero output layer reproduces the plain solver bitwise;
- the batched central-difference gradient of the rollout loss agrees with the oracle's
  forward-mode derivative along a random weight direction;
- training lowers the rollout error on held-out simulations (the measured ratio is printed).
"""
import numpy as np
import pytest

from _helpers import TOL, rel_each, rel_inf, split_packed
from paper_2411_00742_amd import workloads as W

pytestmark = pytest.mark.gpu


def corrected(sizes, scheme=W.SCHEME_SSPRK3, cfl=0.5, seed=0, scale=0.4, t_end=600.0):
    c, _ = W.inloop(n_sims=len(sizes), n_coarse=8, refine=1, t_end=t_end, n_samples=5, seed_offset=60 + seed)
    rng = np.random.default_rng(seed)
    f0 = np.concatenate([W.scale_to_seed_mass(W.seed_sample_1d("lognormal", n, 1000.0, 200.0, 40.0), 5e-3, W.ALPHA,
                                              1000.0, n) for n in sizes])
    w = rng.normal(scale=scale, size=(len(sizes), W.CORR_NW))
    return c.with_(n_cells=np.array(sizes, dtype=np.int32), f0=f0, corr=w, scheme=scheme, cfl=cfl)


def gpu_run(prob, record_f=True):
    import paper_2411_00742_amd as pbe
    s = pbe.Solver(prob, record_f=record_f)
    o = {k: v.cpu().numpy() for k, v in s.solve().items()}
    s.close()
    return o


@pytest.mark.parametrize("scheme,nu", [(W.SCHEME_SSPRK3, 0.5), (W.SCHEME_LW_TVD, 0.9)])
def test_corrected_solve_matches_oracle(torch_cuda, oracle, scheme, nu):
    sizes = [4, 5, 17, 63, 64, 65, 100, 129, 200, 255, 256, 257, 383, 511, 512]
    p = corrected(sizes, scheme=scheme, cfl=nu)
    o = gpu_run(p)
    ns = len(p.t_samples)
    fs = split_packed(o["f"], [n * ns for n in sizes])
    for s, n in enumerate(sizes):
        r = oracle.solve1d(p, s, record_f=True)
        assert int(o["steps"][s]) == r["steps"], (s, o["steps"][s], r["steps"])
        assert rel_inf(fs[s], r["f_samples"].ravel()) <= TOL, (s, n)
        assert rel_each(o["mom"][s], r["mom"]) <= TOL and rel_each(o["C"][s], r["C"]) <= TOL, (s, n)


def test_zero_output_layer_is_the_plain_kernel_bitwise(torch_cuda):
    sizes = [30, 64, 200, 512]
    p = corrected(sizes)
    w = p.corr.copy()
    w[:, 6 * W.CORR_H:] = 0.0
    a = gpu_run(p.with_(corr=w))
    b = gpu_run(p.with_(corr=None))
    for k in ("f", "mom", "C", "steps"):
        np.testing.assert_array_equal(a[k], b[k])


def test_rollout_gradient_matches_oracle_tangent(torch_cuda, oracle):
    import torch
    from paper_2411_00742_amd import inloop as IL
    coarse, fine = W.inloop(n_sims=3, n_coarse=40, refine=4, t_end=300.0, n_samples=6, seed_offset=70)
    target = IL.fine_targets(fine, 4)
    fit = IL.CorrectionFit(coarse, target, [0, 1, 2])
    rng = np.random.default_rng(3)
    w = IL.init_weights(1, scale=0.5)
    w[5 * W.CORR_H:] = rng.normal(scale=0.2, size=W.CORR_NW - 5 * W.CORR_H)
    loss, g = fit.loss_and_grad(torch.tensor(w, device=fit.solver.device))
    fit.close()
    v = rng.normal(size=W.CORR_NW)
    # the same loss and its derivative along v from the oracle's forward mode
    tg = target.cpu().numpy()
    pw = coarse.with_(corr=np.tile(w, (3, 1)))
    L, dL = 0.0, 0.0
    for s in range(3):
        r = oracle.solve1d(pw, s, record_f=True)
        t = oracle.tangent1d_corr(pw, s, v)
        d = r["f_samples"] - tg[s]
        den = (tg[s] ** 2).sum(axis=1)
        L += ((d ** 2).sum(axis=1) / den).sum()
        dL += ((2.0 * d * t["dF"][..., 0]).sum(axis=1) / den).sum()
    n = 3 * tg.shape[1]
    assert abs(float(loss) - L / n) <= 1e-10 * L / n
    gv = float((g.cpu().numpy() * v).sum())
    assert abs(gv - dL / n) <= 1e-6 * abs(dL / n), (gv, dL / n)


def test_training_lowers_the_held_out_error(torch_cuda):
    from paper_2411_00742_amd import inloop as IL
    coarse, fine = W.inloop(n_sims=48, n_coarse=50, refine=16)
    target = IL.fine_targets(fine, 16)
    idx = np.arange(48)
    train, test = idx[:36], idx[36:]
    w, hist = IL.train(coarse, target, train, iters=800)
    ev = IL.evaluate(coarse, target, test, w)
    print("in-the-loop correction: loss", hist[0], "->", hist[-1], "held out", ev)
    assert hist[-1] < 0.6 * hist[0]
    assert ev["corrected"] < 0.6 * ev["plain"], ev

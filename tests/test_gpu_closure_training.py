"""Training the learned closure through the solver, and what it gains.

Ground truth: the power law times an Arrhenius temperature factor (the form of
App. A), shared by all simulations, which run different cooling profiles, seeds
and initial concentrations.  The plain power law has no temperature input, so
no choice of its four shared parameters reproduces all trajectories; the
closure sees T and can.  Both are fitted by Adam through the adjoint on the
same 80% of the simulations and compared on the held-out 20%.  The training
outcome is not pinned to an oracle value (parity unpinned); the gain is the
measured ratio of held-out losses.
"""
import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W

pytestmark = pytest.mark.gpu


def problems(n_sims, n=200, t_end=3600.0):
    truth, split = W.closure(n_sims=n_sims, n=n, t_end=t_end, n_samples=10)
    plain = truth.with_(law=W.LAW_POWER)
    plain.par = truth.par.copy()
    # starting point of both fits: the ground truth frozen at 30 degC
    plain.par[:, W.P_KG] = 4e-7
    plain.par[:, W.P_KB] = 2e9
    mlp = plain.with_(law=W.LAW_MLP, mlp=W.closure_net(), mlp_precision=W.MLP_BF16)
    return truth, plain, mlp, split


def test_training_lowers_the_loss(torch_cuda):
    from paper_2411_00742_amd import closure_train as T
    truth, plain, mlp, split = problems(64, t_end=1200.0)
    mom, C = T.generate_data(truth)
    w, hist = T.fit_closure(mlp, mom, C, split, iters=15, lr=3e-3)
    print("closure loss", hist[0], "->", hist[-1])
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.7 * hist[0]


def test_closure_gain_over_plain_law(torch_cuda):
    import torch
    from paper_2411_00742_amd import closure_train as T
    truth, plain, mlp, split = problems(1024)
    mom, C = T.generate_data(truth)
    vals, hp = T.fit_power_law(plain, mom, C, split, iters=120, lr=0.05, log=print)
    fitted = plain.with_()
    fitted.par = plain.par.copy()
    fitted.par[:, [W.P_KG, W.P_G, W.P_KB, W.P_B]] = vals
    w, hm = T.fit_closure(mlp, mom, C, split, iters=300, lr=3e-3, log=print)
    trained = mlp.with_(mlp=np.concatenate([w.cpu().numpy(), mlp.mlp[W.MLP_NW:]]).astype(np.float32))
    held = ~split
    l_plain = T.evaluate(fitted, mom, C, held)
    l_mlp = T.evaluate(trained, mom, C, held)
    print(f"held-out loss: best-fit power law {l_plain:.4e}, trained closure {l_mlp:.4e}, "
          f"gain {l_plain / l_mlp:.2f}x; fitted (kg, g, kb, b) = {vals}")
    assert np.isfinite(l_mlp) and l_mlp < l_plain

"""In-the-loop correction of a coarse grid (Sec. 4.2, Fig. 5b of the paper): a small network
inside the time loop offsets the discretisation error of each coarse step, so that a coarse
solve follows the fine solution at the coarse solve's cost.

The network (see include/pbe.h, PBE_CORR_*): at every interior face a correction flux
Y = sigma nu (W2 . tanh(W1 x + b1) + b2) from the four surrounding cells scaled by their
largest magnitude and the face's Courant number; the corrected state is
f_i + Y_{i-1/2} - Y_{i+1/2}, so the number balance and the boundary fluxes stay the solver's.

Training follows the solver-in-the-loop idea the paper cites: the loss is taken over whole
coarse rollouts (every recorded sample of the corrected coarse solve against the fine solve's
densities averaged onto the coarse cells), so the network learns from the errors it meets
when its own corrections feed the next steps.  Its 57 weights are few enough for batched
central differences: one launch solves the 2 * 57 + 1 perturbed copies of every training
simulation side by side.  Adam (lr 1e-2) updates the weights.
"""
from __future__ import annotations

import time

import numpy as np

from . import Adam, Solver
from . import workloads as W


def fine_targets(fine: W.Problem, refine: int):
    """Fine-grid densities at the sample times, averaged onto the coarse cells: [S, ns, n_coarse]."""
    s = Solver(fine, record_f=True)
    o = s.solve()
    S, ns = fine.n_sims, len(fine.t_samples)
    nf = int(fine.n_cells[0])
    f = o["f"].reshape(S, ns, nf // refine, refine).mean(dim=3).clone()
    s.close()
    return f


def rollout_errors(f, target):
    """Relative squared error of every sample, [S, ns]."""
    num = ((f - target) ** 2).sum(dim=2)
    den = (target ** 2).sum(dim=2)
    return num / den


class CorrectionFit:
    """Central-difference gradients of the rollout loss over the training simulations."""

    def __init__(self, coarse: W.Problem, target, train_idx, h: float = 1e-5):
        import torch
        self.torch = torch
        self.h = h
        self.train_idx = np.asarray(train_idx)
        self.n = len(self.train_idx)
        self.nb = 2 * W.CORR_NW + 1                        # base, +h e_j, -h e_j
        base = coarse.subset(self.train_idx)
        blocks = base.subset(np.tile(np.arange(self.n), self.nb))
        blocks = blocks.with_(corr=np.zeros((self.n * self.nb, W.CORR_NW)))
        self.solver = Solver(blocks, record_f=True)
        self.target = target[torch.as_tensor(self.train_idx, device=target.device)]
        self.ns, self.nc = self.target.shape[1], self.target.shape[2]
        eye = torch.eye(W.CORR_NW, dtype=torch.float64, device=self.solver.device)
        self.delta = torch.cat([torch.zeros((1, W.CORR_NW), dtype=torch.float64, device=eye.device), h * eye, -h * eye])

    def loss_and_grad(self, w):
        """(mean rollout loss at w, d loss / d w) from one batched solve."""
        t = self.torch
        wb = (w.to(t.float64)[None, :] + self.delta).repeat_interleave(self.n, dim=0).contiguous()
        self.solver.set_corr(wb)
        o = self.solver.solve()
        f = o["f"].reshape(self.nb, self.n, self.ns, self.nc)
        err = rollout_errors(f.reshape(self.nb * self.n, self.ns, self.nc), self.target.repeat(self.nb, 1, 1))
        per = err.reshape(self.nb, self.n * self.ns).mean(dim=1)
        g = (per[1:1 + W.CORR_NW] - per[1 + W.CORR_NW:]) / (2.0 * self.h)
        return per[0], g

    def close(self):
        self.solver.close()


def init_weights(seed: int = 0, scale: float = 0.3):
    """Random first layer, zero output layer: training starts from the uncorrected solver."""
    rng = np.random.default_rng(seed)
    w = np.zeros(W.CORR_NW)
    w[:5 * W.CORR_H] = rng.normal(scale=scale, size=5 * W.CORR_H)
    return w


def train(coarse: W.Problem, target, train_idx, iters: int = 200, lr: float = 1e-2, seed: int = 0):
    """Adam on the correction weights; returns (weights [CORR_NW] float64 array, loss history)."""
    import torch
    fit = CorrectionFit(coarse, target, train_idx)
    opt = Adam(torch.tensor(init_weights(seed), dtype=torch.float32, device=fit.solver.device), lr=lr)
    hist = []
    for _ in range(iters):
        loss, g = fit.loss_and_grad(opt.w)
        hist.append(float(loss))
        opt.step(g)
    fit.close()
    return opt.w.double().cpu().numpy(), hist


def evaluate(coarse: W.Problem, target, idx, w):
    """Mean relative squared rollout error of the plain and of the corrected coarse solve on sims idx."""
    import torch
    sub = coarse.subset(idx)
    tg = target[torch.as_tensor(np.asarray(idx), device=target.device)]
    out = {}
    for name, prob in (("plain", sub), ("corrected", sub.with_(corr=np.tile(w, (len(idx), 1))))):
        s = Solver(prob, record_f=True)
        o = s.solve()
        f = o["f"].reshape(len(idx), tg.shape[1], tg.shape[2])
        out[name] = float(rollout_errors(f, tg).mean())
        s.close()
    return out


def timing(coarse: W.Problem, fine: W.Problem, w, reps: int = 3):
    """Wall time of one solve of every simulation: fine grid, coarse grid, corrected coarse grid."""
    import torch
    res = {}
    for name, prob in (("fine", fine), ("coarse", coarse),
                       ("corrected", coarse.with_(corr=np.tile(w, (coarse.n_sims, 1))))):
        s = Solver(prob)
        o = s.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s.solve(o)
        torch.cuda.synchronize()
        res[name + "_ms"] = 1e3 * (time.perf_counter() - t0) / reps
        s.close()
    return res

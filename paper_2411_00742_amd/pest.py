"""Parameter estimation of a polynomial growth law through the differentiable
solver (Sec. 4.1, App. B and App. C of the paper), and the time per optimizer
iteration with reverse-mode gradients (the library's adjoint, pbe_grad_poly)
against batched forward differences of the solver (one launch that runs the
k + 1 perturbed copies of the experiments side by side).

Experiments (App. B): nine in-silico batch experiments at constant temperature
T in {10, 15, 20} degC and initial supersaturation S0 in {1.15, 1.25, 1.5}
(c0 = S0 c*(T), with the exponential solubility c* = 3.37 exp(0.036 T) g/kg of
App. A), one crystal length on [0, 1000] um, a Gaussian seed of 400 +- 30 um
scaled to 1 g per kg of solvent, no nucleation.  The measurements are the
concentration and the mean crystal length at 600 uniform times over 600 min,
computed by this solver with the paper's Arrhenius growth law (App. A
Eq. (A.2) with the first axis' constants of Table A.1) on 1 um bins; the paper
computes them with the method of moments.

Model (Eq. (poly_growth_rate)): G(S) = a_1 (S - 1) + ... + a_k (S - 1)^k in
um/min, one coefficient vector shared by the nine experiments, solved on 5 um
bins.  Loss: sum over experiments and samples of the squared relative errors
of the concentration and of the mean length (the residual sum of squares of
App. C in relative form).  Optimizer: Adam (App. C) with learning rate 0.01 on
theta = a / 100 um/min, theta projected onto theta >= 0 (the paper's only
constraint).  Units of these problems: minutes, g per kg of solvent, number
density per um and kg of solvent (alpha = rho_c k_v).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import Adam, Solver
from . import workloads as W

TEMPS = (10.0, 15.0, 20.0)
S0S = (1.15, 1.25, 1.5)
A_SCALE = 100.0                      # um/min per unit of theta
CS0, CS1 = 3.37, 0.036               # App. A solubility, g/kg and 1/degC
TRUTH = dict(kg=8.86e6 / 1e6, g=3.7, Eg=2.45e3)   # Table A.1, first axis (kg in the solver's units)


def experiments(n: int = 200, L_max: float = 1000.0, t_end: float = 600.0, n_samples: int = 600,
                law: int = W.LAW_POLY, poly=None) -> W.Problem:
    """The nine experiments on n bins; law LAW_POLY (coefficients poly[k] shared) or LAW_ARRHENIUS (truth)."""
    rho_kv = W.PAPER_RHO_C * W.PAPER_KV
    f = W.gaussian_seed_1d(n, L_max, 400.0, 30.0, 1.0)
    dL = L_max / n
    L = (np.arange(n) + 0.5) * dL
    f = f / (rho_kv * float((L ** 3 * f).sum() * dL))      # seed mass 1 g
    pars, C0 = [], []
    for T in TEMPS:
        for S0 in S0S:
            pars.append(W._par_row(TRUTH["kg"], TRUTH["g"], 0.0, 1.0, 0.0, Eg=TRUTH["Eg"], T0=T, T1=T, t_ramp=0.0))
            C0.append(S0 * CS0 * math.exp(CS1 * T))
    S = len(pars)
    prob = W.Problem(ndim=1, n_cells=np.full(S, n, dtype=np.int32), L_max=np.full(S, L_max), f0=np.tile(f, S),
                     C0=np.array(C0), par=np.array(pars), t_samples=W.uniform_samples(n_samples, t_end),
                     t_end=t_end, law=law, sol_law=W.SOL_EXP, cs0=CS0, cs1=CS1, alpha=rho_kv, dt_max=1.0,
                     name=f"pest-9x{n}")
    if law == W.LAW_POLY:
        prob.poly = np.tile(np.asarray(poly, dtype=np.float64), (S, 1))
    return prob


def measurements():
    """Concentration and mean length of the truth law at the 600 sample times: (C, Lmean) [9, 600]."""
    truth = experiments(n=1000, law=W.LAW_ARRHENIUS)
    s = Solver(truth)
    o = s.solve()
    mom, C = o["mom"], o["C"]
    Lm = mom[:, :, 1] / mom[:, :, 0]
    out = (C.clone(), Lm.clone())
    s.close()
    return out


def loss_and_cotangents(mom, C, C_ref, L_ref):
    """Loss [sims] (per experiment) and the cotangents of mom and C (torch tensors)."""
    import torch
    Lm = mom[:, :, 1] / mom[:, :, 0]
    rc = (C - C_ref) / C_ref
    rl = (Lm - L_ref) / L_ref
    loss = (rc ** 2).sum(dim=1) + (rl ** 2).sum(dim=1)
    gC = 2.0 * rc / C_ref
    gL = 2.0 * rl / L_ref
    gmom = torch.zeros_like(mom)
    gmom[:, :, 1] = gL / mom[:, :, 0]
    gmom[:, :, 0] = -gL * mom[:, :, 1] / mom[:, :, 0] ** 2
    return loss, gmom, gC


class PolyFit:
    """Gradients of the estimation loss with respect to theta (k coefficients), by the
    adjoint or by batched forward differences, on solver handles built once."""

    def __init__(self, k: int, C_ref, L_ref, theta0=None, max_steps: int = 100000, ckpt_every: int = 32,
                 nd: bool = True):
        import torch
        self.k = k
        self.C_ref, self.L_ref = C_ref, L_ref
        th = np.full(k, 0.5) if theta0 is None else np.asarray(theta0, dtype=np.float64)
        self.prob = experiments(poly=A_SCALE * th)
        self.ad = Solver(self.prob, ckpt_every=ckpt_every, max_steps=max_steps)
        self.dev = self.ad.device
        self.nd = None
        if nd:
            # k + 1 blocks of the nine experiments: the base point, then theta_j + h
            self.nd = Solver(self.prob.subset(np.tile(np.arange(9), k + 1)), max_steps=max_steps)
        self.torch = torch

    def _coeffs(self, theta, blocks=1):
        a = (A_SCALE * theta.to(self.torch.float64)).reshape(1, -1)
        return a.expand(9 * blocks, -1).contiguous()

    def grad_ad(self, theta):
        """(loss, dloss/dtheta [k]) from one solve and the adjoint."""
        self.ad.set_poly(self._coeffs(theta))
        o = self.ad.solve()
        loss, gmom, gC = loss_and_cotangents(o["mom"], o["C"], self.C_ref, self.L_ref)
        gp, _ = self.ad.grad_poly(None, gmom, gC)
        return loss.sum(), A_SCALE * gp.sum(dim=0)

    def grad_nd(self, theta, h: float = 1e-6):
        """(loss, forward-difference dloss/dtheta [k]) from one batched solve of the k + 1 points."""
        t = self.torch
        k = self.k
        th = theta.to(t.float64).reshape(1, -1).repeat(k + 1, 1)
        th[1:] += h * t.eye(k, dtype=t.float64, device=theta.device)
        a = (A_SCALE * th).repeat_interleave(9, dim=0).contiguous()
        self.nd.set_poly(a)
        o = self.nd.solve()
        loss, _, _ = loss_and_cotangents(o["mom"], o["C"], self.C_ref.repeat(k + 1, 1), self.L_ref.repeat(k + 1, 1))
        per = loss.reshape(k + 1, 9).sum(dim=1)
        return per[0], (per[1:] - per[0]) / h

    def close(self):
        self.ad.close()
        if self.nd is not None:
            self.nd.close()


def iteration_times(ks, C_ref, L_ref, reps: int = 3):
    """Mean time of one optimizer iteration (gradient + Adam step) per k, adjoint vs forward differences."""
    import torch
    out = []
    for k in ks:
        fit = PolyFit(k, C_ref, L_ref)
        theta = torch.full((k,), 0.5, dtype=torch.float32, device=fit.dev)
        res = {"k": k}
        for name, fn in (("ad", fit.grad_ad), ("nd", fit.grad_nd)):
            warm = Adam(theta.clone(), lr=1e-2)   # warm-up: graph capture, first launch of every kernel
            _, g = fn(warm.w)
            warm.step(g)
            warm.w.clamp_(min=0.0)
            opt = Adam(theta.clone(), lr=1e-2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                _, g = fn(opt.w)
                opt.step(g)
                opt.w.clamp_(min=0.0)
            torch.cuda.synchronize()
            res[name + "_ms"] = 1e3 * (time.perf_counter() - t0) / reps
        fit.close()
        out.append(res)
    return out


def fit(k: int, C_ref, L_ref, iters: int = 100, lr: float = 1e-2, theta0=None):
    """Adam on theta with the adjoint gradient; returns (theta, loss history)."""
    import torch
    f = PolyFit(k, C_ref, L_ref, theta0=theta0, nd=False)
    th0 = np.full(k, 0.5) if theta0 is None else np.asarray(theta0)
    opt = Adam(torch.tensor(th0, dtype=torch.float32, device=f.dev), lr=lr)
    hist = []
    for _ in range(iters):
        loss, g = f.grad_ad(opt.w)
        hist.append(float(loss))
        opt.step(g)
        opt.w.clamp_(min=0.0)
    f.close()
    return opt.w, hist

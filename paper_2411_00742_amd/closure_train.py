"""Training through the differentiable solver: the learned closure and, for
comparison, the plain power law with shared kinetics.

Both fits minimise the same loss over the training simulations, the sum of
squared relative errors of the sampled moments mu_0..mu_3 and of the
concentration against measured trajectories (the residual sum of squares of
Sec. 4.1 / App. C, in relative form), with Adam (App. C).  Gradients come from
the library's discrete adjoint (pbe_grad); the closure's weight gradient and
the Adam step run in the library's kernels.  torch supplies device buffers
and the few elementwise operations that form the loss and its cotangents.
"""
from __future__ import annotations

import numpy as np

from . import Adam, MLP_NW, Solver
from . import workloads as W


def relative_loss(mom, C, mom_ref, C_ref, weight):
    """Per-sim weighted loss and its cotangents (torch tensors on the device).

    weight[s] scales sim s (0 excludes it); returns (loss, gmom, gC)."""
    rm = (mom - mom_ref) / mom_ref
    rc = (C - C_ref) / C_ref
    w = weight.reshape(-1, 1)
    loss = (w * (rm ** 2).sum(dim=2)).sum() + (w * rc ** 2).sum()
    gmom = 2.0 * w.unsqueeze(2) * rm / mom_ref
    gC = 2.0 * w * rc / C_ref
    return loss, gmom, gC


def per_sim_loss(mom, C, mom_ref, C_ref):
    rm = (mom - mom_ref) / mom_ref
    rc = (C - C_ref) / C_ref
    return (rm ** 2).sum(dim=(1, 2)) + (rc ** 2).sum(dim=1)


def generate_data(prob_truth):
    """Trajectories of the ground-truth law (the plain solver's output)."""
    s = Solver(prob_truth)
    o = s.solve()
    mom, C = o["mom"].clone(), o["C"].clone()
    s.close()
    return mom, C


def fit_closure(prob_mlp, mom_ref, C_ref, train, iters=200, lr=3e-3, ckpt_every=32, log=None):
    """Train the closure weights of prob_mlp (law LAW_MLP) on the sims where train is True.

    Returns (weights [MLP_NW] float32 device tensor, loss history)."""
    import torch
    s = Solver(prob_mlp, ckpt_every=ckpt_every)
    dev = s.device
    w = torch.tensor(np.asarray(prob_mlp.mlp[:MLP_NW], dtype=np.float32), device=dev)
    weight = torch.tensor(train.astype(np.float64) / max(int(train.sum()), 1), device=dev)
    opt = Adam(w, lr=lr)
    hist = []
    for it in range(iters):
        o = s.solve()
        loss, gmom, gC = relative_loss(o["mom"], o["C"], mom_ref, C_ref, weight)
        _, gw = s.grad(None, gmom, gC, with_mlp=True)
        opt.step(gw)
        s.set_mlp(w)
        hist.append(float(loss.item()))
        if log and (it % 20 == 0 or it == iters - 1):
            log(f"closure it {it}: loss {hist[-1]:.4e}")
    s.close()
    return w, hist


def fit_power_law(prob_plain, mom_ref, C_ref, train, iters=150, lr=0.05, ckpt_every=32, log=None):
    """Fit shared (kg, g, kb, b) of the power law (in log space, so they stay
    positive, the paper's only constraint) on the training sims."""
    import torch
    s = Solver(prob_plain, ckpt_every=ckpt_every)
    dev = s.device
    idx = [W.P_KG, W.P_G, W.P_KB, W.P_B]
    theta = torch.tensor(np.log(prob_plain.par[0, idx]), dtype=torch.float32, device=dev)
    weight = torch.tensor(train.astype(np.float64) / max(int(train.sum()), 1), device=dev)
    opt = Adam(theta, lr=lr)
    par = np.array(prob_plain.par, dtype=np.float64, copy=True)
    hist = []
    for it in range(iters):
        vals = np.exp(theta.cpu().numpy().astype(np.float64))
        par[:, idx] = vals
        s.set_par(par)
        o = s.solve()
        loss, gmom, gC = relative_loss(o["mom"], o["C"], mom_ref, C_ref, weight)
        gpar = s.grad(None, gmom, gC)
        # shared parameters: sum the per-sim gradients; chain rule to log space
        g = gpar[:, :4].sum(dim=0) * torch.tensor(vals, device=dev)
        opt.step(g)
        hist.append(float(loss.item()))
        if log and (it % 20 == 0 or it == iters - 1):
            log(f"power law it {it}: loss {hist[-1]:.4e}")
    vals = np.exp(theta.cpu().numpy().astype(np.float64))
    s.close()
    return vals, hist


def fit_arrhenius_fd(prob_arr, mom_ref, C_ref, train, iters=150, lr=0.05, h=1e-5, log=None):
    """Fit shared (kg, g, kb, b, Eg, Eb) of the Arrhenius law (App. A, Eq. (A.2): the power law
    times exp(-E/(T + 273.15)) for growth and nucleation) on the training sims.  The adjoint
    returns derivatives for (kg, g, kb, b, gamma) only, so all six come from batched central
    differences: one launch solves the 13 copies (base, +h, -h per parameter) of every training
    simulation.  Parameters at a reference temperature, where the rate constants decouple from
    the activation temperatures: theta = (ln kg_ref, g, ln kb_ref, b, Eg / 1000 K, Eb / 1000 K),
    kg = kg_ref exp(Eg / T_ref), kb = kb_ref exp(Eb / T_ref), T_ref = 30 degC."""
    import torch
    tr = np.flatnonzero(train)
    n = len(tr)
    base = prob_arr.subset(tr)
    copies = base.subset(np.tile(np.arange(n), 13))
    # an explicit step budget: the bound derived from the kinetics takes the Arrhenius factor as 1,
    # which the growing kg = kg_ref exp(Eg / T_ref) would soon exceed
    s = Solver(copies, max_steps=4 * int(np.ceil(prob_arr.t_end / prob_arr.dt_max)) + 64)
    dev = s.device
    idx = [W.P_KG, W.P_G, W.P_KB, W.P_B, W.P_EG, W.P_EB]

    Tref = 30.0 + 273.15

    def to_par(th):
        Eg, Eb = 1e3 * th[4], 1e3 * th[5]
        return np.array([np.exp(th[0] + Eg / Tref), th[1], np.exp(th[2] + Eb / Tref), th[3], Eg, Eb])

    p0 = prob_arr.par[0, idx]
    theta = torch.tensor([np.log(p0[0]) - p0[4] / Tref, p0[1], np.log(p0[2]) - p0[5] / Tref, p0[3], p0[4] / 1e3,
                          p0[5] / 1e3], dtype=torch.float32, device=dev)
    opt = Adam(theta, lr=lr)
    par = np.array(copies.par, dtype=np.float64, copy=True)
    mref, cref = mom_ref[torch.as_tensor(tr, device=mom_ref.device)], C_ref[torch.as_tensor(tr, device=C_ref.device)]
    hist = []
    for it in range(iters):
        th = theta.cpu().numpy().astype(np.float64)
        for b in range(13):
            tb = th.copy()
            if b > 0:
                tb[(b - 1) % 6] += h if b <= 6 else -h
            par[b * n:(b + 1) * n][:, idx] = to_par(tb)
        s.set_par(par)
        o = s.solve()
        per = per_sim_loss(o["mom"], o["C"], mref.repeat(13, 1, 1), cref.repeat(13, 1)).reshape(13, n).mean(dim=1)
        g = (per[1:7] - per[7:13]) / (2.0 * h)
        opt.step(g)
        hist.append(float(per[0].item()))
        if log and (it % 20 == 0 or it == iters - 1):
            log(f"arrhenius it {it}: loss {hist[-1]:.4e}")
    vals = to_par(theta.cpu().numpy().astype(np.float64))
    s.close()
    return vals, hist


def evaluate(prob, mom_ref, C_ref, mask):
    """Mean per-sim loss over the sims where mask is True."""
    import torch
    s = Solver(prob)
    o = s.solve()
    l = per_sim_loss(o["mom"], o["C"], mom_ref, C_ref)
    m = torch.tensor(mask, device=l.device)
    out = float(l[m].mean().item())
    s.close()
    return out

"""Host logic of the differentiable solve (no GPU): PBESolve.backward refuses to
differentiate a solve that a later forward on the same solver has replaced."""
import numpy as np
import pytest
import torch

import paper_2411_00742_amd as pbe


class FakeSolver:
    """Stands in for Solver on the CPU: the same generation bookkeeping, outputs that are
    linear in the parameters so the gradient is known."""

    def __init__(self, S=3):
        self.prob = type("P", (), {})()
        self.prob.par = np.ones((S, pbe.NPAR))
        self.generation = 0
        self.S = S

    def set_par(self, par):
        self.generation += 1
        self.par = par.copy()

    def solve(self):
        self.generation += 1
        p = torch.tensor(self.par[:, :pbe.NGRAD])
        return dict(f=p.sum(1).clone(), mom=p[:, :4].reshape(self.S, 1, 4).clone(), C=p[:, :1].clone())

    def grad(self, gf, gmom, gC):
        g = torch.zeros(self.S, pbe.NGRAD, dtype=torch.float64)
        g += gf[:, None]
        g[:, :4] += gmom.reshape(self.S, 4)
        g[:, 0] += gC.reshape(self.S)
        return g


def test_backward_of_the_current_solve():
    s = FakeSolver()
    par5 = torch.ones(3, pbe.NGRAD, dtype=torch.float64, requires_grad=True)
    f, mom, C = pbe.pbe_solve_autograd(par5, s)
    (g,) = torch.autograd.grad(f.sum() + mom.sum() + C.sum(), par5)
    want = torch.ones(3, pbe.NGRAD, dtype=torch.float64)
    want[:, :4] += 1
    want[:, 0] += 1
    assert torch.equal(g, want)


def test_backward_after_a_second_forward_is_refused():
    s = FakeSolver()
    par5 = torch.ones(3, pbe.NGRAD, dtype=torch.float64, requires_grad=True)
    f1, _, _ = pbe.pbe_solve_autograd(par5, s)
    f2, _, _ = pbe.pbe_solve_autograd(par5 * 2, s)
    with pytest.raises(RuntimeError, match="another solve"):
        torch.autograd.grad(f1.sum(), par5)
    (g,) = torch.autograd.grad(f2.sum(), par5)   # the latest solve is still differentiable
    assert torch.all(g == 2)

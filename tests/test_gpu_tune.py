"""The autotuner (pbe_tune): 1D launch shapes give bitwise-identical results
(each simulation runs the same code on one wavefront whatever the grid size),
2D tile lengths agree to rounding, the chosen shape is no slower than the
default in its own trial, and the per-process cache returns the choice
without timing."""
import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W

pytestmark = pytest.mark.gpu


def outputs(s):
    return {k: v.cpu().numpy() for k, v in s.solve().items()}


def test_tuned_1d_launch_gives_identical_results(torch_cuda):
    import paper_2411_00742_amd as pbe
    prob = W.batched(n_sims=300, n_lo=64, n_hi=2048, t_end=300.0, n_samples=3)
    s = pbe.Solver(prob)
    a = outputs(s)
    t = s.tune()
    print("1D tuning", t)
    assert t["n_candidates"] == 4 and t["best_ms"] <= t["default_ms"] * 1.0001
    b = outputs(s)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    again = s.tune(use_cache=True)
    assert again["n_candidates"] == 0 and again["blocks"] == t["blocks"]
    s.close()
    s2 = pbe.Solver(prob, autotune=True)
    c = outputs(s2)
    s2.close()
    for k in a:
        assert np.array_equal(a[k], c[k]), k


def test_tuned_2d_tiles_give_identical_results(torch_cuda):
    import paper_2411_00742_amd as pbe
    prob = W.shape_2d(n_sims=3, n_lo=100, n_hi=300, t_end=120.0, n_samples=2)
    s = pbe.Solver(prob)
    a = outputs(s)
    t = s.tune(trial_steps=10)
    print("2D tuning", t)
    assert t["n_candidates"] == 4 and t["seg_2d"] in (64, 128, 256, 512)
    b = outputs(s)
    # the column blocks group the moment partial sums, so another tile length
    # changes mu_12 (and through C everything else) at rounding level only
    assert np.array_equal(a["steps"], b["steps"]) and np.array_equal(a["status"], b["status"])
    assert np.abs(a["f"] - b["f"]).max() <= 1e-12 * np.abs(a["f"]).max()
    np.testing.assert_allclose(b["mom"], a["mom"], rtol=1e-12)
    np.testing.assert_allclose(b["C"], a["C"], rtol=1e-13)
    s.close()

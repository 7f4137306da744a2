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


@pytest.mark.skip(reason="an earlier form of the 1D autotuner (graph-captured trials with wave-pair candidates) "
                         "crashed the host process inside the HIP runtime (SIGSEGV in pbe_tune, no GPU fault); the "
                         "cause has not been shown, so 1D tuning returns PBE_EUNSUPPORTED and this case stays off "
                         "the GPU")
def test_tuned_1d_launch_gives_identical_results(torch_cuda):
    import paper_2411_00742_amd as pbe
    prob = W.batched(n_sims=300, n_lo=64, n_hi=2048, t_end=300.0, n_samples=3)
    s = pbe.Solver(prob)
    a = outputs(s)
    t = s.tune()
    print("1D tuning", t)
    assert t["n_candidates"] == 4 and t["best_ms"] <= t["default_ms"] * 1.0001
    b = outputs(s)
    same_partition_as_default(a, b, t["pair_long"])
    again = s.tune(use_cache=True)
    assert again["n_candidates"] == 0 and again["blocks"] == t["blocks"]
    s.close()
    s2 = pbe.Solver(prob, autotune=True)
    c = outputs(s2)
    s2.close()
    same_partition_as_default(a, c, t["pair_long"])


def test_1d_tuning_is_switched_off(torch_cuda):
    """pbe_tune and PBE_FLAG_AUTOTUNE refuse 1D handles (before any device work)."""
    import paper_2411_00742_amd as pbe
    prob = W.batched(n_sims=4, n_lo=64, n_hi=300, t_end=60.0, n_samples=2)
    s = pbe.Solver(prob)
    with pytest.raises(pbe.PBEError) as e:
        s.tune()
    assert e.value.code == pbe.PBE_EUNSUPPORTED
    a = outputs(s)                         # the handle is unaffected
    s.set_launch(blocks=(8, 8, 8, 8))      # shapes are still applied without timing
    b = outputs(s)
    same_partition_as_default(a, b, False)
    s.close()
    with pytest.raises(pbe.PBEError) as e:
        pbe.Solver(prob, autotune=True)
    assert e.value.code == pbe.PBE_EUNSUPPORTED


def same_partition_as_default(a, b, pairs):
    """One wavefront per sim: bitwise equal whatever the grid size.  Wave pairs sum the
    moments in two halves, so those sims agree to rounding."""
    if not pairs:
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        return
    assert np.array_equal(a["steps"], b["steps"]) and np.array_equal(a["status"], b["status"])
    np.testing.assert_allclose(b["mom"], a["mom"], rtol=1e-12)
    np.testing.assert_allclose(b["C"], a["C"], rtol=1e-13)


def test_wave_pairs_match_oracle(torch_cuda, oracle):
    """Grids over 1024 cells on wave pairs (K = ceil(N/128) per lane) against the oracle."""
    import paper_2411_00742_amd as pbe
    sizes = [1025, 1100, 1151, 1279, 1280, 1281, 1500, 1536, 1537, 1791, 1999, 2047, 2048, 64, 700]
    base = W.batched(n_sims=len(sizes), n_lo=200, n_hi=300, t_end=240.0, n_samples=3)
    seeds = [W.gaussian_seed_1d(n, 1000.0, 200.0, 30.0, 1e9) for n in sizes]
    prob = base.with_(n_cells=np.array(sizes, dtype=np.int32), f0=np.concatenate(seeds))
    prob.C0[:] = W.csat_linear(40.0) * 1.15
    s = pbe.Solver(prob)
    s.set_launch(pair_long=True)
    o = outputs(s)
    s.set_launch(pair_long=False)
    single = outputs(s)
    s.close()
    off = prob.offsets()
    for i in range(prob.n_sims):
        r = oracle.solve1d(prob, i)
        assert int(o["steps"][i]) == r["steps"] and int(o["status"][i]) == r["status"]
        f = o["f"][off[i]:off[i + 1]]
        assert np.abs(f - r["f_final"]).max() <= 1e-10 * np.abs(r["f_final"]).max()
        np.testing.assert_allclose(o["mom"][i], r["mom"], rtol=1e-10)
        np.testing.assert_allclose(o["C"][i], r["C"], rtol=1e-10)
    same_partition_as_default(single, o, True)


def test_tuned_2d_tiles_give_identical_results(torch_cuda):
    import paper_2411_00742_amd as pbe
    prob = W.shape_2d(n_sims=3, n_lo=100, n_hi=300, t_end=120.0, n_samples=2)
    s = pbe.Solver(prob)
    a = outputs(s)
    t = s.tune(trial_steps=10)
    print("2D tuning", t)
    assert t["n_candidates"] == 4 and t["seg_2d"] in (32, 64, 128, 256)
    b = outputs(s)
    # the column blocks group the moment partial sums, so another tile length
    # changes mu_12 (and through C everything else) at rounding level only
    assert np.array_equal(a["steps"], b["steps"]) and np.array_equal(a["status"], b["status"])
    assert np.abs(a["f"] - b["f"]).max() <= 1e-12 * np.abs(a["f"]).max()
    np.testing.assert_allclose(b["mom"], a["mom"], rtol=1e-12)
    np.testing.assert_allclose(b["C"], a["C"], rtol=1e-13)
    s.close()

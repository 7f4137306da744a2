"""pbe_mlp_vjp_noalloc (the closure weight gradient without device allocation)
against pbe_mlp_vjp, called through the C ABI: two calls in a row, the second on
fewer rows, in both precisions.  The two entry points run the same kernels with
the same tiling, so the results are compared bitwise; sizes beyond the scratch
limit are refused on the host."""
import ctypes as C

import numpy as np
import pytest

from paper_2411_00742_amd import workloads as W

pytestmark = pytest.mark.gpu


def blob():
    b = W.closure_net(seed_offset=5, out_gain=0.5)
    o, H = W.MLP_OFF, W.MLP_H
    b[o["b1"]:o["b1"] + H] = np.linspace(-0.2, 0.25, H)
    b[o["b2"]:o["b2"] + H] = np.linspace(0.15, -0.1, H)
    return b


def call(name, bl, prec, z, yb):
    import torch
    import paper_2411_00742_amd as pbe
    zt = torch.tensor(z, dtype=torch.float64, device="cuda").contiguous()
    yt = torch.tensor(yb, dtype=torch.float64, device="cuda").contiguous()
    gw = torch.full((W.MLP_NW,), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    b = np.ascontiguousarray(bl, dtype=np.float32)
    rc = getattr(pbe.lib(), name)(b.ctypes.data_as(C.POINTER(C.c_float)), prec, z.shape[0],
                                  C.c_void_p(zt.data_ptr()), C.c_void_p(yt.data_ptr()), C.c_void_p(gw.data_ptr()),
                                  C.c_void_p(st.cuda_stream))
    return rc, gw.cpu().numpy()


@pytest.mark.parametrize("prec", [W.MLP_BF16, W.MLP_FP64])
def test_noalloc_matches_allocating_entry_point(torch_cuda, prec):
    import paper_2411_00742_amd as pbe
    rng = np.random.default_rng(5)
    bl = blob()
    for n in (4096, 333):      # the second call is smaller: nothing of the first may leak into it
        z = rng.uniform(-1.5, 1.5, size=(n, 3))
        yb = rng.normal(size=(n, 2))
        rc_a, a = call("pbe_mlp_vjp", bl, prec, z, yb)
        rc_b, b = call("pbe_mlp_vjp_noalloc", bl, prec, z, yb)
        assert rc_a == pbe.PBE_OK and rc_b == pbe.PBE_OK, (rc_a, rc_b)
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), (n, np.max(np.abs(a - b)))


def test_noalloc_refuses_more_rows_than_its_scratch(torch_cuda):
    import paper_2411_00742_amd as pbe
    n = pbe.MLP_VJP_NOALLOC_MAX_ROWS + 1
    z = np.zeros((n, 3))
    yb = np.zeros((n, 2))
    rc, g = call("pbe_mlp_vjp_noalloc", blob(), W.MLP_BF16, z, yb)
    assert rc == pbe.PBE_EINVAL
    assert np.all(np.isnan(g))   # nothing was launched

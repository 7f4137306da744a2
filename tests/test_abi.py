"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/pbe.h, and rejects invalid problems on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2411_00742_amd as pbe
from paper_2411_00742_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(pbe_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_entry_point():
    L = pbe.lib()
    decl = declared_entry_points()
    assert set(decl) == set(pbe.EXPORTS), decl
    for name in decl:
        assert hasattr(L, name), name


def test_strerror_and_null_destroy():
    L = pbe.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, 17):
        assert isinstance(L.pbe_strerror(code), bytes)
    assert L.pbe_strerror(-1) == b"invalid argument"
    L.pbe_destroy(None)


def _create_rc(prob, **kw):
    st, keep = pbe.make_problem_struct(prob, **kw)
    h = C.c_void_p()
    rc = pbe.lib().pbe_create(C.byref(st), None, C.byref(h))
    assert not h.value
    return rc


def _mutations():
    base = W.batched(3, 200, 300, t_end=100.0, n_samples=2)
    out = []

    def m(name, **kw):
        out.append((name, base.with_(**kw)))

    m("n_cells too small", n_cells=np.array([3, 200, 250], dtype=np.int32),
      f0=np.concatenate([np.ones(3), base.f0[:450]]))
    m("n_cells too large", n_cells=np.array([2049, 200, 250], dtype=np.int32),
      f0=np.concatenate([np.ones(2049), np.ones(450)]))
    f = base.f0.copy(); f[5] = np.nan
    m("nan in f0", f0=f)
    f = base.f0.copy(); f[7] = -1.0
    m("negative f0", f0=f)
    m("unsorted samples", t_samples=np.array([60.0, 50.0]))
    m("sample beyond t_end", t_samples=np.array([50.0, 150.0]))
    m("zero sample time", t_samples=np.array([0.0, 50.0]))
    m("cfl above one", cfl=1.5)
    m("cfl zero", cfl=0.0)
    m("dt_max zero", dt_max=0.0)
    m("t_end negative", t_end=-1.0)
    par = base.par.copy(); par[1, W.P_KG] = -1e-7
    m("negative kg", par=par)
    par = base.par.copy(); par[0, W.P_G] = 0.0
    m("zero growth exponent", par=par)
    par = base.par.copy(); par[2, W.P_GAMMA] = -1e-3
    m("negative gamma", par=par)
    m("zero C0", C0=np.array([0.18, 0.0, 0.18]))
    m("bad law", law=7)
    m("bad scheme", scheme=3)
    m("negative alpha", alpha=-1.0)
    m("solubility non-positive", cs0=-1.0)
    par = base.par.copy(); par[1, W.P_KD] = -1e-7
    m("negative kd", par=par)
    par = base.par.copy(); par[0, W.P_KD] = 1e-7; par[0, W.P_D] = 0.0
    m("zero dissolution exponent", par=par)
    return out


@pytest.mark.parametrize("name,prob", _mutations(), ids=[n for n, _ in _mutations()])
def test_invalid_problems_rejected_on_host(name, prob):
    assert _create_rc(prob) == pbe.PBE_EINVAL, name


def test_invalid_flags_and_counts():
    base = W.batched(2, 200, 300, t_end=100.0, n_samples=2)
    st, keep = pbe.make_problem_struct(base)
    st.flags = 1 << 5
    h = C.c_void_p()
    assert pbe.lib().pbe_create(C.byref(st), None, C.byref(h)) == pbe.PBE_EINVAL
    st, keep = pbe.make_problem_struct(base)
    st.n_sims = 0
    assert pbe.lib().pbe_create(C.byref(st), None, C.byref(h)) == pbe.PBE_EINVAL
    assert pbe.lib().pbe_create(None, None, C.byref(h)) == pbe.PBE_EINVAL
    st, keep = pbe.make_problem_struct(base, ckpt_every=-1)
    assert pbe.lib().pbe_create(C.byref(st), None, C.byref(h)) == pbe.PBE_EINVAL


def test_null_handle_calls_are_rejected():
    L = pbe.lib()
    assert L.pbe_step(None, 1, None) == pbe.PBE_EINVAL
    assert L.pbe_solve(None, None, None, None, None, None) == pbe.PBE_EINVAL
    assert L.pbe_fetch(None, None, None, None, None, None) == pbe.PBE_EINVAL
    assert L.pbe_grad(None, None, None, None, None, None) == pbe.PBE_EINVAL
    assert L.pbe_reset(None) == pbe.PBE_EINVAL
    assert L.pbe_set_par(None, None) == pbe.PBE_EINVAL


def test_gradient_options_rejected_on_host():
    base = W.batched(2, 200, 300, t_end=100.0, n_samples=2)
    assert _create_rc(base.with_(scheme=W.SCHEME_LW_TVD), ckpt_every=16) == pbe.PBE_EUNSUPPORTED
    big = W.batched(2, 1500, 1600, t_end=100.0, n_samples=2)
    assert _create_rc(big, ckpt_every=16) == pbe.PBE_EUNSUPPORTED
    # the 2D split solver is forward-only and records moments, not densities
    two = W.shape_2d(2, 16, 24, t_end=100.0, n_samples=2)
    assert _create_rc(two, ckpt_every=16) == pbe.PBE_EUNSUPPORTED
    assert _create_rc(two, record_f=True) == pbe.PBE_EUNSUPPORTED
    assert _create_rc(two, record_rates=True) == pbe.PBE_EUNSUPPORTED


def test_dissolution_options_rejected_on_host():
    """Dissolution runs the plain laws forward in 1D: no adjoint, no 2D, no other law."""
    dis = W.dissolution(3, 100, 300)
    assert _create_rc(dis, ckpt_every=16) == pbe.PBE_EUNSUPPORTED
    assert _create_rc(dis.with_(law=W.LAW_POLY, poly=np.ones((3, 2)))) == pbe.PBE_EUNSUPPORTED
    two = W.shape_2d(2, 16, 24, t_end=100.0, n_samples=2)
    par = two.par.copy(); par[1, W.P_KD] = 1e-7
    assert _create_rc(two.with_(par=par)) == pbe.PBE_EUNSUPPORTED


def test_strang_is_a_2d_option():
    one = W.batched(2, 200, 300, t_end=100.0, n_samples=2).with_(splitting=W.SPLIT_STRANG)
    assert _create_rc(one) == pbe.PBE_EUNSUPPORTED

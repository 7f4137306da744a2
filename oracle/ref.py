"""ctypes wrapper of the FP64 CPU oracle (libpbe_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and
by the benchmark's CPU-baseline leg.  The solver package never imports it.

Inputs are `Problem` objects from the seeded workload module; outputs are
numpy arrays.  See pbe_oracle.h for the meaning of every field.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbe_oracle.so")
SOURCES = [os.path.join(HERE, "pbe_oracle.cpp")]
NPAR = 15
NTAN = 5
DT_DIFF, DT_FROZEN = 0, 1
MLP_NC = 18

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
           "-Wall", "-o", LIB_PATH + ".tmp"] + SOURCES
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Process(C.Structure):
    _fields_ = [("law", C.c_int32), ("scheme", C.c_int32), ("sol_law", C.c_int32), ("mlp_precision", C.c_int32),
                ("cs0", C.c_double), ("cs1", C.c_double), ("alpha", C.c_double),
                ("cfl", C.c_double), ("dt_max", C.c_double), ("t_end", C.c_double),
                ("mlp", C.POINTER(C.c_float)), ("splitting", C.c_int32)]


class Sim1D(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_samples", C.c_int32), ("max_steps", C.c_int32), ("n_replay", C.c_int32),
                ("n_rates_replay", C.c_int32),
                ("L_max", C.c_double), ("C0", C.c_double),
                ("f0", _dp), ("par", _dp), ("t_samples", _dp), ("dt_replay", _dp),
                ("G0_replay", _dp), ("B_replay", _dp), ("n_poly", C.c_int32), ("poly", _dp),
                ("f_samples", _dp), ("mom", _dp), ("C", _dp), ("f_final", _dp), ("dt_log", _dp),
                ("G0_log", _dp), ("B_log", _dp),
                ("steps", _ip), ("status", _ip),
                ("C_final", _dp), ("t_final", _dp), ("outflow", _dp), ("corr", _dp)]


class Sim2D(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n_samples", C.c_int32), ("max_steps", C.c_int32),
                ("L1_max", C.c_double), ("L2_max", C.c_double), ("C0", C.c_double),
                ("f0", _dp), ("par", _dp), ("t_samples", _dp),
                ("mom", _dp), ("C", _dp), ("f_final", _dp), ("dt_log", _dp),
                ("steps", _ip), ("status", _ip),
                ("C_final", _dp), ("t_final", _dp), ("outflow", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.ref_phi_vanleer.restype = C.c_double
        L.ref_phi_vanleer.argtypes = [C.c_double]
        L.ref_limited_slope.restype = C.c_double
        L.ref_limited_slope.argtypes = [C.c_double, C.c_double]
        L.ref_solve1d.argtypes = [C.POINTER(Process), C.POINTER(Sim1D)]
        L.ref_solve1d_batch.argtypes = [C.POINTER(Process), C.POINTER(Sim1D), C.c_int32, C.c_int32]
        L.ref_tangent1d.argtypes = [C.POINTER(Process), C.POINTER(Sim1D), C.c_int32, _dp, _dp, _dp]
        L.ref_solve2d.argtypes = [C.POINTER(Process), C.POINTER(Sim2D)]
        L.ref_solve2d_batch.argtypes = [C.POINTER(Process), C.POINTER(Sim2D), C.c_int32, C.c_int32]
        L.ref_mom1d.argtypes = [C.POINTER(Process), _dp, C.c_double, _dp, C.c_int32, _dp, C.c_double, C.c_double,
                                _dp, _dp]
        L.ref_mom2d.argtypes = L.ref_mom1d.argtypes
        L.ref_dual_example.argtypes = [C.c_double, C.c_double, _dp]
        L.ref_bf16.restype = C.c_double
        L.ref_bf16.argtypes = [C.c_double]
        _fp = C.POINTER(C.c_float)
        L.ref_mlp_forward.argtypes = [_fp, C.c_int32, C.c_int32, _dp, _dp, _dp]
        L.ref_mlp_vjp.argtypes = [_fp, C.c_int32, C.c_int32, _dp, _dp, _dp]
        L.ref_tangent1d_mlp.argtypes = [C.POINTER(Process), C.POINTER(Sim1D), C.c_int32, _dp, _dp, _dp, _dp]
        L.ref_tangent1d_poly.argtypes = [C.POINTER(Process), C.POINTER(Sim1D), C.c_int32, _dp, _dp, _dp, _dp]
        L.ref_tangent1d_corr.argtypes = [C.POINTER(Process), C.POINTER(Sim1D), C.c_int32, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    return a.ctypes.data_as(_dp)


def process_of(prob) -> Process:
    """Process struct for a Problem; for the closure law it points into prob.mlp (kept alive by prob)."""
    mlp = None
    if getattr(prob, "mlp", None) is not None:
        assert prob.mlp.dtype == np.float32 and prob.mlp.flags.c_contiguous
        mlp = prob.mlp.ctypes.data_as(C.POINTER(C.c_float))
    return Process(law=prob.law, scheme=prob.scheme, sol_law=prob.sol_law,
                   mlp_precision=int(getattr(prob, "mlp_precision", 0)), cs0=prob.cs0, cs1=prob.cs1,
                   alpha=prob.alpha, cfl=prob.cfl, dt_max=prob.dt_max, t_end=prob.t_end, mlp=mlp,
                   splitting=int(getattr(prob, "splitting", 0)))


def phi_vanleer(theta: float) -> float:
    return lib().ref_phi_vanleer(theta)


def limited_slope(a: float, b: float) -> float:
    return lib().ref_limited_slope(a, b)


def dual_example(x1: float, x2: float) -> np.ndarray:
    out = np.zeros(6)
    lib().ref_dual_example(x1, x2, _ptr(out))
    return out


class _Sim1DBuffers:
    """Owns the numpy arrays a Sim1D struct points into."""

    def __init__(self, prob, s, record_f, max_steps, dt_replay, log_steps, rates_replay=None):
        n = int(prob.n_cells[s])
        ns = len(prob.t_samples)
        self.f0 = np.ascontiguousarray(prob.f0_of(s), dtype=np.float64)
        self.par = np.ascontiguousarray(prob.par[s], dtype=np.float64)
        self.ts = np.ascontiguousarray(prob.t_samples, dtype=np.float64)
        self.replay = None if dt_replay is None else np.ascontiguousarray(dt_replay, dtype=np.float64)
        if rates_replay is None:
            self.G0r = self.Br = None
        else:
            self.G0r = np.ascontiguousarray(rates_replay[0], dtype=np.float64)
            self.Br = np.ascontiguousarray(rates_replay[1], dtype=np.float64)
            assert self.G0r.shape == self.Br.shape
        poly = getattr(prob, "poly", None)
        self.poly = None if poly is None else np.ascontiguousarray(poly[s], dtype=np.float64)
        corr = getattr(prob, "corr", None)
        self.corr = None if corr is None else np.ascontiguousarray(corr[s], dtype=np.float64)
        self.f_samples = np.zeros((ns, n)) if record_f else None
        self.mom = np.zeros((ns, 4))
        self.C = np.zeros(ns)
        self.f_final = np.zeros(n)
        cap = log_steps if log_steps else 0
        self.dt_log = np.zeros(cap) if cap else None
        self.G0_log = np.zeros(cap) if cap else None
        self.B_log = np.zeros(cap) if cap else None
        self.steps = np.zeros(1, dtype=np.int32)
        self.status = np.zeros(1, dtype=np.int32)
        self.C_final = np.zeros(1)
        self.t_final = np.zeros(1)
        self.outflow = np.zeros(1)
        ms = max_steps if max_steps else 0
        if cap and (ms == 0 or ms > cap):
            ms = cap
        self.struct = Sim1D(n=n, n_samples=ns, max_steps=ms,
                            n_replay=0 if self.replay is None else len(self.replay),
                            n_rates_replay=0 if self.G0r is None else len(self.G0r),
                            L_max=float(prob.L_max[s]), C0=float(prob.C0[s]),
                            f0=_ptr(self.f0), par=_ptr(self.par), t_samples=_ptr(self.ts),
                            dt_replay=_ptr(self.replay), G0_replay=_ptr(self.G0r), B_replay=_ptr(self.Br),
                            n_poly=0 if self.poly is None else len(self.poly), poly=_ptr(self.poly),
                            f_samples=_ptr(self.f_samples), mom=_ptr(self.mom),
                            C=_ptr(self.C), f_final=_ptr(self.f_final), dt_log=_ptr(self.dt_log),
                            G0_log=_ptr(self.G0_log), B_log=_ptr(self.B_log),
                            steps=_ptr(self.steps), status=_ptr(self.status), C_final=_ptr(self.C_final),
                            t_final=_ptr(self.t_final), outflow=_ptr(self.outflow), corr=_ptr(self.corr))

    def result(self) -> dict:
        st = int(self.steps[0])
        r = dict(mom=self.mom, C=self.C, f_final=self.f_final, steps=st, status=int(self.status[0]),
                 C_final=float(self.C_final[0]), t_final=float(self.t_final[0]), outflow=float(self.outflow[0]))
        if self.f_samples is not None:
            r["f_samples"] = self.f_samples
        if self.dt_log is not None:
            r["dt"] = self.dt_log[:st].copy()
            r["G0"] = self.G0_log[:st].copy()
            r["B"] = self.B_log[:st].copy()
        return r


DEFAULT_LOG = 400000


def solve1d(prob, s: int = 0, record_f: bool = False, max_steps: int | None = None, dt_replay=None,
            log_steps: int = DEFAULT_LOG, rates_replay=None) -> dict:
    """Run one 1D simulation of `prob` on the CPU; returns samples and final state.

    rates_replay = (G0[steps], B[steps]): use these rates at the first steps instead of the law."""
    assert prob.ndim == 1
    buf = _Sim1DBuffers(prob, s, record_f, max_steps, dt_replay, log_steps, rates_replay)
    p = process_of(prob)
    rc = lib().ref_solve1d(C.byref(p), C.byref(buf.struct))
    if rc != 0:
        raise RuntimeError(f"ref_solve1d failed ({rc})")
    return buf.result()


def solve1d_batch(prob, idx=None, n_threads: int = 0, record_f: bool = False, max_steps: int | None = None,
                  log_steps: int = 0):
    """Run several sims over a thread pool. Returns (list of result dicts, threads used)."""
    idx = range(prob.n_sims) if idx is None else idx
    bufs = [_Sim1DBuffers(prob, int(s), record_f, max_steps, None, log_steps) for s in idx]
    arr = (Sim1D * len(bufs))(*[b.struct for b in bufs])
    p = process_of(prob)
    used = lib().ref_solve1d_batch(C.byref(p), arr, len(bufs), n_threads)
    # copy back scalar outputs written through the array copy of the structs (pointers are shared)
    return [b.result() for b in bufs], used


def tangent1d(prob, s: int = 0, with_f: bool = True, max_steps: int | None = None, frozen_dt: bool = False):
    """Forward-mode derivatives of the samples w.r.t. (kg, g, kb, b, gamma).

    frozen_dt=False differentiates the step sizes in the branch each step takes (see
    pbe_oracle.h); True replays the primal run's step sizes as constants.
    Returns dict with dF [ns, n, 5] (if with_f), dM [ns, 4, 5], dC [ns, 5].
    """
    buf = _Sim1DBuffers(prob, s, False, max_steps, None, 0)
    n = int(prob.n_cells[s])
    ns = len(prob.t_samples)
    dF = np.zeros((ns, n, NTAN)) if with_f else None
    dM = np.zeros((ns, 4, NTAN))
    dC = np.zeros((ns, NTAN))
    p = process_of(prob)
    rc = lib().ref_tangent1d(C.byref(p), C.byref(buf.struct), DT_FROZEN if frozen_dt else DT_DIFF, _ptr(dF),
                             _ptr(dM), _ptr(dC))
    if rc != 0:
        raise RuntimeError(f"ref_tangent1d failed ({rc})")
    out = dict(dM=dM, dC=dC)
    if with_f:
        out["dF"] = dF
    return out


class _Sim2DBuffers:
    def __init__(self, prob, s, max_steps, log_steps):
        n1, n2 = int(prob.n_cells[s, 0]), int(prob.n_cells[s, 1])
        ns = len(prob.t_samples)
        self.f0 = np.ascontiguousarray(prob.f0_of(s), dtype=np.float64)
        self.par = np.ascontiguousarray(prob.par[s], dtype=np.float64)
        self.ts = np.ascontiguousarray(prob.t_samples, dtype=np.float64)
        self.mom = np.zeros((ns, 4))
        self.C = np.zeros(ns)
        self.f_final = np.zeros((n2, n1))
        self.dt_log = np.zeros(log_steps) if log_steps else None
        self.steps = np.zeros(1, dtype=np.int32)
        self.status = np.zeros(1, dtype=np.int32)
        self.C_final = np.zeros(1)
        self.t_final = np.zeros(1)
        self.outflow = np.zeros(1)
        ms = max_steps if max_steps else 0
        if log_steps and (ms == 0 or ms > log_steps):
            ms = log_steps
        self.struct = Sim2D(n1=n1, n2=n2, n_samples=ns, max_steps=ms, L1_max=float(prob.L_max[s, 0]),
                            L2_max=float(prob.L_max[s, 1]), C0=float(prob.C0[s]), f0=_ptr(self.f0),
                            par=_ptr(self.par), t_samples=_ptr(self.ts), mom=_ptr(self.mom), C=_ptr(self.C),
                            f_final=_ptr(self.f_final), dt_log=_ptr(self.dt_log), steps=_ptr(self.steps),
                            status=_ptr(self.status), C_final=_ptr(self.C_final), t_final=_ptr(self.t_final),
                            outflow=_ptr(self.outflow))

    def result(self):
        st = int(self.steps[0])
        r = dict(mom=self.mom, C=self.C, f_final=self.f_final, steps=st, status=int(self.status[0]),
                 C_final=float(self.C_final[0]), t_final=float(self.t_final[0]), outflow=float(self.outflow[0]))
        if self.dt_log is not None:
            r["dt"] = self.dt_log[:st].copy()
        return r


def solve2d(prob, s: int = 0, max_steps: int | None = None, log_steps: int = DEFAULT_LOG) -> dict:
    assert prob.ndim == 2
    buf = _Sim2DBuffers(prob, s, max_steps, log_steps)
    p = process_of(prob)
    rc = lib().ref_solve2d(C.byref(p), C.byref(buf.struct))
    if rc != 0:
        raise RuntimeError(f"ref_solve2d failed ({rc})")
    return buf.result()


def solve2d_batch(prob, idx=None, n_threads: int = 0, max_steps: int | None = None):
    idx = range(prob.n_sims) if idx is None else idx
    bufs = [_Sim2DBuffers(prob, int(s), max_steps, 0) for s in idx]
    arr = (Sim2D * len(bufs))(*[b.struct for b in bufs])
    p = process_of(prob)
    used = lib().ref_solve2d_batch(C.byref(p), arr, len(bufs), n_threads)
    return [b.result() for b in bufs], used


def mom1d(prob, s: int, mu_init, t_samples=None, rtol: float = 1e-12, atol: float = 1e-30):
    ts = np.ascontiguousarray(prob.t_samples if t_samples is None else t_samples, dtype=np.float64)
    mu0 = np.ascontiguousarray(mu_init, dtype=np.float64)
    par = np.ascontiguousarray(prob.par[s], dtype=np.float64)
    mu = np.zeros((len(ts), 4))
    Cq = np.zeros(len(ts))
    p = process_of(prob)
    rc = lib().ref_mom1d(C.byref(p), _ptr(par), float(prob.C0[s]), _ptr(mu0), len(ts), _ptr(ts), rtol, atol,
                         _ptr(mu), _ptr(Cq))
    if rc != 0:
        raise RuntimeError("ref_mom1d did not converge")
    return mu, Cq


def mom2d(prob, s: int, mu_init, t_samples=None, rtol: float = 1e-12, atol: float = 1e-30):
    ts = np.ascontiguousarray(prob.t_samples if t_samples is None else t_samples, dtype=np.float64)
    mu0 = np.ascontiguousarray(mu_init, dtype=np.float64)
    par = np.ascontiguousarray(prob.par[s], dtype=np.float64)
    mu = np.zeros((len(ts), 6))
    Cq = np.zeros(len(ts))
    p = process_of(prob)
    rc = lib().ref_mom2d(C.byref(p), _ptr(par), float(prob.C0[s]), _ptr(mu0), len(ts), _ptr(ts), rtol, atol,
                         _ptr(mu), _ptr(Cq))
    if rc != 0:
        raise RuntimeError("ref_mom2d did not converge")
    return mu, Cq


def _blob(w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    return w, w.ctypes.data_as(C.POINTER(C.c_float))


def mlp_forward(blob, precision: int, x, with_jac: bool = False):
    """Closure network on raw inputs x[n, 3] = (S, T, log10 mu_2): y[n, 2] (and dy/dz [n, 2, 3])."""
    w, wp = _blob(blob)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    n = x.shape[0]
    y = np.zeros((n, 2))
    dy = np.zeros((n, 2, 3)) if with_jac else None
    rc = lib().ref_mlp_forward(wp, precision, n, _ptr(x), _ptr(y), _ptr(dy))
    assert rc == 0
    return (y, dy) if with_jac else y


def mlp_vjp(blob, precision: int, z, ybar):
    """Weight gradient of sum_r ybar[r] . y(z[r]) for normalised inputs z[n, 3]."""
    w, wp = _blob(blob)
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 3)
    ybar = np.ascontiguousarray(ybar, dtype=np.float64).reshape(-1, 2)
    g = np.zeros(4546)
    rc = lib().ref_mlp_vjp(wp, precision, z.shape[0], _ptr(z), _ptr(ybar), _ptr(g))
    assert rc == 0
    return g


def tangent1d_mlp(prob, s: int, v, with_f: bool = True, max_steps: int | None = None, frozen_dt: bool = False):
    """Closure-law solve: derivatives along the weight direction v (tangent 0) and gamma (tangent 1)."""
    n, ns = int(prob.n_cells[s]), len(prob.t_samples)
    b = _Sim1DBuffers(prob, s, False, max_steps, None, 0)
    st = b.struct
    v = np.ascontiguousarray(v, dtype=np.float64)
    dF = np.zeros((ns, n, 2)) if with_f else None
    dM = np.zeros((ns, 4, 2))
    dC = np.zeros((ns, 2))
    p = process_of(prob)
    rc = lib().ref_tangent1d_mlp(C.byref(p), C.byref(st), DT_FROZEN if frozen_dt else DT_DIFF, _ptr(v), _ptr(dF),
                                 _ptr(dM), _ptr(dC))
    assert rc == 0, rc
    return dict(dF=dF, dM=dM, dC=dC)


def bf16(x: float) -> float:
    return lib().ref_bf16(float(x))


def tangent1d_poly(prob, s: int, v, with_f: bool = True, max_steps: int | None = None, frozen_dt: bool = False):
    """Polynomial growth law: derivatives along the coefficient direction v (tangent 0) and gamma
    (tangent 1).  Returns dict with dF [ns, n, 2] (if with_f), dM [ns, 4, 2], dC [ns, 2]."""
    buf = _Sim1DBuffers(prob, s, False, max_steps, None, 0)
    n, ns = int(prob.n_cells[s]), len(prob.t_samples)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert buf.poly is not None and v.shape == buf.poly.shape
    dF = np.zeros((ns, n, 2)) if with_f else None
    dM = np.zeros((ns, 4, 2))
    dC = np.zeros((ns, 2))
    p = process_of(prob)
    rc = lib().ref_tangent1d_poly(C.byref(p), C.byref(buf.struct), DT_FROZEN if frozen_dt else DT_DIFF, _ptr(v),
                                  _ptr(dF), _ptr(dM), _ptr(dC))
    if rc != 0:
        raise RuntimeError(f"ref_tangent1d_poly failed ({rc})")
    out = dict(dM=dM, dC=dC)
    if with_f:
        out["dF"] = dF
    return out


def tangent1d_corr(prob, s: int, v, with_f: bool = True, max_steps: int | None = None, frozen_dt: bool = False):
    """In-the-loop correction: derivatives along the weight direction v (tangent 0) and gamma
    (tangent 1).  Returns dict with dF [ns, n, 2] (if with_f), dM [ns, 4, 2], dC [ns, 2]."""
    buf = _Sim1DBuffers(prob, s, False, max_steps, None, 0)
    n, ns = int(prob.n_cells[s]), len(prob.t_samples)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert buf.corr is not None and v.shape == buf.corr.shape
    dF = np.zeros((ns, n, 2)) if with_f else None
    dM = np.zeros((ns, 4, 2))
    dC = np.zeros((ns, 2))
    p = process_of(prob)
    rc = lib().ref_tangent1d_corr(C.byref(p), C.byref(buf.struct), DT_FROZEN if frozen_dt else DT_DIFF, _ptr(v),
                                  _ptr(dF), _ptr(dM), _ptr(dC))
    if rc != 0:
        raise RuntimeError(f"ref_tangent1d_corr failed ({rc})")
    out = dict(dM=dM, dC=dC)
    if with_f:
        out["dF"] = dF
    return out

"""MI355X (gfx950) crystallization population-balance solver.

Thin ctypes binding of the C ABI in include/pbe.h (libpbe.so, built in-tree
by paper_2411_00742_amd/build.py).  The binding only marshals arguments:
torch supplies device memory for the outputs and the HIP stream; every step of
the solve runs in the library's HIP kernels.  There is no CPU fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import workloads  # noqa: F401  (seeded input generators)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbe.so")

PBE_OK, PBE_EINVAL, PBE_ENOMEM, PBE_EDEVICE, PBE_ENONFINITE, PBE_ESTATE, PBE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FLAG_DEVICE_PTRS, FLAG_RECORD_F, FLAG_AUTOTUNE, FLAG_RECORD_RATES, FLAG_STRANG = 1, 2, 4, 8, 16
SIM_OK, SIM_NONFINITE, SIM_OUTFLOW, SIM_FALLBACK, SIM_STEPCAP = 0, 1, 2, 4, 8
NPAR = 15
NGRAD = 5

# every entry point of include/pbe.h
EXPORTS = ["pbe_create", "pbe_step", "pbe_reset", "pbe_solve", "pbe_fetch", "pbe_grad", "pbe_set_par",
           "pbe_set_mlp", "pbe_mlp_forward", "pbe_adam", "pbe_tune", "pbe_set_launch", "pbe_destroy", "pbe_strerror",
           "pbe_last_kernel_ms", "pbe_rate_log", "pbe_mlp_vjp", "pbe_mlp_vjp_noalloc", "pbe_set_poly",
           "pbe_grad_poly", "pbe_set_corr"]
MLP_VJP_NOALLOC_MAX_ROWS = 4096
CORR_H, CORR_NW = 8, 57
MLP_NW, MLP_NC = 4546, 18
MLP_BF16, MLP_FP64 = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class PbeProblem(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n_sims", C.c_int32),
                ("n_cells", _ip), ("L_max", _dp), ("f0", _dp), ("C0", _dp), ("par", _dp),
                ("mlp", C.POINTER(C.c_float)),
                ("law", C.c_int32), ("scheme", C.c_int32), ("sol_law", C.c_int32), ("n_samples", C.c_int32),
                ("cs0", C.c_double), ("cs1", C.c_double), ("alpha", C.c_double), ("cfl", C.c_double),
                ("dt_max", C.c_double), ("t_end", C.c_double), ("t_samples", _dp),
                ("ckpt_every", C.c_int32), ("max_steps", C.c_int32), ("flags", C.c_int32),
                ("mlp_precision", C.c_int32), ("n_poly", C.c_int32), ("poly", _dp), ("corr", _dp)]


class PbeTuning(C.Structure):
    _fields_ = [("blocks", C.c_int32 * 4), ("seg_2d", C.c_int32), ("pair_long", C.c_int32), ("n_candidates", C.c_int32),
                ("best_ms", C.c_float), ("default_ms", C.c_float)]


class PBEError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().pbe_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


_lib = None


def lib():
    """Load libpbe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2411_00742_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.pbe_create.argtypes = [C.POINTER(PbeProblem), vp, C.POINTER(vp)]
        L.pbe_step.argtypes = [vp, C.c_int32, _ip]
        L.pbe_reset.argtypes = [vp]
        L.pbe_solve.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pbe_fetch.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pbe_grad.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pbe_set_par.argtypes = [vp, _dp]
        L.pbe_set_mlp.argtypes = [vp, vp]
        L.pbe_mlp_forward.argtypes = [C.POINTER(C.c_float), C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.pbe_tune.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(PbeTuning)]
        L.pbe_set_launch.argtypes = [vp, C.POINTER(PbeTuning)]
        L.pbe_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.pbe_destroy.argtypes = [vp]
        L.pbe_destroy.restype = None
        L.pbe_strerror.argtypes = [C.c_int]
        L.pbe_strerror.restype = C.c_char_p
        L.pbe_last_kernel_ms.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.pbe_rate_log.argtypes = [vp, C.c_int32, vp]
        L.pbe_mlp_vjp.argtypes = [C.POINTER(C.c_float), C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.pbe_mlp_vjp_noalloc.argtypes = [C.POINTER(C.c_float), C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.pbe_set_poly.argtypes = [vp, vp]
        L.pbe_grad_poly.argtypes = [vp, vp, vp, vp, vp, vp]
        L.pbe_set_corr.argtypes = [vp, vp]
        for name in EXPORTS:
            if name not in ("pbe_destroy", "pbe_strerror"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != PBE_OK:
        raise PBEError(rc, what)


def _arr(x, dtype):
    return np.ascontiguousarray(x, dtype=dtype)


def make_problem_struct(prob, ckpt_every=0, record_f=False, device_ptrs=True, max_steps=0, autotune=False,
                        record_rates=False):
    """Build the pbe_problem struct for a workloads.Problem; returns (struct, keepalive)."""
    keep = dict(n_cells=_arr(prob.n_cells.reshape(-1), np.int32), L_max=_arr(prob.L_max.reshape(-1), np.float64),
                f0=_arr(prob.f0, np.float64), C0=_arr(prob.C0, np.float64), par=_arr(prob.par, np.float64),
                t_samples=_arr(prob.t_samples, np.float64))
    mlp = getattr(prob, "mlp", None)
    if mlp is not None:
        keep["mlp"] = _arr(mlp, np.float32)
    poly = getattr(prob, "poly", None)
    if poly is not None:
        keep["poly"] = _arr(poly, np.float64)
    corr = getattr(prob, "corr", None)
    if corr is not None:
        keep["corr"] = _arr(corr, np.float64)
    flags = (FLAG_DEVICE_PTRS if device_ptrs else 0) | (FLAG_RECORD_F if record_f else 0) | \
        (FLAG_AUTOTUNE if autotune else 0) | (FLAG_RECORD_RATES if record_rates else 0) | \
        (FLAG_STRANG if getattr(prob, "splitting", 0) == 1 else 0)
    st = PbeProblem(ndim=prob.ndim, n_sims=prob.n_sims,
                    n_cells=keep["n_cells"].ctypes.data_as(_ip), L_max=keep["L_max"].ctypes.data_as(_dp),
                    f0=keep["f0"].ctypes.data_as(_dp), C0=keep["C0"].ctypes.data_as(_dp),
                    par=keep["par"].ctypes.data_as(_dp),
                    mlp=keep["mlp"].ctypes.data_as(C.POINTER(C.c_float)) if "mlp" in keep else None,
                    law=prob.law, scheme=prob.scheme, sol_law=prob.sol_law, n_samples=len(prob.t_samples),
                    cs0=prob.cs0, cs1=prob.cs1, alpha=prob.alpha, cfl=prob.cfl, dt_max=prob.dt_max,
                    t_end=prob.t_end, t_samples=keep["t_samples"].ctypes.data_as(_dp),
                    ckpt_every=ckpt_every, max_steps=max_steps, flags=flags,
                    mlp_precision=int(getattr(prob, "mlp_precision", 0)),
                    n_poly=0 if poly is None else int(keep["poly"].shape[1]),
                    poly=keep["poly"].ctypes.data_as(_dp) if "poly" in keep else None,
                    corr=keep["corr"].ctypes.data_as(_dp) if "corr" in keep else None)
    return st, keep


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Solver:
    """One pbe_handle: a batch of simulations resident on the GPU.

    Outputs are torch tensors on the current CUDA (HIP) device; all work is
    ordered on torch's current stream.
    """

    def __init__(self, prob, ckpt_every: int = 0, record_f: bool = False, max_steps: int = 0, stream=None,
                 autotune: bool = False, record_rates: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2411_00742_amd needs a ROCm GPU; none is visible")
        self.torch = torch
        self.prob = prob
        self.record_f = record_f
        self.ckpt_every = ckpt_every
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.generation = 0   # bumped by every call that replaces the recorded solve
        st, keep = make_problem_struct(prob, ckpt_every, record_f, True, max_steps, autotune, record_rates)
        self._h = C.c_void_p()
        _check(lib().pbe_create(C.byref(st), C.c_void_p(self.stream.cuda_stream), C.byref(self._h)), "pbe_create")
        del keep
        self.S = prob.n_sims
        self.ns = len(prob.t_samples)
        poly = getattr(prob, "poly", None)
        self.n_poly = 0 if poly is None else int(np.asarray(poly).shape[1])
        self.total = int(prob.cells_per_sim().sum())

    # --- output buffers -------------------------------------------------------
    def _outputs(self):
        t = self.torch
        nf = self.total * self.ns if self.record_f else self.total
        kw = dict(device=self.device)
        return dict(f=t.empty(nf, dtype=t.float64, **kw), mom=t.empty((self.S, self.ns, 4), dtype=t.float64, **kw),
                    C=t.empty((self.S, self.ns), dtype=t.float64, **kw), steps=t.empty(self.S, dtype=t.int32, **kw),
                    status=t.empty(self.S, dtype=t.int32, **kw))

    def solve(self, out=None):
        """Solve every simulation from the initial condition; returns dict of device tensors."""
        o = out if out is not None else self._outputs()
        self.generation += 1
        _check(lib().pbe_solve(self._h, _ptr(o["f"]), _ptr(o["mom"]), _ptr(o["C"]), _ptr(o["steps"]),
                               _ptr(o["status"])), "pbe_solve")
        return o

    def step(self, n_steps: int) -> int:
        n_active = C.c_int32()
        self.generation += 1
        _check(lib().pbe_step(self._h, n_steps, C.byref(n_active)), "pbe_step")
        return n_active.value

    def fetch(self):
        o = self._outputs()
        _check(lib().pbe_fetch(self._h, _ptr(o["f"]), _ptr(o["mom"]), _ptr(o["C"]), _ptr(o["steps"]),
                               _ptr(o["status"])), "pbe_fetch")
        return o

    def reset(self):
        self.generation += 1
        _check(lib().pbe_reset(self._h), "pbe_reset")

    def set_par(self, par):
        self.generation += 1
        p = _arr(par, np.float64)
        assert p.shape == (self.S, NPAR)
        _check(lib().pbe_set_par(self._h, p.ctypes.data_as(_dp)), "pbe_set_par")

    def grad(self, gf=None, gmom=None, gC=None, with_mlp: bool = False):
        """d<cotangents, outputs>/d(kg, g, kb, b, gamma) per sim, as a [S, 5] device tensor;
        with_mlp (closure law): also d/d(closure weights) [MLP_NW], summed over sims."""
        t = self.torch
        g = t.empty((self.S, NGRAD), dtype=t.float64, device=self.device)
        gw = t.empty(MLP_NW, dtype=t.float64, device=self.device) if with_mlp else None
        cot = [None if x is None else x.to(device=self.device, dtype=t.float64).contiguous() for x in (gf, gmom, gC)]
        _check(lib().pbe_grad(self._h, _ptr(cot[0]), _ptr(cot[1]), _ptr(cot[2]), _ptr(g), _ptr(gw)), "pbe_grad")
        return (g, gw) if with_mlp else g

    def set_poly(self, poly):
        """New polynomial growth coefficients [S, n_poly] (device tensor or host array)."""
        self.generation += 1
        t = self.torch
        c = t.as_tensor(poly, dtype=t.float64).to(self.device).contiguous()
        assert c.shape == (self.S, self.n_poly)
        _check(lib().pbe_set_poly(self._h, _ptr(c)), "pbe_set_poly")
        self._poly_keep = c

    def set_corr(self, corr):
        """New in-the-loop correction weights [S, CORR_NW] (device tensor or host array)."""
        self.generation += 1
        t = self.torch
        c = t.as_tensor(corr, dtype=t.float64).to(self.device).contiguous()
        assert c.shape == (self.S, CORR_NW)
        _check(lib().pbe_set_corr(self._h, _ptr(c)), "pbe_set_corr")
        self._corr_keep = c

    def grad_poly(self, gf=None, gmom=None, gC=None):
        """d<cotangents, outputs>/d(polynomial coefficients) per sim [S, n_poly], and the
        (kg, g, kb, b, gamma) gradient [S, 5] (device tensors)."""
        t = self.torch
        g = t.empty((self.S, NGRAD), dtype=t.float64, device=self.device)
        gp = t.empty((self.S, self.n_poly), dtype=t.float64, device=self.device)
        cot = [None if x is None else x.to(device=self.device, dtype=t.float64).contiguous() for x in (gf, gmom, gC)]
        _check(lib().pbe_grad_poly(self._h, _ptr(cot[0]), _ptr(cot[1]), _ptr(cot[2]), _ptr(g), _ptr(gp)),
               "pbe_grad_poly")
        return gp, g

    def set_mlp(self, w):
        """New closure weights: a float32 device tensor (or array) of MLP_NW values."""
        self.generation += 1
        t = self.torch
        w = t.as_tensor(w, dtype=t.float32).to(self.device).contiguous()
        assert w.numel() == MLP_NW
        _check(lib().pbe_set_mlp(self._h, _ptr(w)), "pbe_set_mlp")
        self._mlp_keep = w

    def tune(self, trial_steps: int = 0, use_cache: bool = False) -> dict:
        """Run the autotuner (pbe_tune); returns the chosen launch shape and trial times."""
        t = PbeTuning()
        _check(lib().pbe_tune(self._h, trial_steps, 1 if use_cache else 0, C.byref(t)), "pbe_tune")
        return dict(blocks=list(t.blocks), seg_2d=t.seg_2d, pair_long=t.pair_long, n_candidates=t.n_candidates,
                    best_ms=t.best_ms,
                    default_ms=t.default_ms)

    def set_launch(self, blocks=(0, 0, 0, 0), seg_2d: int = 128, pair_long: bool = False):
        """Apply a launch shape (pbe_set_launch); 0 blocks means what fits the device."""
        t = PbeTuning()
        for i, b in enumerate(blocks):
            t.blocks[i] = int(b)
        t.seg_2d = seg_2d
        t.pair_long = 1 if pair_long else 0
        _check(lib().pbe_set_launch(self._h, C.byref(t)), "pbe_set_launch")

    def rate_log(self, n_steps: int):
        """(dt, G0, B) of the first n_steps steps of every sim in the last solve: [S, n_steps, 3]."""
        t = self.torch
        o = t.empty((self.S, n_steps, 3), dtype=t.float64, device=self.device)
        _check(lib().pbe_rate_log(self._h, n_steps, _ptr(o)), "pbe_rate_log")
        return o

    def last_kernel_ms(self):
        a, b = C.c_float(), C.c_float()
        _check(lib().pbe_last_kernel_ms(self._h, C.byref(a), C.byref(b)), "pbe_last_kernel_ms")
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pbe_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward(blob, precision: int, x):
    """The closure network on raw inputs x[n, 3] = (S, T, log10 mu_2) (device tensor or array):
    returns device tensors y [n, 2] and dy [n, 2, 3] = dy_o/dz_i."""
    import torch
    b = _arr(blob, np.float32)
    assert b.size == MLP_NW + MLP_NC
    dev = torch.device("cuda", torch.cuda.current_device())
    xt = torch.as_tensor(x, dtype=torch.float64).to(dev).contiguous().reshape(-1, 3)
    n = xt.shape[0]
    y = torch.empty((n, 2), dtype=torch.float64, device=dev)
    dy = torch.empty((n, 2, 3), dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream()
    _check(lib().pbe_mlp_forward(b.ctypes.data_as(C.POINTER(C.c_float)), precision, n, _ptr(xt), _ptr(y), _ptr(dy),
                                 C.c_void_p(st.cuda_stream)), "pbe_mlp_forward")
    return y, dy


def mlp_vjp(blob, precision: int, z, ybar, noalloc: bool = False):
    """Weight gradient sum_r (dy/dW at z_r)^T ybar_r of the closure network over rows of
    normalised inputs z[n, 3] and output cotangents ybar[n, 2]: a [MLP_NW] device tensor.
    noalloc: use pbe_mlp_vjp_noalloc (no device allocation in the library; n <= 4096)."""
    import torch
    b = _arr(blob, np.float32)
    assert b.size == MLP_NW + MLP_NC
    dev = torch.device("cuda", torch.cuda.current_device())
    zt = torch.as_tensor(z, dtype=torch.float64).to(dev).contiguous().reshape(-1, 3)
    yt = torch.as_tensor(ybar, dtype=torch.float64).to(dev).contiguous().reshape(-1, 2)
    assert zt.shape[0] == yt.shape[0]
    gw = torch.empty(MLP_NW, dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream()
    fn = lib().pbe_mlp_vjp_noalloc if noalloc else lib().pbe_mlp_vjp
    _check(fn(b.ctypes.data_as(C.POINTER(C.c_float)), precision, zt.shape[0], _ptr(zt), _ptr(yt), _ptr(gw),
              C.c_void_p(st.cuda_stream)), "pbe_mlp_vjp_noalloc" if noalloc else "pbe_mlp_vjp")
    return gw


class Adam:
    """Adam state for a float32 device parameter vector, stepped by the library's kernel."""

    def __init__(self, w, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        self.w = w
        self.m = torch.zeros_like(w)
        self.v = torch.zeros_like(w)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0

    def step(self, g):
        import torch
        self.t += 1
        g = g.to(dtype=torch.float64).contiguous()
        st = torch.cuda.current_stream()
        _check(lib().pbe_adam(_ptr(self.w), _ptr(self.m), _ptr(self.v), _ptr(g), self.w.numel(), self.t, self.lr,
                              self.b1, self.b2, self.eps, C.c_void_p(st.cuda_stream)), "pbe_adam")


def _autograd_function():
    import torch

    class PBESolve(torch.autograd.Function):
        """Differentiable batched solve: kinetics (kg, g, kb, b, gamma) per sim -> recorded outputs.

        forward(par5 [S, 5] float64, solver) -> (f, mom, C); backward runs the
        library's discrete adjoint (pbe_grad), which differentiates every step size
        in the branch the solve took.  The solver must have been created with
        ckpt_every > 0.
        """

        @staticmethod
        def forward(ctx, par5, solver):
            par = np.array(solver.prob.par, dtype=np.float64, copy=True)
            par[:, :NGRAD] = par5.detach().cpu().numpy()
            solver.set_par(par)
            out = solver.solve()
            ctx.solver = solver
            ctx.generation = solver.generation
            ctx.par_device = par5.device
            return out["f"], out["mom"], out["C"]

        @staticmethod
        def backward(ctx, gf, gmom, gC):
            # pbe_grad differentiates the handle's last solve: a later solve on the same
            # solver (another forward before this backward) has replaced it
            if ctx.solver.generation != ctx.generation:
                raise RuntimeError("PBESolve.backward: the solver ran another solve after this forward; "
                                   "use one Solver per differentiable solve that is still to be back-propagated")
            g = ctx.solver.grad(gf, gmom, gC)
            return g.to(ctx.par_device), None

    return PBESolve


def pbe_solve_autograd(par5, solver):
    """Apply the differentiable solve (see PBESolve)."""
    return _autograd_function().apply(par5, solver)

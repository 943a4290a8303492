"""Thin ctypes binding of librt4d.so (the C ABI declared in include/rt4d.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions carry the C names (``rt_plan_create``, ``rt_forward``,
``rt_adjoint``, ``tv_grad``, ``tv_div``, ``shrink``, ``solve``, the job
calls ...) and take torch tensors for device arrays; ``Plan`` and ``Job``
wrap the handles.  Tensors must be float32, contiguous, on the plan's GPU.
The call is issued on torch's current stream of that device.

If librt4d.so is not built this module raises on first use: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RT4D_LIBRARY names another build of the same library (the host-sanitizer
# build that `python -m paper_1809_09725_amd.build --sanitize` writes)
LIB_PATH = os.environ.get("RT4D_LIBRARY") or os.path.join(_HERE, "librt4d.so")

RT_OK, RT_E_ARG, RT_E_SHAPE, RT_E_HIP, RT_E_OOM, RT_E_NONFINITE = 0, -1, -2, -3, -4, -5
RT_FORM_PF, RT_FORM_SF, RT_FORM_AUTO = 0, 1, 2
RT_PREC_FP32, RT_PREC_BF16MFMA = 0, 1
RT_CP_PLAIN, RT_CP_ACCEL = 0, 1

EXPORTS = ("rt_plan_create", "rt_plan_destroy", "rt_plan_bytes", "rt_tables", "rt_forward",
           "rt_adjoint", "tv_grad", "tv_div", "shrink", "solve", "rt_job_bytes",
           "rt_job_create", "rt_job_step", "rt_job_done", "rt_job_iters", "rt_job_report",
           "rt_job_checkpoint_bytes", "rt_job_checkpoint", "rt_job_restore", "rt_job_destroy",
           "rt_dot", "rt_timing_enable", "rt_timing_reset", "rt_timing_read", "rt_last_error",
           "rt_fbp_filter", "rt_fbp", "rt_solve_ooc", "rt_calib_fma", "rt_form_pick", "rt_plan_form", "rt_basis_fourier", "rt_dot_noalloc")


class RtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rt4d error {code}: {msg}")
        self.code = code


class rt_geom(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("N", "Nz", "Ns", "Ntheta", "Npi", "K", "Nt")]


class rt_solve_params(ctypes.Structure):
    _fields_ = [("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("tol", ctypes.c_double), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("n_iter", ctypes.c_int32), ("n_pow", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("mu", ctypes.c_double), ("variant", ctypes.c_int32)]


class rt_solve_report(ctypes.Structure):
    _fields_ = [("L_R", ctypes.c_double), ("L_G", ctypes.c_double), ("tau", ctypes.c_double),
                ("sigma", ctypes.c_double), ("residual", ctypes.c_double),
                ("objective", ctypes.c_double), ("rel_change", ctypes.c_double),
                ("iters_done", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load librt4d.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1809_09725_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
    f32, c_int = ctypes.c_float, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "rt_plan_create": (c_int, [P(rt_geom), c_int, c_int, vp, vp, P(vp)]),
        "rt_plan_destroy": (None, [vp]),
        "rt_plan_bytes": (c_int, [vp, P(sz)]),
        "rt_tables": (c_int, [vp, vp, vp, vp, vp, vp]),
        "rt_forward": (c_int, [vp, vp, vp, vp]),
        "rt_adjoint": (c_int, [vp, vp, vp, vp]),
        "tv_grad": (c_int, [vp, vp, f32, vp, vp]),
        "tv_div": (c_int, [vp, vp, f32, vp, vp]),
        "shrink": (c_int, [vp, vp, f32, vp]),
        "solve": (c_int, [vp, P(rt_solve_params), vp, vp, P(rt_solve_report), vp]),
        "rt_job_bytes": (c_int, [P(rt_geom), c_int, c_int, P(sz)]),
        "rt_job_create": (c_int, [vp, P(rt_solve_params), vp, vp, vp, P(vp)]),
        "rt_job_step": (c_int, [vp, i32, vp]),
        "rt_job_done": (c_int, [vp]),
        "rt_job_iters": (c_int, [vp]),
        "rt_job_report": (c_int, [vp, P(rt_solve_report), vp]),
        "rt_job_checkpoint_bytes": (c_int, [vp, P(sz)]),
        "rt_job_checkpoint": (c_int, [vp, vp, vp]),
        "rt_job_restore": (c_int, [vp, vp, vp]),
        "rt_job_destroy": (None, [vp]),
        "rt_dot": (c_int, [vp, vp, sz, P(ctypes.c_double), vp]),
        "rt_dot_noalloc": (c_int, [vp, vp, sz, P(ctypes.c_double), vp]),
        "rt_fbp_filter": (c_int, [vp, vp, vp, vp]),
        "rt_fbp": (c_int, [vp, vp, vp, vp]),
        "rt_solve_ooc": (c_int, [P(rt_geom), vp, vp, P(rt_solve_params), vp, vp, i32,
                                 P(rt_solve_report), vp]),
        "rt_form_pick": (c_int, [P(rt_geom), c_int, c_int, P(c_int), P(c_int)]),
        "rt_plan_form": (c_int, [vp, P(c_int), P(c_int)]),
        "rt_basis_fourier": (c_int, [P(rt_geom), i32, vp, vp]),
        "rt_calib_fma": (c_int, [i32, i32, vp, P(ctypes.c_double), P(ctypes.c_double), vp]),
        "rt_timing_enable": (c_int, [c_int]),
        "rt_timing_reset": (c_int, []),
        "rt_timing_read": (c_int, [ctypes.c_char_p, P(ctypes.c_double), P(ctypes.c_int64)]),
        "rt_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _ = u64
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != RT_OK:
        raise RtError(rc, lib().rt_last_error().decode())


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


@dataclass(frozen=True)
class Geom:
    N: int
    Nz: int
    Ns: int
    Ntheta: int
    Npi: int
    K: int
    Nt: int

    @property
    def n0(self) -> int:
        return self.Ntheta // self.Npi

    @property
    def f_shape(self):
        return (self.Nz, self.N, self.N, self.K)

    @property
    def g_shape(self):
        return (self.Ntheta, self.Nz, self.Ns)

    @property
    def p_shape(self):
        return (self.Nz, self.Nt, 4, self.N, self.N)

    def c(self) -> rt_geom:
        return rt_geom(self.N, self.Nz, self.Ns, self.Ntheta, self.Npi, self.K, self.Nt)


def _ptr(t: torch.Tensor | None, shape, dev: torch.device, name: str) -> ctypes.c_void_p:
    if t is None:
        raise ValueError(f"{name} is None")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if t.device != dev:
        raise ValueError(f"{name} is on {t.device}, the plan is on {dev}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------- C-named calls

def rt_plan_create(geom: Geom, form: int = RT_FORM_PF, prec: int = RT_PREC_FP32,
                   phi=None, S=None) -> ctypes.c_void_p:
    import numpy as np
    h = ctypes.c_void_p()
    keep = []
    pp = ps = None
    if phi is not None:
        a = np.ascontiguousarray(phi, dtype=np.float64)
        assert a.shape == (geom.Ntheta, geom.K)
        keep.append(a)
        pp = a.ctypes.data_as(ctypes.c_void_p)
    if S is not None:
        a = np.ascontiguousarray(S, dtype=np.float64)
        assert a.shape == (geom.Nt, geom.K)
        keep.append(a)
        ps = a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().rt_plan_create(ctypes.byref(geom.c()), form, prec, pp, ps, ctypes.byref(h)))
    return h


def rt_plan_destroy(h) -> None:
    lib().rt_plan_destroy(h)


def rt_forward(plan: "Plan", f: torch.Tensor, g: torch.Tensor) -> None:
    _check(lib().rt_forward(plan.h, _ptr(f, plan.geom.f_shape, plan.device, "f"),
                            _ptr(g, plan.geom.g_shape, plan.device, "g"), _stream(plan.device)))


def rt_adjoint(plan: "Plan", g: torch.Tensor, f_out: torch.Tensor) -> None:
    _check(lib().rt_adjoint(plan.h, _ptr(g, plan.geom.g_shape, plan.device, "g"),
                            _ptr(f_out, plan.geom.f_shape, plan.device, "f_out"),
                            _stream(plan.device)))


def solve_ooc(geom: "Geom", g: torch.Tensor, f: torch.Tensor, slab: int, phi=None, S=None,
              device=None, **kw) -> dict:
    """Out-of-core solve: g and f are host (CPU) float32 tensors, f is updated
    in place; the volume streams through the GPU in z-slabs of `slab` slices."""
    import numpy as np
    for name, t, shape in (("g", g, geom.g_shape), ("f", f, geom.f_shape)):
        if t.device.type != "cpu" or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CPU tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    keep = []

    def host(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(ctypes.c_void_p)

    dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                       torch.device(device).index or 0)
    rep = rt_solve_report()
    prm = make_params(**kw)
    with torch.cuda.device(dev):
        _check(lib().rt_solve_ooc(ctypes.byref(geom.c()), host(phi), host(S), ctypes.byref(prm),
                                  ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                  int(slab), ctypes.byref(rep), _stream(dev)))
    return rep.as_dict()


def rt_fbp_filter(plan: "Plan", g: torch.Tensor, q: torch.Tensor) -> None:
    _check(lib().rt_fbp_filter(plan.h, _ptr(g, plan.geom.g_shape, plan.device, "g"),
                               _ptr(q, plan.geom.g_shape, plan.device, "q"), _stream(plan.device)))


def rt_fbp(plan: "Plan", g: torch.Tensor, f_out: torch.Tensor) -> None:
    _check(lib().rt_fbp(plan.h, _ptr(g, plan.geom.g_shape, plan.device, "g"),
                        _ptr(f_out, plan.geom.f_shape, plan.device, "f_out"), _stream(plan.device)))


def tv_grad(plan: "Plan", f: torch.Tensor, lambda2: float, p: torch.Tensor) -> None:
    _check(lib().tv_grad(plan.h, _ptr(f, plan.geom.f_shape, plan.device, "f"), lambda2,
                         _ptr(p, plan.geom.p_shape, plan.device, "p"), _stream(plan.device)))


def tv_div(plan: "Plan", p: torch.Tensor, lambda2: float, f_out: torch.Tensor) -> None:
    _check(lib().tv_div(plan.h, _ptr(p, plan.geom.p_shape, plan.device, "p"), lambda2,
                        _ptr(f_out, plan.geom.f_shape, plan.device, "f_out"),
                        _stream(plan.device)))


def shrink(plan: "Plan", p: torch.Tensor, lambda1: float) -> None:
    _check(lib().shrink(plan.h, _ptr(p, plan.geom.p_shape, plan.device, "p"), lambda1,
                        _stream(plan.device)))


def make_params(*, lambda1: float, lambda2: float, n_iter: int, tau: float = 0.0,
                sigma: float = 0.0, tol: float = 0.0, n_pow: int = 20, check_every: int = 0,
                seed: int = 0, mu: float = 0.0, variant: str = "plain") -> rt_solve_params:
    """variant: "plain" (theta = 1, fixed steps) or "accel" (the accelerated
    form with adaptive theta, tau, sigma for the uniformly convex model with
    mu > 0)."""
    v = {"plain": RT_CP_PLAIN, "accel": RT_CP_ACCEL}[variant]
    return rt_solve_params(lambda1, lambda2, tol, tau, sigma, n_iter, n_pow, check_every, seed,
                           mu, v)


def solve(plan: "Plan", params: rt_solve_params, g: torch.Tensor, f: torch.Tensor) -> dict:
    rep = rt_solve_report()
    _check(lib().solve(plan.h, ctypes.byref(params), _ptr(g, plan.geom.g_shape, plan.device, "g"),
                       _ptr(f, plan.geom.f_shape, plan.device, "f"), ctypes.byref(rep),
                       _stream(plan.device)))
    return rep.as_dict()


def form_pick(geom: Geom, form: int = RT_FORM_AUTO, prec: int = RT_PREC_BF16MFMA) -> tuple[int, int]:
    """(form, precision) a plan of this geometry runs for the requested pair;
    RT_FORM_AUTO is resolved by the library's rule.  Host only."""
    fo, po = ctypes.c_int(), ctypes.c_int()
    _check(lib().rt_form_pick(ctypes.byref(geom.c()), form, prec, ctypes.byref(fo), ctypes.byref(po)))
    return fo.value, po.value


def basis_fourier(geom: Geom, M: int):
    """(phi [Ntheta][K], S [Nt][K]) FP64 host tables of the real form of the
    paper's Fourier basis of M functions (K = M - 1), for Plan(phi=, S=)."""
    import numpy as np
    phi = np.empty((geom.Ntheta, geom.K), np.float64)
    S = np.empty((geom.Nt, geom.K), np.float64)
    _check(lib().rt_basis_fourier(ctypes.byref(geom.c()), M, ctypes.c_void_p(phi.ctypes.data),
                                  ctypes.c_void_p(S.ctypes.data)))
    return phi, S


def fourier_complex_coeffs(f_real: torch.Tensor, M: int) -> torch.Tensor:
    """Complex coefficients c_j, j = 0 .. M-1 (frequency j - M/2), of the
    paper's basis from the real-form coefficients [..., K = M - 1] (last
    axis): c_0 = a_0, c_v = (a_v - i b_v)/2, c_{-v} = (a_v + i b_v)/2,
    c_{-M/2} = 0."""
    K = f_real.shape[-1]
    if K != M - 1:
        raise ValueError(f"K = {K} real coefficients are the span of M = K + 1 functions")
    c = torch.zeros(*f_real.shape[:-1], M, dtype=torch.complex64, device=f_real.device)
    c[..., M // 2] = f_real[..., 0]
    for v in range(1, M // 2):
        a, b = f_real[..., 2 * v - 1], f_real[..., 2 * v]
        c[..., M // 2 + v] = torch.complex(a, -b) / 2
        c[..., M // 2 - v] = torch.complex(a, b) / 2
    return c


def rt_job_bytes(geom: Geom, form: int = RT_FORM_PF, prec: int = RT_PREC_FP32) -> int:
    b = ctypes.c_size_t()
    _check(lib().rt_job_bytes(ctypes.byref(geom.c()), form, prec, ctypes.byref(b)))
    return b.value


def rt_dot(x: torch.Tensor, y: torch.Tensor) -> float:
    if x.dtype != torch.float32 or y.dtype != torch.float32 or x.numel() != y.numel():
        raise ValueError("rt_dot needs two float32 tensors of equal size")
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("rt_dot needs contiguous tensors")
    out = ctypes.c_double()
    _check(lib().rt_dot(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel(),
                        ctypes.byref(out), _stream(x.device)))
    return out.value


def calib_fma(n_blocks: int, n_iter: int, out: torch.Tensor) -> tuple[float, float]:
    """(milliseconds, flops) of the FP32 FMA issue-rate kernel; out holds
    n_blocks * 256 float32 values on the device."""
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < 256 * n_blocks:
        raise ValueError("calib_fma needs a contiguous float32 tensor of n_blocks * 256 values")
    ms, fl = ctypes.c_double(), ctypes.c_double()
    _check(lib().rt_calib_fma(n_blocks, n_iter, ctypes.c_void_p(out.data_ptr()), ctypes.byref(ms),
                              ctypes.byref(fl), _stream(out.device)))
    return ms.value, fl.value


def timing_enable(on: bool = True) -> None:
    _check(lib().rt_timing_enable(1 if on else 0))


def timing_reset() -> None:
    _check(lib().rt_timing_reset())


def timing_read(kernel: str) -> tuple[float, int]:
    """(total milliseconds, launches) of the named kernel since the last reset."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().rt_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------------ objects

class Plan:
    """Owns an rt_plan on one GPU (tables + scratch)."""

    def __init__(self, geom: Geom, form: int = RT_FORM_PF, prec: int = RT_PREC_FP32,
                 phi=None, S=None, device=None):
        self.geom = geom
        self.form, self.prec = form, prec
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            self.h = rt_plan_create(geom, form, prec, phi, S)
        fo, po = ctypes.c_int(), ctypes.c_int()
        _check(lib().rt_plan_form(self.h, ctypes.byref(fo), ctypes.byref(po)))
        self.form, self.prec = fo.value, po.value   # RT_FORM_AUTO resolved by the library

    def close(self) -> None:
        if getattr(self, "h", None):
            rt_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().rt_plan_bytes(self.h, ctypes.byref(b)))
        return b.value

    def tables(self) -> dict:
        import numpy as np
        n = self.geom.Ntheta
        th, t = np.zeros(n), np.zeros(n)
        cls, rot, flip = (np.zeros(n, np.int32) for _ in range(3))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().rt_tables(self.h, p(th), p(t), p(cls), p(rot), p(flip)))
        return dict(theta=th, t=t, cls=cls, rot=rot, flip=flip)

    def _new(self, shape):
        return torch.empty(shape, dtype=torch.float32, device=self.device)

    def forward(self, f, out=None):
        out = self._new(self.geom.g_shape) if out is None else out
        rt_forward(self, f, out)
        return out

    def adjoint(self, g, out=None):
        out = self._new(self.geom.f_shape) if out is None else out
        rt_adjoint(self, g, out)
        return out

    def fbp_filter(self, g, out=None):
        out = self._new(self.geom.g_shape) if out is None else out
        rt_fbp_filter(self, g, out)
        return out

    def fbp(self, g, out=None):
        """FBP initial guess in coefficient form (blocks until it is ready)."""
        out = self._new(self.geom.f_shape) if out is None else out
        rt_fbp(self, g, out)
        return out

    def tv_grad(self, f, lambda2, out=None):
        out = self._new(self.geom.p_shape) if out is None else out
        tv_grad(self, f, lambda2, out)
        return out

    def tv_div(self, p, lambda2, out=None):
        out = self._new(self.geom.f_shape) if out is None else out
        tv_div(self, p, lambda2, out)
        return out

    def shrink(self, p, lambda1):
        shrink(self, p, lambda1)
        return p

    def solve(self, g, f, **kw) -> dict:
        return solve(self, make_params(**kw), g, f)


class Job:
    """Resumable solver state (rt_job); the caller keeps g and f alive."""

    def __init__(self, plan: Plan, g: torch.Tensor, f: torch.Tensor, **kw):
        self.plan, self.g, self.f = plan, g, f
        self.params = make_params(**kw)
        self.h = ctypes.c_void_p()
        _check(lib().rt_job_create(plan.h, ctypes.byref(self.params),
                                   _ptr(g, plan.geom.g_shape, plan.device, "g"),
                                   _ptr(f, plan.geom.f_shape, plan.device, "f"),
                                   _stream(plan.device), ctypes.byref(self.h)))

    def step(self, n: int = 1, stream=None) -> None:
        s = _stream(self.plan.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(lib().rt_job_step(self.h, n, s))

    @property
    def done(self) -> bool:
        r = lib().rt_job_done(self.h)
        if r < 0:
            _check(r)
        return r == 1

    @property
    def iters(self) -> int:
        return lib().rt_job_iters(self.h)

    def report(self, stream=None) -> dict:
        rep = rt_solve_report()
        s = _stream(self.plan.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(lib().rt_job_report(self.h, ctypes.byref(rep), s))
        return rep.as_dict()

    def checkpoint(self) -> bytearray:
        n = ctypes.c_size_t()
        _check(lib().rt_job_checkpoint_bytes(self.h, ctypes.byref(n)))
        buf = bytearray(n.value)
        cbuf = (ctypes.c_char * n.value).from_buffer(buf)
        _check(lib().rt_job_checkpoint(self.h, ctypes.cast(cbuf, ctypes.c_void_p),
                                       _stream(self.plan.device)))
        return buf

    def restore(self, buf: bytearray) -> None:
        cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
        _check(lib().rt_job_restore(self.h, ctypes.cast(cbuf, ctypes.c_void_p),
                                    _stream(self.plan.device)))

    def close(self) -> None:
        if getattr(self, "h", None):
            lib().rt_job_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

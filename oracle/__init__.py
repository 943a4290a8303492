"""FP64 CPU oracle (test infrastructure only).

This package wraps ``oracle.c``, a plain double-precision implementation of
the decomposed-time Radon operator, its adjoint, the 4D TV operators and the
adapted Chambolle-Pock loop (Nikitin et al., Sec. 2-4 and Fig. 2).  It is the
independent reference the GPU library is checked against: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  It shares no code with the product library and never calls it.

Array conventions (numpy, C order):
  f   : (Nz, N, N, K)         coefficient volumes f_k
  g   : (Ntheta, Nz, Ns)      sinogram
  p   : (Nz, N, N, Nt, 4)     4D gradient field, components (x, y, z, t)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                        "-Wall", "-fno-fast-math", "-ffp-contract=off",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("N", "Nz", "Ns", "Ntheta", "Npi", "K", "Nt")]


class _Params(ctypes.Structure):
    _fields_ = [("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double),
                ("tol", ctypes.c_double), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("n_iter", ctypes.c_int32), ("n_pow", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("route", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("mu", ctypes.c_double), ("variant", ctypes.c_int32)]


class _Report(ctypes.Structure):
    _fields_ = [("L_R", ctypes.c_double), ("L_G", ctypes.c_double), ("tau", ctypes.c_double),
                ("sigma", ctypes.c_double), ("residual", ctypes.c_double),
                ("objective", ctypes.c_double), ("rel_change", ctypes.c_double),
                ("iters_done", ctypes.c_int32)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d, i, u64 = ctypes.c_double, ctypes.c_int, ctypes.c_uint64
        _lib.or_weight.restype = d
        _lib.or_weight.argtypes = [d, d, i, i, i, i, i]
        _lib.or_tv_norm.restype = d
        _lib.or_power.restype = d
        _lib.or_S_norm.restype = d
        _lib.or_seeded_uniform.restype = d
        _lib.or_seeded_uniform.argtypes = [u64, u64]
        _lib.or_shrink.argtypes = [ctypes.c_size_t, ctypes.c_void_p, d]
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass(frozen=True)
class Geom:
    """Problem sizes: N x N pixels per slice, Nz slices, Ns detector bins,
    Ntheta = Npi * Ntheta0 projections over Npi half-turns, K basis
    functions, Nt time frames for the TV (Nt <= Npi)."""
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

    def c(self) -> _Geom:
        return _Geom(self.N, self.Nz, self.Ns, self.Ntheta, self.Npi, self.K, self.Nt)


def tables(g: Geom):
    """Angle, time, class, half-turn and flip tables plus Phi and S (Sec. 4, eq. discrt)."""
    th = np.zeros(g.Ntheta); t = np.zeros(g.Ntheta)
    cls = np.zeros(g.Ntheta, np.int32); rot = np.zeros(g.Ntheta, np.int32)
    flip = np.zeros(g.Ntheta, np.int32)
    phi = np.zeros((g.Ntheta, g.K)); S = np.zeros((g.Nt, g.K))
    rc = _L().or_tables(ctypes.byref(g.c()), _p(th), _p(t), _p(cls), _p(rot), _p(flip),
                        _p(phi), _p(S))
    if rc != 0:
        raise ValueError("or_tables: bad geometry")
    return dict(theta=th, t=t, cls=cls, rot=rot, flip=flip, phi=phi, S=S)


def weight(theta: float, b: int, q: int, r: int, N: int, Ns: int) -> float:
    return _L().or_weight(np.cos(theta), np.sin(theta), b, q, r, N, Ns)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def forward(g: Geom, f, phi=None, route: str = "direct") -> np.ndarray:
    """R_T f: (Nz,N,N,K) -> (Ntheta,Nz,Ns)."""
    T = tables(g)
    phi = T["phi"] if phi is None else _f64(phi)
    f = _f64(f).reshape(g.Nz, g.N, g.N, g.K)
    out = np.zeros((g.Ntheta, g.Nz, g.Ns))
    if route == "direct":
        _L().or_forward_direct(ctypes.byref(g.c()), _p(T["theta"]), _p(phi), _p(f), _p(out))
    elif route == "folded":
        _L().or_forward_folded(ctypes.byref(g.c()), _p(phi), _p(f), _p(out))
    else:
        raise ValueError(route)
    return out


def adjoint(g: Geom, s, phi=None, route: str = "direct") -> np.ndarray:
    """R_T* g: (Ntheta,Nz,Ns) -> (Nz,N,N,K)."""
    T = tables(g)
    phi = T["phi"] if phi is None else _f64(phi)
    s = _f64(s).reshape(g.Ntheta, g.Nz, g.Ns)
    out = np.zeros((g.Nz, g.N, g.N, g.K))
    if route == "direct":
        _L().or_adjoint_direct(ctypes.byref(g.c()), _p(T["theta"]), _p(phi), _p(s), _p(out))
    elif route == "folded":
        _L().or_adjoint_folded(ctypes.byref(g.c()), _p(phi), _p(s), _p(out))
    else:
        raise ValueError(route)
    return out


def tv_grad(g: Geom, f, lambda2: float, S=None) -> np.ndarray:
    S = tables(g)["S"] if S is None else _f64(S)
    f = _f64(f).reshape(g.Nz, g.N, g.N, g.K)
    p = np.zeros((g.Nz, g.N, g.N, g.Nt, 4))
    _L().or_tv_grad(ctypes.byref(g.c()), _p(S), ctypes.c_double(lambda2), _p(f), _p(p))
    return p


def tv_div(g: Geom, p, lambda2: float, S=None) -> np.ndarray:
    S = tables(g)["S"] if S is None else _f64(S)
    p = _f64(p).reshape(g.Nz, g.N, g.N, g.Nt, 4)
    out = np.zeros((g.Nz, g.N, g.N, g.K))
    _L().or_tv_div(ctypes.byref(g.c()), _p(S), ctypes.c_double(lambda2), _p(p), _p(out))
    return out


def shrink(p, lambda1: float) -> np.ndarray:
    q = _f64(p).copy()
    assert q.size % 4 == 0
    _L().or_shrink(q.size // 4, _p(q), lambda1)
    return q


def tv_norm(g: Geom, f, lambda2: float, S=None) -> float:
    S = tables(g)["S"] if S is None else _f64(S)
    f = _f64(f).reshape(g.Nz, g.N, g.N, g.K)
    return _L().or_tv_norm(ctypes.byref(g.c()), _p(S), ctypes.c_double(lambda2), _p(f))


def S_norm(g: Geom, S=None) -> float:
    S = tables(g)["S"] if S is None else _f64(S)
    return _L().or_S_norm(ctypes.byref(g.c()), _p(S))


def seeded_uniform(seed: int, n: int) -> np.ndarray:
    """Values 0..n-1 of the counter-based SplitMix64 uniform(-1,1) stream."""
    f = _L().or_seeded_uniform
    return np.array([f(seed, j) for j in range(n)])


def power(g: Geom, n_pow: int = 20, seed: int = 0, route: str = "direct") -> float:
    T = tables(g)
    return _L().or_power(ctypes.byref(g.c()), 1 if route == "folded" else 0,
                         _p(T["theta"]), _p(T["phi"]), ctypes.c_int(n_pow),
                         ctypes.c_uint64(seed))


def solve(g: Geom, data, *, lambda1: float, lambda2: float, n_iter: int, f0=None,
          tau: float = 0.0, sigma: float = 0.0, tol: float = 0.0, n_pow: int = 20,
          check_every: int = 0, seed: int = 0, route: str = "direct", phi=None, S=None,
          mu: float = 0.0, variant: str = "plain"):
    """Adapted Chambolle-Pock loop (Sec. 3, Fig. 2).  Returns (f, report dict).

    mu > 0 adds the uniformly convex term mu/2 |f|^2 (the primal step becomes
    its prox); variant="accel" is the accelerated form with adaptive theta,
    tau and sigma (the O(1/N^2) variant that Secs. 1 and 8 name)."""
    T = tables(g)
    phi = T["phi"] if phi is None else _f64(phi)
    S = T["S"] if S is None else _f64(S)
    data = _f64(data).reshape(g.Ntheta, g.Nz, g.Ns)
    f = np.zeros((g.Nz, g.N, g.N, g.K)) if f0 is None else _f64(f0).reshape(g.Nz, g.N, g.N, g.K).copy()
    if variant not in ("plain", "accel"):
        raise ValueError(variant)
    prm = _Params(lambda1, lambda2, tol, tau, sigma, n_iter, n_pow, check_every,
                  1 if route == "folded" else 0, seed, mu, 1 if variant == "accel" else 0)
    rep = _Report()
    _L().or_solve(ctypes.byref(g.c()), _p(T["theta"]), _p(phi), _p(S), ctypes.byref(prm),
                  _p(data), _p(f), ctypes.byref(rep))
    return f, {n: getattr(rep, n) for n, _ in _Report._fields_}


def shepp_logan(g: Geom, s) -> np.ndarray:
    """Projections convolved with the Shepp-Logan kernel over the detector
    (the filter of the FBP initial guess, Secs. 5-6)."""
    s = _f64(s).reshape(g.Ntheta, g.Nz, g.Ns)
    out = np.zeros((g.Ntheta, g.Nz, g.Ns))
    _L().or_shepp_logan(ctypes.byref(g.c()), _p(s), _p(out))
    return out


def half_turn_means(g: Geom, phi=None) -> np.ndarray:
    """B[m][k]: the mean of phi_k over the projections of half-turn m.  A
    frame reconstructed from one half-turn sees the object averaged over
    that half-turn, sum_k B[m][k] f_k."""
    phi = tables(g)["phi"] if phi is None else _f64(phi)
    return phi.reshape(g.Npi, g.n0, g.K).mean(axis=1)


def fbp_frames(g: Geom, s) -> np.ndarray:
    """One static FBP per half-turn (Sec. 5: frame m from the projections in
    [m pi, (m+1) pi)): the filtered projections of half-turn m, back-projected
    with the transpose of the projector and weighted by the angle step
    pi / Ntheta0.  Returns (Nz, N, N, Npi)."""
    q = shepp_logan(g, s)
    gm = Geom(g.N, g.Nz, g.Ns, g.Ntheta, g.Npi, g.Npi, g.Npi)
    rot = tables(g)["rot"]
    ind = np.zeros((g.Ntheta, g.Npi))
    ind[np.arange(g.Ntheta), rot] = np.pi / g.n0
    return adjoint(gm, q, phi=ind)


def fbp(g: Geom, s, phi=None) -> np.ndarray:
    """Initial guess f_k (Secs. 5-6): the half-turn FBP frames F_m, then the
    minimum-norm least-squares coefficients of sum_k B[m][k] f_k = F_m
    (numpy's pseudo-inverse of B).  Returns (Nz, N, N, K)."""
    F = fbp_frames(g, s)
    A = np.linalg.pinv(half_turn_means(g, phi))      # (K, Npi)
    return F @ A.T


def num_threads() -> int:
    return _L().or_num_threads()

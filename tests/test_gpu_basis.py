"""A caller-supplied temporal basis: the real Fourier basis of the paper's
validation (Sec. 5 uses a Fourier basis of M functions; for a real object its
complex exponentials pair into cos/sin), passed through the ABI's phi and S
arguments, against the FP64 oracle given the same tables."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1809_09725_amd import inputs, rt4d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def fourier(G):
    """phi[i][k]: 1, cos(2 pi j t_i), sin(2 pi j t_i) for j = 1 .. (K-1)/2, t_i = i/Ntheta;
    S: the basis at the start of each half-turn."""
    t = np.arange(G.Ntheta) / G.Ntheta
    cols = [np.ones_like(t)]
    for j in range(1, (G.K - 1) // 2 + 1):
        cols += [np.cos(2 * math.pi * j * t), np.sin(2 * math.pi * j * t)]
    phi = np.stack(cols[:G.K], axis=1)
    n0 = G.Ntheta // G.Npi
    S = phi[[m * n0 for m in range(G.Nt)]]
    return phi, S


def og(G):
    return O.Geom(**G.__dict__)


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)


G7 = rt4d.Geom(N=48, Nz=2, Ns=50, Ntheta=8 * 12, Npi=8, K=7, Nt=8)


@pytest.mark.parametrize("form", ["pf", "sf"])
def test_fourier_basis_operator_parity(form):
    torch.cuda.set_device(DEV)
    phi, S = fourier(G7)
    plan = rt4d.Plan(G7, form=rt4d.RT_FORM_PF if form == "pf" else rt4d.RT_FORM_SF,
                     prec=rt4d.RT_PREC_FP32 if form == "pf" else rt4d.RT_PREC_BF16MFMA,
                     phi=phi, S=S)
    f = inputs.uniform(G7.f_shape, 71)
    s = inputs.uniform(G7.g_shape, 72)
    ef = rel(plan.forward(T(f)).cpu().numpy(), O.forward(og(G7), f, phi=phi))
    ea = rel(plan.adjoint(T(s)).cpu().numpy(), O.adjoint(og(G7), s, phi=phi))
    tol = 1e-5 if form == "pf" else 3e-3
    print(f"{form}: forward {ef:.2e} adjoint {ea:.2e}")
    assert ef <= tol and ea <= tol
    if form == "pf":
        p = plan.tv_grad(T(f), 4.0)
        ref = O.tv_grad(og(G7), f, 4.0, S=S).transpose(0, 3, 4, 1, 2)   # oracle (Nz,N,N,Nt,4)
        assert rel(p.cpu().numpy(), ref) <= 1e-5


def test_fourier_basis_solve_parity():
    torch.cuda.set_device(DEV)
    G = G7
    phi, S = fourier(G)
    g = inputs.uniform(G.g_shape, 73, 0.0, 1.0)
    _, r0 = O.solve(og(G), g, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=5,
                    phi=phi, S=S)
    kw = dict(lambda1=2.0 ** -9 * r0["L_R"] ** 2, lambda2=4.0, n_iter=20, tau=r0["tau"],
              sigma=r0["sigma"])
    plan = rt4d.Plan(G, phi=phi, S=S)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = plan.solve(T(g), f, **kw)
    fo, ro = O.solve(og(G), g, phi=phi, S=S, **kw)
    e = rel(f.cpu().numpy(), fo)
    print(f"Fourier-basis solve rel {e:.2e}")
    assert e <= 1e-3
    assert abs(rep["objective"] - ro["objective"]) <= 1e-4 * abs(ro["objective"])


def test_paper_fourier_m16_many_half_turns_operators():
    """The paper's M = 16 Fourier basis (Sec. 6; K = 15 real functions from
    the library's table) over its 130 half-turns: synthesise-first refuses
    Npi > 32, so the automatic form choice runs project-first in FP32;
    forward and adjoint against the FP64 oracle given the same tables."""
    torch.cuda.set_device(DEV)
    G = rt4d.Geom(N=40, Nz=2, Ns=44, Ntheta=130 * 3, Npi=130, K=15, Nt=2)
    phi, S = rt4d.basis_fourier(G, 16)
    plan = rt4d.Plan(G, form=rt4d.RT_FORM_AUTO, prec=rt4d.RT_PREC_BF16MFMA, phi=phi, S=S)
    assert (plan.form, plan.prec) == (rt4d.RT_FORM_PF, rt4d.RT_PREC_FP32)
    f = inputs.uniform(G.f_shape, 74)
    s = inputs.uniform(G.g_shape, 75)
    ef = rel(plan.forward(T(f)).cpu().numpy(), O.forward(og(G), f, phi=phi, route="folded"))
    ea = rel(plan.adjoint(T(s)).cpu().numpy(), O.adjoint(og(G), s, phi=phi, route="folded"))
    print(f"M=16 over 130 half-turns: forward {ef:.2e} adjoint {ea:.2e}")
    assert ef <= 1e-5 and ea <= 1e-5
    plan.close()


def test_paper_fourier_m16_solve():
    """M = 16 (K = 15) with 40 half-turns and the TV on 40 frames: 20
    iterations of the automatically chosen (project-first FP32) loop against
    the oracle's, iterate within 1e-3."""
    torch.cuda.set_device(DEV)
    G = rt4d.Geom(N=32, Nz=2, Ns=36, Ntheta=40 * 4, Npi=40, K=15, Nt=40)
    phi, S = rt4d.basis_fourier(G, 16)
    g = inputs.uniform(G.g_shape, 76, 0.0, 1.0)
    _, r0 = O.solve(og(G), g, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=5,
                    phi=phi, S=S, route="folded")
    kw = dict(lambda1=2.0 ** -9 * r0["L_R"] ** 2, lambda2=4.0, n_iter=20, tau=r0["tau"],
              sigma=r0["sigma"])
    plan = rt4d.Plan(G, form=rt4d.RT_FORM_AUTO, prec=rt4d.RT_PREC_BF16MFMA, phi=phi, S=S)
    assert plan.form == rt4d.RT_FORM_PF
    f = torch.zeros(G.f_shape, device=DEV)
    rep = plan.solve(T(g), f, **kw)
    fo, ro = O.solve(og(G), g, phi=phi, S=S, route="folded", **kw)
    e = rel(f.cpu().numpy(), fo)
    m = float(np.abs(f.cpu().numpy() - fo).max() / np.abs(fo).max())
    print(f"M=16 solve: rel {e:.2e}, scaled max-abs {m:.2e}")
    assert e <= 1e-3 and m <= 1e-3
    assert abs(rep["objective"] - ro["objective"]) <= 1e-4 * abs(ro["objective"])
    plan.close()

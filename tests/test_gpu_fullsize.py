"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times.

Slices are independent under parallel-beam geometry, so the operators are
checked slice by slice: a few sampled slices carry seeded random data and are
compared with the FP64 oracle on that slice alone; every other slice is zero
and must come out exactly zero (no cross-slice leakage).  The 2048^2 slab,
whose slices the oracle cannot finish in seconds, is checked on properties
that hold at any size: the adjoint identity in FP64, agreement of the two
forms, and the zero slices."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1809_09725_amd import inputs, rt4d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)

C2 = rt4d.Geom(N=512, Nz=128, Ns=512, Ntheta=1800, Npi=10, K=16, Nt=10)
C3 = rt4d.Geom(N=1024, Nz=64, Ns=1024, Ntheta=3600, Npi=12, K=16, Nt=12)
C5 = rt4d.Geom(N=2048, Nz=32, Ns=2048, Ntheta=3600, Npi=12, K=32, Nt=12)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def close(got, want, tol, what=""):
    """rel-L2 <= tol and max |got - want| <= tol * max |want|."""
    a = np.asarray(got, np.float64)
    b = np.asarray(want, np.float64)
    e = rel(a, b)
    m = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
    print(f"  {what}: rel-L2 {e:.3e}, scaled max-abs {m:.3e} (tol {tol:.0e})", flush=True)
    assert e <= tol and m <= tol, (what, e, m, tol)


def slice_geom(G):
    return O.Geom(N=G.N, Nz=1, Ns=G.Ns, Ntheta=G.Ntheta, Npi=G.Npi, K=G.K, Nt=G.Nt)


def sparse_f(G, zs, seed):
    f = torch.zeros(G.f_shape, device=DEV)
    host = {}
    for z in zs:
        h = inputs.uniform((G.N, G.N, G.K), seed + z)
        host[z] = h
        f[z].copy_(torch.from_numpy(h))
    return f, host


def sparse_g(G, zs, seed):
    g = torch.zeros(G.g_shape, device=DEV)
    host = {}
    for z in zs:
        h = inputs.uniform((G.Ntheta, G.Ns), seed + z)
        host[z] = h
        g[:, z, :].copy_(torch.from_numpy(h))
    return g, host


def others_zero_forward(g, zs):
    mask = torch.ones(g.shape[1], dtype=torch.bool, device=DEV)
    mask[list(zs)] = False
    return bool((g[:, mask, :] == 0).all().item())


def others_zero_adjoint(f, zs):
    mask = torch.ones(f.shape[0], dtype=torch.bool, device=DEV)
    mask[list(zs)] = False
    return bool((f[mask] == 0).all().item())


def check_sampled(G, form, prec, zf, za, tol, route="direct"):
    torch.cuda.set_device(DEV)
    plan = rt4d.Plan(G, form=form, prec=prec)
    og = slice_geom(G)
    f, fh = sparse_f(G, zf, 11)
    g = plan.forward(f)
    torch.cuda.synchronize()
    assert others_zero_forward(g, zf)
    for z in zf:
        ref = O.forward(og, fh[z][None], route=route)[:, 0, :]
        close(g[:, z, :].cpu().numpy(), ref, tol, f"forward slice {z}")
    del f, g
    gi, gh = sparse_g(G, za, 23)
    fo = plan.adjoint(gi)
    torch.cuda.synchronize()
    assert others_zero_adjoint(fo, za)
    for z in za:
        ref = O.adjoint(og, gh[z][:, None, :], route=route)[0]
        close(fo[z].cpu().numpy(), ref, tol, f"adjoint slice {z}")
    plan.close()


def test_c2_plain_sampled_slices():
    check_sampled(C2, rt4d.RT_FORM_PF, rt4d.RT_PREC_FP32, (0, 77, 127), (0, 127), 1e-5)


def test_c2_precision_sampled_slices():
    check_sampled(C2, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA, (5,), (5,), 3e-3)


def test_c3_precision_sampled_slices():
    # the precision form's error against the FP64 oracle on a subset of the 64 slices
    check_sampled(C3, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA, (0, 9, 18, 27, 36, 45, 54, 63),
                  (0, 63), 3e-3)


def test_c5_launch_configurations_against_oracle():
    """The 2048^2, 2048-bin, K = 32 slab's launch configurations (plain form:
    one class per group, 2048-bin tiles, 8-channel chunks; precision form: 4
    bins per thread, 2 MFMA k-steps, the staged B ring, 4 line parts) depend
    on N, Ns, K and Npi but not on the number of classes per half-turn, so a
    slab of the same sizes with 25 classes per half-turn (300 projections
    over the 12 half-turns) runs the very kernels of the full workload.  One
    slice of seeded data against the FP64 oracle's folded route: <= 1e-5
    plain, <= 3e-3 precision."""
    G = rt4d.Geom(N=2048, Nz=2, Ns=2048, Ntheta=12 * 25, Npi=12, K=32, Nt=12)
    check_sampled(G, rt4d.RT_FORM_PF, rt4d.RT_PREC_FP32, (1,), (0,), 1e-5, route="folded")
    check_sampled(G, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA, (0,), (1,), 3e-3, route="folded")


def test_c2_solve_four_slices():
    """The solver at the 512^2 workload on a 4-slice subset (the TV couples
    the slices): 20 iterations of the plain form from the noisy sinogram of
    a moving phantom with the workload's step rule, against the FP64
    oracle's 20 iterations (folded route), iterate within 1e-3."""
    torch.cuda.set_device(DEV)
    G = rt4d.Geom(N=512, Nz=4, Ns=512, Ntheta=1800, Npi=10, K=16, Nt=10)
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, 40, seed=2, axis_range=(G.N / 64, G.N / 16),
                             z_axis_range=(1.0, 2.0), rho_range=(0.1, 0.5),
                             speed_per_halfturn=G.N / 64)
    g = inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=2,
                        device="cuda").float().contiguous()
    # the workload's steps: tau = sigma = 1/sqrt((1.01 L_R)^2 + L_G^2) with
    # L_R = 940.06 (power iteration of the full workload), L_G = 36.13
    tau = 1.0 / np.hypot(1.01 * 940.06, 36.13)
    kw = dict(lambda1=2.0 ** -9 * 940.0 ** 2, lambda2=4.0, n_iter=20, tau=tau, sigma=tau)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = rt4d.Plan(G).solve(g, f, **kw)
    og = O.Geom(N=G.N, Nz=G.Nz, Ns=G.Ns, Ntheta=G.Ntheta, Npi=G.Npi, K=G.K, Nt=G.Nt)
    fo, ro = O.solve(og, g.cpu().numpy(), route="folded", **kw)
    print(f"C2 4-slice solve, 20 iterations: objective {rep['objective']:.9e} "
          f"vs {ro['objective']:.9e}", flush=True)
    close(f.cpu().numpy(), fo, 1e-3, "C2 4-slice solve iterate")
    assert abs(rep["objective"] - ro["objective"]) <= 1e-4 * abs(ro["objective"])


def test_c3_precision_every_slice():
    """All 64 slices of the 1024^2 x 64 workload: the precision form against
    the plain FP32 form, slice by slice (the plain form is within 1e-5 of the
    FP64 oracle on the sampled slices, so this is the precision form's error
    to within that)."""
    torch.cuda.set_device(DEV)
    G = C3
    f = torch.from_numpy(inputs.uniform(G.f_shape, 53)).to(DEV)
    pf = rt4d.Plan(G, form=rt4d.RT_FORM_PF, prec=rt4d.RT_PREC_FP32)
    ref = pf.forward(f)
    ra = pf.adjoint(ref)
    pf.close()
    sf = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    got = sf.forward(f)
    ga = sf.adjoint(ref)
    torch.cuda.synchronize()
    num = torch.linalg.vector_norm((got - ref).double(), dim=(0, 2))
    den = torch.linalg.vector_norm(ref.double(), dim=(0, 2))
    e = (num / den).cpu().numpy()
    numa = torch.linalg.vector_norm((ga - ra).double(), dim=(1, 2, 3))
    dena = torch.linalg.vector_norm(ra.double(), dim=(1, 2, 3))
    ea = (numa / dena).cpu().numpy()
    print(f"precision forward, 64 slices: rel {e.min():.3e} .. {e.max():.3e}; "
          f"adjoint: rel {ea.min():.3e} .. {ea.max():.3e}", flush=True)
    assert e.shape == (64,) and float(e.max()) <= 3e-3
    assert float(ea.max()) <= 3e-3
    sf.close()


def test_c5_properties():
    """2048^2 x 32 slab, K = 32: adjoint identity in FP64, precision vs plain
    form, exact zeros in the empty slices."""
    torch.cuda.set_device(DEV)
    G = C5
    zs = (0, 31)
    f, _ = sparse_f(G, zs, 31)
    g, _ = sparse_g(G, zs, 37)
    pf = rt4d.Plan(G, form=rt4d.RT_FORM_PF, prec=rt4d.RT_PREC_FP32)
    Rf = pf.forward(f)
    Rg = pf.adjoint(g)
    torch.cuda.synchronize()
    assert others_zero_forward(Rf, zs) and others_zero_adjoint(Rg, zs)
    lhs = rt4d.rt_dot(Rf, g)
    rhs = rt4d.rt_dot(f, Rg)
    scale = np.sqrt(rt4d.rt_dot(Rf, Rf) * rt4d.rt_dot(g, g))
    print(f"adjoint identity: |lhs-rhs|/scale = {abs(lhs - rhs) / scale:.3e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale   # Cauchy-Schwarz on the FP32 operator bar
    del Rg
    pf.close()
    sf = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    Rf16 = sf.forward(f)
    torch.cuda.synchronize()
    assert others_zero_forward(Rf16, zs)
    d = torch.linalg.vector_norm((Rf16 - Rf).double()) / torch.linalg.vector_norm(Rf.double())
    print(f"precision vs plain forward: rel {d.item():.3e}", flush=True)
    assert d.item() <= 3e-3
    sf.close()

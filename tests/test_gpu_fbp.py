"""The FBP initial guess on the GPU (rt_fbp_filter, rt_fbp) against the FP64
oracle: small shapes element by element, the 512^2 x 128 workload on sampled
slices, error paths, and its use as a warm start of the solver."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_1809_09725_amd import inputs, rt4d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def og(G, **kw):
    d = dict(N=G.N, Nz=G.Nz, Ns=G.Ns, Ntheta=G.Ntheta, Npi=G.Npi, K=G.K, Nt=G.Nt)
    d.update(kw)
    return O.Geom(**d)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch.cuda.set_device(DEV)
    yield
    torch.cuda.synchronize()


FILTER_SHAPES = [(1, 1), (3, 7), (50, 5), (512, 3), (1100, 2), (2100, 1)]   # (Ns, rows)


@pytest.mark.parametrize("Ns,nth", FILTER_SHAPES, ids=lambda v: str(v))
def test_filter_parity(Ns, nth):
    G = rt4d.Geom(N=4, Nz=1, Ns=Ns, Ntheta=nth, Npi=1, K=1, Nt=1)
    p = rt4d.Plan(G)
    g = inputs.uniform(G.g_shape, 70 + Ns)
    q = p.fbp_filter(T(g)).cpu().numpy()
    want = O.shepp_logan(og(G), g)
    e = rel(q, want)
    print(f"Ns={Ns}: rel {e:.2e}", flush=True)
    assert e <= 1e-5


FBP_SHAPES = [
    rt4d.Geom(N=64, Nz=1, Ns=64, Ntheta=720, Npi=8, K=8, Nt=8),
    rt4d.Geom(N=45, Nz=3, Ns=50, Ntheta=3 * 37, Npi=3, K=5, Nt=3),      # ragged, K % 4 != 0
    rt4d.Geom(N=32, Nz=2, Ns=40, Ntheta=6 * 20, Npi=6, K=4, Nt=6),      # K < Npi: least squares
    rt4d.Geom(N=33, Nz=2, Ns=40, Ntheta=2 * 45, Npi=2, K=16, Nt=2),     # K > Npi: minimum norm
    rt4d.Geom(N=20, Nz=1, Ns=23, Ntheta=12, Npi=1, K=1, Nt=1),          # static
]


@pytest.mark.parametrize("G", FBP_SHAPES, ids=lambda G: f"N{G.N}z{G.Nz}s{G.Ns}t{G.Ntheta}k{G.K}")
@pytest.mark.parametrize("form", ["pf", "sf"])
def test_fbp_parity(G, form):
    p = rt4d.Plan(G, form=rt4d.RT_FORM_SF if form == "sf" else rt4d.RT_FORM_PF,
                  prec=rt4d.RT_PREC_BF16MFMA if form == "sf" else rt4d.RT_PREC_FP32)
    g = inputs.uniform(G.g_shape, 80 + G.N)
    f0 = p.fbp(T(g)).cpu().numpy()
    want = O.fbp(og(G), g)
    e = rel(f0, want)
    print(f"{G} {form}: rel {e:.2e}", flush=True)
    assert e <= 1e-5


def test_fbp_with_a_supplied_basis():
    """A real Fourier basis (1, cos, sin pairs over the scan) passed in Phi."""
    G = rt4d.Geom(N=32, Nz=2, Ns=36, Ntheta=4 * 24, Npi=4, K=5, Nt=4)
    t = np.arange(G.Ntheta) / G.Ntheta
    cols = [np.ones_like(t)]
    for j in (1, 2):
        cols += [np.cos(2 * np.pi * j * t), np.sin(2 * np.pi * j * t)]
    phi = np.stack(cols, axis=1)
    p = rt4d.Plan(G, phi=phi)
    g = inputs.uniform(G.g_shape, 91)
    f0 = p.fbp(T(g)).cpu().numpy()
    e = rel(f0, O.fbp(og(G), g, phi=phi))
    print(f"Fourier basis: rel {e:.2e}", flush=True)
    assert e <= 1e-5


def test_fbp_c2_sampled_slices():
    """512^2 x 128, K = 16, 1800 projections over 10 half-turns: slices 0 and
    77 carry data and match the oracle slice by slice; every other slice is
    exactly zero."""
    G = rt4d.Geom(N=512, Nz=128, Ns=512, Ntheta=1800, Npi=10, K=16, Nt=10)
    zs = (0, 77)
    g = torch.zeros(G.g_shape, device=DEV)
    host = {}
    for z in zs:
        h = inputs.uniform((G.Ntheta, G.Ns), 500 + z)
        host[z] = h
        g[:, z, :].copy_(torch.from_numpy(h))
    p = rt4d.Plan(G)
    f0 = p.fbp(g)
    torch.cuda.synchronize()
    mask = torch.ones(G.Nz, dtype=torch.bool, device=DEV)
    mask[list(zs)] = False
    assert bool((f0[mask] == 0).all().item())
    for z in zs:
        want = O.fbp(og(G, Nz=1), host[z][:, None, :])[0]
        e = rel(f0[z].cpu().numpy(), want)
        print(f"slice {z}: rel {e:.2e}", flush=True)
        assert e <= 1e-5
    p.close()


def test_fbp_errors():
    L = rt4d.lib()
    G = rt4d.Geom(N=8, Nz=1, Ns=8, Ntheta=65, Npi=65, K=2, Nt=2)
    p = rt4d.Plan(G)
    g = torch.zeros(G.g_shape, device=DEV)
    f = torch.zeros(G.f_shape, device=DEV)
    rc = L.rt_fbp(p.h, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()), None)
    assert rc == rt4d.RT_E_SHAPE
    # two equal basis columns: the half-turn means are rank deficient
    G2 = rt4d.Geom(N=8, Nz=1, Ns=8, Ntheta=8, Npi=4, K=3, Nt=4)
    phi = np.ones((G2.Ntheta, G2.K))
    phi[:, 2] = np.arange(G2.Ntheta)
    p2 = rt4d.Plan(G2, phi=phi)
    g2 = torch.zeros(G2.g_shape, device=DEV)
    f2 = torch.zeros(G2.f_shape, device=DEV)
    rc = L.rt_fbp(p2.h, ctypes.c_void_p(g2.data_ptr()), ctypes.c_void_p(f2.data_ptr()), None)
    assert rc == rt4d.RT_E_ARG
    assert "rank" in L.rt_last_error().decode()
    # empty volume: nothing to do
    G3 = rt4d.Geom(N=8, Nz=0, Ns=8, Ntheta=8, Npi=2, K=2, Nt=2)
    p3 = rt4d.Plan(G3)
    assert L.rt_fbp(p3.h, None, None, None) == rt4d.RT_OK


def test_fbp_warm_start_lowers_the_objective():
    """Twenty iterations from the FBP guess end below twenty from zero, on the
    noisy sinogram of a moving phantom."""
    G = rt4d.Geom(N=64, Nz=4, Ns=64, Ntheta=8 * 48, Npi=8, K=8, Nt=8)
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, 6, seed=9, axis_range=(4, 14),
                             z_axis_range=(1, 3), rho_range=(0.2, 0.6), speed_per_halfturn=2.0)
    g = inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=9,
                        device="cuda").float().contiguous()
    p = rt4d.Plan(G)
    kw = dict(lambda1=2.0 ** -9 * 4 * 64.0 ** 2, lambda2=4.0, n_iter=20, n_pow=20, check_every=0, seed=1)
    f_zero = torch.zeros(G.f_shape, device=DEV)
    r_zero = p.solve(g, f_zero, **kw)
    f_fbp = p.fbp(g)
    r_fbp = p.solve(g, f_fbp, **kw)
    print(f"objective after 20 iterations: from 0 {r_zero['objective']:.4e}, "
          f"from FBP {r_fbp['objective']:.4e}", flush=True)
    assert r_fbp["objective"] < r_zero["objective"]

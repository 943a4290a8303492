"""The out-of-core solve (rt_solve_ooc) against the in-core solve: the same
iterate bit for bit, for every slab height from one slice to the whole
volume, and the same step sizes and report; and against the FP64 oracle's
solve, iterate within 1e-3."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1809_09725_amd import inputs, rt4d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def case(G, seed):
    g = torch.from_numpy(inputs.uniform(G.g_shape, seed, 0.0, 1.0))
    f0 = torch.from_numpy(0.1 * inputs.uniform(G.f_shape, seed + 1))
    return g.contiguous(), f0.contiguous()


def in_core(G, g, f0, **kw):
    p = rt4d.Plan(G)
    f = f0.to(DEV)
    rep = p.solve(g.to(DEV), f, **kw)
    torch.cuda.synchronize()
    p.close()
    return f.cpu(), rep


G7 = rt4d.Geom(N=48, Nz=7, Ns=50, Ntheta=4 * 30, Npi=4, K=6, Nt=4)


@pytest.mark.parametrize("slab", [1, 2, 3, 7, 10])
def test_ooc_equals_in_core(slab):
    torch.cuda.set_device(DEV)
    g, f0 = case(G7, 61)
    kw = dict(lambda1=2.0 ** -9 * 48.0 ** 2, lambda2=4.0, n_iter=6, n_pow=20, seed=3)
    ref, rr = in_core(G7, g, f0, **kw)
    f = f0.clone()
    ro = rt4d.solve_ooc(G7, g, f, slab, **kw)
    print(f"slab {slab}: max |diff| {float((f - ref).abs().max()):.3e}, "
          f"objective {ro['objective']:.9e} vs {rr['objective']:.9e}", flush=True)
    assert torch.equal(f, ref)
    assert ro["L_R"] == rr["L_R"] and ro["tau"] == rr["tau"] and ro["sigma"] == rr["sigma"]
    assert abs(ro["residual"] - rr["residual"]) <= 1e-12 * rr["residual"]
    assert abs(ro["objective"] - rr["objective"]) <= 1e-12 * rr["objective"]
    assert ro["iters_done"] == 6


G35 = rt4d.Geom(N=40, Nz=35, Ns=42, Ntheta=5 * 16, Npi=5, K=8, Nt=5)


@pytest.mark.parametrize("variant", ["plain", "accel"])
def test_ooc_ragged_slabs_equal_in_core(variant):
    """35 slices in slabs of 12 (the last one ragged, the middle one with
    both halos), N = 40 with Nt = 5 frames and K = 8, plain and with the
    uniformly convex term under the accelerated loop: the out-of-core
    iterate equals the in-core one bit for bit."""
    torch.cuda.set_device(DEV)
    g, f0 = case(G35, 131)
    kw = dict(lambda1=2.0 ** -9 * 40.0 ** 2, lambda2=3.0, n_iter=5, n_pow=10, seed=4)
    if variant == "accel":
        kw.update(mu=1.5, variant="accel")
    ref, rr = in_core(G35, g, f0, **kw)
    f = f0.clone()
    ro = rt4d.solve_ooc(G35, g, f, 12, **kw)
    print(f"{variant}: max |diff| {float((f - ref).abs().max()):.3e}", flush=True)
    assert torch.equal(f, ref)
    assert abs(ro["objective"] - rr["objective"]) <= 1e-12 * abs(rr["objective"])


def test_ooc_explicit_steps_supplied_basis_static_volume():
    """Explicit tau/sigma, a supplied real Fourier basis and S, and K = 1 on
    one slice (no z coupling) all reproduce the in-core iterate."""
    torch.cuda.set_device(DEV)
    G = rt4d.Geom(N=32, Nz=5, Ns=36, Ntheta=4 * 24, Npi=4, K=5, Nt=4)
    t = np.arange(G.Ntheta) / G.Ntheta
    cols = [np.ones_like(t)]
    for j in (1, 2):
        cols += [np.cos(2 * np.pi * j * t), np.sin(2 * np.pi * j * t)]
    phi = np.stack(cols, axis=1)
    S = phi[:: G.Ntheta // G.Nt][: G.Nt]
    g, f0 = case(G, 71)
    kw = dict(lambda1=0.5, lambda2=2.0, n_iter=4, tau=0.02, sigma=0.02)
    p = rt4d.Plan(G, phi=phi, S=S)
    ref = f0.to(DEV)
    p.solve(g.to(DEV), ref, **kw)
    f = f0.clone()
    rt4d.solve_ooc(G, g, f, 2, phi=phi, S=S, **kw)
    assert torch.equal(f, ref.cpu())
    G1 = rt4d.Geom(N=40, Nz=1, Ns=31, Ntheta=12, Npi=1, K=1, Nt=1)
    g1, f1 = case(G1, 81)
    ref1, _ = in_core(G1, g1, f1, lambda1=0.1, lambda2=1.0, n_iter=3, n_pow=5)
    f = f1.clone()
    rt4d.solve_ooc(G1, g1, f, 4, lambda1=0.1, lambda2=1.0, n_iter=3, n_pow=5)
    assert torch.equal(f, ref1)


def test_ooc_errors():
    torch.cuda.set_device(DEV)
    g, f0 = case(G7, 91)
    with pytest.raises(rt4d.RtError) as e:
        rt4d.solve_ooc(G7, g, f0.clone(), 0, lambda1=1.0, lambda2=1.0, n_iter=1)
    assert e.value.code == rt4d.RT_E_ARG
    with pytest.raises(rt4d.RtError) as e:
        rt4d.solve_ooc(G7, g, f0.clone(), 2, lambda1=1.0, lambda2=1.0, n_iter=1, check_every=1)
    assert e.value.code == rt4d.RT_E_ARG
    with pytest.raises(ValueError):
        rt4d.solve_ooc(G7, g.to(DEV), f0.clone(), 2, lambda1=1.0, lambda2=1.0, n_iter=1)


@pytest.mark.parametrize("variant", ["plain", "accel"])
def test_ooc_against_oracle(variant):
    """Slabs of 3 slices (three slabs, two of them with both halos) for 8
    iterations of the default step rule, plain and with the uniformly convex
    term under the accelerated loop: the iterate within 1e-3 of the oracle's
    (rel-L2, and the largest element error scaled by the largest value), the
    objective within 1e-4."""
    torch.cuda.set_device(DEV)
    g, f0 = case(G7, 101)
    og = O.Geom(**G7.__dict__)
    # steps from the oracle's own step rule (20 power steps), given to both
    _, r0 = O.solve(og, g.numpy(), lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=3,
                    route="folded")
    kw = dict(lambda1=2.0 ** -9 * 48.0 ** 2, lambda2=4.0, n_iter=8, tau=r0["tau"],
              sigma=r0["sigma"])
    if variant == "accel":
        kw.update(mu=2.0, variant="accel")
    f = f0.clone()
    ro = rt4d.solve_ooc(G7, g, f, 3, **kw)
    fo, rr = O.solve(og, g.numpy(), f0=f0.numpy(), route="folded", **kw)
    a, b = f.numpy().astype(np.float64), fo
    e = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    m = float(np.abs(a - b).max() / np.abs(b).max())
    print(f"{variant}: out-of-core vs oracle rel-L2 {e:.3e}, scaled max-abs {m:.3e}; objective "
          f"{ro['objective']:.9e} vs {rr['objective']:.9e}", flush=True)
    assert e <= 1e-3 and m <= 1e-3
    assert abs(ro["objective"] - rr["objective"]) <= 1e-4 * abs(rr["objective"])

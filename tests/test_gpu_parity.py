"""GPU parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances: tables bit-exact; operators rel-L2 <= 1e-5 (FP32 arithmetic
against FP64) and <= 3e-3 with the BF16 contraction; TV operators <= 1e-6;
reconstructions after a fixed iteration count rel-L2 <= 1e-3, in both forms.
Every array comparison also bounds the largest element error, scaled by the
largest reference value, so that a few wrong elements cannot hide in the norm:
max |got - want| <= tol * max |want| for FP32 results, and <= BF16_ELEM for
every result that passes through the BF16 contraction (the operator bar of that
form: one rounding of f~ to BF16 moves an element by up to 2^-9 of itself,
about 2e-3, which the norm averages and a single element does not)."""
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


BF16_ELEM = 3e-3   # element bar of results that pass through the BF16 contraction


def close(got, want, tol, what="", elem=None):
    """rel-L2 <= tol and max |got - want| <= elem * max |want| (elem defaults
    to tol); returns both."""
    elem = tol if elem is None else elem
    a = np.asarray(got, np.float64)
    b = np.asarray(want, np.float64)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    e = rel(a, b)
    m = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) if b.size else 0.0
    print(f"  {what}: rel-L2 {e:.2e} (tol {tol:.0e}), scaled max-abs {m:.2e} (tol {elem:.0e})",
          flush=True)
    assert e <= tol and m <= elem, (what, e, m, tol, elem)
    return e, m


def og(G):
    return O.Geom(**G.__dict__)


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(DEV)


C1 = rt4d.Geom(N=64, Nz=1, Ns=64, Ntheta=720, Npi=8, K=8, Nt=8)
SHAPES = [
    C1,
    rt4d.Geom(N=45, Nz=3, Ns=50, Ntheta=3 * 37, Npi=3, K=5, Nt=3),     # ragged, K % 4 != 0
    rt4d.Geom(N=70, Nz=2, Ns=70, Ntheta=4 * 25, Npi=4, K=12, Nt=4),    # two channel chunks
    rt4d.Geom(N=33, Nz=2, Ns=40, Ntheta=2 * 45, Npi=2, K=16, Nt=2),
    rt4d.Geom(N=40, Nz=1, Ns=31, Ntheta=12, Npi=1, K=1, Nt=1),         # static, K = 1
    rt4d.Geom(N=16, Nz=2, Ns=2100, Ntheta=4 * 4, Npi=4, K=4, Nt=4),    # 2 bin tiles
    rt4d.Geom(N=96, Nz=2, Ns=100, Ntheta=2 * 60, Npi=2, K=16, Nt=2),   # 1024 threads x 2 rays
    rt4d.Geom(N=150, Nz=2, Ns=192, Ntheta=2 * 90, Npi=2, K=16, Nt=2),  # ... lanes reordered in blocks of 64 bins
    rt4d.Geom(N=1024, Nz=1, Ns=96, Ntheta=2 * 8, Npi=2, K=8, Nt=2),    # 8 rays per thread
    rt4d.Geom(N=600, Nz=1, Ns=700, Ntheta=2 * 8, Npi=2, K=16, Nt=2),   # 16 channels in two chunks, block sums
    rt4d.Geom(N=1024, Nz=1, Ns=1024, Ntheta=2 * 4, Npi=2, K=16, Nt=2), # ... over 1024 positions and bins
    rt4d.Geom(N=2048, Nz=1, Ns=64, Ntheta=2 * 4, Npi=2, K=16, Nt=2),   # ... and one line buffer
    rt4d.Geom(N=1, Nz=1, Ns=1, Ntheta=1, Npi=1, K=1, Nt=1),            # one ray
]


@pytest.fixture(scope="module", autouse=True)
def _device():
    torch.cuda.set_device(DEV)
    yield
    torch.cuda.synchronize()


def test_tables_bit_exact():
    for G in (C1, SHAPES[1]):
        p = rt4d.Plan(G)
        got = p.tables()
        want = O.tables(og(G))
        for k in ("theta", "t", "cls", "rot", "flip"):
            assert np.array_equal(got[k], want[k]), k


@pytest.mark.parametrize("G", SHAPES, ids=lambda G: f"N{G.N}z{G.Nz}s{G.Ns}t{G.Ntheta}k{G.K}")
def test_forward_adjoint_parity(G):
    print(f"case {G}", flush=True)
    p = rt4d.Plan(G)
    for seed, maker in ((11, "uniform"), (12, "smooth")):
        if maker == "uniform":
            f = inputs.uniform(G.f_shape, seed)
        else:
            f = inputs.smooth_coeffs(G.N, G.Nz, G.K, seed)
        s = inputs.uniform(G.g_shape, seed + 100)
        Rf = p.forward(T(f)).cpu().numpy()
        Rs = p.adjoint(T(s)).cpu().numpy()
        close(Rf, O.forward(og(G), f), 1e-5, f"{maker} forward")
        close(Rs, O.adjoint(og(G), s), 1e-5, f"{maker} adjoint")


def test_adjoint_identity_on_gpu():
    G = SHAPES[2]
    p = rt4d.Plan(G)
    f = T(inputs.uniform(G.f_shape, 3))
    s = T(inputs.uniform(G.g_shape, 4))
    Rf, Rs = p.forward(f), p.adjoint(s)
    lhs, rhs = rt4d.rt_dot(Rf, s), rt4d.rt_dot(f, Rs)
    scale = np.sqrt(rt4d.rt_dot(Rf, Rf) * rt4d.rt_dot(s, s))
    assert abs(lhs - rhs) <= 2e-6 * scale


def test_rt_dot_fp64():
    x = torch.rand(1_000_003, device=DEV) - 0.5
    y = torch.rand(1_000_003, device=DEV) - 0.5
    want = float(np.dot(x.cpu().double().numpy(), y.cpu().double().numpy()))
    assert abs(rt4d.rt_dot(x, y) - want) <= 1e-12 * abs(want) + 1e-12
    assert rt4d.rt_dot(x[:0], y[:0]) == 0.0


@pytest.mark.parametrize("G", [SHAPES[1], SHAPES[2], rt4d.Geom(N=20, Nz=4, Ns=20, Ntheta=60, Npi=6, K=32, Nt=5),
                               rt4d.Geom(N=9, Nz=1, Ns=9, Ntheta=8, Npi=8, K=3, Nt=1)],
                         ids=lambda G: f"N{G.N}z{G.Nz}k{G.K}t{G.Nt}")
def test_tv_parity(G):
    p = rt4d.Plan(G)
    lam1, lam2 = 0.3, 2.5
    f = inputs.uniform(G.f_shape, 5)
    q = inputs.uniform(G.p_shape, 6)                  # library layout (Nz, Nt, 4, N, N)
    qo = np.ascontiguousarray(q.transpose(0, 3, 4, 1, 2))   # oracle layout (Nz, N, N, Nt, 4)
    pg = p.tv_grad(T(f), lam2).cpu().numpy()
    close(pg, O.tv_grad(og(G), f, lam2).transpose(0, 3, 4, 1, 2), 1e-6, "tv_grad")
    dv = p.tv_div(T(q), lam2).cpu().numpy()
    close(dv, O.tv_div(og(G), qo, lam2), 1e-6, "tv_div")
    sh = p.shrink(T(q), lam1).cpu().numpy()
    close(sh, O.shrink(qo, lam1).transpose(0, 3, 4, 1, 2), 1e-6, "shrink")
    assert np.abs(p.shrink(T(q), 0.0).cpu().numpy()).max() == 0.0


def test_solve_parity_c1():
    """C1 workload: moving ellipses, 50 iterations, explicit steps."""
    G = C1
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, 3, seed=1, axis_range=(2, 8), rho_range=(0.5, 1.0),
                             speed_per_halfturn=1.0)
    g = inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=1).numpy()
    p = rt4d.Plan(G)
    _, r0 = O.solve(og(G), g, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=9)
    L = r0["L_R"]
    lam1 = 2.0 ** -9 * L * L
    kw = dict(lambda1=lam1, lambda2=4.0, n_iter=50, tau=r0["tau"], sigma=r0["sigma"])
    f = torch.zeros(G.f_shape, device=DEV)
    rep = p.solve(T(g), f, **kw)
    fo, ro = O.solve(og(G), g, route="folded", **kw)
    print(f"C1 solve: objective {rep['objective']:.6e} vs {ro['objective']:.6e}")
    close(f.cpu().numpy(), fo, 1e-3, "C1 solve iterate")
    assert abs(rep["objective"] - ro["objective"]) <= 1e-4 * abs(ro["objective"])
    assert rep["iters_done"] == 50


def c1_problem():
    G = C1
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, 3, seed=1, axis_range=(2, 8), rho_range=(0.5, 1.0),
                             speed_per_halfturn=1.0)
    g = inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=1).numpy()
    _, r0 = O.solve(og(G), g, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=9)
    return G, g, r0


@pytest.mark.parametrize("variant", ["plain", "accel"])
def test_uniformly_convex_solve_c1(variant):
    """The model with the uniformly convex term mu/2 |f|^2 (mu = 1e-3 L_R^2),
    plain and accelerated loops (adaptive theta, tau, sigma): 60 iterations
    of the C1 workload against the oracle's, iterate within 1e-3, the
    objective (with the mu term) within 1e-4, and the report's steps are the
    initial ones."""
    G, g, r0 = c1_problem()
    L = r0["L_R"]
    kw = dict(lambda1=2.0 ** -9 * L * L, lambda2=4.0, n_iter=60, tau=r0["tau"], sigma=r0["sigma"],
              mu=1e-3 * L * L, variant=variant)
    p = rt4d.Plan(G)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = p.solve(T(g), f, **kw)
    fo, ro = O.solve(og(G), g, route="folded", **kw)
    print(f"{variant}: objective {rep['objective']:.9e} vs {ro['objective']:.9e}")
    close(f.cpu().numpy(), fo, 1e-3, f"mu > 0, {variant} iterate")
    assert abs(rep["objective"] - ro["objective"]) <= 1e-4 * abs(ro["objective"])
    assert rep["tau"] == r0["tau"] and rep["sigma"] == r0["sigma"]


def test_accelerated_checkpoint_resume_bitwise():
    """The accelerated loop's adapted steps survive a checkpoint: 20 + 20
    iterations through a restored job equal 40 in one go, bit for bit."""
    G = SHAPES[1]
    p = rt4d.Plan(G)
    g0 = inputs.uniform(G.g_shape, 33)
    g = T(g0)
    st = safe_steps(G, g0, 2.0)
    kw = dict(lambda1=0.1, lambda2=2.0, n_iter=40, tau=st, sigma=st, mu=0.5, variant="accel")
    fa = torch.zeros(G.f_shape, device=DEV)
    ja = rt4d.Job(p, g, fa, **kw)
    ja.step(40)
    fb = torch.zeros(G.f_shape, device=DEV)
    jb = rt4d.Job(p, g, fb, **kw)
    jb.step(20)
    ck = jb.checkpoint()
    jb.close()
    fc = torch.zeros(G.f_shape, device=DEV)
    jc = rt4d.Job(p, g, fc, **kw)
    jc.restore(ck)
    jc.step(40)
    torch.cuda.synchronize()
    assert jc.iters == 40 and torch.equal(fa, fc)
    assert ja.report() == jc.report()


def test_step_rule_power_iteration():
    G = SHAPES[1]
    p = rt4d.Plan(G)
    g = inputs.uniform(G.g_shape, 8)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = p.solve(T(g), f, lambda1=0.01, lambda2=1.0, n_iter=2, n_pow=20, seed=77)
    _, ro = O.solve(og(G), g, lambda1=0.01, lambda2=1.0, n_iter=2, n_pow=20, seed=77)
    assert abs(rep["L_R"] - ro["L_R"]) <= 1e-5 * ro["L_R"]
    assert abs(rep["L_G"] - ro["L_G"]) <= 1e-12 * ro["L_G"]
    assert abs(rep["tau"] - ro["tau"]) <= 1e-5 * ro["tau"]


def safe_steps(G, g, lambda2):
    """tau = sigma from the oracle's default rule (tau sigma |K|^2 < 1)."""
    _, r = O.solve(og(G), g, lambda1=0.0, lambda2=lambda2, n_iter=0, n_pow=30, seed=5)
    return r["tau"]


def test_solve_monitors_and_tolerance():
    G = SHAPES[1]
    p = rt4d.Plan(G)
    g = inputs.uniform(G.g_shape, 8)
    st = safe_steps(G, g, 2.0)
    kw = dict(lambda1=0.1, lambda2=2.0, n_iter=30, tau=st, sigma=st, check_every=5)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = p.solve(T(g), f, **kw)
    fo, ro = O.solve(og(G), g, **kw)
    assert rel(f.cpu().numpy(), fo) <= 1e-4
    assert abs(rep["rel_change"] - ro["rel_change"]) <= 1e-3 * ro["rel_change"]
    assert abs(rep["residual"] - ro["residual"]) <= 1e-5 * ro["residual"]
    kw.update(n_iter=1000, check_every=1, tol=1e-3)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = p.solve(T(g), f, **kw)
    _, ro = O.solve(og(G), g, **kw)
    assert abs(rep["iters_done"] - ro["iters_done"]) <= 1


def test_deterministic_bitwise():
    G = SHAPES[2]
    p = rt4d.Plan(G)
    f = T(inputs.uniform(G.f_shape, 21))
    s = T(inputs.uniform(G.g_shape, 22))
    assert torch.equal(p.forward(f), p.forward(f))
    assert torch.equal(p.adjoint(s), p.adjoint(s))
    a = torch.zeros(G.f_shape, device=DEV)
    b = torch.zeros(G.f_shape, device=DEV)
    r1 = p.solve(s, a, lambda1=0.1, lambda2=2.0, n_iter=7, check_every=7)
    r2 = p.solve(s, b, lambda1=0.1, lambda2=2.0, n_iter=7, check_every=7)
    assert torch.equal(a, b) and r1 == r2


def test_empty_and_errors():
    G = rt4d.Geom(N=16, Nz=0, Ns=16, Ntheta=16, Npi=2, K=4, Nt=2)
    p = rt4d.Plan(G)
    f = torch.zeros(G.f_shape, device=DEV)
    g = torch.zeros(G.g_shape, device=DEV)
    p.forward(f, g)
    p.adjoint(g, f)
    rep = p.solve(g, f, lambda1=0.1, lambda2=1.0, n_iter=3, tau=0.1, sigma=0.1)
    assert rep["iters_done"] == 3 and rep["residual"] == 0.0
    G = SHAPES[1]
    p = rt4d.Plan(G)
    f = torch.zeros(G.f_shape, device=DEV)
    with pytest.raises(ValueError):
        p.forward(f[:, :, :, :-1])
    big = torch.zeros(G.f_shape[0] * G.f_shape[1] * G.f_shape[2] * G.f_shape[3] + 1, device=DEV)
    g = torch.zeros(G.g_shape, device=DEV)
    with pytest.raises(rt4d.RtError) as ei:   # 4-byte offset: not 16-byte aligned
        rt4d.lib()
        rc = rt4d.lib().rt_forward(p.h, rt4d.ctypes.c_void_p(big.data_ptr() + 4),
                                   rt4d.ctypes.c_void_p(g.data_ptr()), None)
        rt4d._check(rc)
    assert ei.value.code == rt4d.RT_E_ARG
    with pytest.raises(rt4d.RtError):
        p.solve(g, f, lambda1=-1.0, lambda2=1.0, n_iter=1)
    with pytest.raises(rt4d.RtError):
        p.shrink(torch.zeros(G.p_shape, device=DEV), -0.5)


def test_checkpoint_resume_bitwise():
    G = SHAPES[1]
    p = rt4d.Plan(G)
    g0 = inputs.uniform(G.g_shape, 31)
    g = T(g0)
    st = safe_steps(G, g0, 2.0)
    kw = dict(lambda1=0.1, lambda2=2.0, n_iter=50, tau=st, sigma=st)
    fa = torch.zeros(G.f_shape, device=DEV)
    ja = rt4d.Job(p, g, fa, **kw)
    ja.step(50)
    fb = torch.zeros(G.f_shape, device=DEV)
    jb = rt4d.Job(p, g, fb, **kw)
    jb.step(25)
    ck = jb.checkpoint()
    jb.close()
    fc = torch.full(G.f_shape, 3.0, device=DEV)
    jc = rt4d.Job(p, g, fc, **kw)
    jc.restore(ck)
    assert jc.iters == 25
    jc.step(100)
    assert jc.done and jc.iters == 50
    torch.cuda.synchronize()
    assert torch.equal(fa, fc)


# ------------------------------------------------- precision form (BF16 MFMA)

SF_SHAPES = [
    C1,
    rt4d.Geom(N=45, Nz=3, Ns=50, Ntheta=3 * 37, Npi=3, K=5, Nt=3),
    rt4d.Geom(N=70, Nz=2, Ns=70, Ntheta=4 * 25, Npi=4, K=12, Nt=4),
    rt4d.Geom(N=600, Nz=1, Ns=530, Ntheta=12 * 6, Npi=12, K=16, Nt=12),   # 2 chunks, 2 bins/thread
    rt4d.Geom(N=48, Nz=2, Ns=48, Ntheta=12 * 20, Npi=12, K=32, Nt=6),
    rt4d.Geom(N=40, Nz=1, Ns=1100, Ntheta=8 * 3, Npi=8, K=8, Nt=8),       # 4 bins per thread
    rt4d.Geom(N=16, Nz=2, Ns=2100, Ntheta=4 * 4, Npi=4, K=4, Nt=4),       # 2 bin tiles of 2048
    rt4d.Geom(N=1, Nz=1, Ns=1, Ntheta=1, Npi=1, K=1, Nt=1),
]


@pytest.mark.parametrize("G", SF_SHAPES, ids=lambda G: f"N{G.N}z{G.Nz}s{G.Ns}t{G.Ntheta}k{G.K}")
def test_precision_form_parity(G):
    """Synthesise-first forward and MFMA fold-sum adjoint: rel-L2 <= 3e-3
    against the FP64 oracle (BF16 f_k and sinogram, Phi as BF16 hi + lo)."""
    p = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    for seed, maker in ((41, "uniform"), (42, "smooth")):
        f = inputs.uniform(G.f_shape, seed) if maker == "uniform" else \
            inputs.smooth_coeffs(G.N, G.Nz, G.K, seed)
        s = inputs.uniform(G.g_shape, seed + 100)
        print(f"case {G} {maker}", flush=True)
        close(p.forward(T(f)).cpu().numpy(), O.forward(og(G), f), 3e-3, "precision forward")
        close(p.adjoint(T(s)).cpu().numpy(), O.adjoint(og(G), s), 3e-3, "precision adjoint")


def test_precision_form_line_parts():
    """A 2048^2 slice with K = 32 holds 256 MiB in BF16, so each workgroup
    walks a quarter of the lines and k_sf_finish adds the four partial ray
    sums: forward within 3e-3 of the oracle on two slices, and the h1 prox
    (with its FP64 residual monitor) of a short solve agrees with the plain
    form's."""
    G = rt4d.Geom(N=2048, Nz=2, Ns=64, Ntheta=2 * 4, Npi=2, K=32, Nt=2)
    p = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    f = inputs.uniform(G.f_shape, 43)
    close(p.forward(T(f)).cpu().numpy(), O.forward(og(G), f), 3e-3, "line parts: precision forward")
    g0 = inputs.uniform(G.g_shape, 44, 0.0, 1.0)
    kw = dict(lambda1=0.5, lambda2=1.0, n_iter=3, tau=1e-4, sigma=1e-4, check_every=1)
    f_sf = torch.zeros(G.f_shape, device=DEV)
    r_sf = p.solve(T(g0), f_sf, **kw)
    fo, ro = O.solve(og(G), g0, route="folded", **kw)
    close(f_sf.cpu().numpy(), fo, 1e-3, "line parts: precision solve iterate", BF16_ELEM)
    print(f"line parts: residual {r_sf['residual']:.9e} vs {ro['residual']:.9e}", flush=True)
    assert abs(r_sf["residual"] - ro["residual"]) <= 3e-3 * ro["residual"]


def test_precision_form_solve_c1():
    G = C1
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, 3, seed=1, axis_range=(2, 8), rho_range=(0.5, 1.0),
                             speed_per_halfturn=1.0)
    g = inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=1).numpy()
    _, r0 = O.solve(og(G), g, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=9)
    lam1 = 2.0 ** -9 * r0["L_R"] ** 2
    kw = dict(lambda1=lam1, lambda2=4.0, n_iter=50, tau=r0["tau"], sigma=r0["sigma"])
    p = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    f = torch.zeros(G.f_shape, device=DEV)
    rep = p.solve(T(g), f, **kw)
    fo, ro = O.solve(og(G), g, route="folded", **kw)
    print(f"precision-form C1 solve: objective {rep['objective']:.6e} vs {ro['objective']:.6e}")
    close(f.cpu().numpy(), fo, 1e-3, "precision-form C1 solve iterate", BF16_ELEM)
    assert abs(rep["objective"] - ro["objective"]) <= 1e-3 * abs(ro["objective"])


def test_precision_form_deterministic():
    G = SF_SHAPES[2]
    p = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    f = T(inputs.uniform(G.f_shape, 5))
    s = T(inputs.uniform(G.g_shape, 6))
    assert torch.equal(p.forward(f), p.forward(f))
    assert torch.equal(p.adjoint(s), p.adjoint(s))

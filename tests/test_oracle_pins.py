"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed-form Radon transforms, special angles that reduce to numpy sums, a
dense brute-force ray walk, exact identities of the paper (adjointness,
pi-periodicity fold), textbook TV identities, numpy/scipy linear algebra and
an independent optimiser for the regularised problem."""
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import Geom

RNG = np.random.default_rng(12345)


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ------------------------------------------------------------------ tables

def test_tables_invariants():
    g = Geom(N=8, Nz=1, Ns=8, Ntheta=720, Npi=8, K=8, Nt=8)
    T = O.tables(g)
    i = np.arange(g.Ntheta)
    assert (T["cls"] + g.n0 * T["rot"] == i).all()
    assert ((T["cls"] >= 0) & (T["cls"] < g.n0)).all()
    assert (T["flip"] == T["rot"] % 2).all()
    # theta = alpha t, alpha = Npi*pi (Sec. 2 and Sec. 4 eq. discrt)
    np.testing.assert_allclose(T["theta"], g.Npi * np.pi * T["t"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.diff(T["theta"]), np.pi / g.n0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(T["theta"][::g.n0], np.pi * np.arange(g.Npi), rtol=0, atol=1e-12)
    assert T["t"][0] == 0.0 and T["t"][-1] < 1.0
    # phi_0 == 1, every phi_k(0) == 1, cos(pi k / 2) at t = 1/2
    assert (T["phi"][:, 0] == 1.0).all() and (T["phi"][0, :] == 1.0).all()
    half = g.Ntheta // 2
    np.testing.assert_allclose(T["phi"][half, :4], [1, 0, -1, 0], atol=1e-15)
    # S: frames at the half-turn starts
    np.testing.assert_array_equal(T["S"], T["phi"][::g.n0][:g.Nt])


def test_tables_reject_non_multiple():
    with pytest.raises(ValueError):
        O.tables(Geom(N=8, Nz=1, Ns=8, Ntheta=10, Npi=3, K=2, Nt=2))


def test_splitmix64_golden():
    here = os.path.dirname(__file__)
    vals = [int(l, 16) for l in open(os.path.join(here, "golden", "splitmix64_seed0.txt"))
            if l.startswith("0x")]
    got = O.seeded_uniform(0, 3)
    want = [2.0 * ((v >> 40) / 16777216.0) - 1.0 for v in vals]
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------ projector geometry

def test_special_angles_reduce_to_sums():
    N = 9
    g = Geom(N=N, Nz=2, Ns=N, Ntheta=4, Npi=1, K=1, Nt=1)   # 0, 45, 90, 135 degrees
    f = RNG.uniform(-1, 1, (2, N, N, 1))
    out = O.forward(g, f)
    img = f[..., 0]
    # theta = 0: s = x, every ray is one column (sum over rows)
    np.testing.assert_allclose(out[0], img.sum(axis=1), rtol=1e-13, atol=1e-13)
    # theta = pi/2: s = y, every ray is one row
    np.testing.assert_allclose(out[2], img.sum(axis=2), rtol=1e-12, atol=1e-12)
    # theta = pi/4 with N = Ns odd: the central ray crosses the pixel centres
    # of the anti-diagonal (x + y = 0) with weight sqrt(2) each
    c = (N - 1) // 2
    anti = np.array([img[:, r, N - 1 - r] for r in range(N)]).sum(axis=0)
    np.testing.assert_allclose(out[1][:, c], math.sqrt(2) * anti, rtol=1e-12)


def joseph_matrix(N, Ns, thetas):
    """Dense system matrix by stepping each ray through the rows (or columns)
    and interpolating linearly between the two nearest pixel centres."""
    h = 0.5 * (N - 1)
    A = np.zeros((len(thetas) * Ns, N * N))
    for i, th in enumerate(thetas):
        c, s = math.cos(th), math.sin(th)
        for b in range(Ns):
            sb = b - 0.5 * (Ns - 1)
            row = i * Ns + b
            if abs(c) >= abs(s):
                for r in range(N):
                    pos = (sb - (r - h) * s) / c + h
                    q0 = math.floor(pos)
                    for q, w in ((q0, 1 - (pos - q0)), (q0 + 1, pos - q0)):
                        if 0 <= q < N:
                            A[row, r * N + q] += w / abs(c)
            else:
                for q in range(N):
                    pos = (sb - (q - h) * c) / s + h
                    r0 = math.floor(pos)
                    for r, w in ((r0, 1 - (pos - r0)), (r0 + 1, pos - r0)):
                        if 0 <= r < N:
                            A[row, r * N + q] += w / abs(s)
    return A


def weight_matrix(N, Ns, thetas):
    """Dense matrix from the single weight formula over every (bin, pixel)."""
    A = np.zeros((len(thetas) * Ns, N * N))
    for i, th in enumerate(thetas):
        for b in range(Ns):
            for r in range(N):
                for q in range(N):
                    A[i * Ns + b, r * N + q] = O.weight(th, b, q, r, N, Ns)
    return A


@pytest.mark.parametrize("N,Ns", [(8, 8), (7, 10)])
def test_dense_8x8_three_ways(N, Ns):
    """K = 1 (phi == 1) reduces R_T to the static projector over all angles;
    its matrix from the oracle equals the ray walk and the weight formula."""
    Npi, n0 = 2, 9
    g = Geom(N=N, Nz=1, Ns=Ns, Ntheta=Npi * n0, Npi=Npi, K=1, Nt=1)
    th = O.tables(g)["theta"]
    J = joseph_matrix(N, Ns, th)
    W = weight_matrix(N, Ns, th)
    np.testing.assert_allclose(W, J, atol=1e-13)
    cols = []
    for j in range(N * N):
        e = np.zeros((1, N, N, 1)); e.flat[j] = 1.0
        cols.append(O.forward(g, e).ravel())
    A = np.stack(cols, axis=1)
    np.testing.assert_allclose(A, J, atol=1e-13)
    Af = np.stack([O.forward(g, np.eye(N * N)[j].reshape(1, N, N, 1), route="folded").ravel()
                   for j in range(N * N)], axis=1)
    np.testing.assert_allclose(Af, J, atol=1e-12)
    # adjoint is the transpose, both routes
    rows = []
    for j in range(g.Ntheta * Ns):
        e = np.zeros((g.Ntheta, 1, Ns)); e.flat[j] = 1.0
        rows.append(O.adjoint(g, e).ravel())
    np.testing.assert_allclose(np.stack(rows, axis=0), J, atol=1e-13)
    rows = [O.adjoint(g, np.eye(g.Ntheta * Ns)[j].reshape(g.Ntheta, 1, Ns), route="folded").ravel()
            for j in range(g.Ntheta * Ns)]
    np.testing.assert_allclose(np.stack(rows, axis=0), J, atol=1e-12)


def gaussian_image(N, sigma, x0=0.0, y0=0.0):
    x = np.arange(N) - 0.5 * (N - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    return np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * sigma ** 2))


def gaussian_radon(theta, s, sigma, x0=0.0, y0=0.0):
    """Radon transform of exp(-|p - p0|^2 / (2 sigma^2)) (closed form)."""
    sh = x0 * np.cos(theta) + y0 * np.sin(theta)
    return math.sqrt(2 * math.pi) * sigma * np.exp(-(s - sh) ** 2 / (2 * sigma ** 2))


def test_gaussian_closed_form_second_order():
    errs = []
    for N in (32, 64, 128):
        sigma = N / 10
        x0, y0 = 0.11 * N, -0.07 * N
        g = Geom(N=N, Nz=1, Ns=N, Ntheta=12, Npi=1, K=1, Nt=1)
        th = O.tables(g)["theta"]
        f = gaussian_image(N, sigma, x0, y0)[None, :, :, None]
        out = O.forward(g, f)[:, 0, :]
        s = np.arange(N) - 0.5 * (N - 1)
        ref = np.stack([gaussian_radon(t, s, sigma, x0, y0) for t in th])
        errs.append(np.abs(out - ref).max() / ref.max())
    assert errs[0] < 1e-2
    # O(h^2) in units of the blob width: doubling the resolution quarters the error
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3, errs


def test_time_modulated_gaussian_closed_form():
    """f(x,y,t) = G(x,y) cos(3 pi t) is f_3 = G in the cosine basis, so
    R_T f (i, b) = cos(3 pi t_i) R G(theta_i, s_b) (Sec. 4 eq. radapr, exact
    for a represented object).  Pins the angle-time coupling and Phi."""
    N, Npi, n0, K = 64, 4, 15, 5
    g = Geom(N=N, Nz=1, Ns=N, Ntheta=Npi * n0, Npi=Npi, K=K, Nt=Npi)
    sigma, x0, y0 = 6.0, 9.0, -5.0
    f = np.zeros((1, N, N, K))
    f[0, :, :, 3] = gaussian_image(N, sigma, x0, y0)
    s = np.arange(N) - 0.5 * (N - 1)
    i = np.arange(g.Ntheta)
    th = i * np.pi / n0
    t = i / g.Ntheta
    ref = np.cos(3 * np.pi * t)[:, None] * np.stack([gaussian_radon(a, s, sigma, x0, y0) for a in th])
    for route in ("direct", "folded"):
        out = O.forward(g, f, route=route)[:, 0, :]
        assert np.abs(out - ref).max() < 3e-3 * np.abs(ref).max()


def ellipse_image(N, A, B, psi, x0, y0):
    x = np.arange(N) - 0.5 * (N - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = (X - x0) * math.cos(psi) + (Y - y0) * math.sin(psi)
    v = -(X - x0) * math.sin(psi) + (Y - y0) * math.cos(psi)
    return ((u / A) ** 2 + (v / B) ** 2 <= 1.0).astype(float)


def ellipse_radon(theta, s, A, B, psi, x0, y0):
    """Kak & Slaney: 2AB sqrt(a^2 - s'^2)/a^2, a^2 = A^2 cos^2(theta-psi) + B^2 sin^2."""
    a2 = (A * math.cos(theta - psi)) ** 2 + (B * math.sin(theta - psi)) ** 2
    sp = s - (x0 * math.cos(theta) + y0 * math.sin(theta))
    return np.where(sp * sp < a2, 2 * A * B * np.sqrt(np.maximum(a2 - sp * sp, 0)) / a2, 0.0)


def test_ellipse_closed_form_converges():
    errs = []
    for N in (64, 128, 256):
        sc = N / 64
        A, B, psi, x0, y0 = 17 * sc, 9 * sc, 0.6, 5.3 * sc, -3.1 * sc
        g = Geom(N=N, Nz=1, Ns=N, Ntheta=6, Npi=1, K=1, Nt=1)
        th = O.tables(g)["theta"]
        out = O.forward(g, ellipse_image(N, A, B, psi, x0, y0)[None, :, :, None], route="folded")[:, 0]
        s = np.arange(N) - 0.5 * (N - 1)
        ref = np.stack([ellipse_radon(t, s, A, B, psi, x0, y0) for t in th])
        errs.append(np.abs(out - ref).sum() / np.abs(ref).sum())
    assert errs[0] < 0.05
    assert errs[1] < 0.75 * errs[0] and errs[2] < 0.75 * errs[1], errs


# --------------------------------------------- identities of the paper (Sec. 4)

RAGGED = Geom(N=9, Nz=3, Ns=11, Ntheta=21, Npi=3, K=5, Nt=3)


@pytest.mark.parametrize("route", ["direct", "folded"])
def test_adjoint_identity(route):
    g = RAGGED
    f = RNG.uniform(-1, 1, (g.Nz, g.N, g.N, g.K))
    s = RNG.uniform(-1, 1, (g.Ntheta, g.Nz, g.Ns))
    Rf = O.forward(g, f, route=route)
    Rs = O.adjoint(g, s, route=route)
    lhs, rhs = np.vdot(Rf, s), np.vdot(f, Rs)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Rf) * np.linalg.norm(s)


def test_fold_equals_direct():
    """pi-periodicity with the s-flip (Sec. 4) and the fold-sum are exact."""
    g = RAGGED
    f = RNG.uniform(-1, 1, (g.Nz, g.N, g.N, g.K))
    s = RNG.uniform(-1, 1, (g.Ntheta, g.Nz, g.Ns))
    assert rel(O.forward(g, f, route="folded"), O.forward(g, f)) < 1e-12
    assert rel(O.adjoint(g, s, route="folded"), O.adjoint(g, s)) < 1e-12


def test_forward_is_linear_and_slices_independent():
    g = RAGGED
    f1 = RNG.uniform(-1, 1, (g.Nz, g.N, g.N, g.K))
    f2 = RNG.uniform(-1, 1, (g.Nz, g.N, g.N, g.K))
    a, b = 0.7, -1.9
    np.testing.assert_allclose(O.forward(g, a * f1 + b * f2),
                               a * O.forward(g, f1) + b * O.forward(g, f2), atol=1e-12)
    one = Geom(g.N, 1, g.Ns, g.Ntheta, g.Npi, g.K, g.Nt)
    np.testing.assert_allclose(O.forward(g, f1)[:, 1:2], O.forward(one, f1[1:2]), atol=1e-13)


# ---------------------------------------------------------------------- TV

TVG = Geom(N=7, Nz=4, Ns=7, Ntheta=20, Npi=5, K=6, Nt=4)


@pytest.mark.parametrize("g", [TVG, Geom(N=6, Nz=1, Ns=6, Ntheta=8, Npi=4, K=3, Nt=4),
                               Geom(N=5, Nz=3, Ns=5, Ntheta=6, Npi=1, K=2, Nt=1)])
def test_div_is_negative_adjoint_of_grad(g):
    lam2 = 2.5
    u = RNG.uniform(-1, 1, (g.Nz, g.N, g.N, g.K))
    p = RNG.uniform(-1, 1, (g.Nz, g.N, g.N, g.Nt, 4))
    lhs = np.vdot(O.tv_grad(g, u, lam2), p)
    rhs = -np.vdot(u, O.tv_div(g, p, lam2))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0) * 10


def test_grad_constant_and_ramp():
    g = TVG
    lam2 = 3.0
    S = O.tables(g)["S"]
    # constant field in k=0 (phi_0 = 1 in every frame): zero gradient everywhere
    f = np.zeros((g.Nz, g.N, g.N, g.K)); f[..., 0] = 4.2
    assert np.abs(O.tv_grad(g, f, lam2)).max() == 0.0
    # ramp along x in k=0: constant x-difference except the last column
    x = np.arange(g.N) - 3.0
    f[..., 0] = 0.5 * x[None, None, :]
    p = O.tv_grad(g, f, lam2)
    np.testing.assert_allclose(p[:, :, :-1, :, 0], 0.5, atol=1e-14)
    assert np.abs(p[:, :, -1, :, 0]).max() == 0.0
    assert np.abs(p[..., 1:]).max() == 0.0
    # ramp along z in k=1: frames scale by S[m,1] = cos(pi m / Npi)
    f = np.zeros((g.Nz, g.N, g.N, g.K)); f[..., 1] = 2.0 * np.arange(g.Nz)[:, None, None]
    p = O.tv_grad(g, f, lam2)
    cm = np.cos(np.pi * np.arange(g.Nt) / g.Npi)
    np.testing.assert_allclose(p[:-1, :, :, :, 2], np.broadcast_to(2.0 * cm, p[:-1, :, :, :, 2].shape),
                               atol=1e-14)
    # time difference of a static-in-space field in k=1: lambda2 (S[m+1,1]-S[m,1]) u
    u = RNG.uniform(-1, 1, (g.Nz, g.N, g.N))
    f = np.zeros((g.Nz, g.N, g.N, g.K)); f[..., 1] = u
    p = O.tv_grad(g, f, lam2)
    for m in range(g.Nt - 1):
        np.testing.assert_allclose(p[..., m, 3], lam2 * (cm[m + 1] - cm[m]) * u, atol=1e-13)
    assert np.abs(p[..., g.Nt - 1, 3]).max() == 0.0
    np.testing.assert_allclose(S[:, 1], cm, atol=1e-15)


def test_shrink_closed_form():
    p = RNG.normal(size=(50, 4)) * 3
    lam = 1.7
    q = O.shrink(p, lam).reshape(50, 4)
    n = np.linalg.norm(p, axis=1)
    for j in range(50):
        if n[j] <= lam:
            np.testing.assert_array_equal(q[j], p[j])        # identity inside the ball
        else:
            np.testing.assert_allclose(q[j], p[j] * lam / n[j], rtol=1e-15)
    assert (np.linalg.norm(q, axis=1) <= lam * (1 + 1e-15)).all()
    np.testing.assert_allclose(O.shrink(q, lam), q, rtol=1e-15)  # idempotent (to rounding)
    assert np.abs(O.shrink(p, 0.0)).max() == 0.0                # lambda1 = 0: ball {0}


def test_S_norm_matches_numpy():
    for g in (TVG, Geom(N=4, Nz=1, Ns=4, Ntheta=1800, Npi=10, K=16, Nt=10)):
        S = O.tables(g)["S"]
        assert abs(O.S_norm(g) - np.linalg.norm(S, 2)) < 1e-12 * np.linalg.norm(S, 2)


# ------------------------------------------------------------------ solver

TINY = Geom(N=5, Nz=2, Ns=6, Ntheta=12, Npi=3, K=3, Nt=3)


def dense_R(g):
    nf = g.Nz * g.N * g.N * g.K
    return np.stack([O.forward(g, np.eye(nf)[j].reshape(g.Nz, g.N, g.N, g.K)).ravel()
                     for j in range(nf)], axis=1)


def test_power_iteration_matches_svd():
    g = Geom(N=4, Nz=1, Ns=5, Ntheta=6, Npi=2, K=2, Nt=2)
    A = dense_R(g)
    smax = np.linalg.svd(A, compute_uv=False)[0]
    L = O.power(g, n_pow=3000, seed=7)
    assert abs(L - smax) <= 1e-10 * smax


def test_power_iteration_on_one_slice_is_the_full_norm():
    # the power iteration runs on slice 0 alone; the dense operator of all
    # slices (block-diagonal, identical blocks) has the same top singular value
    g = Geom(N=4, Nz=3, Ns=5, Ntheta=6, Npi=2, K=2, Nt=2)
    smax = np.linalg.svd(dense_R(g), compute_uv=False)[0]
    L = O.power(g, n_pow=3000, seed=7)
    assert abs(L - smax) <= 1e-10 * smax


def test_solve_least_squares_limit_is_pinv():
    """lambda1 = 0: h2 is projected to 0, the loop is CP for 1/2|Af-g|^2 from
    f0 = 0, whose iterates stay in range(A^T) and converge to pinv(A) g."""
    g = TINY
    A = dense_R(g)
    data = RNG.uniform(-1, 1, (g.Ntheta, g.Nz, g.Ns))
    f, rep = O.solve(g, data, lambda1=0.0, lambda2=1.0, n_iter=40000, n_pow=200)
    ref = np.linalg.pinv(A) @ data.ravel()
    assert rel(f.ravel(), ref) < 1e-6
    assert rep["iters_done"] == 40000
    assert rep["tau"] == rep["sigma"] > 0


def test_solve_matches_independent_optimiser():
    """lambda1 > 0: the CP limit minimises eq. lr12; compare its objective with
    SLSQP on the smooth epigraph form min 1/2|Af-g|^2 + lambda1 sum t_j,
    |D_j f|^2 <= t_j^2, t >= 0 (D_j the 4-vector of voxel-frame j)."""
    scipy_opt = pytest.importorskip("scipy.optimize")
    g = Geom(N=4, Nz=1, Ns=5, Ntheta=8, Npi=2, K=2, Nt=2)
    lam1, lam2 = 0.05, 2.0
    A = dense_R(g)
    nf = A.shape[1]
    D = np.stack([O.tv_grad(g, np.eye(nf)[j].reshape(g.Nz, g.N, g.N, g.K), lam2).ravel()
                  for j in range(nf)], axis=1)           # (n4*4, nf)
    truth = RNG.uniform(0, 1, nf)
    data = (A @ truth + 0.05 * RNG.normal(size=A.shape[0])).reshape(g.Ntheta, g.Nz, g.Ns)
    f, rep = O.solve(g, data, lambda1=lam1, lambda2=lam2, n_iter=60000, n_pow=200)

    def obj(fv):
        return 0.5 * np.sum((A @ fv - data.ravel()) ** 2) + \
            lam1 * np.sum(np.linalg.norm((D @ fv).reshape(-1, 4), axis=1))

    nj = D.shape[0] // 4
    x0 = np.concatenate([np.linalg.lstsq(A, data.ravel(), rcond=None)[0], np.ones(nj)])
    Dj = D.reshape(nj, 4, nf)
    cons = [{"type": "ineq",
             "fun": lambda x: x[nf:] ** 2 - np.einsum("jcn,n->jc", Dj, x[:nf]).__pow__(2).sum(1),
             "jac": lambda x: np.hstack([-2 * np.einsum("jc,jcn->jn", np.einsum("jcn,n->jc", Dj, x[:nf]), Dj),
                                         np.diag(2 * x[nf:])])},
            {"type": "ineq", "fun": lambda x: x[nf:], "jac": lambda x: np.hstack([np.zeros((nj, nf)), np.eye(nj)])}]

    def epi(x):
        r = A @ x[:nf] - data.ravel()
        return 0.5 * r @ r + lam1 * x[nf:].sum()

    def epi_jac(x):
        return np.concatenate([A.T @ (A @ x[:nf] - data.ravel()), lam1 * np.ones(nj)])

    res = scipy_opt.minimize(epi, x0, jac=epi_jac, constraints=cons, method="SLSQP",
                             options={"maxiter": 2000, "ftol": 1e-15})
    e_cp, e_ref = obj(f.ravel()), obj(res.x[:nf])
    assert e_cp <= e_ref * (1 + 1e-6) + 1e-12
    assert abs(rep["objective"] - e_cp) <= 1e-10 * e_cp
    # a wrong sign anywhere would leave the loop far from the minimum
    assert e_cp < obj(np.linalg.lstsq(A, data.ravel(), rcond=None)[0])


def test_solve_fixed_count_and_monitors():
    g = TINY
    data = RNG.uniform(-1, 1, (g.Ntheta, g.Nz, g.Ns))
    f1, r1 = O.solve(g, data, lambda1=0.1, lambda2=2.0, n_iter=30, tau=0.05, sigma=0.05,
                     check_every=5)
    f2, r2 = O.solve(g, data, lambda1=0.1, lambda2=2.0, n_iter=30, tau=0.05, sigma=0.05)
    np.testing.assert_array_equal(f1, f2)      # monitors do not change the iterates
    assert r1["rel_change"] > 0 and r2["rel_change"] == 0
    assert r1["L_R"] == 0.0                     # explicit tau/sigma: no power iteration
    Rf = O.forward(g, f1)
    assert abs(r1["residual"] - np.linalg.norm(Rf - data)) < 1e-12 * r1["residual"]
    f3, r3 = O.solve(g, data, lambda1=0.1, lambda2=2.0, n_iter=1000, tau=0.05, sigma=0.05,
                     check_every=1, tol=1e-3)
    assert 0 < r3["iters_done"] < 1000


def test_solve_scalar_worked_example():
    """Hand-worked iterates of Fig. 2 on the one-pixel problem (golden file)."""
    here = os.path.dirname(__file__)
    rows = [l.split() for l in open(os.path.join(here, "golden", "cp_scalar_hand.txt"))
            if l.strip() and not l.startswith("#")]
    g = Geom(N=1, Nz=1, Ns=1, Ntheta=1, Npi=1, K=1, Nt=1)
    assert O.forward(g, np.ones((1, 1, 1, 1)))[0, 0, 0] == 1.0
    for n, num, den in rows:
        f, _ = O.solve(g, np.ones((1, 1, 1)), lambda1=0.3, lambda2=1.0, n_iter=int(n),
                       tau=0.5, sigma=0.5)
        assert abs(f.item() - int(num) / int(den)) < 1e-15


# ---------------------------------------- accelerated form (uniformly convex G)

def test_accel_scalar_worked_example():
    """Hand-worked iterates of the accelerated loop on the one-pixel problem
    (golden file): adaptive theta, tau and sigma and the prox of mu/2 |f|^2."""
    here = os.path.dirname(__file__)
    rows = [l.split() for l in open(os.path.join(here, "golden", "cp_accel_scalar_hand.txt"))
            if l.strip() and not l.startswith("#")]
    g = Geom(N=1, Nz=1, Ns=1, Ntheta=1, Npi=1, K=1, Nt=1)
    for n, val in rows:
        f, rep = O.solve(g, np.ones((1, 1, 1)), lambda1=0.3, lambda2=1.0, n_iter=int(n),
                         tau=0.5, sigma=0.5, mu=8.0, variant="accel")
        assert abs(f.item() - float(val)) < 1e-15
        assert rep["tau"] == 0.5 and rep["sigma"] == 0.5      # the step rule's values
    # the plain loop on the same uniformly convex problem keeps theta = 1 and
    # fixed steps: its first iterate is the same, its second is not
    f1, _ = O.solve(g, np.ones((1, 1, 1)), lambda1=0.3, lambda2=1.0, n_iter=1, tau=0.5,
                    sigma=0.5, mu=8.0)
    f2, _ = O.solve(g, np.ones((1, 1, 1)), lambda1=0.3, lambda2=1.0, n_iter=2, tau=0.5,
                    sigma=0.5, mu=8.0)
    assert abs(f1.item() - 1 / 30) < 1e-16 and abs(f2.item() - 0.06476190476190476) > 1e-3


def test_accel_with_mu_zero_is_the_plain_loop():
    """mu = 0: theta_n = 1 and the steps stay fixed, so the accelerated form
    is the loop of Fig. 2 (up to the rounding of f+ + 1 (f+ - f) vs 2 f+ - f)."""
    g = TINY
    data = RNG.uniform(-1, 1, (g.Ntheta, g.Nz, g.Ns))
    kw = dict(lambda1=0.1, lambda2=2.0, n_iter=60, tau=0.05, sigma=0.05, check_every=10)
    fp, rp = O.solve(g, data, **kw)
    fa, ra = O.solve(g, data, variant="accel", mu=0.0, **kw)
    assert rel(fa, fp) < 1e-13
    assert abs(ra["objective"] - rp["objective"]) < 1e-12 * rp["objective"]


def test_tikhonov_limit_is_the_regularised_normal_equations():
    """lambda1 = 0, mu > 0: both forms converge to the unique minimiser of
    1/2 |Af - g|^2 + mu/2 |f|^2, i.e. (A^T A + mu I)^-1 A^T g (numpy solve)."""
    g = TINY
    A = dense_R(g)
    data = RNG.uniform(-1, 1, (g.Ntheta, g.Nz, g.Ns))
    mu = 1.0
    ref = np.linalg.solve(A.T @ A + mu * np.eye(A.shape[1]), A.T @ data.ravel())
    want = 0.5 * np.sum((A @ ref - data.ravel()) ** 2) + 0.5 * mu * ref @ ref
    f, rep = O.solve(g, data, lambda1=0.0, lambda2=1.0, n_iter=4000, n_pow=200, mu=mu)
    assert rel(f.ravel(), ref) < 1e-8
    assert abs(rep["objective"] - want) < 1e-12 * want
    # the accelerated form: |f_n - f*| = O(1/n)
    errs = []
    for n in (5000, 20000):
        f, rep = O.solve(g, data, lambda1=0.0, lambda2=1.0, n_iter=n, n_pow=200, mu=mu,
                         variant="accel")
        errs.append(rel(f.ravel(), ref))
    assert errs[1] < 3e-4 and errs[1] <= errs[0] / 3, errs
    assert abs(rep["objective"] - want) < 1e-6 * want


def test_accel_rate_and_minimiser_on_a_tv_problem():
    """lambda1 > 0, mu > 0 (the uniformly convex case of the accelerated
    method): the minimiser is unique; the plain loop converges to it, SLSQP on
    the epigraph form agrees, and the accelerated iterates approach it at
    least as fast as C/n (the O(1/N^2) bound on |f_n - f*|^2): every doubling
    of n at least halves the error."""
    scipy_opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(5)
    g = Geom(N=4, Nz=1, Ns=5, Ntheta=8, Npi=2, K=2, Nt=2)
    lam1, lam2, mu = 0.05, 2.0, 0.5
    A = dense_R(g)
    nf = A.shape[1]
    truth = rng.uniform(0, 1, nf)
    data = (A @ truth + 0.05 * rng.normal(size=A.shape[0])).reshape(g.Ntheta, g.Nz, g.Ns)
    star, _ = O.solve(g, data, lambda1=lam1, lambda2=lam2, n_iter=40000, n_pow=200, mu=mu)
    star = star.ravel()
    D = np.stack([O.tv_grad(g, np.eye(nf)[j].reshape(g.Nz, g.N, g.N, g.K), lam2).ravel()
                  for j in range(nf)], axis=1)
    nj = D.shape[0] // 4
    Dj = D.reshape(nj, 4, nf)

    def epi(x):
        r = A @ x[:nf] - data.ravel()
        return 0.5 * r @ r + lam1 * x[nf:].sum() + 0.5 * mu * x[:nf] @ x[:nf]

    def epi_jac(x):
        return np.concatenate([A.T @ (A @ x[:nf] - data.ravel()) + mu * x[:nf], lam1 * np.ones(nj)])

    cons = [{"type": "ineq",
             "fun": lambda x: x[nf:] ** 2 - np.einsum("jcn,n->jc", Dj, x[:nf]).__pow__(2).sum(1),
             "jac": lambda x: np.hstack([-2 * np.einsum("jc,jcn->jn", np.einsum("jcn,n->jc", Dj, x[:nf]), Dj),
                                         np.diag(2 * x[nf:])])},
            {"type": "ineq", "fun": lambda x: x[nf:], "jac": lambda x: np.hstack([np.zeros((nj, nf)), np.eye(nj)])}]
    x0 = np.concatenate([np.zeros(nf), np.ones(nj)])
    res = scipy_opt.minimize(epi, x0, jac=epi_jac, constraints=cons, method="SLSQP",
                             options={"maxiter": 3000, "ftol": 1e-16})

    def obj(fv):
        return 0.5 * np.sum((A @ fv - data.ravel()) ** 2) + 0.5 * mu * fv @ fv + \
            lam1 * np.sum(np.linalg.norm((D @ fv).reshape(-1, 4), axis=1))

    # the plain loop's limit is at least as good as SLSQP's point, and mu-strong
    # convexity bounds their distance: |x - x*|^2 <= 2 (E(x) - E(x*)) / mu
    e_star, e_ref = obj(star), obj(res.x[:nf])
    assert e_star <= e_ref * (1 + 1e-9)
    assert np.linalg.norm(res.x[:nf] - star) <= np.sqrt(2 * (e_ref - e_star) / mu) + 1e-6
    assert rel(res.x[:nf], star) < 2e-3
    errs = []
    for n in (50, 100, 200, 400, 800, 1600):
        f, _ = O.solve(g, data, lambda1=lam1, lambda2=lam2, n_iter=n, n_pow=200, mu=mu,
                       variant="accel")
        errs.append(rel(f.ravel(), star))
    assert all(b <= 0.5 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4

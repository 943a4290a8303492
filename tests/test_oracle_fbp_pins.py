"""Pins of the oracle's FBP initial guess (Secs. 5-6) against facts that do
not come from the oracle itself: the Shepp-Logan filter's closed-form
frequency response, the reconstruction of an analytic disc, the half-turn
symmetry of a static object, and the closed form of the half-turn means of
the cosine basis."""
import numpy as np
import pytest

import oracle as O


def test_shepp_logan_frequency_response():
    """The discrete Shepp-Logan kernel h(n) = -2/(pi^2 (4n^2-1)) has the
    response (1/pi)|sin(w/2)| (Shepp and Logan, 1974): the ramp |w|/(2 pi)
    near w = 0, rolled off towards the Nyquist frequency."""
    Ns = 4001
    g = O.Geom(N=1, Nz=1, Ns=Ns, Ntheta=1, Npi=1, K=1, Nt=1)
    row = np.zeros((1, 1, Ns))
    row[0, 0, Ns // 2] = 1.0
    h = O.shepp_logan(g, row)[0, 0]
    n = np.arange(Ns) - Ns // 2
    tail = 1.0 / (np.pi ** 2 * (Ns // 2))            # bound of the truncated sum
    for w in (0.0, 0.3, 1.0, 2.0, 3.0, np.pi):
        H = float(np.sum(h * np.cos(w * n)))
        assert abs(H - abs(np.sin(w / 2)) / np.pi) <= tail, w
    assert np.allclose(h, h[::-1], rtol=0, atol=1e-15)      # even kernel


def test_fbp_of_an_off_centre_disc():
    """Analytic projections of a disc (chord lengths 2 sqrt(R^2 - (s - s0)^2),
    s0 = x0 cos + y0 sin with x the column and y the row) reconstruct to its
    density inside and to zero outside."""
    N, n0 = 96, 120
    g = O.Geom(N=N, Nz=1, Ns=N, Ntheta=n0, Npi=1, K=1, Nt=1)
    th = O.tables(g)["theta"]
    sb = np.arange(N) - (N - 1) / 2
    R, x0, y0 = 30.0, 10.0, -5.0
    u = sb[None, :] - (x0 * np.cos(th) + y0 * np.sin(th))[:, None]
    p = np.where(np.abs(u) < R, 2 * np.sqrt(np.maximum(R * R - u * u, 0.0)), 0.0)
    F = O.fbp_frames(g, p[:, None, :])[0, :, :, 0]
    X, Y = np.meshgrid(sb, sb)                      # X: column, Y: row
    rr = np.hypot(X - x0, Y - y0)
    inside = F[rr < 0.8 * R]
    outside = F[(rr > 1.2 * R) & (np.hypot(X, Y) < 0.45 * N)]
    assert abs(inside.mean() - 1.0) < 5e-3
    assert np.abs(inside - 1.0).max() < 0.05
    assert abs(outside.mean()) < 0.01 and np.abs(outside).max() < 0.1


def test_static_object_gives_equal_frames():
    """Half-turn m sees the same object at theta0 + m pi, i.e. the same
    projections with the detector reversed on odd half-turns: every half-turn
    frame is the same image."""
    g = O.Geom(N=20, Nz=2, Ns=23, Ntheta=4 * 15, Npi=4, K=3, Nt=4)
    g0 = np.random.default_rng(3).random((g.n0, g.Nz, g.Ns))
    s = np.concatenate([g0 if m % 2 == 0 else g0[:, :, ::-1] for m in range(g.Npi)])
    F = O.fbp_frames(g, s)
    for m in range(1, g.Npi):
        assert np.abs(F[..., m] - F[..., 0]).max() <= 1e-12 * np.abs(F).max()
    # a moving object does not: the frames differ
    s2 = s.copy()
    s2[g.n0:2 * g.n0] *= 2.0
    F2 = O.fbp_frames(g, s2)
    assert np.abs(F2[..., 1] - 2 * F2[..., 0]).max() <= 1e-12 * np.abs(F2).max()


@pytest.mark.parametrize("Npi,n0,K", [(10, 18, 16), (3, 7, 5), (1, 9, 1)])
def test_half_turn_means_closed_form(Npi, n0, K):
    """Mean of cos(pi k i / Ntheta) over i in [m n0, (m+1) n0): the sum of a
    cosine series, sin(n0 d / 2) / sin(d / 2) cos(a + (n0 - 1) d / 2) / n0
    with a = pi k m n0 / Ntheta, d = pi k / Ntheta (and 1 for k = 0)."""
    Nth = Npi * n0
    g = O.Geom(N=4, Nz=1, Ns=4, Ntheta=Nth, Npi=Npi, K=K, Nt=1)
    B = O.half_turn_means(g)
    for m in range(Npi):
        for k in range(K):
            if k == 0:
                want = 1.0
            else:
                d = np.pi * k / Nth
                a = np.pi * k * m * n0 / Nth
                want = np.sin(n0 * d / 2) / np.sin(d / 2) * np.cos(a + (n0 - 1) * d / 2) / n0
            assert abs(B[m, k] - want) <= 1e-13


def test_initial_guess_reproduces_the_frames_and_fits_the_data():
    """The coefficients re-synthesise the half-turn frames (B has full row
    rank when K >= Npi), and the initial guess explains most of the data of a
    moving object."""
    from paper_1809_09725_amd import inputs
    g = O.Geom(N=32, Nz=2, Ns=36, Ntheta=4 * 24, Npi=4, K=6, Nt=4)
    f_true = inputs.smooth_coeffs(g.N, g.Nz, g.K, 5)
    s = O.forward(g, f_true)
    f0 = O.fbp(g, s)
    F = O.fbp_frames(g, s)
    B = O.half_turn_means(g)
    assert np.abs(f0 @ B.T - F).max() <= 1e-10 * np.abs(F).max()
    r0 = np.linalg.norm(O.forward(g, f0) - s) / np.linalg.norm(s)
    assert r0 < 0.5

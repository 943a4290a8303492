"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad geometry before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_1809_09725_amd import rt4d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rt4d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    L = rt4d.lib()
    names = header_functions()
    assert len(names) >= 20, names
    for n in names:
        assert hasattr(L, n), f"librt4d.so does not export {n}"
    assert set(names) == set(rt4d.EXPORTS)


def test_no_oracle_in_the_library():
    """The product library must not link or embed the oracle."""
    data = open(rt4d.LIB_PATH, "rb").read()
    for sym in (b"or_forward_direct", b"or_adjoint_direct", b"or_solve", b"liboracle"):
        assert sym not in data


@pytest.mark.parametrize("bad,code", [
    (dict(Ntheta=10, Npi=3), rt4d.RT_E_SHAPE),        # not whole half-turns
    (dict(Nt=9, Npi=8), rt4d.RT_E_SHAPE),             # more frames than half-turns
    (dict(N=0), rt4d.RT_E_SHAPE),
    (dict(K=0), rt4d.RT_E_SHAPE),
    (dict(Nz=-1), rt4d.RT_E_SHAPE),
    (dict(K=65), rt4d.RT_E_SHAPE),
    # lines longer than 2048 positions are staged as float4 only: K % 4 == 0
    (dict(N=3000, Ns=3000, K=15), rt4d.RT_E_SHAPE),
    (dict(N=4096, Ns=64, K=5), rt4d.RT_E_SHAPE),
])
def test_bad_geometry_rejected_before_any_launch(bad, code):
    g = dict(N=16, Nz=2, Ns=16, Ntheta=24, Npi=8, K=8, Nt=8)
    g.update(bad)
    geom = rt4d.Geom(**g)
    b = ctypes.c_size_t()
    rc = rt4d.lib().rt_job_bytes(ctypes.byref(geom.c()), 0, 0, ctypes.byref(b))
    assert rc == code
    assert rt4d.lib().rt_last_error().decode()
    h = ctypes.c_void_p()
    rc = rt4d.lib().rt_plan_create(ctypes.byref(geom.c()), 0, 0, None, None, ctypes.byref(h))
    assert rc == code and not h.value


def test_long_lines_accepted_with_float4_channels():
    """Above N = 2048 the plan needs K % 4 == 0; such shapes pass the host checks."""
    for n, k in ((3000, 16), (4096, 4), (2048, 15)):
        geom = rt4d.Geom(N=n, Nz=1, Ns=64, Ntheta=8, Npi=2, K=k, Nt=2)
        b = ctypes.c_size_t()
        assert rt4d.lib().rt_job_bytes(ctypes.byref(geom.c()), 0, 0, ctypes.byref(b)) == rt4d.RT_OK


def test_bad_enums_rejected():
    geom = rt4d.Geom(N=16, Nz=2, Ns=16, Ntheta=24, Npi=8, K=8, Nt=8)
    h = ctypes.c_void_p()
    assert rt4d.lib().rt_plan_create(ctypes.byref(geom.c()), 7, 0, None, None, ctypes.byref(h)) == rt4d.RT_E_ARG
    assert rt4d.lib().rt_plan_create(ctypes.byref(geom.c()), 0, 9, None, None, ctypes.byref(h)) == rt4d.RT_E_ARG
    # BF16 contraction only exists in the synthesise-first form
    assert rt4d.lib().rt_plan_create(ctypes.byref(geom.c()), rt4d.RT_FORM_PF, rt4d.RT_PREC_BF16MFMA,
                                     None, None, ctypes.byref(h)) == rt4d.RT_E_ARG


def test_job_bytes_accounts_for_state():
    geom = rt4d.Geom(N=512, Nz=128, Ns=512, Ntheta=1800, Npi=10, K=16, Nt=10)
    b = rt4d.rt_job_bytes(geom)
    nf = 128 * 512 * 512 * 16
    ng = 1800 * 128 * 512
    n4 = 128 * 512 * 512 * 10
    state = (2 * nf + 2 * ng + 5 * n4) * 4
    scratch = 180 * 128 * 512 * 16 * 4 + n4 * 4
    assert state + scratch <= b <= state + scratch + 64 * 2 ** 20
    # the precision form adds the BF16 shadow of f~ (K rounded up to 16 channels)
    b16 = rt4d.rt_job_bytes(geom, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA)
    assert b16 - b == 128 * 512 * 512 * 16 * 2
    # a 2048^2 slice at K = 32 is 256 MiB in BF16: four line parts of partial ray sums
    c5 = rt4d.Geom(N=2048, Nz=32, Ns=2048, Ntheta=3600, Npi=12, K=32, Nt=12)
    d5 = (rt4d.rt_job_bytes(c5, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA) - rt4d.rt_job_bytes(c5))
    assert d5 == 32 * 2048 * 2048 * 32 * 2 + 4 * 3600 * 32 * 2048 * 4
    g5 = rt4d.Geom(N=64, Nz=2, Ns=64, Ntheta=80, Npi=8, K=5, Nt=8)
    assert (rt4d.rt_job_bytes(g5, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA) -
            rt4d.rt_job_bytes(g5)) == 2 * 64 * 64 * 16 * 2


def test_null_handles():
    L = rt4d.lib()
    assert L.rt_forward(None, None, None, None) == rt4d.RT_E_ARG
    assert L.rt_job_step(None, 1, None) == rt4d.RT_E_ARG
    L.rt_plan_destroy(None)
    L.rt_job_destroy(None)


def test_ooc_rejects_bad_arguments_before_any_launch():
    """The out-of-core solve checks its arguments on the host first."""
    L = rt4d.lib()
    geom = rt4d.Geom(N=16, Nz=4, Ns=16, Ntheta=24, Npi=8, K=8, Nt=8)
    prm = rt4d.make_params(lambda1=1.0, lambda2=1.0, n_iter=1)
    rep = rt4d.rt_solve_report()
    buf = ctypes.c_void_p(1 << 20)   # never dereferenced: the checks fail first
    rc = L.rt_solve_ooc(ctypes.byref(geom.c()), None, None, ctypes.byref(prm), buf, buf, 0,
                        ctypes.byref(rep), None)
    assert rc == rt4d.RT_E_ARG and "slab" in L.rt_last_error().decode()
    prm2 = rt4d.make_params(lambda1=1.0, lambda2=1.0, n_iter=1, check_every=2)
    rc = L.rt_solve_ooc(ctypes.byref(geom.c()), None, None, ctypes.byref(prm2), buf, buf, 2,
                        ctypes.byref(rep), None)
    assert rc == rt4d.RT_E_ARG
    bad = rt4d.Geom(N=16, Nz=4, Ns=16, Ntheta=10, Npi=3, K=8, Nt=3)
    rc = L.rt_solve_ooc(ctypes.byref(bad.c()), None, None, ctypes.byref(prm), buf, buf, 2,
                        ctypes.byref(rep), None)
    assert rc == rt4d.RT_E_SHAPE
    rc = L.rt_solve_ooc(ctypes.byref(geom.c()), None, None, ctypes.byref(prm), None, None, 2,
                        ctypes.byref(rep), None)
    assert rc == rt4d.RT_E_ARG
    empty = rt4d.Geom(N=16, Nz=0, Ns=16, Ntheta=24, Npi=8, K=8, Nt=8)
    assert L.rt_solve_ooc(ctypes.byref(empty.c()), None, None, ctypes.byref(prm), None, None, 2,
                          ctypes.byref(rep), None) == rt4d.RT_OK


# ------------------------------------------------ form choice and Fourier basis (host only)

@pytest.mark.parametrize("K,Npi,prec,want", [
    (16, 8, rt4d.RT_PREC_BF16MFMA, rt4d.RT_FORM_SF),    # K >= 2 Npi
    (32, 8, rt4d.RT_PREC_BF16MFMA, rt4d.RT_FORM_SF),
    (15, 8, rt4d.RT_PREC_BF16MFMA, rt4d.RT_FORM_PF),    # K < 2 Npi
    (16, 12, rt4d.RT_PREC_BF16MFMA, rt4d.RT_FORM_PF),
    (64, 32, rt4d.RT_PREC_BF16MFMA, rt4d.RT_FORM_SF),
    (64, 33, rt4d.RT_PREC_BF16MFMA, rt4d.RT_FORM_PF),   # synthesise-first needs Npi <= 32
    (32, 8, rt4d.RT_PREC_FP32, rt4d.RT_FORM_PF),        # FP32: project-first only
])
def test_auto_form_rule(K, Npi, prec, want):
    G = rt4d.Geom(N=32, Nz=1, Ns=32, Ntheta=Npi * 4, Npi=Npi, K=K, Nt=1)
    fo, po = rt4d.form_pick(G, rt4d.RT_FORM_AUTO, prec)
    assert fo == want
    assert po == (rt4d.RT_PREC_BF16MFMA if want == rt4d.RT_FORM_SF else rt4d.RT_PREC_FP32)
    # explicit forms are checked, not changed
    assert rt4d.form_pick(G, rt4d.RT_FORM_PF, rt4d.RT_PREC_FP32) == (rt4d.RT_FORM_PF, rt4d.RT_PREC_FP32)
    with pytest.raises(rt4d.RtError):
        rt4d.form_pick(G, rt4d.RT_FORM_PF, rt4d.RT_PREC_BF16MFMA)
    with pytest.raises(rt4d.RtError):
        rt4d.form_pick(G, 7, rt4d.RT_PREC_FP32)


def test_auto_job_bytes_match_the_chosen_form():
    G = rt4d.Geom(N=64, Nz=4, Ns=64, Ntheta=8 * 16, Npi=8, K=32, Nt=8)
    assert rt4d.rt_job_bytes(G, rt4d.RT_FORM_AUTO, rt4d.RT_PREC_BF16MFMA) == \
        rt4d.rt_job_bytes(G, rt4d.RT_FORM_SF, rt4d.RT_PREC_BF16MFMA)
    assert rt4d.rt_job_bytes(G, rt4d.RT_FORM_AUTO, rt4d.RT_PREC_FP32) == \
        rt4d.rt_job_bytes(G, rt4d.RT_FORM_PF, rt4d.RT_PREC_FP32)


def test_fourier_tables_span_the_complex_basis():
    """The real table of M = 16 functions (K = 15) against numpy's complex
    exponentials exp(2 pi i t (j - M/2)) at t_i = i/Ntheta: every real-form
    synthesis equals the complex synthesis with the stated coefficients, and
    the table's columns are the real and imaginary parts."""
    import numpy as np
    import torch
    M = 16
    G = rt4d.Geom(N=8, Nz=1, Ns=8, Ntheta=130 * 3, Npi=130, K=M - 1, Nt=40)
    phi, S = rt4d.basis_fourier(G, M)
    t = np.arange(G.Ntheta) / G.Ntheta
    E = np.exp(2j * np.pi * np.outer(t, np.arange(M) - M // 2))     # [Ntheta][M]
    assert np.abs(phi[:, 0] - 1).max() == 0
    for v in range(1, M // 2):
        assert np.abs(phi[:, 2 * v - 1] - E[:, M // 2 + v].real).max() < 1e-13
        assert np.abs(phi[:, 2 * v] - E[:, M // 2 + v].imag).max() < 1e-13
    n0 = G.Ntheta // G.Npi
    assert np.array_equal(S, phi[[m * n0 for m in range(G.Nt)]])
    rs = np.random.default_rng(3)
    a = rs.standard_normal((5, M - 1))
    c = rt4d.fourier_complex_coeffs(torch.from_numpy(a.astype(np.float32)), M).numpy().astype(np.complex128)
    assert np.all(c[:, 0] == 0)                                        # frequency -M/2
    real_form = a.astype(np.float32).astype(np.float64) @ phi.T
    complex_form = c @ E.T
    assert np.abs(complex_form.imag).max() < 1e-6 * np.abs(complex_form).max()
    assert np.abs(complex_form.real - real_form).max() < 1e-6 * np.abs(real_form).max()
    with pytest.raises(rt4d.RtError):
        rt4d.basis_fourier(rt4d.Geom(N=8, Nz=1, Ns=8, Ntheta=16, Npi=4, K=15, Nt=4), 15)
    with pytest.raises(rt4d.RtError):
        rt4d.basis_fourier(rt4d.Geom(N=8, Nz=1, Ns=8, Ntheta=16, Npi=4, K=14, Nt=4), 16)

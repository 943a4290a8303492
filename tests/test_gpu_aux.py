"""The measurement aids of the C ABI on the GPU: the FMA issue-rate kernel
(rt_calib_fma) against an FP32 emulation of its chains on the host, and the
per-kernel timing counters (rt_timing_*) around a forward projection."""
import numpy as np
import pytest
import torch

from paper_1809_09725_amd import inputs, rt4d

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def test_calib_fma_chains_and_flop_count():
    torch.cuda.set_device(DEV)
    nb, it = 4, 3
    out = torch.empty(nb * 256, device=DEV)
    ms, flop = rt4d.calib_fma(nb, it, out)
    assert ms > 0.0
    assert flop == 2.0 * 8 * 16 * it * 256 * nb
    # eight chains x <- fma(x, 0.999, 0.001) from x = thread + chain, 16 per
    # iteration, summed in chain order; each fma rounds once to FP32 (the
    # FP64 product of two floats is exact, so only the final rounding counts
    # except in rare double-rounding cases: compared to 2 ulp)
    a, b = np.float32(0.999), np.float32(0.001)
    tid = np.arange(256, dtype=np.float64)
    s = np.zeros(256, np.float32)
    for c in range(8):
        x = (tid + c).astype(np.float32)
        for _ in range(16 * it):
            x = (x.astype(np.float64) * np.float64(a) + np.float64(b)).astype(np.float32)
        s = (s + x).astype(np.float32)
    got = out.cpu().numpy().reshape(nb, 256)
    for blk in range(nb):
        np.testing.assert_allclose(got[blk], s, rtol=2.5e-7, atol=0)


def test_timing_counters_around_a_forward():
    torch.cuda.set_device(DEV)
    G = rt4d.Geom(N=48, Nz=2, Ns=50, Ntheta=4 * 30, Npi=4, K=6, Nt=4)
    plan = rt4d.Plan(G)
    f = torch.from_numpy(inputs.uniform(G.f_shape, 5)).to(DEV)
    rt4d.timing_reset()
    rt4d.timing_enable(True)
    plan.forward(f)
    plan.forward(f)
    torch.cuda.synchronize()
    rt4d.timing_enable(False)
    ms, n = rt4d.timing_read("k_project")
    assert n == 2 and ms > 0.0
    plan.forward(f)   # not counted while disabled
    torch.cuda.synchronize()
    assert rt4d.timing_read("k_project")[1] == 2
    assert rt4d.timing_read("no_such_kernel") == (0.0, 0)
    rt4d.timing_reset()
    assert rt4d.timing_read("k_project") == (0.0, 0)
    plan.close()

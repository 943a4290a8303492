"""Serving loop on the GPU: each job's result is the same alone and in the mix."""
import pytest
import torch

from paper_1809_09725_amd import inputs, rt4d
from paper_1809_09725_amd.serving import GpuBackend, JobSpec, Scheduler, pick_form, serial_baseline

pytestmark = pytest.mark.gpu


def tiny_trace():
    shapes = [(32, 1, 4), (48, 2, 8), (32, 2, 16), (48, 1, 8), (32, 1, 8)]
    return [JobSpec(jid=j, arrival=0.002 * j, N=N, Nz=Nz, K=K, Ntheta=4 * N, Npi=8, n_iter=6,
                    seed=40 + j, lambda1=2.0 ** -9 * 4 * N * N)
            for j, (N, Nz, K) in enumerate(shapes)]


def payload(s):
    G = s.geom()
    return torch.from_numpy(inputs.uniform(G.g_shape, 1000 + s.jid, 0.0, 1.0))


def alone(s, form):
    G = s.geom()
    dev = torch.device("cuda", 0)
    g = payload(s).to(dev)
    f = torch.zeros(G.f_shape, device=dev)
    plan = rt4d.Plan(G, form=rt4d.RT_FORM_SF if form == "sf" else rt4d.RT_FORM_PF,
                     prec=rt4d.RT_PREC_BF16MFMA if form == "sf" else rt4d.RT_PREC_FP32)
    plan.solve(g, f, lambda1=s.lambda1, lambda2=s.lambda2, n_iter=s.n_iter, n_pow=20,
               check_every=0, seed=s.seed)
    torch.cuda.synchronize()
    plan.close()
    return f


@pytest.mark.parametrize("form", ["sf", "pf", "auto"])
def test_served_equals_alone(form):
    torch.cuda.set_device(0)
    tr = tiny_trace()
    be = GpuBackend(payload, form=form, keep_results=True)
    recs, st = Scheduler(be, 8 << 30, max_active=4, depth=2, form=form).run(tr)
    be.close()
    assert st["jobs"] == len(tr)
    assert st["max_resident"] >= 2      # jobs were resident (and stepped) together
    for s, r in zip(tr, recs):
        assert r.iters == s.n_iter
        ref = alone(s, pick_form(s, form))
        got = be.results[s.jid]
        # same kernels, same order, per-job scratch: the results agree bitwise
        assert torch.equal(got, ref), f"job {s.jid}: max diff {(got - ref).abs().max().item()}"


def test_serial_baseline_matches_plain_solver():
    torch.cuda.set_device(0)
    tr = tiny_trace()[:3]
    recs, st, res = serial_baseline(tr, payload, keep_results=True)
    assert st["jobs"] == 3
    fins = [r.finished for r in recs]
    assert fins == sorted(fins)
    for s in tr:
        assert torch.equal(res[s.jid], alone(s, "pf"))


def test_nonfinite_job_fails_alone():
    """A job whose sinogram holds a NaN is caught by the FP64 finiteness check
    at admission and marked failed; every other job of the mix is bitwise the
    same as alone (NaN here is only data: no kernel sees it)."""
    torch.cuda.set_device(0)
    tr = tiny_trace()
    bad = tr[2].jid

    def pay(s):
        p = payload(s)
        if s.jid == bad:
            p = p.clone()
            p[5, 0, 3] = float("nan")
        return p

    be = GpuBackend(pay, form="auto", keep_results=True)
    recs, st = Scheduler(be, 8 << 30, max_active=4, depth=2, form="auto").run(tr)
    be.close()
    r = {x.jid: x for x in recs}
    assert r[bad].status == "failed" and "non-finite" in r[bad].error, r[bad]
    assert st["failed"] == 1 and st["jobs"] == len(tr) - 1
    for s in tr:
        if s.jid == bad:
            assert s.jid not in be.results
            continue
        assert r[s.jid].status == "done"
        assert torch.equal(be.results[s.jid], alone(s, pick_form(s, "auto")))

"""Scheduler logic of the serving loop on a simulated device (no GPU)."""
import numpy as np
import pytest

from paper_1809_09725_amd.serving import FakeBackend, JobSpec, Scheduler, c4_trace


def spec(jid, arrival, N=64, Nz=4, K=8, n_iter=10):
    return JobSpec(jid=jid, arrival=arrival, N=N, Nz=Nz, K=K, Ntheta=4 * N, Npi=8, n_iter=n_iter,
                   seed=jid, lambda1=1.0)


def cost(s):   # seconds per iteration on the fake device
    return 1e-9 * s.work_per_iter(True)


def test_c4_trace_shape():
    tr = c4_trace()
    assert len(tr) == 64
    arr = np.array([s.arrival for s in tr])
    assert np.all(np.diff(arr) > 0)
    # mean inter-arrival 0.5 s (rate 2/s): loose statistical bound for 64 samples
    assert 0.3 < arr[-1] / 64 < 0.8
    for s in tr:
        assert s.N in (256, 512, 1024) and s.Nz in (8, 32, 128) and s.K in (8, 16, 32)
        assert s.Ntheta == 4 * s.N and s.Ntheta % s.Npi == 0 and s.Nt == s.Npi
        assert s.n_iter == 60
    assert c4_trace()[5] == tr[5]          # seeded
    assert c4_trace(seed=5)[5] != tr[5]


def test_all_jobs_complete_and_accounting():
    tr = [spec(j, 0.01 * j, N=32 * (1 + j % 3), K=8 << (j % 2)) for j in range(12)]
    be = FakeBackend(cost, setup_s=0.001)
    budget = 3 * max(be.bytes_needed(s) for s in tr)
    recs, st = Scheduler(be, budget, max_active=4).run(tr)
    assert st["jobs"] == 12
    for s, r in zip(tr, recs):
        assert r.jid == s.jid and r.iters == s.n_iter
        assert r.arrival <= r.admitted <= r.ready <= r.finished
        assert r.latency >= s.n_iter * cost(s) - 1e-12
    assert be.peak_bytes <= budget
    assert be.live_bytes == 0
    assert st["makespan_s"] == pytest.approx(max(r.finished for r in recs))
    assert st["p50_latency_s"] <= st["p99_latency_s"]
    assert 2 <= st["max_resident"] <= 4
    # every issued iteration ran exactly once
    assert sorted(be.order) == sorted(j for s in tr for j in [s.jid] * s.n_iter)


def test_short_job_overtakes_long_one():
    long_ = spec(0, 0.0, N=256, Nz=32, n_iter=50)
    short = spec(1, 0.5 * 50 * cost(long_) / 2, N=32, Nz=1, n_iter=5)
    be = FakeBackend(cost)
    recs, _ = Scheduler(be, 1 << 40, max_active=4).run([long_, short])
    r = {x.jid: x for x in recs}
    assert r[1].finished < r[0].finished
    # the short job did not wait for the long one to drain
    assert r[1].latency < 0.2 * r[0].latency


def test_budget_limits_residency():
    tr = [spec(j, 0.0, N=128, Nz=8) for j in range(6)]
    be = FakeBackend(cost)
    one = be.bytes_needed(tr[0])
    recs, _ = Scheduler(be, 2 * one + one // 2, max_active=8).run(tr)
    assert be.peak_bytes <= 2 * one + one // 2
    # at most two resident at a time: admissions come in pairs
    adm = sorted(r.admitted for r in recs)
    fin = sorted(r.finished for r in recs)
    for k in range(2, 6):
        assert adm[k] >= fin[k - 2] - 1e-12


def test_oldest_job_not_starved_by_backfill():
    first = spec(100, 0.0, N=32, Nz=1, n_iter=20)
    big = spec(0, 0.001, N=256, Nz=16, n_iter=3)
    smalls = [spec(j, 0.001 + 0.002 * j, N=32, Nz=1, n_iter=20) for j in range(1, 80)]
    tr = [first, big] + smalls
    be = FakeBackend(cost)
    nb, ns = be.bytes_needed(big), be.bytes_needed(first)
    assert nb >= 4 * ns
    budget = nb + ns // 2        # the big job never fits beside a small one

    def finish_rank(starve_s):
        be = FakeBackend(cost)
        recs, _ = Scheduler(be, budget, max_active=8, starve_s=starve_s).run(tr)
        order = sorted(recs, key=lambda r: r.finished)
        return [r.jid for r in order].index(0)

    # with back-fill unlimited the stream of small jobs keeps the big one out to the end
    assert finish_rank(1e9) == len(tr) - 1
    # once it has waited starve_s, freed memory is held for it
    assert finish_rank(0.01) < len(tr) // 2


def test_concurrency_beats_serial_when_jobs_share_the_device():
    tr = [spec(j, 0.0, N=32, Nz=1, n_iter=20) for j in range(8)]
    be1 = FakeBackend(cost, overlap=3.0)
    _, serial = Scheduler(be1, 1 << 40, max_active=1).run(tr)
    be2 = FakeBackend(cost, overlap=3.0)
    _, served = Scheduler(be2, 1 << 40, max_active=8).run(tr)
    assert served["makespan_s"] < serial["makespan_s"]
    assert served["jobs_per_hour"] > serial["jobs_per_hour"]


def test_job_larger_than_budget_rejected_alone():
    big = spec(0, 0.0, N=256, Nz=32)
    small = [spec(j, 0.001 * j, N=32, Nz=1) for j in range(1, 4)]
    be = FakeBackend(cost)
    recs, st = Scheduler(be, be.bytes_needed(big) - 1).run([big] + small)
    r = {x.jid: x for x in recs}
    assert r[0].status == "rejected" and "budget" in r[0].error and r[0].iters == 0
    assert all(r[j].status == "done" and r[j].iters == 10 for j in (1, 2, 3))
    assert st["jobs"] == 3 and st["rejected"] == 1 and st["failed"] == 0
    assert 0 not in be.order and be.live_bytes == 0
    with pytest.raises(ValueError):
        Scheduler(be, 0)


def test_failures_are_isolated():
    """A job whose setup raises (e.g. a non-finite sinogram) and one whose
    fourth iteration raises are marked failed and freed; the others finish
    with exactly the iterations they would have run without them."""
    tr = [spec(j, 0.001 * j, N=32 * (1 + j % 2), Nz=1 + j % 3) for j in range(8)]
    be = FakeBackend(cost, setup_s=0.001, fail_setup={2}, fail_at={5: 4})
    budget = 3 * max(be.bytes_needed(s) for s in tr)
    recs, st = Scheduler(be, budget, max_active=4).run(tr)
    r = {x.jid: x for x in recs}
    assert r[2].status == "failed" and "setup" in r[2].error and r[2].iters == 0
    assert r[5].status == "failed" and "iteration 4" in r[5].error and r[5].iters <= 3
    for j in (0, 1, 3, 4, 6, 7):
        assert r[j].status == "done" and r[j].iters == 10
        assert be.order.count(j) == 10
    assert be.order.count(2) == 0 and be.order.count(5) <= 3
    assert st["jobs"] == 6 and st["failed"] == 2
    assert be.live_bytes == 0 and be.peak_bytes <= budget
    assert st["makespan_s"] == pytest.approx(max(r[j].finished for j in (0, 1, 3, 4, 6, 7)))


def test_cancellation_while_waiting_and_while_running():
    tr = [spec(0, 0.0, N=64, Nz=4, n_iter=40), spec(1, 0.0, N=64, Nz=4, n_iter=40),
          spec(2, 0.0, N=32, Nz=1, n_iter=10)]
    one_iter = cost(tr[0])
    tr[0].cancel_at = 5.5 * one_iter         # running: withdrawn after a few iterations
    be = FakeBackend(cost)
    # budget for one job at a time: job 1 waits, and is cancelled from outside
    sched = Scheduler(be, be.bytes_needed(tr[0]), max_active=4)
    sched.cancel(1)
    recs, st = sched.run(tr)
    r = {x.jid: x for x in recs}
    assert r[0].status == "cancelled" and 0 < r[0].iters < 40
    assert r[1].status == "cancelled" and r[1].iters == 0 and be.order.count(1) == 0
    assert r[2].status == "done" and r[2].iters == 10
    assert st["cancelled"] == 2 and st["jobs"] == 1 and be.live_bytes == 0
    # a cancelled job's queued iterations were dropped, not run
    assert be.order.count(0) == r[0].iters


def test_window_one_runs_shortest_remaining_first():
    # all resident from the start; window = 1 runs them one at a time, shortest first
    tr = [spec(0, 0.0, N=128, Nz=8, n_iter=10), spec(1, 0.0, N=32, Nz=1, n_iter=10),
          spec(2, 0.0, N=64, Nz=4, n_iter=10)]
    be = FakeBackend(cost)
    recs, _ = Scheduler(be, 1 << 40, max_active=8, window=1).run(tr)
    fin = {r.jid: r.finished for r in recs}
    assert fin[1] < fin[2] < fin[0]
    # strictly one job's iterations at a time
    seq = be.order
    assert seq == sorted(seq, key=lambda j: [1, 2, 0].index(j))


def test_auto_form_picks_precision_only_for_at_least_two_channels_per_half_turn():
    import dataclasses
    from paper_1809_09725_amd.serving import pick_form
    assert pick_form(spec(0, 0.0, K=16), "auto") == "sf"       # Npi = 8
    assert pick_form(spec(0, 0.0, K=32), "auto") == "sf"
    assert pick_form(spec(0, 0.0, K=8), "auto") == "pf"
    assert pick_form(dataclasses.replace(spec(0, 0.0, K=16), Npi=12, Ntheta=12 * 64), "auto") == "pf"
    assert pick_form(spec(0, 0.0, K=8), "sf") == "sf"

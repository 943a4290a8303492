"""Serving form: a continuous-batching request loop over the resumable solver.

Reconstruction requests (jobs) of different sizes arrive over time.  Each job
is the iteration of Fig. 2 for its own geometry (N, Nz, Ntheta, K), run for a
fixed number of iterations through the rt_job API of librt4d.  The loop

  * admits arrived jobs while their resident state fits the HBM budget
    (rt_job_bytes + the caller's f and g), oldest first; a younger job may
    back-fill memory the oldest cannot use yet, until the oldest has waited
    `starve_s` seconds;
  * keeps every admitted job's f_k, duals and sinogram resident in device
    memory, each job on its own stream (default priority);
  * interleaves iterations of the co-resident jobs: the `window` jobs with
    the least remaining work (shortest remaining processing time first) may
    each have up to `depth` iterations queued on the device, so short jobs
    overtake long ones while two or three jobs together keep the device
    busy; the device has no notion of priority, so the host does the
    ordering by what it queues;
  * runs the setup of a job (plan tables, power iteration for the step size)
    on a worker thread, so that admission never stalls the issue loop;
  * isolates failures: a job larger than the whole budget is rejected on its
    own, a job whose setup or iteration raises (a non-finite sinogram found
    by the FP64 finiteness check at admission, a library error, a device
    allocation failure) is marked failed and its memory freed, and a job can
    be cancelled while waiting, in setup or running; every other job goes on
    as if that job had never been there.

The same loop drives a fake device in the CPU tests (`FakeBackend`), which
checks the admission, ordering and accounting logic without a GPU.

`serial_baseline` is the comparison: the plain FP32 solver (`solve`) run on
one job at a time in arrival order.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------- jobs

@dataclass
class JobSpec:
    """One reconstruction request.  Ns = N, Nt = Npi (frames at the half-turn
    starts), Ntheta = Npi * Ntheta0."""
    jid: int
    arrival: float            # seconds after the start of the trace
    N: int
    Nz: int
    K: int
    Ntheta: int
    Npi: int
    n_iter: int
    seed: int
    lambda1: float
    lambda2: float = 4.0
    cancel_at: float = math.inf   # the client withdraws the request at this time

    @property
    def Ns(self) -> int:
        return self.N

    @property
    def Nt(self) -> int:
        return self.Npi

    def geom(self):
        from . import rt4d
        return rt4d.Geom(N=self.N, Nz=self.Nz, Ns=self.Ns, Ntheta=self.Ntheta, Npi=self.Npi,
                         K=self.K, Nt=self.Nt)

    def samples_per_iter(self) -> float:
        """Delivered ray-samples of one R_T + R_T* pair."""
        return 2.0 * self.Ntheta * self.Nz * self.Ns * self.N

    def work_per_iter(self, sf: bool) -> float:
        """Relative cost of one iteration: executed projector taps (K channels
        per class for project-first, one frame per projection for
        synthesise-first) plus the streaming TV bytes in tap-equivalents."""
        n0 = self.Ntheta // self.Npi
        taps = 2.0 * self.Nz * self.Ns * self.N * (self.Ntheta if sf else n0 * self.K)
        stream = 4.0 * self.Nz * self.N * self.N * (2 * self.K + 8 * self.Nt)
        return taps + stream


def c4_trace(n_jobs: int = 64, rate: float = 2.0, seed: int = 4, n_iter: int = 60,
             sizes=(256, 512, 1024), slices=(8, 32, 128), channels=(8, 16, 32),
             Npi: int = 8) -> list[JobSpec]:
    """Poisson arrivals (mean `rate` jobs/s) of jobs with N, Nz, K drawn
    uniformly from the given sets; Ntheta = 4N angles over Npi = 8 half-turns.
    lambda1 = 2^-9 * Ntheta * N, the paper's 2^-9 (Sec. 6) scaled by
    Ntheta * N, which tracks |R_T|^2 of this projector to within ~5%."""
    rs = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(n_jobs):
        t += float(rs.exponential(1.0 / rate))
        N = int(rs.choice(sizes))
        Nz = int(rs.choice(slices))
        K = int(rs.choice(channels))
        out.append(JobSpec(jid=j, arrival=t, N=N, Nz=Nz, K=K, Ntheta=4 * N, Npi=Npi,
                           n_iter=n_iter, seed=seed * 1000 + j,
                           lambda1=2.0 ** -9 * (4 * N) * N))
    return out


# --------------------------------------------------------------------------- records

@dataclass
class Record:
    jid: int
    arrival: float
    admitted: float = math.nan
    ready: float = math.nan
    finished: float = math.nan
    bytes: int = 0
    iters: int = 0
    report: dict = field(default_factory=dict)
    status: str = "pending"   # done | failed | rejected | cancelled
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def summarize(records: list[Record], makespan: float) -> dict:
    """Throughput and latency over the jobs that completed; the others are
    counted by status."""
    ok = [r for r in records if r.status == "done"]
    lat = np.array([r.latency for r in ok])
    out = {"jobs": len(ok), "makespan_s": makespan,
           "jobs_per_hour": 3600.0 * len(ok) / makespan if makespan > 0 else math.inf,
           "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else math.nan,
           "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else math.nan,
           "mean_latency_s": float(lat.mean()) if len(lat) else math.nan}
    for st in ("failed", "rejected", "cancelled"):
        out[st] = sum(r.status == st for r in records)
    return out


# --------------------------------------------------------------------------- scheduler

class _Active:
    __slots__ = ("spec", "h", "issued", "done", "est", "rec")

    def __init__(self, spec, h, est, rec):
        self.spec, self.h, self.est, self.rec = spec, h, est, rec
        self.issued = 0
        self.done = 0

    def remaining(self) -> float:
        return (self.spec.n_iter - self.issued) * self.est


class Scheduler:
    """Continuous batching of solver iterations under an HBM budget."""

    def __init__(self, backend, budget_bytes: int, max_active: int = 8, depth: int = 2,
                 window: int = 2, starve_s: float = 30.0, form: str = "sf", log=None):
        if budget_bytes <= 0 or max_active < 1 or depth < 1 or window < 1:
            raise ValueError("budget, max_active, depth and window must be positive")
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.depth = depth
        self.window = window
        self.log = log           # called with a line per finished job
        self.starve_s = starve_s
        self.form = form         # for the work estimate of each job
        self._cancel: set[int] = set()
        self._cancel_lock = threading.Lock()

    def cancel(self, jid: int) -> None:
        """Withdraw job `jid` (safe from any thread): a waiting job leaves the
        queue, a job in setup is released when its setup ends, a running job
        is released at once (its queued iterations drain first)."""
        with self._cancel_lock:
            self._cancel.add(jid)

    def _cancelled(self, jid: int) -> bool:
        with self._cancel_lock:
            return jid in self._cancel

    def run(self, trace: list[JobSpec]) -> tuple[list[Record], dict]:
        be = self.be
        future = deque(sorted(trace, key=lambda s: (s.arrival, s.jid)))
        waiting: deque[JobSpec] = deque()
        setting_up: list[_Active] = []
        active: list[_Active] = []
        records: dict[int, Record] = {}
        used = 0
        max_resident = 0
        t0 = be.now()

        def close(a: _Active, status: str, err: str = "") -> None:
            nonlocal used
            a.rec.status, a.rec.error = status, err
            a.rec.iters = a.done
            a.rec.finished = be.now() - t0
            try:
                be.release(a.h)
            except Exception as e:      # the memory is the backend's to reclaim; keep serving
                a.rec.error += f"; release: {e}"
            used -= a.rec.bytes
            if self.log:
                s = a.spec
                self.log(f"served job {s.jid} (N={s.N} Nz={s.Nz} K={s.K}) {status} at "
                         f"{a.rec.finished:.1f} s{': ' + err if err else ''}")

        while future or waiting or setting_up or active:
            now = be.now() - t0
            while future and future[0].arrival <= now:
                s = future.popleft()
                rec = records[s.jid] = Record(jid=s.jid, arrival=s.arrival)
                need = be.bytes_needed(s)
                if need > self.budget:
                    rec.status, rec.finished = "rejected", now
                    rec.error = f"needs {need} bytes, more than the whole budget {self.budget}"
                    if self.log:
                        self.log(f"job {s.jid} rejected: {rec.error}")
                    continue
                waiting.append(s)
            # ---- cancellations (client requests and the trace's own)
            for s in list(waiting):
                if s.cancel_at <= now or self._cancelled(s.jid):
                    waiting.remove(s)
                    r = records[s.jid]
                    r.status, r.finished = "cancelled", now
            for a in list(active):
                if a.spec.cancel_at <= now or self._cancelled(a.spec.jid):
                    active.remove(a)
                    a.done = be.completed(a.h)
                    close(a, "cancelled")
            # ---- admission: oldest first, back-fill while the oldest is not starving
            n_res = len(active) + len(setting_up)
            i = 0
            while i < len(waiting) and n_res < self.max_active:
                s = waiting[i]
                need = be.bytes_needed(s)
                if used + need <= self.budget:
                    del waiting[i]
                    used += need
                    rec = records[s.jid]
                    rec.admitted, rec.bytes = be.now() - t0, need
                    est = s.work_per_iter(pick_form(s, self.form) == "sf")
                    setting_up.append(_Active(s, be.start_admit(s), est, rec))
                    n_res += 1
                    continue
                if i == 0 and now - s.arrival >= self.starve_s:
                    break          # reserve freed memory for the oldest job
                i += 1
            max_resident = max(max_resident, len(active) + len(setting_up))
            # ---- jobs whose setup finished join the active set (or fail alone)
            for a in list(setting_up):
                try:
                    ok = be.ready(a.h)
                except Exception as e:
                    setting_up.remove(a)
                    close(a, "failed", f"setup: {e}")
                    continue
                if ok:
                    setting_up.remove(a)
                    a.rec.ready = be.now() - t0
                    if a.spec.cancel_at <= be.now() - t0 or self._cancelled(a.spec.jid):
                        close(a, "cancelled")
                    else:
                        active.append(a)
            # ---- completions
            for a in list(active):
                try:
                    a.done = be.completed(a.h)
                    if a.done < a.spec.n_iter:
                        continue
                    a.rec.report = be.finish(a.h)
                except Exception as e:
                    active.remove(a)
                    close(a, "failed", f"iteration {a.done}: {e}")
                    continue
                active.remove(a)
                close(a, "done")
            # ---- issue: the `window` jobs with least remaining work, `depth` queued each
            issued = False
            order = sorted(active, key=lambda a: (a.remaining(), a.spec.jid))
            for a in order[:self.window]:
                try:
                    while a.issued < a.spec.n_iter and a.issued - a.done < self.depth:
                        be.issue(a.h)
                        a.issued += 1
                        issued = True
                except Exception as e:
                    active.remove(a)
                    close(a, "failed", f"issue of iteration {a.issued + 1}: {e}")
            if not issued:
                nxt = future[0].arrival - (be.now() - t0) if future else None
                be.wait(nxt)
        makespan = max((r.finished for r in records.values() if r.status == "done"), default=0.0)
        recs = [records[s.jid] for s in trace]
        st = summarize(recs, makespan)
        st["max_resident"] = max_resident
        return recs, st


# --------------------------------------------------------------------------- GPU backend

class _Slot:
    __slots__ = ("spec", "stream", "future", "plan", "job", "g", "f", "events", "done")

    def __init__(self, spec):
        self.spec = spec
        self.events = deque()
        self.done = 0
        self.plan = self.job = self.g = self.f = None


def pick_form(s: JobSpec, form: str) -> str:
    """'sf' or 'pf' for one job.  'auto' asks the library (rt_form_pick with
    RT_FORM_AUTO and the BF16 contraction allowed): the synthesise-first
    precision form when K >= 2 Npi and Npi <= 32, the plain FP32 form
    otherwise."""
    if form == "auto":
        from . import rt4d
        fo, _ = rt4d.form_pick(s.geom(), rt4d.RT_FORM_AUTO, rt4d.RT_PREC_BF16MFMA)
        return "sf" if fo == rt4d.RT_FORM_SF else "pf"
    return form


class GpuBackend:
    """Runs jobs through librt4d on one GPU.  `payload(spec)` returns the
    job's sinogram as a host (preferably pinned) FP32 tensor.  form: 'sf'
    (precision), 'pf' (plain FP32) or 'auto' (per job, see pick_form)."""

    def __init__(self, payload, form: str = "sf", device: int = 0, n_pow: int = 20,
                 keep_results: bool = False, setup_threads: int = 2, poll_s: float = 2e-4):
        import torch

        from . import rt4d
        if form not in ("sf", "pf", "auto"):
            raise ValueError(form)
        self.torch, self.rt = torch, rt4d
        self.payload = payload
        self.form_name = form
        self.dev = torch.device("cuda", device)
        self.n_pow = n_pow
        self.keep = keep_results
        self.poll_s = poll_s
        self.pool = ThreadPoolExecutor(max_workers=setup_threads)
        self.results: dict = {}          # jid -> final f (keep_results)

    def now(self) -> float:
        return time.perf_counter()

    def _form(self, s: JobSpec):
        rt = self.rt
        if pick_form(s, self.form_name) == "sf":
            return rt.RT_FORM_SF, rt.RT_PREC_BF16MFMA
        return rt.RT_FORM_PF, rt.RT_PREC_FP32

    def bytes_needed(self, s: JobSpec) -> int:
        G = s.geom()
        nf = G.Nz * G.N * G.N * G.K
        ng = G.Ntheta * G.Nz * G.Ns
        return self.rt.rt_job_bytes(G, *self._form(s)) + 4 * (nf + ng)

    def _setup(self, sl: _Slot) -> None:
        torch, rt = self.torch, self.rt
        torch.cuda.set_device(self.dev)
        s = sl.spec
        G = s.geom()
        with torch.cuda.stream(sl.stream):
            host = self.payload(s)
            sl.g = host.to(self.dev, non_blocking=True)
            if tuple(sl.g.shape) != tuple(G.g_shape) or sl.g.dtype != torch.float32:
                raise ValueError(f"sinogram of shape {tuple(sl.g.shape)} ({sl.g.dtype}), expected "
                                 f"{tuple(G.g_shape)} float32")
            # admission check: sum g^2 in FP64 on the device is finite exactly
            # when every sample is (the iteration has no monitor to notice)
            if not math.isfinite(rt.rt_dot(sl.g.view(-1), sl.g.view(-1))):
                raise ValueError("non-finite sinogram")
            sl.f = torch.zeros(G.f_shape, device=self.dev)
            form, prec = self._form(s)
            sl.plan = rt.Plan(G, form=form, prec=prec)
            sl.job = rt.Job(sl.plan, sl.g, sl.f, lambda1=s.lambda1, lambda2=s.lambda2,
                            n_iter=s.n_iter, n_pow=self.n_pow, check_every=0, seed=s.seed)
        sl.stream.synchronize()

    def start_admit(self, s: JobSpec) -> _Slot:
        sl = _Slot(s)
        sl.stream = self.torch.cuda.Stream(self.dev)   # default priority
        sl.future = self.pool.submit(self._setup, sl)
        return sl

    def ready(self, sl: _Slot) -> bool:
        if not sl.future.done():
            return False
        sl.future.result()      # re-raises a setup failure
        return True

    def issue(self, sl: _Slot) -> None:
        sl.job.step(1, stream=sl.stream)
        ev = self.torch.cuda.Event()
        ev.record(sl.stream)
        sl.events.append(ev)

    def completed(self, sl: _Slot) -> int:
        while sl.events and sl.events[0].query():
            sl.events.popleft()
            sl.done += 1
        return sl.done

    def finish(self, sl: _Slot) -> dict:
        rep = sl.job.report(stream=sl.stream)
        if self.keep:
            with self.torch.cuda.stream(sl.stream):
                self.results[sl.spec.jid] = sl.f.clone()
        sl.stream.synchronize()
        return rep

    def release(self, sl: _Slot) -> None:
        """Free the job's device state; works on a slot whose setup failed
        part way (whatever was created is closed)."""
        if sl.future is not None and not sl.future.done():
            sl.future.exception()          # wait for the setup thread to let go
        sl.stream.synchronize()
        if sl.job is not None:
            sl.job.close()
        if sl.plan is not None:
            sl.plan.close()
        sl.g = sl.f = None
        sl.job = sl.plan = None
        sl.events.clear()

    def wait(self, until_next_arrival) -> None:
        dt = self.poll_s if until_next_arrival is None else min(self.poll_s, max(0.0, until_next_arrival))
        if dt > 0:
            time.sleep(dt)

    def close(self) -> None:
        self.pool.shutdown(wait=True)


def serial_baseline(trace: list[JobSpec], payload, device: int = 0, n_pow: int = 20,
                    keep_results: bool = False, log=None) -> tuple[list[Record], dict, dict]:
    """The plain FP32 solver, one job at a time in arrival order: each job
    starts when it has arrived and the previous one has finished."""
    import torch

    from . import rt4d
    dev = torch.device("cuda", device)
    results = {}
    recs = []
    t0 = time.perf_counter()
    for s in sorted(trace, key=lambda s: (s.arrival, s.jid)):
        rec = Record(jid=s.jid, arrival=s.arrival)
        while time.perf_counter() - t0 < s.arrival:
            time.sleep(min(1e-3, s.arrival - (time.perf_counter() - t0)))
        rec.admitted = rec.ready = time.perf_counter() - t0
        G = s.geom()
        g = payload(s).to(dev)
        f = torch.zeros(G.f_shape, device=dev)
        plan = rt4d.Plan(G, form=rt4d.RT_FORM_PF, prec=rt4d.RT_PREC_FP32)
        rec.report = plan.solve(g, f, lambda1=s.lambda1, lambda2=s.lambda2, n_iter=s.n_iter,
                                n_pow=n_pow, check_every=0, seed=s.seed)
        plan.close()
        if keep_results:
            results[s.jid] = f
        torch.cuda.synchronize(dev)
        rec.finished = time.perf_counter() - t0
        rec.iters = s.n_iter
        rec.status = "done"
        recs.append(rec)
        if log:
            log(f"plain job {s.jid} (N={s.N} Nz={s.Nz} K={s.K}) done at {rec.finished:.1f} s, "
                f"latency {rec.latency:.1f} s")
    makespan = max(r.finished for r in recs) if recs else 0.0
    by_id = {r.jid: r for r in recs}
    ordered = [by_id[s.jid] for s in trace]
    return ordered, summarize(ordered, makespan), results


# --------------------------------------------------------------------------- fake device

class FakeBackend:
    """A simulated device for testing the scheduler on the CPU.

    Time is virtual.  Queued iterations of all jobs run in issue order on one
    simulated engine, each taking `cost(spec)` seconds, optionally sped up by
    `overlap` when several jobs are queued (a crude model of small jobs
    sharing the device).  Setup takes `setup_s` seconds."""

    def __init__(self, cost, setup_s: float = 0.0, overlap: float = 1.0, bytes_fn=None,
                 fail_setup=(), fail_at=None):
        self.cost = cost
        self.fail_setup = set(fail_setup)     # jids whose setup raises
        self.fail_at = dict(fail_at or {})    # jid -> iteration whose issue raises
        self.setup_s = setup_s
        self.overlap = overlap
        self.bytes_fn = bytes_fn or (lambda s: s.Nz * s.N * s.N * s.K * 4 * 6)
        self.t = 0.0
        self.queue: deque = deque()      # (slot, cost) in issue order
        self.busy_until = 0.0
        self.live_bytes = 0
        self.peak_bytes = 0
        self.order: list[int] = []       # jid of every finished iteration, in order
        self.pending: list = []          # slots still in setup

    class Slot:
        def __init__(self, spec, ready_at):
            self.spec, self.ready_at = spec, ready_at
            self.done = 0
            self.issued = 0

    def now(self) -> float:
        return self.t

    def bytes_needed(self, s) -> int:
        return int(self.bytes_fn(s))

    def start_admit(self, s):
        self.live_bytes += self.bytes_needed(s)
        self.peak_bytes = max(self.peak_bytes, self.live_bytes)
        sl = FakeBackend.Slot(s, self.t + self.setup_s)
        self.pending.append(sl)
        return sl

    def ready(self, sl) -> bool:
        if self.t >= sl.ready_at:
            if sl in self.pending:
                self.pending.remove(sl)
            if sl.spec.jid in self.fail_setup:
                raise ValueError("non-finite sinogram")
            return True
        return False

    def issue(self, sl) -> None:
        if self.fail_at.get(sl.spec.jid) == sl.issued + 1:
            raise RuntimeError("simulated library error")
        sl.issued += 1
        self.queue.append(sl)

    def _advance(self, dt: float) -> None:
        end = self.t + dt
        while self.queue:
            sl = self.queue[0]
            jobs = len({id(q) for q in self.queue})
            c = self.cost(sl.spec) / (self.overlap if jobs > 1 else 1.0)
            start = max(self.busy_until, self.t)
            if start + c > end + 1e-12:
                break
            self.queue.popleft()
            self.busy_until = start + c
            self.t = self.busy_until
            sl.done += 1
            self.order.append(sl.spec.jid)
        self.t = max(self.t, end)

    def completed(self, sl) -> int:
        return sl.done

    def finish(self, sl) -> dict:
        return {"iters": sl.done}

    def release(self, sl) -> None:
        self.live_bytes -= self.bytes_needed(sl.spec)
        if sl in self.pending:
            self.pending.remove(sl)
        # iterations of a released job still queued are dropped
        self.queue = deque(q for q in self.queue if q is not sl)

    def wait(self, until_next_arrival) -> None:
        # advance to the next event: the head iteration's end, a setup end or an arrival
        cands = []
        if self.queue:
            sl = self.queue[0]
            jobs = len({id(q) for q in self.queue})
            c = self.cost(sl.spec) / (self.overlap if jobs > 1 else 1.0)
            cands.append(max(self.busy_until, self.t) + c - self.t)
        if until_next_arrival is not None:
            cands.append(max(until_next_arrival, 0.0))
        cands += [sl.ready_at - self.t for sl in self.pending if sl.ready_at > self.t]
        dt = min(cands) if cands else 1e-3
        self._advance(max(dt, 1e-9))

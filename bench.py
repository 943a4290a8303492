#!/usr/bin/env python3
"""Benchmark of the decomposed-time tomography hot path on one MI355X.

One step = one iteration of the adapted Chambolle-Pock loop (Sec. 3, Fig. 2)
on the plain FP32 workload: 512 x 512 x 128 volume, K = 16 cosine basis
functions, 1800 projections over 10 half-turns (180 per half-turn), 512
detector bins, 10 time frames; synthetic data from 40 moving ellipsoids and
a growing sphere with 1% Gaussian noise.  A step runs R_T with the h1 prox,
the 4D gradient with the shrink, R_T*, the divergence with the primal update
and extrapolation, and the FP64 monitors (residual, TV, relative change).

value = delivered R_T + R_T* ray-samples per second / 1e9 (2 Ntheta Nz Ns N
per iteration), inputs resident in HBM.  Prints one JSON line on stdout.

  python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
  python bench.py --copy-calib     # plain copy kernel for counter calibration
  python bench.py --form sf        # the precision form on the same workload
  python bench.py --serve [--jobs 64 --rate 2 --iters 60]
        # serving form: a Poisson trace of jobs of mixed size served with the
        # precision form under continuous batching, against the plain FP32
        # solver one job at a time; prints its own JSON line
  python bench.py --ooc 16 [--steps 4 --warmup 1]
        # out-of-core form: the state in host memory, streamed through the GPU
        # in z-slabs of 16 slices; prints its own JSON line
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "R_T+R_T* Gray-samples/s, solver iters/s; served p50/p99 latency vs plain"
PEAK_HBM = 8.0e12                               # B/s, MI355X HBM3E
# published FP32 vector peak of MI355X: 256 CU x 4 SIMD x 16 lanes x 2 flop x
# 2 (packed) x 2.4 GHz = 157.3 TFLOP/s.  This build issues unpacked FMAs only,
# so half of it (78.6) is the most its FMA kernels can reach; `--valu-calib`
# measures that rate on the device.
PEAK_FP32_VALU = 157.3e12
# unpacked FP32 FMA rate measured on MI355X with `bench.py --valu-calib`
# (8 independent chains per thread, 4096 workgroups): 76.41 TFLOP/s, 0.975
# VALU instructions per clock per CU at the 2.39 GHz the counters give
FP32_UNPACKED_MEASURED = 76.41e12
KERNELS = ("k_project", "k_contract", "k_fold", "k_backproject", "k_grad_shrink",
           "k_div_update", "k_project_sf", "k_fold_mfma")
SOURCES = {"k_project": "proj_pf.hip", "k_contract": "proj_pf.hip", "k_fold": "proj_pf.hip",
           "k_backproject": "backproject.hip", "k_grad_shrink": "tv.hip", "k_div_update": "tv.hip",
           "k_project_sf": "proj_sf.hip", "k_fold_mfma": "proj_sf.hip",
           "k_shepp_logan": "fbp.hip", "k_analysis": "fbp.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Workloads: (N, Nz, Ns, Ntheta, Npi, K, Nt), the form they are quoted in, and
# the moving-phantom family that makes their data.
WORKLOADS = {
    "c2": dict(geom=(512, 128, 512, 1800, 10, 16, 10), form="pf", n_ell=40, drift=0.0,
               sphere=(10.0, 60.0, 0.5), seed=2,
               desc="plain FP32 R_T/R_T* + 4D TV Chambolle-Pock iteration, 512x512x128 volume, "
                    "K=16 cosine basis, 1800 projections over 10 half-turns, 512 bins, 10 TV "
                    "frames, 40 moving ellipsoids + growing sphere, 1% noise"),
    "c3": dict(geom=(1024, 64, 1024, 3600, 12, 16, 12), form="sf", n_ell=40, drift=0.0,
               sphere=(20.0, 120.0, 0.5), seed=3,
               desc="precision form (BF16 MFMA basis contraction, FP32 projection) iteration, "
                    "1024x1024x64 volume, K=16, 3600 projections over 12 half-turns, 1024 bins, "
                    "12 TV frames, 40 moving ellipsoids + growing sphere, 1% noise"),
    "c5": dict(geom=(2048, 32, 2048, 3600, 12, 32, 12), form="sf", n_ell=200, drift=0.5,
               sphere=None, seed=5,
               desc="large slab, precision form iteration, 2048x2048x32 volume, K=32, 3600 "
                    "projections over 12 half-turns, 2048 bins, 12 TV frames, 200 ellipsoids "
                    "with linear motion and density drift, 1% noise, all state resident in HBM"),
}


def workload_geom(name: str):
    from paper_1809_09725_amd import rt4d
    N, Nz, Ns, Nth, Npi, K, Nt = WORKLOADS[name]["geom"]
    return rt4d.Geom(N=N, Nz=Nz, Ns=Ns, Ntheta=Nth, Npi=Npi, K=K, Nt=Nt)


def c2_geom():
    return workload_geom("c2")


def algorithmic(kernel: str, G, sf: bool = False) -> tuple[str, float]:
    """(bound, algorithmic flops or bytes of one launch); sf: precision form."""
    n0 = G.Ntheta // G.Npi
    nvox = G.Nz * G.N * G.N
    if kernel == "k_project":       # 2 taps x 1 FMA per channel-sample on every ray step
        return "alu", 4.0 * G.K * n0 * G.Nz * G.Ns * G.N
    if kernel == "k_project_sf":    # 2 taps x 1 FMA per half-turn on every ray step
        return "alu", 4.0 * G.Npi * n0 * G.Nz * G.Ns * G.N
    if kernel == "k_fold_mfma":     # read g, write g~
        return "hbm", G.Ntheta * G.Nz * G.Ns * 4.0 + n0 * G.Nz * G.Ns * 4.0 * G.K
    if kernel == "k_backproject":   # 2 taps x 1 FMA per channel per voxel and class
        return "alu", 4.0 * G.K * n0 * G.Nz * G.N * G.N
    if kernel == "k_grad_shrink":   # read the frames of f~, read + write h2
        return "hbm", nvox * (4.0 * G.Nt + 2 * 16.0 * G.Nt)
    if kernel == "k_div_update":    # read h2, f, R*h1; write f, f~ and the frames of f~
        shadow = 2.0 * ((G.K + 15) // 16 * 16) if sf else 0.0   # + the BF16 shadow of f~
        return "hbm", nvox * (16.0 * G.Nt + 4 * 4.0 * G.K + 4.0 * G.Nt + shadow)
    if kernel == "k_contract":      # read P, g, h1; write h1
        return "hbm", n0 * G.Nz * G.Ns * 4.0 * G.K + G.Ntheta * G.Nz * G.Ns * 12.0
    if kernel == "k_fold":          # read g, write g~
        return "hbm", G.Ntheta * G.Nz * G.Ns * 4.0 + n0 * G.Nz * G.Ns * 4.0 * G.K
    if kernel == "k_shepp_logan":   # every output bin sums the Ns bins of its row
        return "alu", 2.0 * G.Ntheta * G.Nz * G.Ns * G.Ns
    if kernel == "k_analysis":      # read the Npi frames, write the K coefficients
        return "hbm", nvox * 4.0 * (G.Npi + G.K)
    raise KeyError(kernel)


def fbp_measure(plan, G, g) -> dict:
    """The FBP initial guess (rt_fbp) on the workload's sinogram: wall time of
    one blocking call after an untimed one, and its kernels.  The half-turn
    back-projection runs the fold-sum and back-projection with Npi channels."""
    import dataclasses

    import torch

    from paper_1809_09725_amd import rt4d
    f0 = torch.empty(G.f_shape, device=g.device)
    plan.fbp(g, out=f0)
    torch.cuda.synchronize()
    rt4d.timing_reset()
    rt4d.timing_enable(True)
    t0 = time.perf_counter()
    plan.fbp(g, out=f0)
    t1 = time.perf_counter()
    rt4d.timing_enable(False)
    Gm = dataclasses.replace(G, K=G.Npi, Nt=G.Npi)
    kern = {}
    for k, geom in (("k_shepp_logan", G), ("k_fold", Gm), ("k_backproject", Gm), ("k_analysis", G)):
        ms, n = rt4d.timing_read(k)
        if not n:
            continue
        b, w = algorithmic(k, geom)
        peak = PEAK_HBM if b == "hbm" else PEAK_FP32_VALU
        kern[k] = {"ms": round(ms, 4), "launches": n, "bound": b,
                   "frac": round(w / (ms * 1e-3) / peak, 4)}
    rt4d.timing_reset()
    log("FBP initial guess: " + f"{(t1 - t0) * 1e3:.1f} ms, " +
        ", ".join(f"{k} {v['ms']:.3f} ms" for k, v in kern.items()))
    return {"what": "FBP initial guess (rt_fbp): Shepp-Logan filter, one frame per half-turn, "
                    "least-squares coefficients; blocking call incl. its temporaries",
            "ms": round((t1 - t0) * 1e3, 3), "kernels": kern}


def source_sha(kernel: str) -> str:
    p = os.path.join(ROOT, "paper_1809_09725_amd", "csrc", SOURCES[kernel])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload: str = "c2"):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha") != source_sha(kernel):
            return None
        return 1024.0 * (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"]) +
                         float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"]))
    except (KeyError, ValueError):
        return None


CPU_SLICES = 16   # slices of the oracle sample: about 20 s of FP64 work (both routes) on 16 host cores


def cpu_baseline(G, g_slices, seed: int) -> dict:
    """The FP64 oracle, as it stands, on a bounded sample: R_T and R_T* over
    all projections of the first CPU_SLICES slices (slices are independent
    under parallel-beam geometry, so the rate is that of the whole volume),
    by both of its routes: direct (each projection's frame synthesised and
    projected) and folded (the K channels projected once per angle class,
    Sec. 4).  The value is the faster route's rate."""
    import numpy as np

    import oracle as O
    from paper_1809_09725_amd import inputs
    nz = g_slices.shape[1]
    og = O.Geom(N=G.N, Nz=nz, Ns=G.Ns, Ntheta=G.Ntheta, Npi=G.Npi, K=G.K, Nt=G.Nt)
    f = inputs.uniform((nz, G.N, G.N, G.K), seed)
    gs = np.asarray(g_slices, np.float64)
    O.build()
    samples = 2.0 * G.Ntheta * nz * G.Ns * G.N
    t = {}
    for route in ("folded", "direct"):
        t0 = time.perf_counter()
        O.forward(og, f, route=route)
        t1 = time.perf_counter()
        O.adjoint(og, gs, route=route)
        t2 = time.perf_counter()
        t[route] = (t1 - t0, t2 - t1)
    rate = {r: samples / sum(v) / 1e9 for r, v in t.items()}
    best = max(rate, key=rate.get)
    return {"value": rate[best], "unit": "Gray-samples/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{nz} of {G.Nz} slices of the workload (seeded uniform f, the workload's "
                      f"sinogram): R_T then R_T* over all {G.Ntheta} projections, FP64; value from "
                      f"the {best} route; folded (Sec. 4) forward {t['folded'][0]:.2f} s, adjoint "
                      f"{t['folded'][1]:.2f} s ({rate['folded']:.3f} Gray-samples/s); direct forward "
                      f"{t['direct'][0]:.2f} s, adjoint {t['direct'][1]:.2f} s "
                      f"({rate['direct']:.3f} Gray-samples/s)"}


def copy_calib():
    import torch
    n = 1 << 28                      # 1 GiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calib_bytes_per_direction": 4 * n, "dispatches": 3}))


def valu_calib():
    """Unpacked FP32 FMA issue rate: a launch of 8 independent FMA chains per
    thread over 16 workgroups per CU; flops / event time.  Under rocprofv3
    --pmc GRBM_GUI_ACTIVE the same launch gives the clock."""
    import torch

    from paper_1809_09725_amd import rt4d
    blocks, n_iter = 256 * 16, 4096
    out = torch.empty(blocks * 256, device="cuda")
    rt4d.calib_fma(blocks, 64, out)                      # warm-up
    best = None
    for _ in range(3):
        ms, fl = rt4d.calib_fma(blocks, n_iter, out)
        best = ms if best is None else min(best, ms)
    rate = fl / (best * 1e-3)
    print(json.dumps({"valu_calib": "unpacked FP32 FMA", "flop": fl, "ms": round(best, 4),
                      "tflops": round(rate / 1e12, 3),
                      "fma_per_clk_per_cu_at_2p4GHz": round(rate / 2 / 256 / 2.4e9, 2),
                      "frac_of_published_157p3": round(rate / PEAK_FP32_VALU, 4)}), flush=True)


def serve_main(args) -> int:
    """Serving form: the C4 trace of Poisson-arriving jobs, served with the
    precision form under continuous batching, against the plain FP32 solver
    run one job at a time in arrival order on the same trace."""
    import torch

    from paper_1809_09725_amd import inputs, serving
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    trace = serving.c4_trace(n_jobs=args.jobs, rate=args.rate, seed=4, n_iter=args.iters)
    log(f"trace: {len(trace)} jobs over {trace[-1].arrival:.1f} s, {args.iters} iterations each")
    payloads = {}
    t0 = time.perf_counter()
    for s in trace:     # each job's sinogram, made before the clock starts (the request payload)
        ph = inputs.make_phantom(s.N, s.Nz, s.Npi, 12, seed=4000 + s.jid,
                                 axis_range=(s.N / 64, s.N / 16),
                                 z_axis_range=(max(1.0, s.Nz / 16), max(1.0, s.Nz / 4)),
                                 rho_range=(0.1, 0.5), speed_per_halfturn=s.N / 64)
        g = inputs.sinogram(ph, s.N, s.Nz, s.Ns, s.Ntheta, s.Npi, noise=0.01, seed=4000 + s.jid,
                            device="cuda")
        payloads[s.jid] = g.float().cpu()
        del g
        log(f"payload {s.jid}: N={s.N} Nz={s.Nz} K={s.K} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    payload = lambda s: payloads[s.jid]
    free, total = torch.cuda.mem_get_info(dev)
    budget = int(args.budget_gb * 2**30) if args.budget_gb > 0 else int(0.8 * free)
    log(f"HBM budget {budget / 2**30:.1f} GiB of {total / 2**30:.1f} GiB")

    be = serving.GpuBackend(payload, form=args.serve_form)
    sched = serving.Scheduler(be, budget, max_active=args.max_active, depth=2,
                              window=args.window, form=args.serve_form, log=log)
    recs_s, st_s = sched.run(trace)
    be.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"served: {json.dumps(st_s)}")
    recs_p, st_p, _ = serving.serial_baseline(trace, payload, log=log)
    log(f"plain serial: {json.dumps(st_p)}")
    # equal accuracy: final objectives of the two runs of every job
    dobj = [abs(a.report["objective"] - b.report["objective"]) / abs(b.report["objective"])
            for a, b in zip(recs_s, recs_p)]
    out = {
        "metric": "served p50/p99 latency vs plain; jobs/hour",
        "unit": "jobs/hour", "value": round(st_s["jobs_per_hour"], 2),
        "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
        "config": {"workload": f"{len(trace)} jobs, Poisson arrivals {args.rate}/s, N in "
                               "{256,512,1024}, Nz in {8,32,128}, K in {8,16,32}, Ntheta = 4N over "
                               f"8 half-turns, {args.iters} iterations each, 12 moving ellipsoids, "
                               "1% noise",
                   "budget_gib": round(budget / 2**30, 1), "max_active": args.max_active,
                   "window": args.window},
        "served": {"form": {"auto": "per job: SF (bf16 contraction, fp32 projection) when K >= 2 Npi, "
                                    "else PF fp32", "sf": "SF (bf16 contraction, fp32 projection)",
                            "pf": "PF fp32"}[args.serve_form],
                   "jobs_sf": sum(serving.pick_form(s, args.serve_form) == "sf" for s in trace),
                   **{k: round(v, 3) for k, v in st_s.items()}},
        "plain_serial": {"form": "PF fp32, one job at a time", **{k: round(v, 3) for k, v in st_p.items()}},
        "jobs_per_hour_vs_plain": round(st_s["jobs_per_hour"] / st_p["jobs_per_hour"], 3),
        "p50_vs_plain": round(st_s["p50_latency_s"] / st_p["p50_latency_s"], 3),
        "p99_vs_plain": round(st_s["p99_latency_s"] / st_p["p99_latency_s"], 3),
        "objective_rel_diff_max": float(f"{max(dobj):.3e}"),
        "objective_rel_diff_median": float(f"{sorted(dobj)[len(dobj) // 2]:.3e}"),
    }
    print(json.dumps(out), flush=True)
    return 0


def ooc_main(args) -> int:
    """Out-of-core form: the iteration state stays in host memory and every
    iteration streams the volume through the GPU in z-slabs (rt_solve_ooc).
    Two calls of W and W + K iterations from the same start; their time
    difference over K is the per-iteration cost (set-up, step rule and the
    final report cancel)."""
    import torch

    from paper_1809_09725_amd import inputs, rt4d
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    W = WORKLOADS[args.workload]
    G = workload_geom(args.workload)
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, W["n_ell"], seed=W["seed"],
                             axis_range=(G.N / 64, G.N / 16),
                             z_axis_range=(G.Nz / 16, G.Nz / 4), rho_range=(0.1, 0.5),
                             speed_per_halfturn=G.N / 64, drift=W["drift"], sphere=W["sphere"])
    g = inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=W["seed"],
                        device="cuda").cpu().contiguous()
    torch.cuda.empty_cache()
    log(f"out-of-core: workload {args.workload} {G}, slabs of {args.ooc} slices")
    times = []
    rep = None
    for n in (args.warmup, args.warmup + args.steps):
        f = torch.zeros(G.f_shape)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = rt4d.solve_ooc(G, g, f, args.ooc, lambda1=2.0 ** -9 * 940.0 ** 2, lambda2=4.0,
                             n_iter=n, n_pow=20, seed=2)
        times.append(time.perf_counter() - t0)
        log(f"  {n} iterations: {times[-1]:.3f} s (residual {rep['residual']:.6g})")
    ms_it = (times[1] - times[0]) * 1e3 / args.steps
    nf, ng = G.Nz * G.N * G.N * G.K, G.Ntheta * G.Nz * G.Ns
    nh2 = 4 * G.Nz * G.N * G.N * G.Nt
    nslab = (G.Nz + args.ooc - 1) // args.ooc
    h2d = 4.0 * (2 * nf + (nslab - 1) * G.N * G.N * G.K + nh2 + 2 * ng)
    d2h = 4.0 * (2 * nf + nh2 + ng)
    samples = 2.0 * G.Ntheta * G.Nz * G.Ns * G.N
    out = {"metric": "out-of-core R_T+R_T* Gray-samples/s (state in host memory)",
           "value": round(samples / (ms_it * 1e-3) / 1e9, 3),
           "unit": "Gray-samples/s (1e9 ray-samples/s)", "higher_is_better": True, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_iter": round(ms_it, 3),
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": W["desc"], "slab": args.ooc, "slabs": nslab,
                      "state": "pinned host memory; two device slab sets, three streams"},
           "pcie": {"h2d_GB_per_iter": round(h2d / 1e9, 3), "d2h_GB_per_iter": round(d2h / 1e9, 3),
                    "h2d_GBps": round(h2d / (ms_it * 1e-3) / 1e9, 2),
                    "d2h_GBps": round(d2h / (ms_it * 1e-3) / 1e9, 2)},
           "setup_s": round(times[0], 3)}
    print(json.dumps(out), flush=True)
    return 0


def make_workload_sinogram(name: str, G, device="cuda"):
    from paper_1809_09725_amd import inputs
    W = WORKLOADS[name]
    ph = inputs.make_phantom(G.N, G.Nz, G.Npi, W["n_ell"], seed=W["seed"],
                             axis_range=(G.N / 64, G.N / 16),
                             z_axis_range=(max(1.0, G.Nz / 16), max(1.0, G.Nz / 4)),
                             rho_range=(0.1, 0.5), speed_per_halfturn=G.N / 64, drift=W["drift"],
                             sphere=W["sphere"])
    return inputs.sinogram(ph, G.N, G.Nz, G.Ns, G.Ntheta, G.Npi, noise=0.01, seed=W["seed"],
                           device=device)


def timed_iterations(plan, G, g, steps: int, warmup: int, sf: bool, kernels=KERNELS):
    """Step rule (20 power steps), then `warmup` untimed and `steps` timed
    iterations of the loop; returns (ms per iteration, per-kernel timings,
    report of the step rule)."""
    import torch

    from paper_1809_09725_amd import rt4d
    f = torch.zeros(G.f_shape, device=g.device)
    j0 = rt4d.Job(plan, g, f, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=2)
    rep0 = j0.report()
    j0.close()
    lam1 = 2.0 ** -9 * rep0["L_R"] ** 2
    job = rt4d.Job(plan, g, f, lambda1=lam1, lambda2=4.0, n_iter=warmup + steps,
                   tau=rep0["tau"], sigma=rep0["sigma"], check_every=1)
    for _ in range(warmup):
        job.step(1)
    torch.cuda.synchronize()
    rt4d.timing_reset()
    rt4d.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        job.step(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rt4d.timing_enable(False)
    per = {}
    for k in kernels:
        ms, n = rt4d.timing_read(k)
        if n:
            per[k] = (ms, n)
    rt4d.timing_reset()
    job.close()
    del f
    return (t1 - t0) * 1e3 / steps, per, rep0


def roofline_of(per: dict, G, sf: bool, workload: str) -> tuple[dict, dict]:
    """The dominant kernel's roofline object and every kernel's fraction."""
    dom = max((k for k in per if k in KERNELS), key=lambda k: per[k][0])
    bound, work = algorithmic(dom, G, sf)
    dur = per[dom][0] / per[dom][1] * 1e-3
    if bound == "hbm":
        achieved, peak, unit = work / dur / 1e9, PEAK_HBM / 1e9, "GB/s"
    else:
        achieved, peak, unit = work / dur / 1e12, PEAK_FP32_VALU / 1e12, "TFLOP/s"
    roof = {"kernel": dom, "bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": unit, "frac": round(achieved / peak, 4),
            "traffic": traffic_from_profiles(dom, workload), "launch_ms": round(dur * 1e3, 4)}
    if bound == "alu":   # against what unpacked FMAs reach on this device
        roof["frac_of_unpacked_fma"] = round(achieved * 1e12 / FP32_UNPACKED_MEASURED, 4)
    kern = {}
    for k, (ms, n) in per.items():
        if k not in KERNELS:
            continue
        b, w = algorithmic(k, G, sf)
        d = ms / n * 1e-3
        kern[k] = {"ms": round(d * 1e3, 4), "bound": b,
                   "frac": round((w / d) / (PEAK_HBM if b == "hbm" else PEAK_FP32_VALU), 4),
                   "traffic": traffic_from_profiles(k, workload)}
    return roof, kern


PREC_SLICE = 9   # the sampled slice of the precision form's error check


def precision_measure(steps: int = 5, warmup: int = 2) -> tuple[dict, dict]:
    """The precision form (synthesise-first, BF16 basis contraction on MFMA,
    FP32 projection) on its own workload, 1024^2 x 64, K = 16, 3600
    projections over 12 half-turns: timed iterations and the dominant
    kernel's roofline.  Then R_T and R_T* at the same launch configuration
    on a volume (and a sinogram) whose only nonzero slice holds seeded
    uniform values; those slices of the results come back to the host, for
    the oracle to check in the CPU leg.  Returns (object, host arrays)."""
    import torch

    from paper_1809_09725_amd import inputs, rt4d
    G = workload_geom("c3")
    W = WORKLOADS["c3"]
    t0 = time.perf_counter()
    g = make_workload_sinogram("c3", G)
    torch.cuda.synchronize()
    log(f"precision form: {G}, sinogram in {time.perf_counter() - t0:.1f} s")
    plan = rt4d.Plan(G, form=rt4d.RT_FORM_SF, prec=rt4d.RT_PREC_BF16MFMA)
    ms_it, per, rep0 = timed_iterations(plan, G, g, steps, warmup, True)
    del g
    roof, kern = roofline_of(per, G, True, "c3")
    samples = 2.0 * G.Ntheta * G.Nz * G.Ns * G.N
    log(f"precision form: {ms_it:.2f} ms/iteration; " +
        ", ".join(f"{k} {v['ms']:.2f}" for k, v in kern.items()))
    z = PREC_SLICE
    fh = inputs.uniform((G.N, G.N, G.K), 11 + z)
    f = torch.zeros(G.f_shape, device="cuda")
    f[z].copy_(torch.from_numpy(fh))
    gs = plan.forward(f)[:, z, :].cpu().numpy()
    del f
    gh = inputs.uniform((G.Ntheta, G.Ns), 23 + z)
    gi = torch.zeros(G.g_shape, device="cuda")
    gi[:, z, :].copy_(torch.from_numpy(gh))
    fs = plan.adjoint(gi)[z].cpu().numpy()
    del gi
    plan.close()
    torch.cuda.empty_cache()
    obj = {"workload": W["desc"], "form": "SF", "steps": steps, "warmup": warmup,
           "ms_per_step": round(ms_it, 3), "iters_per_s": round(1e3 / ms_it, 4),
           "value": round(samples / (ms_it * 1e-3) / 1e9, 3),
           "unit": "Gray-samples/s (1e9 ray-samples/s)",
           "roofline": roof, "kernels": kern,
           "error_vs_fp64_oracle": None}
    return obj, {"G": G, "z": z, "f": fh, "g": gh, "Rf": gs, "Rg": fs}


def precision_error(host: dict) -> dict:
    """rel-L2 (and largest element error scaled by the largest reference
    value) of the precision form's R_T and R_T* on the sampled slice against
    the FP64 oracle's folded route, with the oracle's time."""
    import numpy as np

    import oracle as O
    G = host["G"]
    og = O.Geom(N=G.N, Nz=1, Ns=G.Ns, Ntheta=G.Ntheta, Npi=G.Npi, K=G.K, Nt=G.Nt)
    t0 = time.perf_counter()
    rf = O.forward(og, host["f"][None], route="folded")[:, 0, :]
    t1 = time.perf_counter()
    ra = O.adjoint(og, host["g"][:, None, :], route="folded")[0]
    t2 = time.perf_counter()

    def err(a, b):
        a = np.asarray(a, np.float64)
        return (float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                float(np.abs(a - b).max() / np.abs(b).max()))
    ef, mf = err(host["Rf"], rf)
    ea, ma = err(host["Rg"], ra)
    return {"R_T_rel_l2": float(f"{ef:.3e}"), "R_T_max_abs_scaled": float(f"{mf:.3e}"),
            "R_T_adj_rel_l2": float(f"{ea:.3e}"), "R_T_adj_max_abs_scaled": float(f"{ma:.3e}"),
            "bar_rel_l2": 3e-3,
            "sample": f"slice {host['z']} of 64 at the full launch configuration, seeded uniform "
                      f"f and g (all other slices zero); oracle: FP64 folded route, "
                      f"{t1 - t0:.1f} s + {t2 - t1:.1f} s on {O.num_threads()} threads"}


def serving_measure(n_jobs: int) -> dict:
    """The serving form on the first n_jobs requests of the C4 trace (Poisson
    arrivals at 2 jobs/s, seed 4, 60 iterations each), three ways on the same
    payloads: served with the per-job form rule (auto), served with the plain
    FP32 form for every job (pf: the gain of batching alone), and the plain
    FP32 solver one job at a time in arrival order.  Each served result is
    compared with that job's plain result (rel-L2 of f)."""
    import torch

    from paper_1809_09725_amd import inputs, rt4d, serving
    dev = torch.device("cuda", 0)
    trace = serving.c4_trace(n_jobs=64, rate=2.0, seed=4, n_iter=60)[:n_jobs]
    payloads = {}
    t0 = time.perf_counter()
    for s in trace:
        ph = inputs.make_phantom(s.N, s.Nz, s.Npi, 12, seed=4000 + s.jid,
                                 axis_range=(s.N / 64, s.N / 16),
                                 z_axis_range=(max(1.0, s.Nz / 16), max(1.0, s.Nz / 4)),
                                 rho_range=(0.1, 0.5), speed_per_halfturn=s.N / 64)
        g = inputs.sinogram(ph, s.N, s.Nz, s.Ns, s.Ntheta, s.Npi, noise=0.01, seed=4000 + s.jid,
                            device="cuda")
        payloads[s.jid] = g.float().cpu().pin_memory()
        del g
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"serving: {len(trace)} payloads in {time.perf_counter() - t0:.1f} s")
    payload = lambda s: payloads[s.jid]
    _, st_p, res_p = serving.serial_baseline(trace, payload, keep_results=True)
    log(f"serving, plain serial: {json.dumps(st_p)}")
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info(dev)
    budget = int(0.8 * free)

    def served(form):
        be = serving.GpuBackend(payload, form=form, keep_results=True)
        sched = serving.Scheduler(be, budget, max_active=8, depth=2, window=2, form=form)
        recs, st = sched.run(trace)
        be.close()
        torch.cuda.synchronize()
        worst = 0.0
        for jid, f in be.results.items():
            ref = res_p[jid]
            d = (f - ref).contiguous().view(-1)
            e = (rt4d.rt_dot(d, d) / max(rt4d.rt_dot(ref.view(-1), ref.view(-1)), 1e-300)) ** 0.5
            worst = max(worst, e)
        be.results.clear()
        torch.cuda.empty_cache()
        log(f"serving, served {form}: {json.dumps(st)}, worst iterate rel-L2 vs plain {worst:.3e}")
        return {**{k: round(v, 3) for k, v in st.items()},
                "worst_iterate_rel_l2_vs_plain": float(f"{worst:.3e}"),
                "jobs_sf": sum(serving.pick_form(s, form) == "sf" for s in trace)}
    out_auto = served("auto")
    out_pf = served("pf")
    res_p.clear()
    torch.cuda.empty_cache()
    return {"metric": "served p50/p99 latency vs plain; jobs/hour",
            "workload": f"first {len(trace)} jobs of the 64-job trace: Poisson arrivals 2/s (seed 4), "
                        "N in {256,512,1024}, Nz in {8,32,128}, K in {8,16,32}, Ntheta = 4N over 8 "
                        "half-turns, 60 iterations each, 12 moving ellipsoids, 1% noise",
            "budget_gib": round(budget / 2**30, 1), "max_active": 8, "window": 2,
            "served_auto": {"form": "per job: SF (bf16 contraction, fp32 projection) when K >= 2 Npi, "
                                    "else PF fp32", **out_auto},
            "served_pf": {"form": "PF fp32 for every job (batching alone)", **out_pf},
            "plain_serial": {"form": "PF fp32, one job at a time", **{k: round(v, 3) for k, v in st_p.items()}},
            "jobs_per_hour_vs_plain": round(out_auto["jobs_per_hour"] / st_p["jobs_per_hour"], 3),
            "p50_vs_plain": round(out_auto["p50_latency_s"] / st_p["p50_latency_s"], 3),
            "p99_vs_plain": round(out_auto["p99_latency_s"] / st_p["p99_latency_s"], 3),
            "pf_jobs_per_hour_vs_plain": round(out_pf["jobs_per_hour"] / st_p["jobs_per_hour"], 3)}


ACCEL_CHECKS = (25, 50, 100, 200, 400, 800, 1600)


def accel_measure(nz: int = 8, n_ref: int = 3200) -> dict:
    """Plain against accelerated primal-dual loop on the model with the
    uniformly convex term mu/2 |f|^2 (mu = 1e-3 L_R^2), the 512^2 workload's
    geometry and phantom on nz slices.  Both loops run from f = 0 with the
    same initial steps; the objective (at f, FP64) is read at the check
    points.  E* = the accelerated loop's objective after n_ref iterations.
    Reported: the relative gap (E - E*)/E* of both at each check point, the
    first check point within 10% and 1% of E*, and, for each check point of
    the plain loop, the first check point at which the accelerated loop has
    reached the same objective."""
    import torch

    from paper_1809_09725_amd import rt4d
    N, _, Ns, Nth, Npi, K, Nt = WORKLOADS["c2"]["geom"]
    G = rt4d.Geom(N=N, Nz=nz, Ns=Ns, Ntheta=Nth, Npi=Npi, K=K, Nt=Nt)
    g = make_workload_sinogram("c2", G)
    plan = rt4d.Plan(G)
    f = torch.zeros(G.f_shape, device="cuda")
    j0 = rt4d.Job(plan, g, f, lambda1=0.0, lambda2=4.0, n_iter=0, n_pow=20, seed=2)
    r0 = j0.report()
    j0.close()
    L = r0["L_R"]
    kw = dict(lambda1=2.0 ** -9 * L * L, lambda2=4.0, tau=r0["tau"], sigma=r0["sigma"],
              mu=1e-3 * L * L)
    curves, t = {}, {}
    for variant, n_max in (("plain", ACCEL_CHECKS[-1]), ("accel", n_ref)):
        f.zero_()
        job = rt4d.Job(plan, g, f, n_iter=n_max, variant=variant, **kw)
        done, objs = 0, {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in ACCEL_CHECKS + ((n_ref,) if variant == "accel" else ()):
            job.step(n - done)
            done = n
            objs[n] = job.report()["objective"]
        t[variant] = time.perf_counter() - t0
        job.close()
        curves[variant] = objs
    plan.close()
    E = curves["accel"][n_ref]

    def first_within(c, frac):
        return next((n for n in ACCEL_CHECKS if c[n] - E <= frac * E), None)
    same = {}
    for n in ACCEL_CHECKS:
        same[str(n)] = next((m for m in ACCEL_CHECKS if curves["accel"][m] <= curves["plain"][n]), None)
    rel = {v: {str(n): float(f"{(c[n] - E) / E:.4e}") for n in ACCEL_CHECKS} for v, c in curves.items()}
    return {"what": "plain loop (theta = 1, fixed steps) against the accelerated loop (adaptive "
                    "theta, tau, sigma) on the model with mu/2 |f|^2, mu = 1e-3 L_R^2, from f = 0 "
                    "with the same initial steps; objective at f in FP64",
            "workload": f"512^2 x {nz} slices of the 512^2 x 128 workload's geometry and phantom, "
                        "K=16, 1800 projections over 10 half-turns",
            "E_star": float(f"{E:.9e}"), "E_star_from": f"accelerated loop, {n_ref} iterations",
            "rel_gap_plain": rel["plain"], "rel_gap_accel": rel["accel"],
            "iters_to_10pct": {"plain": first_within(curves["plain"], 0.1),
                               "accel": first_within(curves["accel"], 0.1)},
            "iters_to_1pct": {"plain": first_within(curves["plain"], 0.01),
                              "accel": first_within(curves["accel"], 0.01)},
            "accel_iters_to_plain_objective": same,
            "seconds": {k: round(v, 2) for k, v in t.items()}}


CPU_SOLVE_SLICES = 4
CPU_SOLVE_ITERS = 2


def cpu_solve_rate(G, g_slices) -> dict:
    """The oracle's solve (folded route, explicit steps so that no power
    iteration runs) on the first CPU_SOLVE_SLICES slices for CPU_SOLVE_ITERS
    iterations; slices are independent in R_T and the TV couples neighbours
    only, so the whole volume's rate is extrapolated by Nz / slices."""
    import numpy as np

    import oracle as O
    nz = g_slices.shape[1]
    og = O.Geom(N=G.N, Nz=nz, Ns=G.Ns, Ntheta=G.Ntheta, Npi=G.Npi, K=G.K, Nt=G.Nt)
    t0 = time.perf_counter()
    O.solve(og, np.asarray(g_slices, np.float64), lambda1=1.0, lambda2=4.0,
            n_iter=CPU_SOLVE_ITERS, tau=1e-3, sigma=1e-3, route="folded")
    dt = time.perf_counter() - t0
    per_it = dt / CPU_SOLVE_ITERS * G.Nz / nz
    return {"iters_per_s": float(f"{1.0 / per_it:.4e}"),
            "sample": f"oracle solve (folded route) on {nz} of {G.Nz} slices, {CPU_SOLVE_ITERS} "
                      f"iterations in {dt:.1f} s, extrapolated to the whole volume "
                      f"(x {G.Nz / nz:g})"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--valu-calib", action="store_true",
                    help="unpacked FP32 FMA issue rate of the device (the ceiling of the FMA kernels)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the precision-form measurement (1024^2 x 64, BF16 contraction)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving measurement (16-job trace, served vs plain serial)")
    ap.add_argument("--no-accel", action="store_true",
                    help="skip the accelerated-loop convergence comparison")
    ap.add_argument("--serve-jobs", type=int, default=16,
                    help="jobs of the serving trace in the default run")
    ap.add_argument("--workload", choices=tuple(WORKLOADS), default="c2",
                    help="c2: 512^2 x 128 plain FP32 (default); c3: 1024^2 x 64 precision "
                         "form; c5: 2048^2 x 32 slab, K=32, precision form")
    ap.add_argument("--form", choices=("pf", "sf"), default=None,
                    help="pf: plain FP32 project-first; sf: precision form (BF16 basis "
                         "contraction on MFMA, FP32 projection); default: the workload's form")
    ap.add_argument("--kernels-only", action="store_true",
                    help="uniform random sinogram instead of the phantom (same kernels and "
                         "launch shapes; fewer auxiliary launches, for counter runs)")
    ap.add_argument("--ooc", type=int, default=0, metavar="SLAB",
                    help="out-of-core form: the state stays in host memory and every iteration "
                         "streams the volume through the GPU in z-slabs of SLAB slices")
    ap.add_argument("--serve", action="store_true",
                    help="serving form: served precision-form trace vs the plain solver serial")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--rate", type=float, default=2.0)
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--serve-form", choices=("auto", "sf", "pf"), default="auto",
                    help="form of the served jobs: auto = precision form when K >= 2 Npi, plain "
                         "FP32 otherwise")
    ap.add_argument("--window", type=int, default=2,
                    help="jobs with the least remaining work that get iterations queued at once")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="HBM budget for resident jobs (default: 80%% of free device memory)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU path "
              "(the z-slab sharding across GPUs is designed, not built)",
              file=sys.stderr)
        return 2
    if args.copy_calib:
        copy_calib()
        return 0
    if args.valu_calib:
        valu_calib()
        return 0
    if args.serve:
        return serve_main(args)
    if args.ooc > 0:
        return ooc_main(args)

    import torch

    from paper_1809_09725_amd import rt4d
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    W = WORKLOADS[args.workload]
    if args.form is None:
        args.form = W["form"]
    sf = args.form == "sf"
    G = workload_geom(args.workload)
    log(f"workload {args.workload}: {G}, form {args.form}")
    t0 = time.perf_counter()
    if args.kernels_only:
        gen = torch.Generator(device=dev)
        gen.manual_seed(2)
        g = torch.rand(G.g_shape, generator=gen, device=dev)
    else:
        g = make_workload_sinogram(args.workload, G)
    torch.cuda.synchronize()
    log(f"sinogram synthesised in {time.perf_counter() - t0:.1f} s")
    form = rt4d.RT_FORM_SF if sf else rt4d.RT_FORM_PF
    prec = rt4d.RT_PREC_BF16MFMA if sf else rt4d.RT_PREC_FP32
    plan = rt4d.Plan(G, form=form, prec=prec)
    ms_step, per, rep0 = timed_iterations(plan, G, g, args.steps, args.warmup, sf,
                                          KERNELS + ("k_tv_norm",))
    log(f"L_R {rep0['L_R']:.6g} L_G {rep0['L_G']:.6g} tau=sigma {rep0['tau']:.6g}")
    samples = 2.0 * G.Ntheta * G.Nz * G.Ns * G.N
    value = samples / (ms_step * 1e-3) / 1e9
    log("per-kernel ms/launch: " + ", ".join(f"{k} {v[0] / v[1]:.3f}" for k, v in per.items()))
    roof, kern = roofline_of(per, G, sf, args.workload)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gray-samples/s (1e9 ray-samples/s)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if not sf else "bf16+f32", "data": "synthetic",
        "config": {"workload": W["desc"],
                   "N": G.N, "Nz": G.Nz, "Ns": G.Ns, "Ntheta": G.Ntheta, "Npi": G.Npi, "K": G.K,
                   "Nt": G.Nt, "form": args.form.upper(),
                   "precision": "fp32" if not sf else "bf16 contraction + fp32 projection",
                   "parallelism": "single GPU"},
        "iters_per_s": round(1e3 / ms_step, 4),
        "roofline": roof, "kernels": kern,
    }
    if not args.kernels_only:
        out["fbp"] = fbp_measure(plan, G, g)
    plan.close()
    nsl = max(1, min(G.Nz, round(CPU_SLICES * (512 / G.N) ** 2 * 1800 / G.Ntheta)))
    g_cpu = g[:, 0:max(nsl, CPU_SOLVE_SLICES), :].cpu().numpy()
    del g
    torch.cuda.empty_cache()
    extras = args.workload == "c2" and not args.kernels_only
    prec_host = None
    if extras and not args.no_precision:
        out["precision"], prec_host = precision_measure()
    if extras and not args.no_accel:
        out["accelerated"] = accel_measure()
        log(f"accelerated loop: {json.dumps(out['accelerated'])}")
    if extras and not args.no_serving:
        out["serving"] = serving_measure(args.serve_jobs)
    if not args.no_cpu_baseline:
        # about 15 s of oracle work: 16 slices at 512^2 x 1800 angles, fewer for larger slices
        log(f"timing the CPU oracle on {nsl} slices ...")
        out["cpu_baseline"] = cpu_baseline(G, g_cpu[:, 0:nsl, :], 3)
        out["cpu_baseline"]["solver"] = cpu_solve_rate(G, g_cpu[:, 0:CPU_SOLVE_SLICES, :])
        out["cpu_baseline"]["solver"]["gpu_iters_per_s"] = out["iters_per_s"]
        if prec_host is not None:
            out["precision"]["error_vs_fp64_oracle"] = precision_error(prec_host)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

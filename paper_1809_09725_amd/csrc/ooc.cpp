// Out-of-core form of the adapted Chambolle-Pock loop (Sec. 3, Fig. 2): the
// iteration state stays in host memory and every iteration streams the
// volume through the device in z-slabs (the slab decomposition of Sec. 7).
//
// Slices are independent for R_T and R_T*; the 4D gradient couples slice z
// to z+1 (forward difference of the frames of f~) and the divergence couples
// z to z-1 (backward difference of h2).  Slabs are processed in increasing
// z, each with one halo slice on either side:
//   upper halo: f~ of the first slice of the next slab, not yet updated in
//               this iteration, as the in-core step reads it;
//   lower halo: h2 of the last slice of the previous slab, already updated
//               in this iteration, as the in-core step reads it.
// The TV kernels compute only the slab's own slices of the extended slab,
// so every voxel sees exactly the operands of the in-core iteration and the
// iterate is the same bit for bit.
//
// Host state (pinned, allocated per call): copies of f and g, f~, h1, h2.
// Device state (per call): two sets of one extended slab of f, f~, R*h1,
// the frames and h2, and of the slab's sinogram rows of g and h1, plus a
// plan per slab height.  Slab k uses set k & 1, and three streams overlap
// the upload of slab k+1, the compute of slab k and the download of slab
// k-1; events order each copy after what it reads or overwrites.  The lower
// halo is copied on the device from the other set, so no upload waits for
// the previous slab's download.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "internal.h"

namespace rt {
namespace {

struct HostBuf {
    void *p = nullptr;
    ~HostBuf() { if (p) (void)hipHostFree(p); }
};
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

// one plan per slab height (own slices, own + halo, halo + own + halo)
struct SlabPlans {
    rt_geom g;
    const double *phi, *S;
    std::map<int, rt_plan *> m;
    ~SlabPlans()
    {
        for (auto &kv : m) rt_plan_destroy(kv.second);
    }
    int get(int nz, const Plan **out)
    {
        auto it = m.find(nz);
        if (it == m.end()) {
            rt_geom gz = g;
            gz.Nz = nz;
            rt_plan *p = nullptr;
            int rc = rt_plan_create(&gz, RT_FORM_PF, RT_PREC_FP32, phi, S, &p);
            if (rc) return rc;
            it = m.emplace(nz, p).first;
        }
        *out = &it->second->impl;
        return RT_OK;
    }
};

int fetch_red(const Plan &p, double *v, hipStream_t s)
{
    RT_HIP(hipMemcpyAsync(v, p.d_red, sizeof(double), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    return RT_OK;
}

// rows [Ntheta] of S consecutive slices of a [Ntheta][Nz][Ns] sinogram
int copy_rows(float *dst, size_t dpitch, const float *src, size_t spitch, size_t width,
              int height, hipMemcpyKind kind, hipStream_t s)
{
    if (!width || !height) return RT_OK;
    RT_HIP(hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, kind, s));
    return RT_OK;
}

int solve_ooc(const rt_geom &G, const double *phi, const double *Smat, const rt_solve_params &P,
              const float *g_host, float *f_host, int slab, rt_solve_report *rep, hipStream_t s)
{
    const int N = G.N, Nz = G.Nz, Ns = G.Ns, K = G.K, Nt = G.Nt, Nth = G.Ntheta;
    const int SL = std::min(slab, Nz);
    const size_t vf = (size_t)N * N * K;        // floats of one slice of f
    const size_t vfr = (size_t)N * N * Nt;      // of one slice of the frames
    const size_t vh2 = 4 * vfr;                 // of one slice of h2
    const size_t nf = vf * Nz, ng = (size_t)Nth * Nz * Ns, nh2 = vh2 * Nz;
    SlabPlans plans{G, phi, Smat, {}};

    // step sizes: the rule of the in-core solver, with its power iteration
    // on one slice of a slab plan and L_G from the whole volume's shape
    const Plan *pown = nullptr;
    int rc = plans.get(SL, &pown);
    if (rc) return rc;
    double tau = P.tau, sigma = P.sigma, L_R = 0.0;
    const double sn = plan_s_norm(*pown);
    const int ds = (N > 1 ? 2 : 0) + (Nz > 1 ? 1 : 0);
    const double LG2 = sn * sn * 4.0 * ((double)ds + (Nt > 1 ? P.lambda2 * P.lambda2 : 0.0));
    if (!(P.tau > 0 && P.sigma > 0)) {
        Job J;
        J.plan = pown;
        J.prm = P;
        rc = job_alloc(J);
        if (!rc) rc = job_power_iteration(J, s);
        (void)hipStreamSynchronize(s);
        L_R = J.L_R;
        job_free(J);
        if (rc) return rc;
        const double L = std::sqrt((1.01 * L_R) * (1.01 * L_R) + LG2);
        tau = sigma = 1.0 / L;
    }

    // host state
    HostBuf fh, gh, fth, h1h, h2h;
    RT_HIP(hipHostMalloc(&fh.p, std::max<size_t>(nf, 1) * sizeof(float)));
    RT_HIP(hipHostMalloc(&gh.p, std::max<size_t>(ng, 1) * sizeof(float)));
    RT_HIP(hipHostMalloc(&fth.p, std::max<size_t>(nf, 1) * sizeof(float)));
    RT_HIP(hipHostMalloc(&h1h.p, std::max<size_t>(ng, 1) * sizeof(float)));
    RT_HIP(hipHostMalloc(&h2h.p, std::max<size_t>(nh2, 1) * sizeof(float)));
    float *F = (float *)fh.p, *Gh = (float *)gh.p, *FT = (float *)fth.p;
    float *H1 = (float *)h1h.p, *H2 = (float *)h2h.p;
    std::memcpy(F, f_host, nf * sizeof(float));
    std::memcpy(Gh, g_host, ng * sizeof(float));
    std::memcpy(FT, f_host, nf * sizeof(float));
    std::memset(H1, 0, ng * sizeof(float));
    std::memset(H2, 0, nh2 * sizeof(float));

    // device slabs, two of them (slab k uses set k & 1): slot 0 = lower
    // halo, slots 1..SL own, slot SL+1 = upper halo
    const size_t slots = (size_t)SL + 2;
    const size_t ngs = std::max<size_t>((size_t)Nth * SL * Ns, 1);
    DevBuf fd[2], ftd[2], wd[2], ffd[2], h2d[2], h1d[2], gd[2], sd;
    for (int b = 0; b < 2; ++b) {
        RT_HIP(hipMalloc(&fd[b].p, slots * vf * sizeof(float)));
        RT_HIP(hipMalloc(&ftd[b].p, slots * vf * sizeof(float)));
        RT_HIP(hipMalloc(&wd[b].p, slots * vf * sizeof(float)));
        RT_HIP(hipMalloc(&ffd[b].p, slots * vfr * sizeof(float)));
        RT_HIP(hipMalloc(&h2d[b].p, slots * vh2 * sizeof(float)));
        RT_HIP(hipMalloc(&h1d[b].p, ngs * sizeof(float)));
        RT_HIP(hipMalloc(&gd[b].p, ngs * sizeof(float)));
    }
    RT_HIP(hipMalloc(&sd.p, ngs * sizeof(float)));
    float *sD = (float *)sd.p;
    // three streams (default priority): uploads, compute, downloads; events
    // per slab set and per slab of the volume
    const int nslab = (Nz + SL - 1) / SL;
    struct Pipe {
        hipStream_t st[3] = {nullptr, nullptr, nullptr};
        std::vector<hipEvent_t> ev;
        ~Pipe()
        {
            for (hipStream_t x : st)
                if (x) (void)hipStreamSynchronize(x);
            for (hipEvent_t e : ev) (void)hipEventDestroy(e);
            for (hipStream_t x : st)
                if (x) (void)hipStreamDestroy(x);
        }
    } pipe;
    for (auto &x : pipe.st) RT_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    // events: 0,1 upload done; 2,3 lower halo taken; 4,5 compute done;
    // 6,7 download done (per set); 8 + s: slab s downloaded
    pipe.ev.resize(8 + nslab);
    for (auto &e : pipe.ev) {
        RT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        RT_HIP(hipEventRecord(e, pipe.st[0]));   // complete at once: the first waits pass
    }
    hipEvent_t *evUp = &pipe.ev[0], *evHalo = &pipe.ev[2], *evComp = &pipe.ev[4];
    hipEvent_t *evDown = &pipe.ev[6], *evSlab = &pipe.ev[8];
    const hipStream_t sH = pipe.st[0], sC = pipe.st[1], sDn = pipe.st[2];
    // every return waits for the streams before the buffers above are released
    struct SyncGuard {
        hipStream_t s;
        ~SyncGuard() { (void)hipStreamSynchronize(s); }
    } sync_guard{s};
    const auto H2D = hipMemcpyHostToDevice, D2H = hipMemcpyDeviceToHost;
    const float l1 = (float)P.lambda1, l2 = (float)P.lambda2;
    double tau_n = tau, sigma_n = sigma;   // the accelerated form adapts the steps per iteration
    const size_t rowb = (size_t)Ns * sizeof(float), pitch = (size_t)Nz * rowb;

    long k = 0;   // slab counter over all iterations
    int Sprev = 0;
    for (int it = 0; it < P.n_iter; ++it) {
        const float tf = (float)tau_n, sf = (float)sigma_n;
        double cinv = 1.0;
        const double theta = cp_steps(P, &tau_n, &sigma_n, &cinv);
        for (int si = 0; si < nslab; ++si, ++k) {
            const int z0 = si * SL, z1 = std::min(Nz, z0 + SL), S = z1 - z0;
            const int lo = z0 > 0, hi = z1 < Nz, b = (int)(k & 1);
            float *fD = (float *)fd[b].p, *ftD = (float *)ftd[b].p, *wD = (float *)wd[b].p;
            float *FfD = (float *)ffd[b].p, *h2D = (float *)h2d[b].p;
            float *h1D = (float *)h1d[b].p, *gD = (float *)gd[b].p;
            const Plan *po = nullptr, *pg = nullptr, *pd = nullptr;
            // projections on the own slices; the gradient on own + upper halo;
            // the divergence on lower halo + own + upper halo (so that the own
            // slices next to a halo are interior slices, as in the volume)
            if ((rc = plans.get(S, &po)) || (rc = plans.get(S + hi, &pg)) ||
                (rc = plans.get(lo + S + hi, &pd)))
                return rc;
            // upload f, f~ (+ upper halo), h2, h1, g into set b once
            //  - set b's previous slab (k-2) is downloaded,
            //  - slab k-1 has copied its lower halo out of set b,
            //  - this slab and the next were downloaded in the last iteration
            RT_HIP(hipStreamWaitEvent(sH, evDown[b], 0));
            RT_HIP(hipStreamWaitEvent(sH, evHalo[b ^ 1], 0));
            RT_HIP(hipStreamWaitEvent(sH, evSlab[si], 0));
            if (hi) RT_HIP(hipStreamWaitEvent(sH, evSlab[si + 1], 0));
            RT_HIP(hipMemcpyAsync(fD + vf, F + z0 * vf, S * vf * sizeof(float), H2D, sH));
            RT_HIP(hipMemcpyAsync(ftD + vf, FT + z0 * vf, (S + hi) * vf * sizeof(float), H2D, sH));
            RT_HIP(hipMemcpyAsync(h2D + vh2, H2 + z0 * vh2, S * vh2 * sizeof(float), H2D, sH));
            if ((rc = copy_rows(h1D, S * rowb, H1 + (size_t)z0 * Ns, pitch, S * rowb, Nth, H2D, sH)) ||
                (rc = copy_rows(gD, S * rowb, Gh + (size_t)z0 * Ns, pitch, S * rowb, Nth, H2D, sH)))
                return rc;
            RT_HIP(hipEventRecord(evUp[b], sH));
            // compute: the lower halo is the updated h2 of the previous slab's
            // last slice, still on the device in the other set
            RT_HIP(hipStreamWaitEvent(sC, evUp[b], 0));
            if (lo)
                RT_HIP(hipMemcpyAsync(h2D, (float *)h2d[b ^ 1].p + (size_t)Sprev * vh2,
                                      vh2 * sizeof(float), hipMemcpyDeviceToDevice, sC));
            RT_HIP(hipEventRecord(evHalo[b], sC));
            if ((rc = launch_frames(*pg, ftD + vf, FfD + vfr, sC))) return rc;
            if ((rc = launch_forward(*po, ftD + vf, nullptr, CONTRACT_PROX, gD, h1D, sf, nullptr, sC)))
                return rc;
            if ((rc = launch_grad_shrink(*pg, FfD + vfr, h2D + vh2, sf, l1, l2, nullptr, sC, 0, S)))
                return rc;
            if ((rc = launch_adjoint(*po, h1D, wD + vf, sC))) return rc;
            const int e0 = 1 - lo;   // first slot of the extended slab
            if ((rc = launch_div_update(*pd, h2D + e0 * vh2, wD + e0 * vf, fD + e0 * vf, ftD + e0 * vf,
                                        FfD + e0 * vfr, tf, l2, nullptr, sC, lo, lo + S, (float)cinv,
                                        (float)theta)))
                return rc;
            RT_HIP(hipEventRecord(evComp[b], sC));
            // download the slab's own slices
            RT_HIP(hipStreamWaitEvent(sDn, evComp[b], 0));
            RT_HIP(hipMemcpyAsync(F + z0 * vf, fD + vf, S * vf * sizeof(float), D2H, sDn));
            RT_HIP(hipMemcpyAsync(FT + z0 * vf, ftD + vf, S * vf * sizeof(float), D2H, sDn));
            RT_HIP(hipMemcpyAsync(H2 + z0 * vh2, h2D + vh2, S * vh2 * sizeof(float), D2H, sDn));
            if ((rc = copy_rows(H1 + (size_t)z0 * Ns, pitch, h1D, S * rowb, S * rowb, Nth, D2H, sDn)))
                return rc;
            RT_HIP(hipEventRecord(evDown[b], sDn));
            RT_HIP(hipEventRecord(evSlab[si], sDn));
            Sprev = S;
        }
    }
    for (hipStream_t x : pipe.st) RT_HIP(hipStreamSynchronize(x));
    float *fD = (float *)fd[0].p, *gD = (float *)gd[0].p;

    // report at the final f: |R_T f - g|^2 and the TV norm, slab by slab (the
    // TV of a slab's last slice reads the next slab's first slice)
    double res2 = 0.0, tv = 0.0, fsq = 0.0;
    for (int z0 = 0; z0 < Nz; z0 += SL) {
        const int z1 = std::min(Nz, z0 + SL), S = z1 - z0, hi = z1 < Nz;
        const Plan *po = nullptr, *pg = nullptr;
        if ((rc = plans.get(S, &po)) || (rc = plans.get(S + hi, &pg))) return rc;
        RT_HIP(hipMemcpyAsync(fD + vf, F + z0 * vf, (S + hi) * vf * sizeof(float), H2D, s));
        if ((rc = copy_rows(gD, S * rowb, Gh + (size_t)z0 * Ns, pitch, S * rowb, Nth, H2D, s))) return rc;
        const size_t n = (size_t)Nth * S * Ns;
        const int nb = reduce_blocks(0, n);
        double v = 0.0;
        if ((rc = launch_forward(*po, fD + vf, sD, CONTRACT_STORE, nullptr, nullptr, 0.f, nullptr, s)) ||
            (rc = launch_diff_sq_partials(sD, gD, n, po->d_part, nb, s)) ||
            (rc = launch_finish(po->d_part, nb, 1, po->d_red, s)) || (rc = fetch_red(*po, &v, s)))
            return rc;
        res2 += v;
        if ((rc = launch_tv_norm(*pg, fD + vf, l2, pg->d_part, s, 0, S)) ||
            (rc = launch_finish(pg->d_part, (int)voxel_blocks(pg->g), 1, pg->d_red, s)) ||
            (rc = fetch_red(*pg, &v, s)))
            return rc;
        tv += v;
        if (P.mu > 0) {   // |f|^2 of the uniformly convex term
            const size_t nfs = (size_t)S * vf;
            const int nbf = reduce_blocks(0, nfs);
            if ((rc = launch_dot_partials(fD + vf, fD + vf, nfs, po->d_part, nbf, s)) ||
                (rc = launch_finish(po->d_part, nbf, 1, po->d_red, s)) || (rc = fetch_red(*po, &v, s)))
                return rc;
            fsq += v;
        }
    }
    RT_HIP(hipStreamSynchronize(s));
    std::memcpy(f_host, F, nf * sizeof(float));
    if (rep) {
        rep->L_R = L_R;
        rep->L_G = std::sqrt(LG2);
        rep->tau = tau;
        rep->sigma = sigma;
        rep->residual = std::sqrt(res2);
        rep->objective = 0.5 * res2 + P.lambda1 * tv + 0.5 * P.mu * fsq;
        rep->rel_change = 0.0;
        rep->iters_done = P.n_iter;
        if (!std::isfinite(rep->residual) || !std::isfinite(rep->objective))
            return fail(RT_E_NONFINITE, "non-finite residual or objective");
    }
    return RT_OK;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" int rt_solve_ooc(const rt_geom *geom, const double *phi, const double *S,
                            const rt_solve_params *params, const float *g, float *f, int32_t slab,
                            rt_solve_report *report, void *stream)
{
    int rc = check_geom(geom);
    if (rc) return rc;
    if ((rc = solve_params_check(params))) return rc;
    if (params->check_every != 0 || params->tol != 0)
        return fail(RT_E_ARG, "the out-of-core solve runs a fixed count: check_every and tol must be 0");
    if (slab < 1) return fail(RT_E_ARG, "slab must be >= 1 (got %d)", (int)slab);
    if (nf_of(*geom) && (!g || !f)) return fail(RT_E_ARG, "g and f must be non-NULL host arrays");
    if (geom->Nz == 0) {
        if (report) *report = rt_solve_report{};
        return RT_OK;
    }
    const hipStream_t s = (hipStream_t)stream;
    rc = solve_ooc(*geom, phi, S, *params, g, f, slab, report, s);
    return rc;
}

// The adapted Chambolle-Pock loop of Sec. 3, Fig. 2, as a resumable job:
// step sizes (power iteration in FP32 operators with FP64 norms), the
// iteration itself on the device, FP64 monitors, report, checkpoint.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace rt;

namespace {

// Slots of Plan::d_part: the h1 prox's partials first, then the shrink's,
// then the (two-wide) primal update's.
size_t off_grad(const Plan &p) { return (size_t)forward_partials(p); }
size_t off_div(const Plan &p) { return off_grad(p) + voxel_blocks(p.g); }

// |S|_2 = sqrt(largest eigenvalue of S^T S), cyclic Jacobi on the K x K matrix.
double s_norm(const Plan &p)
{
    const int K = p.g.K, Nt = p.g.Nt;
    std::vector<double> A((size_t)K * K, 0.0);
    for (int m = 0; m < Nt; ++m)
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) A[i * K + j] += p.T.S[m * K + i] * p.T.S[m * K + j];
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) (i == j ? dia : off) += A[i * K + j] * A[i * K + j];
        if (off <= 1e-30 * std::max(dia, 1e-300)) break;
        for (int a = 0; a < K; ++a)
            for (int b = a + 1; b < K; ++b) {
                const double apq = A[a * K + b];
                if (apq == 0.0) continue;
                const double tau = (A[b * K + b] - A[a * K + a]) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < K; ++k) {
                    const double x = A[k * K + a], y = A[k * K + b];
                    A[k * K + a] = c * x - s * y;
                    A[k * K + b] = s * x + c * y;
                }
                for (int k = 0; k < K; ++k) {
                    const double x = A[a * K + k], y = A[b * K + k];
                    A[a * K + k] = c * x - s * y;
                    A[b * K + k] = s * x + c * y;
                }
            }
    }
    double mx = 0.0;
    for (int i = 0; i < K; ++i) mx = std::max(mx, A[i * K + i]);
    return std::sqrt(mx);
}

int fetch(const Plan &p, int n, double *host, hipStream_t s)
{
    RT_HIP(hipMemcpyAsync(host, p.d_red, n * sizeof(double), hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    return RT_OK;
}

// L_R = |R_T| by power iteration on R_T* R_T from the seeded start vector.
int power_iteration(Job &J, hipStream_t s)
{
    // R_T acts on every slice with the same operator (parallel beam), so it
    // is block-diagonal with identical blocks and ||R_T|| is the norm of the
    // one-slice operator: iterate on slice 0 only, through a view of the plan
    // with Nz = 1 (tables and scratch are shared; scratch is sized for Nz >= 1).
    const Plan &full = *J.plan;
    Plan p = full;
    p.g.Nz = full.g.Nz > 0 ? 1 : 0;
    const size_t nf = nf_of(p.g), ng = ng_of(p.g);
    float *x = J.ft, *y = J.work;
    int rc = launch_seeded_uniform(x, nf, J.prm.seed, s);
    const int nbf = reduce_blocks(0, nf), nbg = reduce_blocks(0, ng);
    for (int it = 0; !rc && it < J.prm.n_pow; ++it) {
        if ((rc = launch_forward(p, x, J.sino, CONTRACT_STORE, nullptr, nullptr, 0.f, nullptr, s))) break;
        if ((rc = launch_adjoint(p, J.sino, y, s))) break;
        if ((rc = launch_dot_partials(y, y, nf, p.d_part, nbf, s))) break;
        if ((rc = launch_finish(p.d_part, nbf, 1, p.d_red, s))) break;
        if ((rc = launch_scale(y, p.d_red, nf, s))) break;
        std::swap(x, y);
    }
    if (!rc) rc = launch_forward(p, x, J.sino, CONTRACT_STORE, nullptr, nullptr, 0.f, nullptr, s);
    if (!rc) rc = launch_dot_partials(J.sino, J.sino, ng, p.d_part, nbg, s);
    if (!rc) rc = launch_finish(p.d_part, nbg, 1, p.d_red, s);
    ++full.shadow_gen;   // the view wrote the plan's BF16 copy of the volume
    double v = 0.0;
    if (!rc) rc = fetch(p, 1, &v, s);
    if (rc) return rc;
    J.L_R = std::sqrt(v);
    if (!std::isfinite(J.L_R)) return fail(RT_E_NONFINITE, "power iteration produced %g", J.L_R);
    return RT_OK;
}

void free_job(Job &J)
{
    for (void *ptr : {(void *)J.ft, (void *)J.work, (void *)J.h1, (void *)J.sino, (void *)J.h2,
                      (void *)J.Ff})
        if (ptr) (void)hipFree(ptr);
    J.ft = J.work = J.h1 = J.sino = J.h2 = J.Ff = nullptr;
}

int alloc_job(Job &J)
{
    const rt_geom &g = J.plan->g;
    const size_t nf = std::max<size_t>(nf_of(g), 4), ng = std::max<size_t>(ng_of(g), 4);
    const size_t n4 = std::max<size_t>(n4_of(g), 1);
    RT_HIP(hipMalloc(&J.ft, nf * sizeof(float)));
    RT_HIP(hipMalloc(&J.work, nf * sizeof(float)));
    RT_HIP(hipMalloc(&J.h1, ng * sizeof(float)));
    RT_HIP(hipMalloc(&J.sino, ng * sizeof(float)));
    RT_HIP(hipMalloc(&J.h2, 4 * n4 * sizeof(float)));
    RT_HIP(hipMalloc(&J.Ff, n4 * sizeof(float)));
    J.bytes = (2 * nf + 2 * ng + 5 * n4) * sizeof(float);
    return RT_OK;
}

int check_params(const rt_solve_params *prm)
{
    if (!prm) return fail(RT_E_ARG, "params is NULL");
    if (!std::isfinite(prm->lambda1) || prm->lambda1 < 0)
        return fail(RT_E_ARG, "lambda1 must be finite and >= 0");
    if (!std::isfinite(prm->lambda2)) return fail(RT_E_ARG, "lambda2 must be finite");
    if (prm->n_iter < 0 || prm->n_pow < 0 || prm->check_every < 0)
        return fail(RT_E_ARG, "negative iteration count");
    if (!(prm->tol >= 0)) return fail(RT_E_ARG, "tol must be >= 0");
    const bool given = prm->tau > 0 && prm->sigma > 0;
    if (!given && (prm->tau != 0 || prm->sigma != 0))
        return fail(RT_E_ARG, "tau and sigma must both be > 0 (explicit) or both 0 (default rule)");
    if (given && !(std::isfinite(prm->tau) && std::isfinite(prm->sigma)))
        return fail(RT_E_ARG, "tau and sigma must be finite");
    if (!given && prm->n_pow < 1) return fail(RT_E_ARG, "the default step rule needs n_pow >= 1");
    if (!std::isfinite(prm->mu) || prm->mu < 0) return fail(RT_E_ARG, "mu must be finite and >= 0");
    if (prm->variant != RT_CP_PLAIN && prm->variant != RT_CP_ACCEL)
        return fail(RT_E_ARG, "unknown variant %d", (int)prm->variant);
    return RT_OK;
}

int create_job(const rt_plan *plan, const rt_solve_params *prm, const float *g, float *f,
               hipStream_t s, rt_job **out)
{
    if (!out) return fail(RT_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_plan(plan);
    if (!rc) rc = check_params(prm);
    if (rc) return rc;
    const Plan &p = plan->impl;
    int dev = -1;
    RT_HIP(hipGetDevice(&dev));
    if (dev != p.device) return fail(RT_E_ARG, "current device is not the plan's device");
    if (nf_of(p.g) && (!g || !f || (uintptr_t)g % 16 || (uintptr_t)f % 16))
        return fail(RT_E_ARG, "g and f must be non-NULL, 16-byte aligned device arrays");
    rt_job *j = new (std::nothrow) rt_job();
    if (!j) return fail(RT_E_OOM, "host allocation failed");
    Job &J = j->impl;
    J.plan = &p;
    J.prm = *prm;
    J.g = g;
    J.f = f;
    rc = alloc_job(J);
    if (!rc) {
        const double sn = s_norm(p);
        const int ds = (p.g.N > 1 ? 2 : 0) + (p.g.Nz > 1 ? 1 : 0);
        const double LG2 =
            sn * sn * 4.0 * ((double)ds + (p.g.Nt > 1 ? prm->lambda2 * prm->lambda2 : 0.0));
        J.L_G = std::sqrt(LG2);
        if (prm->tau > 0 && prm->sigma > 0) {
            J.tau = prm->tau;
            J.sigma = prm->sigma;
        } else {
            rc = power_iteration(J, s);
            const double L = std::sqrt((1.01 * J.L_R) * (1.01 * J.L_R) + LG2);
            J.tau = J.sigma = 1.0 / L;
        }
        J.tau0 = J.tau;
        J.sigma0 = J.sigma;
    }
    // f~ = f, h1 = 0, h2 = 0, frames of f~
    if (!rc) rc = launch_copy(J.ft, f, nf_of(p.g), s);
    if (!rc) rc = launch_frames(p, J.ft, J.Ff, s);
    if (!rc) rc = launch_fill(J.h1, 0.f, ng_of(p.g), s);
    if (!rc) rc = launch_fill(J.h2, 0.f, 4 * n4_of(p.g), s);
    if (rc) {
        (void)hipStreamSynchronize(s);
        free_job(J);
        delete j;
        return rc;
    }
    *out = j;
    return RT_OK;
}

int step_job(Job &J, int n, hipStream_t s)
{
    const Plan &p = *J.plan;
    const rt_solve_params &P = J.prm;
    const float l1 = (float)P.lambda1, l2 = (float)P.lambda2;
    int rc = RT_OK;
    for (int it = 0; it < n && J.iters < P.n_iter && !J.stopped; ++it) {
        // this iteration's steps; the accelerated form adapts them afterwards
        const float tau = (float)J.tau, sigma = (float)J.sigma;
        double cinv = 1.0;
        const double theta = cp_steps(P, &J.tau, &J.sigma, &cinv);
        const bool check = P.check_every > 0 && (J.iters + 1) % P.check_every == 0;
        double *pf = check ? p.d_part : nullptr;
        double *pg = check ? p.d_part + off_grad(p) : nullptr;
        double *pd = check ? p.d_part + off_div(p) : nullptr;
        // step 3: h1 <- (h1 + sigma (R_T f~ - g)) / (1 + sigma)
        if (p.form == RT_FORM_SF) {
            // the BF16 shadow of f~ is current unless another call on the plan wrote it
            if (J.shadow_gen != p.shadow_gen) {
                if ((rc = launch_to_bf16(p, J.ft, s))) return rc;
                J.shadow_gen = p.shadow_gen;
            }
            if ((rc = launch_forward_sf16(p, nullptr, CONTRACT_PROX, J.g, J.h1, sigma, pf, s))) return rc;
        } else if ((rc = launch_forward(p, J.ft, nullptr, CONTRACT_PROX, J.g, J.h1, sigma, pf, s))) {
            return rc;
        }
        // step 4: h2 <- shrink(h2 + sigma grad S f~)
        if ((rc = launch_grad_shrink(p, J.Ff, J.h2, sigma, l1, l2, pg, s))) return rc;
        // steps 5-6: f+ = f - tau R_T* h1 + tau S^T div h2, f~ = 2 f+ - f
        if ((rc = launch_adjoint(p, J.h1, J.work, s))) return rc;
        if ((rc = launch_div_update(p, J.h2, J.work, J.f, J.ft, J.Ff, tau, l2, pd, s, 0, -1,
                                    (float)cinv, (float)theta)))
            return rc;
        J.shadow_gen = p.shadow_gen;
        ++J.iters;
        if (check && p.g.Nz > 0) {
            const int nbv = (int)voxel_blocks(p.g);
            if ((rc = launch_finish(pf, forward_partials(p), 1, p.d_red, s))) return rc;
            if ((rc = launch_finish(pg, nbv, 1, p.d_red + 1, s))) return rc;
            if ((rc = launch_finish(pd, nbv, 2, p.d_red + 2, s))) return rc;
            double m[4];
            if ((rc = fetch(p, 4, m, s))) return rc;
            J.residual = std::sqrt(m[0]);
            J.objective = 0.5 * m[0] + P.lambda1 * m[1] + 0.5 * P.mu * m[3];
            J.rel_change = m[3] > 0 ? std::sqrt(m[2] / m[3]) : 0.0;
            if (!std::isfinite(J.residual) || !std::isfinite(J.objective) || !std::isfinite(J.rel_change))
                return fail(RT_E_NONFINITE, "non-finite monitor at iteration %d", J.iters);
            if (P.tol > 0 && J.rel_change < P.tol) J.stopped = true;
        }
    }
    return rc;
}

int report_job(Job &J, rt_solve_report *rep, hipStream_t s)
{
    const Plan &p = *J.plan;
    const size_t ng = ng_of(p.g), nf = nf_of(p.g);
    double m[3] = {0.0, 0.0, 0.0};
    if (p.g.Nz > 0) {
        const int nbg = reduce_blocks(0, ng), nbf = reduce_blocks(0, nf);
        int rc = launch_forward(p, J.f, J.sino, CONTRACT_STORE, nullptr, nullptr, 0.f, nullptr, s);
        if (!rc) rc = launch_diff_sq_partials(J.sino, J.g, ng, p.d_part, nbg, s);
        if (!rc) rc = launch_finish(p.d_part, nbg, 1, p.d_red, s);
        if (!rc) rc = launch_tv_norm(p, J.f, (float)J.prm.lambda2, p.d_part + off_grad(p), s);
        if (!rc) rc = launch_finish(p.d_part + off_grad(p), (int)voxel_blocks(p.g), 1, p.d_red + 1, s);
        if (!rc && J.prm.mu > 0) rc = launch_dot_partials(J.f, J.f, nf, p.d_part, nbf, s);
        if (!rc && J.prm.mu > 0) rc = launch_finish(p.d_part, nbf, 1, p.d_red + 2, s);
        if (!rc) rc = fetch(p, J.prm.mu > 0 ? 3 : 2, m, s);
        if (rc) return rc;
    }
    rep->L_R = J.L_R;
    rep->L_G = J.L_G;
    rep->tau = J.tau0;
    rep->sigma = J.sigma0;
    rep->residual = std::sqrt(m[0]);
    rep->objective = 0.5 * m[0] + J.prm.lambda1 * m[1] + 0.5 * J.prm.mu * m[2];
    rep->rel_change = J.rel_change;
    rep->iters_done = J.iters;
    if (!std::isfinite(rep->residual) || !std::isfinite(rep->objective))
        return fail(RT_E_NONFINITE, "non-finite residual or objective");
    return RT_OK;
}

struct CkptHeader {
    char magic[8];
    rt_geom g;
    int32_t iters, stopped;
    double tau, sigma, L_R, L_G, residual, objective, rel_change, tau0, sigma0;
};
constexpr char kMagic[9] = "RT4DCKP2";

}  // namespace

namespace rt {
// the step rule and job buffers, for the out-of-core driver (ooc.cpp)
double plan_s_norm(const Plan &p) { return s_norm(p); }
int job_power_iteration(Job &J, hipStream_t s) { return power_iteration(J, s); }
int job_alloc(Job &J) { return alloc_job(J); }
void job_free(Job &J) { free_job(J); }
int solve_params_check(const rt_solve_params *prm) { return check_params(prm); }

double cp_steps(const rt_solve_params &P, double *tau, double *sigma, double *cinv)
{
    *cinv = P.mu > 0 ? 1.0 / (1.0 + P.mu * *tau) : 1.0;
    if (P.variant != RT_CP_ACCEL || !(P.mu > 0)) return 1.0;
    const double th = 1.0 / std::sqrt(1.0 + 2.0 * P.mu * *tau);
    *tau *= th;
    *sigma /= th;
    return th;
}
}  // namespace rt

extern "C" int rt_job_bytes(const rt_geom *geom, rt_form form, rt_prec prec, size_t *bytes)
{
    int rc = pick_form(geom, &form, &prec);
    if (rc) return rc;
    if (!bytes) return fail(RT_E_ARG, "bytes is NULL");
    const rt_geom &g = *geom;
    const size_t tables = ((size_t)g.Ntheta * g.K + (size_t)g.Nt * g.K) * sizeof(float) +
                          (size_t)(g.Ntheta / g.Npi) * (2 * sizeof(double) + 64) + 64 * 1024;
    const size_t parts = ((size_t)1 << 18) * sizeof(double) + 16 * sizeof(double);
    *bytes = tables + parts + plan_scratch_bytes(g) + n4_of(g) * sizeof(float) + job_state_bytes(g) +
             (form == RT_FORM_SF ? shadow_bytes(g) + sf_partial_bytes(g) : 0);
    return RT_OK;
}

extern "C" int rt_job_create(const rt_plan *plan, const rt_solve_params *params, const float *g,
                             float *f, void *stream, rt_job **out)
{
    return create_job(plan, params, g, f, (hipStream_t)stream, out);
}

extern "C" int rt_job_step(rt_job *job, int32_t n, void *stream)
{
    if (!job) return fail(RT_E_ARG, "job is NULL");
    if (n < 0) return fail(RT_E_ARG, "negative step count");
    return step_job(job->impl, n, (hipStream_t)stream);
}

extern "C" int rt_job_done(const rt_job *job)
{
    if (!job) return fail(RT_E_ARG, "job is NULL");
    return (job->impl.stopped || job->impl.iters >= job->impl.prm.n_iter) ? 1 : 0;
}

extern "C" int rt_job_iters(const rt_job *job)
{
    if (!job) return fail(RT_E_ARG, "job is NULL");
    return job->impl.iters;
}

extern "C" int rt_job_report(rt_job *job, rt_solve_report *rep, void *stream)
{
    if (!job || !rep) return fail(RT_E_ARG, "NULL argument");
    return report_job(job->impl, rep, (hipStream_t)stream);
}

extern "C" int rt_job_checkpoint_bytes(const rt_job *job, size_t *bytes)
{
    if (!job || !bytes) return fail(RT_E_ARG, "NULL argument");
    const rt_geom &g = job->impl.plan->g;
    *bytes = sizeof(CkptHeader) + (2 * nf_of(g) + ng_of(g) + 4 * n4_of(g)) * sizeof(float);
    return RT_OK;
}

extern "C" int rt_job_checkpoint(const rt_job *job, void *host_buf, void *stream)
{
    if (!job || !host_buf) return fail(RT_E_ARG, "NULL argument");
    const Job &J = job->impl;
    const rt_geom &g = J.plan->g;
    hipStream_t s = (hipStream_t)stream;
    CkptHeader h{};
    std::memcpy(h.magic, kMagic, 8);
    h.g = g;
    h.iters = J.iters;
    h.stopped = J.stopped;
    h.tau = J.tau; h.sigma = J.sigma; h.L_R = J.L_R; h.L_G = J.L_G;
    h.residual = J.residual; h.objective = J.objective; h.rel_change = J.rel_change;
    h.tau0 = J.tau0; h.sigma0 = J.sigma0;
    char *b = (char *)host_buf;
    std::memcpy(b, &h, sizeof h);
    b += sizeof h;
    const size_t nf = nf_of(g) * sizeof(float), ng = ng_of(g) * sizeof(float);
    const size_t n4 = 4 * n4_of(g) * sizeof(float);
    if (nf) RT_HIP(hipMemcpyAsync(b, J.f, nf, hipMemcpyDeviceToHost, s));
    if (nf) RT_HIP(hipMemcpyAsync(b + nf, J.ft, nf, hipMemcpyDeviceToHost, s));
    if (ng) RT_HIP(hipMemcpyAsync(b + 2 * nf, J.h1, ng, hipMemcpyDeviceToHost, s));
    if (n4) RT_HIP(hipMemcpyAsync(b + 2 * nf + ng, J.h2, n4, hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    return RT_OK;
}

extern "C" int rt_job_restore(rt_job *job, const void *host_buf, void *stream)
{
    if (!job || !host_buf) return fail(RT_E_ARG, "NULL argument");
    Job &J = job->impl;
    const rt_geom &g = J.plan->g;
    hipStream_t s = (hipStream_t)stream;
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof h);
    if (std::memcmp(h.magic, kMagic, 8) != 0 || std::memcmp(&h.g, &g, sizeof g) != 0)
        return fail(RT_E_ARG, "checkpoint does not belong to a job of this geometry");
    const char *b = (const char *)host_buf + sizeof h;
    const size_t nf = nf_of(g) * sizeof(float), ng = ng_of(g) * sizeof(float);
    const size_t n4 = 4 * n4_of(g) * sizeof(float);
    if (nf) RT_HIP(hipMemcpyAsync(J.f, b, nf, hipMemcpyHostToDevice, s));
    if (nf) RT_HIP(hipMemcpyAsync(J.ft, b + nf, nf, hipMemcpyHostToDevice, s));
    if (ng) RT_HIP(hipMemcpyAsync(J.h1, b + 2 * nf, ng, hipMemcpyHostToDevice, s));
    if (n4) RT_HIP(hipMemcpyAsync(J.h2, b + 2 * nf + ng, n4, hipMemcpyHostToDevice, s));
    int rc = launch_frames(*J.plan, J.ft, J.Ff, s);   // frames are a function of f~
    if (rc) return rc;
    RT_HIP(hipStreamSynchronize(s));
    J.iters = h.iters;
    J.stopped = h.stopped != 0;
    J.tau = h.tau; J.sigma = h.sigma; J.L_R = h.L_R; J.L_G = h.L_G;
    J.residual = h.residual; J.objective = h.objective; J.rel_change = h.rel_change;
    J.tau0 = h.tau0; J.sigma0 = h.sigma0;
    J.shadow_gen = ~0ull;   // the BF16 shadow no longer holds this f~
    return RT_OK;
}

extern "C" void rt_job_destroy(rt_job *job)
{
    if (!job) return;
    free_job(job->impl);   // hipFree waits for work still using the memory
    delete job;
}

extern "C" int solve(const rt_plan *plan, const rt_solve_params *params, const float *g, float *f,
                     rt_solve_report *report, void *stream)
{
    if (!report) return fail(RT_E_ARG, "report is NULL");
    hipStream_t s = (hipStream_t)stream;
    rt_job *job = nullptr;
    int rc = create_job(plan, params, g, f, s, &job);
    if (rc) return rc;
    rc = step_job(job->impl, params->n_iter, s);
    if (!rc) rc = report_job(job->impl, report, s);
    if (!rc) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "solve");
    }
    free_job(job->impl);
    delete job;
    return rc;
}

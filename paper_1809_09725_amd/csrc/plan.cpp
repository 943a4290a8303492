// Plan: geometry checks, host tables, kernel configuration, device tables.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace rt {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? RT_E_OOM : RT_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

int check_geom(const rt_geom *g)
{
    if (!g) return fail(RT_E_ARG, "geometry pointer is NULL");
    if (g->N < 1 || g->Ns < 1 || g->Ntheta < 1 || g->Npi < 1 || g->K < 1 || g->Nt < 1 ||
        g->Nz < 0)
        return fail(RT_E_SHAPE, "sizes must be >= 1 (Nz >= 0): N=%d Nz=%d Ns=%d Ntheta=%d "
                    "Npi=%d K=%d Nt=%d", g->N, g->Nz, g->Ns, g->Ntheta, g->Npi, g->K, g->Nt);
    if (g->Ntheta % g->Npi != 0)
        return fail(RT_E_SHAPE, "Ntheta=%d is not a whole number of half-turns Npi=%d",
                    g->Ntheta, g->Npi);
    if (g->Nt > g->Npi)
        return fail(RT_E_SHAPE, "Nt=%d time frames exceed the Npi=%d half-turns", g->Nt, g->Npi);
    if (g->N > 4096 || g->Ns > 8192 || g->K > 64 || g->Nt > 64 || (int64_t)g->Npi * g->K > 16384)
        return fail(RT_E_SHAPE, "size beyond the supported maximum (N<=4096, Ns<=8192, "
                    "K<=64, Nt<=64, Npi*K<=16384)");
    // a staged line of the projector is held in the prefetch registers of its
    // 512 threads: scalar staging (K % 4 != 0) covers lines of N <= 2048
    // positions, float4 staging N <= 4096
    if (g->N > 2048 && g->K % 4 != 0)
        return fail(RT_E_SHAPE, "N=%d > 2048 needs K to be a multiple of 4 (got K=%d)", g->N, g->K);
    return RT_OK;
}

int check_plan(const rt_plan *p)
{
    if (!p) return fail(RT_E_ARG, "plan is NULL");
    return RT_OK;
}

size_t plan_scratch_bytes(const rt_geom &g)
{
    const size_t n0 = (size_t)(g.Ntheta / g.Npi);
    return n0 * g.Nz * g.Ns * g.K * sizeof(float);
}

size_t shadow_bytes(const rt_geom &g)
{
    return (size_t)g.Nz * g.N * g.N * ((g.K + 15) / 16 * 16) * 2;
}

// a slice's BF16 copy in parts of at most 64 MiB of lines
int sf_line_parts(const rt_geom &g)
{
    const size_t slice = (size_t)g.N * g.N * ((g.K + 15) / 16 * 16) * 2;
    const size_t part = (size_t)64 << 20;
    return (int)std::max<size_t>(1, std::min<size_t>({(slice + part - 1) / part, 16, (size_t)std::max(g.N, 1)}));
}

size_t sf_partial_bytes(const rt_geom &g)
{
    const int nlp = sf_line_parts(g);
    return nlp > 1 ? (size_t)nlp * ng_of(g) * sizeof(float) : 0;
}

size_t job_state_bytes(const rt_geom &g)
{
    return (2 * nf_of(g) + 2 * ng_of(g) + 5 * n4_of(g)) * sizeof(float);
}

// Sec. 4, eq. discrt: theta_i = i*pi/Ntheta0, t_i = i/Ntheta (theta = alpha t,
// alpha = Npi*pi); the class a = i mod Ntheta0 of [0,pi) and the half-turn
// rot = i div Ntheta0 of the pi-periodicity identity.
static void build_tables(const rt_geom &g, const double *phi, const double *S, Tables &T)
{
    const int n0 = g.Ntheta / g.Npi;
    T.theta.resize(g.Ntheta);
    T.t.resize(g.Ntheta);
    T.cls.resize(g.Ntheta);
    T.rot.resize(g.Ntheta);
    T.flip.resize(g.Ntheta);
    T.phi.resize((size_t)g.Ntheta * g.K);
    for (int i = 0; i < g.Ntheta; ++i) {
        T.theta[i] = ((double)i * M_PI) / (double)n0;
        T.t[i] = (double)i / (double)g.Ntheta;
        T.cls[i] = i % n0;
        T.rot[i] = i / n0;
        T.flip[i] = (i / n0) & 1;
        for (int k = 0; k < g.K; ++k)
            T.phi[(size_t)i * g.K + k] =
                phi ? phi[(size_t)i * g.K + k] : std::cos(M_PI * (double)k * T.t[i]);
    }
    T.S.resize((size_t)g.Nt * g.K);
    for (int m = 0; m < g.Nt; ++m)
        for (int k = 0; k < g.K; ++k)
            T.S[(size_t)m * g.K + k] = S ? S[(size_t)m * g.K + k] : T.phi[(size_t)m * n0 * g.K + k];
    T.ccos.resize(n0);
    T.csin.resize(n0);
    for (int a = 0; a < n0; ++a) {
        T.ccos[a] = std::cos(T.theta[a]);
        T.csin[a] = std::sin(T.theta[a]);
    }
}

static int configure(Plan &p)
{
    const rt_geom &g = p.g;
    const int n0 = p.n0;
    const size_t budget = 80 * 1024;

    // ---- forward: classes grouped by walk direction
    std::vector<int> rows, cols;
    for (int a = 0; a < n0; ++a)
        (std::fabs(p.T.ccos[a]) >= std::fabs(p.T.csin[a]) ? rows : cols).push_back(a);
    FwdCfg &F = p.fwd;
    // 512 threads x 4 rays; for 512 < N <= 1024, 8 rays of 8-channel chunks:
    // each workgroup streams its whole slice through, so the re-read traffic
    // per channel-sample is 2N / (rays per workgroup).  (Register budget of
    // the two-level ray sums: 16 channels only for N <= 512, 8 rays only with
    // 8 channels and one line of prefetch in 4 float4.)
    const bool wide = g.N > 512 && g.N <= 1024 && g.K % 4 == 0;
    const int pairs_max = 512 * (wide ? 8 : 4);
    F.BT = std::min(g.Ns, pairs_max);
    F.nbt = (g.Ns + F.BT - 1) / F.BT;
    F.A = std::max(1, pairs_max / F.BT);
    F.A = std::min(F.A, (int)std::max(rows.size(), cols.size()));
    std::vector<int> gcls, gwalk;
    for (int w = 0; w < 2; ++w) {
        const std::vector<int> &L = w == 0 ? rows : cols;
        for (size_t i = 0; i < L.size(); i += F.A) {
            for (int j = 0; j < F.A; ++j)
                gcls.push_back(i + j < L.size() ? L[i + j] : -1);
            gwalk.push_back(w);
        }
    }
    F.ngroups = (int)gwalk.size();
    // LDS line buffers with an odd number of 16-byte groups per position
    // (KC = 4: 4 floats, 8: 12, 16: 20), so that 16 consecutive positions
    // fall in distinct bank groups: two buffers when they fit, else one; one
    // line must also fit the 512 threads' prefetch registers (N * KC <= 16384)
    F.KC = 0;
    const int K4 = (g.K + 3) / 4 * 4;
    for (int kc : {16, 8, 4}) {
        const int pfmax = g.K % 4 == 0 && !wide ? 8 : 4;   // float4 of line prefetch per thread
        const int kcmax = g.K % 4 == 0 && g.N <= 512 ? 16 : 8;
        if (F.KC || (kc > K4 && kc != 4) || g.N * kc > 4 * pfmax * 512 || kc > kcmax) continue;
        const int stride = line_stride(kc);
        for (int nbuf : {2, 1})
            if (!F.KC && nbuf * (size_t)(g.N + 2 * LINE_GUARD) * stride * sizeof(float) <= 160 * 1024) {
                F.KC = kc;
                F.stride = stride;
                F.nbuf = nbuf;
            }
    }
    if (F.KC == 0)
        return fail(RT_E_SHAPE, "no staged-line configuration of the projector for N=%d K=%d", g.N, g.K);
    F.pf = g.N * F.KC <= 4 * 4 * 512 ? 4 : 8;
    F.tl = g.N > 512;
    F.nkc = (g.K + F.KC - 1) / F.KC;
    F.vec = (g.K % 4 == 0) ? 4 : 1;
    F.lds = (size_t)F.nbuf * (g.N + 2 * LINE_GUARD) * F.stride * sizeof(float);
    // 16-channel chunks over more than 1024 rays: 1024 threads of 2 rays each.
    // The group (and so the slice re-read traffic) is the same as with 512
    // threads of 4 rays, at half the registers per thread, so twice the
    // waves share the CU's LDS and VALU.
    F.nth = F.KC == 16 && F.vec == 4 && !F.tl && F.A * F.BT > 1024 && g.N <= 512 ? 1024 : 512;

    // Lane order of the forward waves. A wave's 64 rays are 64 consecutive bins
    // of one class when BT is a multiple of 64; their positions on a line are
    // spaced 1/|c| in [1, sqrt 2] apart, and each 16-byte tap read is served 16
    // lanes at a time over 16 bank groups that repeat every 16 positions (the
    // padded stride is an odd number of groups). Consecutive bins in a quarter
    // of the wave span up to 22 positions, so some share a group. Ordering the
    // 64 rays by (r / c) mod 16 and dealing them out in turn to the four
    // quarters spreads each quarter's positions evenly over the 16 groups.
    // The plain form applies the order when BT is a multiple of 64, the
    // precision form to each class slot's bins.
    p.lperm.assign((size_t)n0 * 64, 0);
    for (int a = 0; a < n0; ++a) {
        const double c = std::fabs(p.T.ccos[a]) >= std::fabs(p.T.csin[a]) ? p.T.ccos[a] : p.T.csin[a];
        double ph[64];
        int ord[64];
        for (int r = 0; r < 64; ++r) {
            ph[r] = std::fmod((double)r / c, 16.0);
            if (ph[r] < 0) ph[r] += 16.0;
            ord[r] = r;
        }
        std::stable_sort(ord, ord + 64, [&](int x, int y) { return ph[x] < ph[y]; });
        for (int i = 0; i < 64; ++i) p.lperm[(size_t)a * 64 + (i % 4) * 16 + i / 4] = (uint8_t)ord[i];
    }

    // ---- adjoint: 32x32 pixel tiles, CA classes staged per round
    AdjCfg &B = p.adj;
    B.TQ = 32;
    B.TR = 32;
    B.CA = 8;
    int wmax = 2;
    for (int a = 0; a < n0; ++a) {
        const double span = (B.TQ - 1) * std::fabs(p.T.ccos[a]) + (B.TR - 1) * std::fabs(p.T.csin[a]);
        wmax = std::max(wmax, (int)std::ceil(span) + 6);
    }
    B.WMAX = wmax;
    // KC channels per window row, stride KC + 4 floats; fewer classes per
    // round when the window is wide.  9..12 channels take one 16-channel
    // chunk: the same FMAs as two 8-channel chunks, with the ray geometry
    // and the window staging done once
    {
        const int K4 = (g.K + 3) / 4 * 4;
        B.KC = K4 > 8 ? 16 : K4 > 4 ? 8 : 4;
        B.stride = B.KC + 4;
        while (B.CA > 1 && (size_t)B.CA * B.WMAX * B.stride * sizeof(float) > budget) B.CA /= 2;
        if ((size_t)B.CA * B.WMAX * B.stride * sizeof(float) > budget)
            return fail(RT_E_SHAPE, "back-projection staging does not fit");
    }
    B.nkc = (g.K + B.KC - 1) / B.KC;
    B.vec = (g.K % 4 == 0) ? 4 : 1;
    B.lds = (size_t)B.CA * B.WMAX * B.stride * sizeof(float);

    p.tv.KT = g.K <= 8 ? 8 : g.K <= 16 ? 16 : g.K <= 32 ? 32 : 64;

    // ---- synthesise-first projector: A classes x NPP frame columns in one 32-column tile
    std::vector<int> gcls_sf, gwalk_sf;
    if (p.form == RT_FORM_SF) {
        SfCfg &C = p.sf;
        C.NPP = (g.Npi + 3) / 4 * 4;
        // one workgroup covers all bins up to 2048 (each thread up to 4 bins
        // per class), so that every line's frames are synthesised once
        C.UB = g.Ns <= 512 ? 1 : g.Ns <= 1024 ? 2 : 4;
        const int kb = (g.K + 15) / 16;
        while (C.UB > 1 && C.UB * sf_slots(C.NPP, C.UB, kb) * C.NPP > (kb >= 3 ? 64 : 96))
            C.UB /= 2;   // registers
        C.A = std::min(sf_slots(C.NPP, C.UB, kb), (int)std::max(rows.size(), cols.size()));
        for (int w = 0; w < 2; ++w) {
            const std::vector<int> &L = w == 0 ? rows : cols;
            for (size_t i = 0; i < L.size(); i += C.A) {
                for (int j = 0; j < C.A; ++j) gcls_sf.push_back(i + j < L.size() ? L[i + j] : -1);
                gwalk_sf.push_back(w);
            }
        }
        C.ngroups = (int)gwalk_sf.size();
        C.BT = std::min(g.Ns, 512 * C.UB);
        C.nbt = (g.Ns + C.BT - 1) / C.BT;
        C.PCH = std::min(512, (g.N + 31) / 32 * 32);
        C.KP = (g.K + 15) / 16 * 16;
        // an odd number of 16-byte groups per row: 16 consecutive positions
        // of a b128 access fall in distinct bank groups
        const int c4 = C.A * C.NPP / 4;
        C.CS = 4 * (c4 % 2 ? c4 : c4 + 1);
        C.lds = (size_t)(C.PCH + 2) * C.CS * sizeof(float);
        C.NLP = sf_line_parts(g);
        // the staged B operand (8 waves x 3 stages x 2 KB copies of 1 KiB) for
        // 17..32 channels: there the per-step B loads are twice as large and
        // their latency bounds the step (2048^2 slab: 315 -> 252 ms); with 16
        // channels the ring's LDS costs more than it hides (512^2: one
        // workgroup per CU instead of two, 18.5 -> 28.6 ms)
        const size_t ring = (size_t)8 * 3 * 2 * kb * 1024;
        if (kb == 2 && C.lds + ring <= 160 * 1024) {
            C.DS = 3;
            C.lds += ring;
        }
    }

    // device copies of the group tables
    RT_HIP(hipMalloc(&p.d_gcls, gcls.size() * sizeof(int)));
    RT_HIP(hipMalloc(&p.d_gwalk, gwalk.size() * sizeof(int)));
    RT_HIP(hipMemcpy(p.d_gcls, gcls.data(), gcls.size() * sizeof(int), hipMemcpyHostToDevice));
    RT_HIP(hipMemcpy(p.d_gwalk, gwalk.data(), gwalk.size() * sizeof(int), hipMemcpyHostToDevice));
    p.bytes += (gcls.size() + gwalk.size()) * sizeof(int);
    if (p.form == RT_FORM_SF) {
        RT_HIP(hipMalloc(&p.d_gcls_sf, gcls_sf.size() * sizeof(int)));
        RT_HIP(hipMalloc(&p.d_gwalk_sf, gwalk_sf.size() * sizeof(int)));
        RT_HIP(hipMemcpy(p.d_gcls_sf, gcls_sf.data(), gcls_sf.size() * sizeof(int), hipMemcpyHostToDevice));
        RT_HIP(hipMemcpy(p.d_gwalk_sf, gwalk_sf.data(), gwalk_sf.size() * sizeof(int), hipMemcpyHostToDevice));
        p.bytes += (gcls_sf.size() + gwalk_sf.size()) * sizeof(int);
    }
    return RT_OK;
}

static void free_plan(Plan &p)
{
    for (void *ptr : {(void *)p.d_phi, (void *)p.d_S, (void *)p.d_ccos, (void *)p.d_csin,
                      (void *)p.d_gcls, (void *)p.d_gwalk, (void *)p.d_lperm, (void *)p.d_gcls_sf, (void *)p.d_gwalk_sf,
                      (void *)p.d_scr, (void *)p.d_frames, p.d_f16, (void *)p.d_psf,
                      (void *)p.d_part,
                      (void *)p.d_red})
        if (ptr) (void)hipFree(ptr);
}

template <class T>
static int dev_copy(T **dst, const std::vector<T> &src, size_t *bytes)
{
    const size_t b = std::max<size_t>(src.size(), 1) * sizeof(T);
    RT_HIP(hipMalloc(dst, b));
    if (!src.empty()) RT_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    *bytes += b;
    return RT_OK;
}

static int create(const rt_geom *geom, rt_form form, rt_prec prec, const double *phi,
                  const double *S, Plan &p)
{
    p.g = *geom;
    p.form = form;
    p.prec = prec;
    p.n0 = geom->Ntheta / geom->Npi;
    RT_HIP(hipGetDevice(&p.device));
    build_tables(p.g, phi, S, p.T);
    int rc = configure(p);
    if (rc) return rc;
    std::vector<float> phi32(p.T.phi.begin(), p.T.phi.end()), S32(p.T.S.begin(), p.T.S.end());
    if ((rc = dev_copy(&p.d_phi, phi32, &p.bytes))) return rc;
    if ((rc = dev_copy(&p.d_S, S32, &p.bytes))) return rc;
    if ((rc = dev_copy(&p.d_ccos, p.T.ccos, &p.bytes))) return rc;
    if ((rc = dev_copy(&p.d_csin, p.T.csin, &p.bytes))) return rc;
    if ((rc = dev_copy(&p.d_lperm, p.lperm, &p.bytes))) return rc;
    const size_t scr = std::max<size_t>(plan_scratch_bytes(p.g), 256);
    RT_HIP(hipMalloc(&p.d_scr, scr));
    p.bytes += scr;
    const size_t frb = std::max<size_t>(n4_of(p.g), 1) * sizeof(float);
    RT_HIP(hipMalloc(&p.d_frames, frb));
    p.bytes += frb;
    if (form == RT_FORM_SF) {
        const size_t sb = std::max<size_t>(shadow_bytes(p.g), 256);
        RT_HIP(hipMalloc(&p.d_f16, sb));
        p.bytes += sb;
        if (const size_t pb = sf_partial_bytes(p.g)) {
            RT_HIP(hipMalloc(&p.d_psf, pb));
            p.bytes += pb;
        }
    }
    // FP64 partials: h1 prox, shrink, primal update (two per workgroup), reductions
    p.part_cap = std::max<size_t>((size_t)1 << 18,
                                  (size_t)forward_partials(p) + 3 * (size_t)voxel_blocks(p.g) + 64);
    RT_HIP(hipMalloc(&p.d_part, p.part_cap * sizeof(double)));
    RT_HIP(hipMalloc(&p.d_red, 16 * sizeof(double)));
    p.bytes += (p.part_cap + 16) * sizeof(double);
    return RT_OK;
}

int pick_form(const rt_geom *geom, rt_form *form, rt_prec *prec)
{
    int rc = check_geom(geom);
    if (rc) return rc;
    if (*form != RT_FORM_PF && *form != RT_FORM_SF && *form != RT_FORM_AUTO)
        return fail(RT_E_ARG, "unknown form %d", (int)*form);
    if (*prec != RT_PREC_FP32 && *prec != RT_PREC_BF16MFMA)
        return fail(RT_E_ARG, "unknown precision %d", (int)*prec);
    if (*form == RT_FORM_AUTO) {
        // per ray and line, project-first taps K channels; synthesise-first
        // taps the Npi frames (rounded up to 4) and forms them on the matrix
        // cores, which pays from about K = 2 Npi (measured per iteration at
        // 8 half-turns: SF/PF 0.53-0.95 at K = 32, 0.97-1.08 at K = 16,
        // 1.2-1.7 at K = 8; 1.24 at K = 16 over 12 half-turns)
        const bool sf = *prec == RT_PREC_BF16MFMA && geom->K >= 2 * geom->Npi && geom->Npi <= 32;
        *form = sf ? RT_FORM_SF : RT_FORM_PF;
        *prec = sf ? RT_PREC_BF16MFMA : RT_PREC_FP32;
        return RT_OK;
    }
    if (*prec == RT_PREC_BF16MFMA && *form != RT_FORM_SF)
        return fail(RT_E_ARG, "the BF16 contraction needs the synthesise-first form");
    if (*form == RT_FORM_SF && *prec != RT_PREC_BF16MFMA)
        return fail(RT_E_ARG, "the synthesise-first form is built with the BF16 contraction only");
    if (*form == RT_FORM_SF && geom->Npi > 32)
        return fail(RT_E_SHAPE, "the synthesise-first form needs Npi <= 32 (got %d)", geom->Npi);
    return RT_OK;
}

}  // namespace rt

using namespace rt;

extern "C" int rt_form_pick(const rt_geom *geom, rt_form form, rt_prec prec, rt_form *form_out,
                            rt_prec *prec_out)
{
    if (!form_out || !prec_out) return fail(RT_E_ARG, "NULL output");
    int rc = pick_form(geom, &form, &prec);
    if (rc) return rc;
    *form_out = form;
    *prec_out = prec;
    return RT_OK;
}

extern "C" int rt_basis_fourier(const rt_geom *geom, int32_t M, double *phi, double *S)
{
    int rc = check_geom(geom);
    if (rc) return rc;
    if (!phi || !S) return fail(RT_E_ARG, "NULL table");
    if (M < 2 || M % 2 || geom->K != M - 1)
        return fail(RT_E_ARG, "the real form of M = %d Fourier functions has K = M - 1 (got K = %d)",
                    (int)M, geom->K);
    const int K = geom->K, n0 = geom->Ntheta / geom->Npi;
    auto row = [&](double t, double *out) {
        out[0] = 1.0;
        for (int v = 1; v <= M / 2 - 1; ++v) {
            const double w = 2.0 * M_PI * (double)v * t;
            out[2 * v - 1] = std::cos(w);
            out[2 * v] = std::sin(w);
        }
    };
    for (int i = 0; i < geom->Ntheta; ++i) row((double)i / (double)geom->Ntheta, phi + (size_t)i * K);
    for (int m = 0; m < geom->Nt; ++m)
        row((double)(m * n0) / (double)geom->Ntheta, S + (size_t)m * K);
    return RT_OK;
}

extern "C" int rt_plan_form(const rt_plan *p, rt_form *form, rt_prec *prec)
{
    if (check_plan(p) || !form || !prec) return fail(RT_E_ARG, "NULL argument");
    *form = p->impl.form;
    *prec = p->impl.prec;
    return RT_OK;
}

extern "C" int rt_plan_create(const rt_geom *geom, rt_form form, rt_prec prec, const double *phi,
                              const double *S, rt_plan **out)
{
    if (!out) return fail(RT_E_ARG, "out is NULL");
    *out = nullptr;
    int rc = pick_form(geom, &form, &prec);
    if (rc) return rc;
    if (phi)
        for (size_t e = 0; e < (size_t)geom->Ntheta * geom->K; ++e)
            if (!std::isfinite(phi[e])) return fail(RT_E_ARG, "phi has a non-finite entry");
    if (S)
        for (size_t e = 0; e < (size_t)geom->Nt * geom->K; ++e)
            if (!std::isfinite(S[e])) return fail(RT_E_ARG, "S has a non-finite entry");
    rt_plan *p = new (std::nothrow) rt_plan();
    if (!p) return fail(RT_E_OOM, "host allocation failed");
    rc = create(geom, form, prec, phi, S, p->impl);
    if (rc) {
        free_plan(p->impl);
        delete p;
        return rc;
    }
    *out = p;
    return RT_OK;
}

extern "C" void rt_plan_destroy(rt_plan *p)
{
    if (!p) return;
    free_plan(p->impl);
    delete p;
}

extern "C" int rt_plan_bytes(const rt_plan *p, size_t *bytes)
{
    if (check_plan(p) || !bytes) return fail(RT_E_ARG, "NULL argument");
    *bytes = p->impl.bytes;
    return RT_OK;
}

extern "C" int rt_tables(const rt_plan *p, double *theta, double *t, int32_t *cls, int32_t *rot,
                         int32_t *flip)
{
    if (check_plan(p)) return RT_E_ARG;
    const Tables &T = p->impl.T;
    const size_t n = T.theta.size();
    if (theta) std::memcpy(theta, T.theta.data(), n * sizeof(double));
    if (t) std::memcpy(t, T.t.data(), n * sizeof(double));
    if (cls) std::memcpy(cls, T.cls.data(), n * sizeof(int32_t));
    if (rot) std::memcpy(rot, T.rot.data(), n * sizeof(int32_t));
    if (flip) std::memcpy(flip, T.flip.data(), n * sizeof(int32_t));
    return RT_OK;
}

extern "C" const char *rt_last_error(void) { return rt::g_err.c_str(); }

/*
 * FP64 CPU oracle for time-domain-decomposition 4D tomography
 * (Nikitin, Carlsson, Andersson, Mokso, "Four-dimensional tomographic
 * reconstruction by time domain decomposition").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product library never
 * calls it, and it shares no source, header, table or helper with the
 * library.  Everything here is plain double precision, written for
 * readability: no blocking, no fusion, no reordering beyond what each
 * definition states.
 *
 * Discrete conventions (the paper leaves the static Radon discretisation
 * open, Sec. 7 only names the method it used):
 *   - slice z of the object holds pixels (row r, column q), r,q = 0..N-1,
 *     with centres x_q = q - (N-1)/2, y_r = r - (N-1)/2 (unit pixels);
 *   - detector bin b = 0..Ns-1 has centre s_b = b - (Ns-1)/2;
 *   - coefficient volumes are stored f[z][r][q][k] (k = basis index);
 *   - sinograms are stored g[i][z][b] (i = projection index);
 *   - projection i has angle theta_i = i*pi/Ntheta0 and time t_i = i/Ntheta,
 *     Ntheta0 = Ntheta/Npi angles per half-turn (Sec. 4, eq. discrt);
 *   - basis phi_k(t) = cos(pi k t), so Phi[i][k] = cos(pi k t_i);
 *   - static projector weight of pixel (q,r) for ray (theta,b):
 *       w = Lambda((s_b - s_p)/c)/c,  s_p = x_q cos(theta) + y_r sin(theta),
 *       c = max(|cos theta|, |sin theta|),  Lambda(u) = max(0, 1-|u|),
 *     which is linear interpolation along the ray with the row (or column)
 *     spacing 1/c, i.e. the ray-driven projector of Joseph.
 *
 * Functions (each names the passage it follows):
 *   or_tables            Sec. 4 eq. discrt, fold of Sec. 4
 *   or_forward_direct    Sec. 2 eq. Rfwd, discretised: project the state
 *                        f(t_i) = sum_k Phi[i][k] f_k at theta_i
 *   or_adjoint_direct    Sec. 2 eq. Radj, the exact transpose of the above
 *   or_forward_folded    Sec. 4 eq. radapr + the pi-periodicity identity:
 *                        static projections of each f_k over [0,pi) only,
 *                        distributed to every half-turn with the s-flip
 *   or_adjoint_folded    Sec. 4 eq. radadjapr + the fold-sum g~_j
 *   or_tv_grad           Sec. 2 eq. TV1 on time frames, Sec. 4 time difference
 *   or_tv_div            Sec. 3, K2* = -div (negative adjoint of the gradient)
 *   or_shrink            Sec. 3, prox of sigma F2* (pointwise projection)
 *   or_tv_norm           Sec. 2 eq. TV1 (value of the penalty, unweighted)
 *   or_power             power iteration for ||R_T|| (step-size rule)
 *   or_solve             Sec. 3 Fig. 2 (adapted Chambolle-Pock loop); with a
 *                        uniformly convex term, its accelerated form (Sec. 1,
 *                        Sec. 8: the O(1/N^2) variant of the method)
 *   or_shepp_logan      Secs. 5-6, the FBP initial guess: projections
 *                        convolved with the Shepp-Logan kernel
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t N, Nz, Ns, Ntheta, Npi, K, Nt;
} or_geom;

typedef struct {
    double lambda1, lambda2, tol, tau, sigma;
    int32_t n_iter, n_pow, check_every, route;
    uint64_t seed;
    double mu;          /* weight of the uniformly convex term mu/2 |f|^2 (0: none) */
    int32_t variant;    /* 0: theta = 1, fixed steps; 1: accelerated (adaptive theta, tau, sigma) */
} or_params;

typedef struct {
    double L_R, L_G, tau, sigma;
    double residual, objective, rel_change;
    int32_t iters_done;
} or_report;

/* ---------------------------------------------------------------- tables */

/* Sec. 4 eq. discrt: theta_i = i*dtheta with dtheta = pi/Ntheta0, t_i = i/Ntheta
 * (theta = alpha t with alpha = Npi*pi).  Index of the angle class inside the
 * half-turn, the half-turn number and its parity (Sec. 4, the identity
 * R f(k pi + theta0, s) = R f(theta0, (-1)^k s)).  phi[i][k] = cos(pi k t_i).
 * S[m][k] = phi at the start of half-turn m (time frames t at 0, pi, 2pi ...). */
int or_tables(const or_geom *g, double *theta, double *t, int32_t *cls,
              int32_t *rot, int32_t *flip, double *phi, double *S)
{
    if (g->Npi <= 0 || g->Ntheta % g->Npi != 0) return -2;
    const int n0 = g->Ntheta / g->Npi;
    for (int i = 0; i < g->Ntheta; ++i) {
        if (theta) theta[i] = ((double)i * M_PI) / (double)n0;
        if (t) t[i] = (double)i / (double)g->Ntheta;
        if (cls) cls[i] = i % n0;
        if (rot) rot[i] = i / n0;
        if (flip) flip[i] = (i / n0) & 1;
        if (phi)
            for (int k = 0; k < g->K; ++k)
                phi[(size_t)i * g->K + k] = cos(M_PI * (double)k * ((double)i / (double)g->Ntheta));
    }
    if (S) {
        if (g->Nt > g->Npi) return -2;
        for (int m = 0; m < g->Nt; ++m)
            for (int k = 0; k < g->K; ++k)
                S[(size_t)m * g->K + k] =
                    cos(M_PI * (double)k * ((double)(m * n0) / (double)g->Ntheta));
    }
    return 0;
}

/* ------------------------------------------------------ static projector */

static double tri(double u)
{
    double a = 1.0 - fabs(u);
    return a > 0.0 ? a : 0.0;
}

/* The projector weight w(theta, b, q, r) written out. */
double or_weight(double cs, double sn, int b, int q, int r, int N, int Ns)
{
    const double c = fmax(fabs(cs), fabs(sn));
    const double xq = (double)q - 0.5 * (double)(N - 1);
    const double yr = (double)r - 0.5 * (double)(N - 1);
    const double sb = (double)b - 0.5 * (double)(Ns - 1);
    const double sp = xq * cs + yr * sn;
    return tri((sb - sp) / c) / c;
}

/* Weights of pixel (q,r) at angle (cs,sn): a pixel reaches at most two bins,
 * those whose centre lies within distance c (< = 1) of s_p; every other bin
 * has weight exactly zero.  Returns the two candidate bins and weights. */
static void pixel_bins(double cs, double sn, int q, int r, int N, int Ns,
                       int *b0, double *w0, double *w1)
{
    const double xq = (double)q - 0.5 * (double)(N - 1);
    const double yr = (double)r - 0.5 * (double)(N - 1);
    const double u = xq * cs + yr * sn + 0.5 * (double)(Ns - 1); /* s_p in bin units */
    const int b = (int)floor(u);
    *b0 = b;
    *w0 = or_weight(cs, sn, b, q, r, N, Ns);
    *w1 = or_weight(cs, sn, b + 1, q, r, N, Ns);
}

/* ------------------------------------------------------ direct operators */

/* Sec. 2 eq. Rfwd discretised at the sampled angles: the object state at
 * time t_i is f(t_i) = sum_k phi_k(t_i) f_k (Sec. 4 eq. repr), and g(i,z,b)
 * is its line integral along ray (theta_i, s_b):
 *   g(i,z,b) = sum_{r,q} w(theta_i,b,q,r) sum_k Phi[i][k] f_k(z,r,q). */
void or_forward_direct(const or_geom *g, const double *theta, const double *phi,
                       const double *f, double *out)
{
    const int N = g->N, Nz = g->Nz, Ns = g->Ns, K = g->K;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < g->Ntheta; ++i) {
        const double cs = cos(theta[i]), sn = sin(theta[i]);
        for (int z = 0; z < Nz; ++z) {
            double *row = out + ((size_t)i * Nz + z) * Ns;
            for (int b = 0; b < Ns; ++b) row[b] = 0.0;
            for (int r = 0; r < N; ++r)
                for (int q = 0; q < N; ++q) {
                    const double *fk = f + (((size_t)z * N + r) * N + q) * K;
                    double state = 0.0;
                    for (int k = 0; k < K; ++k) state += phi[(size_t)i * K + k] * fk[k];
                    int b0;
                    double w0, w1;
                    pixel_bins(cs, sn, q, r, N, Ns, &b0, &w0, &w1);
                    if (b0 >= 0 && b0 < Ns) row[b0] += w0 * state;
                    if (b0 + 1 >= 0 && b0 + 1 < Ns) row[b0 + 1] += w1 * state;
                }
        }
    }
}

/* Sec. 2 eq. Radj: the exact transpose of or_forward_direct,
 *   out_k(z,r,q) = sum_i Phi[i][k] sum_b w(theta_i,b,q,r) g(i,z,b). */
void or_adjoint_direct(const or_geom *g, const double *theta, const double *phi,
                       const double *gin, double *out)
{
    const int N = g->N, Nz = g->Nz, Ns = g->Ns, K = g->K, Nth = g->Ntheta;
    double *cs = malloc(sizeof(double) * (size_t)Nth);
    double *sn = malloc(sizeof(double) * (size_t)Nth);
    for (int i = 0; i < Nth; ++i) { cs[i] = cos(theta[i]); sn[i] = sin(theta[i]); }
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int z = 0; z < Nz; ++z)
        for (int r = 0; r < N; ++r)
            for (int q = 0; q < N; ++q) {
                double *ok = out + (((size_t)z * N + r) * N + q) * K;
                for (int k = 0; k < K; ++k) ok[k] = 0.0;
                for (int i = 0; i < Nth; ++i) {
                    int b0;
                    double w0, w1;
                    pixel_bins(cs[i], sn[i], q, r, N, Ns, &b0, &w0, &w1);
                    const double *row = gin + ((size_t)i * Nz + z) * Ns;
                    double v = 0.0;
                    if (b0 >= 0 && b0 < Ns) v += w0 * row[b0];
                    if (b0 + 1 >= 0 && b0 + 1 < Ns) v += w1 * row[b0 + 1];
                    for (int k = 0; k < K; ++k) ok[k] += phi[(size_t)i * K + k] * v;
                }
            }
    free(cs);
    free(sn);
}

/* ---------------------------------------------- folded (paper) operators */

/* Static parallel-beam projection of one ray by the ray-driven walk of
 * Joseph: if |cos| >= |sin| the ray crosses every row once; at row r it sits
 * at column position u = (s - y_r sin)/cos + (N-1)/2 and takes the linearly
 * interpolated value of the two neighbouring columns, times the row spacing
 * along the ray 1/|cos|.  Otherwise the roles of rows and columns swap.
 * The callback form serves both the projection (gather) and its transpose
 * (scatter). */
typedef struct {
    int idx[2];        /* pixel offsets r*N+q of the two taps, -1 if outside */
    double w[2];
} tap2;

static void ray_taps(double cs, double sn, double s, int N, int step, tap2 *t)
{
    const double h = 0.5 * (double)(N - 1);
    if (fabs(cs) >= fabs(sn)) {
        const int r = step;
        const double y = (double)r - h;
        const double u = (s - y * sn) / cs + h;
        const int q0 = (int)floor(u);
        const double fr = u - (double)q0;
        const double inv = 1.0 / fabs(cs);
        t->idx[0] = (q0 >= 0 && q0 < N) ? r * N + q0 : -1;
        t->idx[1] = (q0 + 1 >= 0 && q0 + 1 < N) ? r * N + q0 + 1 : -1;
        t->w[0] = (1.0 - fr) * inv;
        t->w[1] = fr * inv;
    } else {
        const int q = step;
        const double x = (double)q - h;
        const double v = (s - x * cs) / sn + h;
        const int r0 = (int)floor(v);
        const double fr = v - (double)r0;
        const double inv = 1.0 / fabs(sn);
        t->idx[0] = (r0 >= 0 && r0 < N) ? r0 * N + q : -1;
        t->idx[1] = (r0 + 1 >= 0 && r0 + 1 < N) ? (r0 + 1) * N + q : -1;
        t->w[0] = (1.0 - fr) * inv;
        t->w[1] = fr * inv;
    }
}

/* Sec. 4 eq. radapr with the pi-periodicity identity: P(a,z,b,k) is the
 * static Radon transform of f_k at theta0_a = a*pi/Ntheta0 in [0,pi) only;
 * projection i = rot*Ntheta0 + a receives
 *   g(i,z,b) = sum_k Phi[i][k] P(a, z, b', k),  b' = b or Ns-1-b (odd rot),
 * since s_{Ns-1-b} = -s_b. */
void or_forward_folded(const or_geom *g, const double *phi, const double *f, double *out)
{
    const int N = g->N, Nz = g->Nz, Ns = g->Ns, K = g->K, n0 = g->Ntheta / g->Npi;
    double *P = calloc((size_t)n0 * Nz * Ns * K, sizeof(double));
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int a = 0; a < n0; ++a)
        for (int z = 0; z < Nz; ++z) {
            const double th = ((double)a * M_PI) / (double)n0;
            const double cs = cos(th), sn = sin(th);
            for (int b = 0; b < Ns; ++b) {
                const double s = (double)b - 0.5 * (double)(Ns - 1);
                double *pk = P + (((size_t)a * Nz + z) * Ns + b) * K;
                for (int step = 0; step < N; ++step) {
                    tap2 t;
                    ray_taps(cs, sn, s, N, step, &t);
                    for (int j = 0; j < 2; ++j) {
                        if (t.idx[j] < 0) continue;
                        const double *fk = f + ((size_t)z * N * N + (size_t)t.idx[j]) * K;
                        for (int k = 0; k < K; ++k) pk[k] += t.w[j] * fk[k];
                    }
                }
            }
        }
#pragma omp parallel for collapse(2) schedule(static)
    for (int i = 0; i < g->Ntheta; ++i)
        for (int z = 0; z < Nz; ++z) {
            const int a = i % n0, rot = i / n0;
            for (int b = 0; b < Ns; ++b) {
                const int bp = (rot & 1) ? Ns - 1 - b : b;
                const double *pk = P + (((size_t)a * Nz + z) * Ns + bp) * K;
                double v = 0.0;
                for (int k = 0; k < K; ++k) v += phi[(size_t)i * K + k] * pk[k];
                out[((size_t)i * Nz + z) * Ns + b] = v;
            }
        }
    free(P);
}

/* Sec. 4 eq. radadjapr with the fold-sum: g~(a,z,b,k) = sum_rot Phi[i][k]
 * g(i, z, b'), i = rot*Ntheta0 + a, b' as above; then the static
 * back-projection (transpose of the ray walk) of g~ over theta0_a in [0,pi). */
void or_adjoint_folded(const or_geom *g, const double *phi, const double *gin, double *out)
{
    const int N = g->N, Nz = g->Nz, Ns = g->Ns, K = g->K, n0 = g->Ntheta / g->Npi;
    const size_t nvox = (size_t)Nz * N * N * K;
    double *gt = calloc((size_t)n0 * Nz * Ns * K, sizeof(double));
#pragma omp parallel for collapse(2) schedule(static)
    for (int a = 0; a < n0; ++a)
        for (int z = 0; z < Nz; ++z)
            for (int b = 0; b < Ns; ++b) {
                double *gk = gt + (((size_t)a * Nz + z) * Ns + b) * K;
                for (int rot = 0; rot < g->Npi; ++rot) {
                    const int i = rot * n0 + a;
                    const int bp = (rot & 1) ? Ns - 1 - b : b;
                    const double v = gin[((size_t)i * Nz + z) * Ns + bp];
                    for (int k = 0; k < K; ++k) gk[k] += phi[(size_t)i * K + k] * v;
                }
            }
    memset(out, 0, nvox * sizeof(double));
    const int nth = omp_get_max_threads();
    double *priv = calloc((size_t)nth * nvox, sizeof(double));
#pragma omp parallel
    {
        double *mine = priv + (size_t)omp_get_thread_num() * nvox;
#pragma omp for schedule(static)
        for (int a = 0; a < n0; ++a) {
            const double th = ((double)a * M_PI) / (double)n0;
            const double cs = cos(th), sn = sin(th);
            for (int z = 0; z < Nz; ++z)
                for (int b = 0; b < Ns; ++b) {
                    const double s = (double)b - 0.5 * (double)(Ns - 1);
                    const double *gk = gt + (((size_t)a * Nz + z) * Ns + b) * K;
                    for (int step = 0; step < N; ++step) {
                        tap2 t;
                        ray_taps(cs, sn, s, N, step, &t);
                        for (int j = 0; j < 2; ++j) {
                            if (t.idx[j] < 0) continue;
                            double *ok = mine + ((size_t)z * N * N + (size_t)t.idx[j]) * K;
                            for (int k = 0; k < K; ++k) ok[k] += t.w[j] * gk[k];
                        }
                    }
                }
        }
    }
    for (int th = 0; th < nth; ++th)       /* fixed summation order */
        for (size_t e = 0; e < nvox; ++e) out[e] += priv[(size_t)th * nvox + e];
    free(priv);
    free(gt);
}

/* ---------------------------------------------------------------- 4D TV */

/* Time frames F_m = sum_k S[m][k] f_k at the half-turn starts (Sec. 4,
 * eq. discrt), then the gradient of eq. TV1 with forward differences that are
 * zero at the last index (Sec. 4, time difference between adjacent frames,
 * with unit frame spacing; lambda2 multiplies the time component).
 * p layout: p[z][r][q][m][c], c = 0:x(q) 1:y(r) 2:z 3:t. */
void or_tv_grad(const or_geom *g, const double *S, double lambda2, const double *f, double *p)
{
    const int N = g->N, Nz = g->Nz, K = g->K, Nt = g->Nt;
    const size_t nv = (size_t)Nz * N * N;
    double *F = malloc(sizeof(double) * nv * Nt);    /* F[v][m] */
#pragma omp parallel for schedule(static)
    for (size_t v = 0; v < nv; ++v)
        for (int m = 0; m < Nt; ++m) {
            double s = 0.0;
            for (int k = 0; k < K; ++k) s += S[(size_t)m * K + k] * f[v * K + k];
            F[v * Nt + m] = s;
        }
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < Nz; ++z)
        for (int r = 0; r < N; ++r)
            for (int q = 0; q < N; ++q) {
                const size_t v = ((size_t)z * N + r) * N + q;
                for (int m = 0; m < Nt; ++m) {
                    double *pv = p + (v * Nt + m) * 4;
                    const double c = F[v * Nt + m];
                    pv[0] = (q < N - 1) ? F[(v + 1) * Nt + m] - c : 0.0;
                    pv[1] = (r < N - 1) ? F[(v + N) * Nt + m] - c : 0.0;
                    pv[2] = (z < Nz - 1) ? F[(v + (size_t)N * N) * Nt + m] - c : 0.0;
                    pv[3] = (m < Nt - 1) ? lambda2 * (F[v * Nt + m + 1] - c) : 0.0;
                }
            }
    free(F);
}

/* Sec. 3: K2* = -div_{lambda2}, the divergence being the negative adjoint of
 * the gradient above: backward differences with the boundary rows of the
 * discrete TV literature (Chambolle 2004),
 *   (div p)_i = p_i [i < n-1] - p_{i-1} [i > 0]  per axis,
 * lambda2 times that on the time axis, summed, then mapped back to the
 * coefficients by S^T:  out_k = sum_m S[m][k] (div p)_m. */
void or_tv_div(const or_geom *g, const double *S, double lambda2, const double *p, double *out)
{
    const int N = g->N, Nz = g->Nz, K = g->K, Nt = g->Nt;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < Nz; ++z)
        for (int r = 0; r < N; ++r)
            for (int q = 0; q < N; ++q) {
                const size_t v = ((size_t)z * N + r) * N + q;
                double *ok = out + v * K;
                for (int k = 0; k < K; ++k) ok[k] = 0.0;
                for (int m = 0; m < Nt; ++m) {
#define PC(vv, mm, c) p[((size_t)(vv) * Nt + (mm)) * 4 + (c)]
                    double d = 0.0;
                    d += (q < N - 1 ? PC(v, m, 0) : 0.0) - (q > 0 ? PC(v - 1, m, 0) : 0.0);
                    d += (r < N - 1 ? PC(v, m, 1) : 0.0) - (r > 0 ? PC(v - N, m, 1) : 0.0);
                    d += (z < Nz - 1 ? PC(v, m, 2) : 0.0) -
                         (z > 0 ? PC(v - (size_t)N * N, m, 2) : 0.0);
                    d += lambda2 * ((m < Nt - 1 ? PC(v, m, 3) : 0.0) - (m > 0 ? PC(v, m - 1, 3) : 0.0));
#undef PC
                    for (int k = 0; k < K; ++k) ok[k] += S[(size_t)m * K + k] * d;
                }
            }
}

/* Sec. 3, prox of sigma F2*: F2* is the indicator of {|h(x)|_2 <= lambda1 for
 * every voxel and frame}, so its prox is the pointwise projection
 * h / max(1, |h|_2 / lambda1) of each 4-vector. */
void or_shrink(size_t n4, double *p, double lambda1)
{
#pragma omp parallel for schedule(static)
    for (size_t e = 0; e < n4; ++e) {
        double *v = p + e * 4;
        if (lambda1 <= 0.0) { v[0] = v[1] = v[2] = v[3] = 0.0; continue; } /* ball {0} */
        const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
        const double d = nrm / lambda1;
        const double den = d > 1.0 ? d : 1.0;   /* max(1, |h|/lambda1) */
        for (int c = 0; c < 4; ++c) v[c] /= den;
    }
}

/* Sec. 2 eq. TV1 without the lambda1 factor: sum over voxels and frames of
 * the Euclidean length of the lambda2-weighted 4D gradient. */
double or_tv_norm(const or_geom *g, const double *S, double lambda2, const double *f)
{
    const size_t n4 = (size_t)g->Nz * g->N * g->N * g->Nt;
    double *p = malloc(sizeof(double) * n4 * 4);
    or_tv_grad(g, S, lambda2, f, p);
    double s = 0.0;
    for (size_t e = 0; e < n4; ++e) {
        const double *v = p + e * 4;
        s += sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
    }
    free(p);
    return s;
}

/* ------------------------------------------------------------ the solver */

static double dot(size_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t e = 0; e < n; ++e) s += a[e] * b[e];
    return s;
}

static void apply_R(const or_geom *g, int route, const double *theta, const double *phi,
                    const double *f, double *out)
{
    if (route == 1) or_forward_folded(g, phi, f, out);
    else or_forward_direct(g, theta, phi, f, out);
}

static void apply_Rt(const or_geom *g, int route, const double *theta, const double *phi,
                     const double *gin, double *out)
{
    if (route == 1) or_adjoint_folded(g, phi, gin, out);
    else or_adjoint_direct(g, theta, phi, gin, out);
}

/* SplitMix64 (Steele, Lea, Flood 2014), used counter-style: value j of the
 * stream with seed s is the output mix of state s + (j+1)*0x9E3779B97F4A7C15.
 * The top 24 bits give u in [0,1); x = 2u - 1 is exact in single precision. */
double or_seeded_uniform(uint64_t seed, uint64_t j)
{
    uint64_t z = seed + (j + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    const double u = (double)(z >> 40) / 16777216.0;
    return 2.0 * u - 1.0;
}

/* Largest singular value of R_T by power iteration on R_T* R_T from the
 * seeded start vector: x <- R*R x / |R*R x|, n_pow times, then |R x|. */
double or_power(const or_geom *gin, int route, const double *theta, const double *phi,
                int n_pow, uint64_t seed)
{
    /* R_T applies the same operator to every slice (parallel beam, Sec. 2),
     * so it is block-diagonal with identical blocks and its norm is that of
     * the one-slice operator: the iteration runs on slice 0 alone. */
    or_geom g1 = *gin;
    if (g1.Nz > 1) g1.Nz = 1;
    const or_geom *g = &g1;
    const size_t nf = (size_t)g->Nz * g->N * g->N * g->K;
    const size_t ng = (size_t)g->Ntheta * g->Nz * g->Ns;
    double *x = malloc(sizeof(double) * nf), *y = malloc(sizeof(double) * nf);
    double *s = malloc(sizeof(double) * ng);
    for (size_t e = 0; e < nf; ++e) x[e] = or_seeded_uniform(seed, e);
    for (int it = 0; it < n_pow; ++it) {
        apply_R(g, route, theta, phi, x, s);
        apply_Rt(g, route, theta, phi, s, y);
        const double nrm = sqrt(dot(nf, y, y));
        for (size_t e = 0; e < nf; ++e) x[e] = y[e] / nrm;
    }
    apply_R(g, route, theta, phi, x, s);
    const double L = sqrt(dot(ng, s, s));
    free(x); free(y); free(s);
    return L;
}

/* |S|_2: square root of the largest eigenvalue of S^T S (K x K), by cyclic
 * Jacobi rotations until the off-diagonal mass vanishes. */
double or_S_norm(const or_geom *g, const double *S)
{
    const int K = g->K, Nt = g->Nt;
    double *A = calloc((size_t)K * K, sizeof(double));
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j)
            for (int m = 0; m < Nt; ++m) A[i * K + j] += S[m * K + i] * S[m * K + j];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j)
                if (i != j) off += A[i * K + j] * A[i * K + j];
        if (off < 1e-30) break;
        for (int p = 0; p < K; ++p)
            for (int q = p + 1; q < K; ++q) {
                const double apq = A[p * K + q];
                if (fabs(apq) < 1e-300) continue;
                const double th = 0.5 * atan2(2.0 * apq, A[q * K + q] - A[p * K + p]);
                const double c = cos(th), s = sin(th);
                for (int k = 0; k < K; ++k) {         /* A <- A J */
                    const double akp = A[k * K + p], akq = A[k * K + q];
                    A[k * K + p] = c * akp - s * akq;
                    A[k * K + q] = s * akp + c * akq;
                }
                for (int k = 0; k < K; ++k) {         /* A <- J^T A */
                    const double apk = A[p * K + k], aqk = A[q * K + k];
                    A[p * K + k] = c * apk - s * aqk;
                    A[q * K + k] = s * apk + c * aqk;
                }
            }
    }
    double mx = 0.0;
    for (int i = 0; i < K; ++i) mx = fmax(mx, A[i * K + i]);
    free(A);
    return sqrt(mx);
}

/* Sec. 3 Fig. 2, the adapted Chambolle-Pock loop, with theta = 1:
 *   h1 <- (h1 + sigma (R f~ - g)) / (1 + sigma)
 *   h2 <- shrink(h2 + sigma grad f~)
 *   f+ <- f - tau R* h1 + tau div h2
 *   f~ <- 2 f+ - f,  f <- f+
 * With mu > 0 the primal function G of the splitting is mu/2 |f|^2 instead of
 * zero (the model becomes uniformly convex, the condition under which Sec. 1
 * and Sec. 8 quote the O(1/N^2) rate of the method), so the primal step is its
 * prox:  f+ <- (f - tau R* h1 + tau div h2) / (1 + mu tau).
 * variant 1 is the accelerated form of the primal-dual method for a
 * uniformly convex G (Chambolle and Pock 2011, the algorithm with adaptive
 * steps): after the primal step of iteration n, with the steps tau_n, sigma_n
 * it used,
 *   theta_n = 1 / sqrt(1 + 2 mu tau_n),
 *   f~ <- f+ + theta_n (f+ - f),
 *   tau_{n+1} = theta_n tau_n,  sigma_{n+1} = sigma_n / theta_n.
 * (mu = 0 keeps theta_n = 1: the plain loop.)
 * Step sizes (unless given): L_R from or_power, L_G^2 = |S|^2 4 (d + l2^2 [Nt>1])
 * bounds |grad S|^2 (each forward difference has norm <= 2, d = number of
 * spatial axes longer than one sample), tau = sigma = 1/sqrt((1.01 L_R)^2 + L_G^2),
 * which keeps tau sigma |K|^2 < 1.  Every check_every iterations the monitors
 * are taken at the extrapolated point that the step just used:
 *   residual = |R f~ - g|, objective = 1/2 residual^2 + lambda1 TV(f~)
 *   (+ mu/2 |f+|^2, at the point the primal step produced),
 *   rel_change = |f+ - f| / |f+|;  the loop stops when rel_change < tol.
 * After the loop the report's residual and objective are recomputed at f;
 * the report's tau and sigma are those of the step rule (tau_0, sigma_0). */
int or_solve(const or_geom *g, const double *theta, const double *phi, const double *S,
             const or_params *prm, const double *gdata, double *f, or_report *rep)
{
    const size_t nf = (size_t)g->Nz * g->N * g->N * g->K;
    const size_t ng = (size_t)g->Ntheta * g->Nz * g->Ns;
    const size_t n4 = (size_t)g->Nz * g->N * g->N * g->Nt;
    const int route = prm->route;
    memset(rep, 0, sizeof(*rep));

    double tau = prm->tau, sigma = prm->sigma;
    const double sn = or_S_norm(g, S);
    const int ds = (g->N > 1 ? 2 : 0) + (g->Nz > 1 ? 1 : 0);
    const double LG2 = sn * sn * 4.0 * ((double)ds + (g->Nt > 1 ? prm->lambda2 * prm->lambda2 : 0.0));
    rep->L_G = sqrt(LG2);
    if (!(tau > 0.0 && sigma > 0.0)) {
        rep->L_R = or_power(g, route, theta, phi, prm->n_pow, prm->seed);
        const double L = sqrt((1.01 * rep->L_R) * (1.01 * rep->L_R) + LG2);
        tau = sigma = 1.0 / L;
    }
    rep->tau = tau;
    rep->sigma = sigma;

    double *ft = malloc(sizeof(double) * nf), *fn = malloc(sizeof(double) * nf);
    double *h1 = calloc(ng, sizeof(double)), *Rf = malloc(sizeof(double) * ng);
    double *h2 = calloc(n4 * 4, sizeof(double)), *gr = malloc(sizeof(double) * n4 * 4);
    double *adj = malloc(sizeof(double) * nf), *dv = malloc(sizeof(double) * nf);
    memcpy(ft, f, sizeof(double) * nf);

    const double mu = prm->mu;
    int n = 0;
    for (n = 0; n < prm->n_iter; ++n) {
        const int check = prm->check_every > 0 && ((n + 1) % prm->check_every == 0);
        apply_R(g, route, theta, phi, ft, Rf);
        double res2 = 0.0;
        for (size_t e = 0; e < ng; ++e) {
            const double d = Rf[e] - gdata[e];
            res2 += d * d;
            h1[e] = (h1[e] + sigma * d) / (1.0 + sigma);
        }
        or_tv_grad(g, S, prm->lambda2, ft, gr);
        double tvn = 0.0;
        for (size_t e = 0; e < n4; ++e) {
            const double *v = gr + e * 4;
            tvn += sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
        }
        for (size_t e = 0; e < n4 * 4; ++e) h2[e] += sigma * gr[e];
        or_shrink(n4, h2, prm->lambda1);
        apply_Rt(g, route, theta, phi, h1, adj);
        or_tv_div(g, S, prm->lambda2, h2, dv);
        const double th = prm->variant == 1 ? 1.0 / sqrt(1.0 + 2.0 * mu * tau) : 1.0;
        double dn2 = 0.0, fn2 = 0.0;
        for (size_t e = 0; e < nf; ++e) {
            fn[e] = (f[e] - tau * adj[e] + tau * dv[e]) / (1.0 + mu * tau);
            const double d = fn[e] - f[e];
            dn2 += d * d;
            fn2 += fn[e] * fn[e];
            ft[e] = prm->variant == 1 ? fn[e] + th * (fn[e] - f[e]) : 2.0 * fn[e] - f[e];
            f[e] = fn[e];
        }
        if (prm->variant == 1) {
            tau = th * tau;
            sigma = sigma / th;
        }
        if (check) {
            rep->residual = sqrt(res2);
            rep->objective = 0.5 * res2 + prm->lambda1 * tvn + 0.5 * mu * fn2;
            rep->rel_change = fn2 > 0.0 ? sqrt(dn2 / fn2) : 0.0;
            if (prm->tol > 0.0 && rep->rel_change < prm->tol) { ++n; break; }
        }
    }
    rep->iters_done = n;
    apply_R(g, route, theta, phi, f, Rf);
    double res2 = 0.0;
    for (size_t e = 0; e < ng; ++e) { const double d = Rf[e] - gdata[e]; res2 += d * d; }
    rep->residual = sqrt(res2);
    rep->objective = 0.5 * res2 + prm->lambda1 * or_tv_norm(g, S, prm->lambda2, f) +
                     0.5 * mu * dot(nf, f, f);
    free(ft); free(fn); free(h1); free(Rf); free(h2); free(gr); free(adj); free(dv);
    return 0;
}

/* ------------------------------------------------ FBP initial guess */

/* Secs. 5-6 start the iteration from a filtered back-projection that uses
 * the Shepp-Logan filter.  For unit bin spacing its kernel is
 *   h(n) = -2 / (pi^2 (4 n^2 - 1))            (Shepp and Logan, 1974)
 * and each projection row is convolved with it over the detector, bins
 * outside [0, Ns) being zero:
 *   q(i,z,b) = sum_{b'=0}^{Ns-1} h(b - b') g(i,z,b'). */
void or_shepp_logan(const or_geom *g, const double *gin, double *q)
{
    const int Ns = g->Ns;
    const long rows = (long)g->Ntheta * g->Nz;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        const double *in = gin + row * Ns;
        double *out = q + row * Ns;
        for (int b = 0; b < Ns; ++b) {
            double v = 0.0;
            for (int bp = 0; bp < Ns; ++bp) {
                const double n = (double)(b - bp);
                v += -2.0 / (M_PI * M_PI * (4.0 * n * n - 1.0)) * in[bp];
            }
            out[b] = v;
        }
    }
}

int or_num_threads(void) { return omp_get_max_threads(); }

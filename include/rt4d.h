/*
 * rt4d — decomposed-time parallel-beam tomography on one MI355X (gfx950).
 *
 * C ABI of librt4d.so.  The operations follow Nikitin, Carlsson, Andersson,
 * Mokso, "Four-dimensional tomographic reconstruction by time domain
 * decomposition":
 *
 *   the object is f(x,y,z,t) = sum_k phi_k(t) f_k(x,y,z)          (Sec. 4, eq. repr)
 *   projection i is taken at angle theta_i at its own time t_i     (Sec. 2, eq. Rfwd;
 *                                                                   Sec. 4, eq. discrt)
 *   it minimises 1/2 |R_T f - g|^2 + lambda1 |  |grad_lambda2 f|  |_1   (Sec. 2, eq. lr12)
 *   with the adapted Chambolle-Pock loop                            (Sec. 3, Fig. 2).
 *
 * Discrete conventions (fixed by this library; the paper leaves the static
 * projector open):
 *   - slice z holds pixels (row r, column q), 0 <= r,q < N, centred at
 *     x_q = q - (N-1)/2, y_r = r - (N-1)/2; detector bin b at s_b = b - (Ns-1)/2;
 *   - Ntheta = Npi * Ntheta0 projections over Npi half-turns:
 *     theta_i = i*pi/Ntheta0, t_i = i/Ntheta  (theta = alpha t, alpha = Npi*pi);
 *   - default basis phi_k(t) = cos(pi k t): Phi[i][k] = phi_k(t_i);
 *   - static projector: linear interpolation along each ray with the row (or
 *     column) spacing 1/c, c = max(|cos|,|sin|) (Joseph's ray-driven method);
 *     its exact transpose is the pixel-driven back-projector with the triangle
 *     weight max(0, 1 - |s_b - s_p|/c)/c, s_p = x cos(theta) + y sin(theta);
 *   - the TV acts on Nt <= Npi time frames F_m = sum_k S[m][k] f_k, by default
 *     the states at the half-turn starts, S[m][k] = Phi[m*Ntheta0][k]
 *     (Sec. 4: frames at 0, pi, 2pi, ...), with forward differences that are
 *     zero at the last index, and lambda2 on the time difference (eq. TV1).
 *
 * Memory layouts (all row-major, FP32 unless stated; "device" = HIP device
 * memory of the current device, "host" = ordinary host memory):
 *   f   [Nz][N][N][K]       coefficient volumes f_k, basis index innermost
 *   g   [Ntheta][Nz][Ns]    sinogram
 *   p   [Nz][Nt][4][N][N]   4D gradient / dual field: for each slice and time
 *                           frame, four component planes (x, y, z, t)
 *
 * Conventions for every call:
 *   - the caller owns every array passed in; the library never frees them;
 *   - device pointers must be 16-byte aligned (RT_E_ARG otherwise) and may be
 *     NULL only when the array is empty (Nz == 0);
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     calls are asynchronous on that stream unless stated otherwise;
 *   - return RT_OK (0) or a negative rt_status; arguments and shapes are
 *     checked before anything is launched; rt_last_error() returns a
 *     thread-local message for the last failure on the calling thread;
 *   - a plan owns scratch memory: calls on one plan must not overlap in time
 *     (issue them on one stream, or synchronise between streams).
 */
#ifndef RT4D_H
#define RT4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem sizes.  Ntheta % Npi == 0 (the paper assumes whole half-turns,
 * Sec. 4; a remainder is rejected with RT_E_SHAPE).  N, Ns, Ntheta, Npi, K,
 * Nt >= 1, 1 <= Nt <= Npi, Nz >= 0 (Nz == 0: every operator is a no-op). */
typedef struct {
    int32_t N, Nz, Ns, Ntheta, Npi, K, Nt;
} rt_geom;

typedef enum {
    RT_OK = 0,
    RT_E_ARG = -1,        /* bad pointer, enum or parameter value        */
    RT_E_SHAPE = -2,      /* geometry violates the rules above           */
    RT_E_HIP = -3,        /* a HIP runtime call failed                   */
    RT_E_OOM = -4,        /* device allocation failed                    */
    RT_E_NONFINITE = -5   /* a FP64 monitor of solve saw NaN or Inf      */
} rt_status;

/* Order of the two contractions of R_T = sum_k Phi[i][k] R(f_k)(theta_i):
 * project-first projects the K coefficient volumes over the Ntheta0 angles
 * of [0,pi) and distributes them with the s-flip to every half-turn (Sec. 4,
 * eq. radapr and the pi-periodicity); synthesise-first forms the states
 * sum_k Phi[i][k] f_k and projects those.  RT_FORM_AUTO lets the library
 * choose (rt_form_pick): project-first taps K channels per ray and line,
 * synthesise-first taps Npi frames (rounded up to 4) and also forms them, so
 * with RT_PREC_BF16MFMA it takes synthesise-first when K >= 2 Npi and
 * Npi <= 32, and project-first in FP32 otherwise; with RT_PREC_FP32 it is
 * project-first. */
/* (The _RT_*_I32 members make every 32-bit value a value of the enum type,
 * so a caller's out-of-range argument reaches the library's check and its
 * RT_E_ARG without undefined behaviour in the C++ that reads it.) */
typedef enum { RT_FORM_PF = 0, RT_FORM_SF = 1, RT_FORM_AUTO = 2, _RT_FORM_I32 = 0x7fffffff } rt_form;

/* RT_PREC_FP32: every product in FP32.  RT_PREC_BF16MFMA: the basis
 * contraction sum_k Phi f_k (and its transpose) in BF16 on the matrix cores
 * with FP32 accumulation (f_k rounded to BF16 with round-to-nearest-even,
 * Phi split into BF16 hi+lo), the projection itself in FP32.  BF16 requires
 * RT_FORM_SF, and RT_FORM_SF requires BF16 and Npi <= 32.  An SF plan keeps a
 * BF16 copy of the volume it last projected ([Nz][N][N][K rounded up to 16]);
 * rt_forward converts its input into it, a job refreshes it in the primal
 * update. */
typedef enum { RT_PREC_FP32 = 0, RT_PREC_BF16MFMA = 1, _RT_PREC_I32 = 0x7fffffff } rt_prec;

typedef struct rt_plan rt_plan;

/* Build the tables (angles, times, classes, Phi, S) and allocate scratch on
 * the current device.  phi: host FP64 [Ntheta][K] or NULL for the cosine
 * basis; S: host FP64 [Nt][K] or NULL for the half-turn frames.  Both are
 * copied.  On success *out owns device memory until rt_plan_destroy. */
int rt_plan_create(const rt_geom *geom, rt_form form, rt_prec prec,
                   const double *phi, const double *S, rt_plan **out);
void rt_plan_destroy(rt_plan *plan);

/* Device bytes the plan holds (tables + scratch). */
int rt_plan_bytes(const rt_plan *plan, size_t *bytes);

/* The form and precision a plan of this geometry runs for the requested
 * pair: RT_FORM_AUTO resolved as stated at rt_form, the other forms checked
 * and returned as they are (RT_E_ARG / RT_E_SHAPE as rt_plan_create would
 * give).  Host only; the outputs may not be NULL. */
int rt_form_pick(const rt_geom *geom, rt_form form, rt_prec prec, rt_form *form_out,
                 rt_prec *prec_out);

/* The form and precision the plan runs (never RT_FORM_AUTO).  Host only. */
int rt_plan_form(const rt_plan *plan, rt_form *form, rt_prec *prec);

/* Tables of the paper's Fourier basis of M functions (Sec. 5:
 * phi_j(t) = exp(2 pi i t (j - M/2)), j = 0 .. M-1; Sec. 6 takes M = 16) in
 * the real form that spans the same real-valued objects: a real f(t) has
 * coefficients with c_{-v} = conj(c_v), and the lone frequency -M/2 carries
 * no real function, so the span is the K = M - 1 functions
 *   1, cos(2 pi v t), sin(2 pi v t)   for v = 1 .. M/2 - 1, in that order.
 * Real coefficients (a_0, a_v, b_v) and the complex ones are related by
 * c_0 = a_0, c_v = (a_v - i b_v) / 2, c_{-v} = (a_v + i b_v) / 2,
 * c_{-M/2} = 0; the adjoint's conj(phi) (Sec. 4) is the transpose of this
 * real table.  Fills host FP64 phi[Ntheta][K] at t_i = i/Ntheta and
 * S[Nt][K] at the half-turn starts (t = m Ntheta0 / Ntheta), for
 * rt_plan_create.  M even, M >= 2, and geom->K == M - 1 (RT_E_ARG else).
 * Host only. */
int rt_basis_fourier(const rt_geom *geom, int32_t M, double *phi, double *S);

/* Copy the host tables (Sec. 4, eq. discrt): theta[Ntheta] = i*pi/Ntheta0,
 * t[Ntheta] = i/Ntheta, cls[Ntheta] = i mod Ntheta0, rot[Ntheta] =
 * i div Ntheta0, flip[Ntheta] = rot & 1.  Any pointer may be NULL. Host only. */
int rt_tables(const rt_plan *plan, double *theta, double *t, int32_t *cls,
              int32_t *rot, int32_t *flip);

/* g = R_T f (Sec. 2, eq. Rfwd discretised; Sec. 4, eq. radapr).  Device f, g. */
int rt_forward(const rt_plan *plan, const float *f, float *g, void *stream);

/* f_out = R_T* g, the exact transpose of rt_forward (Sec. 2, eq. Radj;
 * Sec. 4, eq. radadjapr with the fold-sum).  Device g, f_out. */
int rt_adjoint(const rt_plan *plan, const float *g, float *f_out, void *stream);

/* p = grad_lambda2(S f) on the Nt time frames (Sec. 2, eq. TV1).  Device. */
int tv_grad(const rt_plan *plan, const float *f, float lambda2, float *p, void *stream);

/* f_out = S^T div_lambda2 p, with div = -grad^T (Sec. 3: K2* = -div).  Device. */
int tv_div(const rt_plan *plan, const float *p, float lambda2, float *f_out, void *stream);

/* In place p <- p / max(1, |p|_2 / lambda1) for every voxel and frame
 * 4-vector: the prox of sigma F2* (Sec. 3).  lambda1 >= 0.  Device. */
int shrink(const rt_plan *plan, float *p, float lambda1, void *stream);

/* Solver parameters.  lambda1, lambda2: penalty weights of eq. lr12.
 * tau, sigma: step sizes; both > 0 overrides the default rule
 * tau = sigma = 1/sqrt((1.01 L_R)^2 + L_G^2) with L_R = |R_T| by n_pow steps
 * of power iteration from the seeded start vector (SplitMix64, value j =
 * output j+1 of the stream with state `seed`, mapped to 2u-1, u = top 24
 * bits / 2^24) and L_G^2 = |S|_2^2 * 4 * (spatial axes longer than 1 +
 * lambda2^2 [Nt > 1]).  check_every > 0: FP64 monitors every so many
 * iterations, stop when rel_change < tol.  0 = fixed count.
 * mu >= 0: weight of a uniformly convex term mu/2 |f|^2 added to the model
 * (0: the model of eq. lr12 as it stands).  variant: RT_CP_PLAIN (theta = 1,
 * fixed steps) or RT_CP_ACCEL, the accelerated form of the primal-dual
 * method for a uniformly convex primal term, whose O(1/N^2) rate Secs. 1
 * and 8 of the paper name (Chambolle and Pock 2011, adaptive steps): after
 * the primal step of iteration n, taken with tau_n and sigma_n,
 *   theta_n = 1 / sqrt(1 + 2 mu tau_n),  f~ = f+ + theta_n (f+ - f),
 *   tau_{n+1} = theta_n tau_n,  sigma_{n+1} = sigma_n / theta_n.
 * With mu = 0 both variants are the plain loop. */
typedef enum { RT_CP_PLAIN = 0, RT_CP_ACCEL = 1, _RT_CP_I32 = 0x7fffffff } rt_cp_variant;

typedef struct {
    double lambda1, lambda2, tol, tau, sigma;
    int32_t n_iter, n_pow, check_every;
    uint64_t seed;
    double mu;
    int32_t variant;
} rt_solve_params;

/* Report (FP64).  residual = |R_T f - g|, objective = 1/2 residual^2 +
 * lambda1 TV(f) + mu/2 |f|^2, taken at the returned f; rel_change =
 * |f_n - f_{n-1}| / |f_n| at the last monitored iteration (0 if none); tau
 * and sigma are the initial steps (those of the step rule, or the given
 * ones). */
typedef struct {
    double L_R, L_G, tau, sigma, residual, objective, rel_change;
    int32_t iters_done;
} rt_solve_report;

/* The adapted Chambolle-Pock loop of Sec. 3, Fig. 2 with theta = 1:
 *   h1 <- (h1 + sigma (R_T f~ - g)) / (1 + sigma)
 *   h2 <- shrink(h2 + sigma grad_lambda2 S f~, lambda1)
 *   f+ <- (f - tau R_T* h1 + tau S^T div_lambda2 h2) / (1 + mu tau)
 *   f~ <- 2 f+ - f,   f <- f+
 * (RT_CP_ACCEL: f~ and the steps as stated at rt_solve_params)
 * from f = f~ = f (input), h1 = 0, h2 = 0.  Device g, f (in: start, out:
 * result).  Allocates its state on the device for the duration of the call
 * and blocks until the report is ready. */
int solve(const rt_plan *plan, const rt_solve_params *params, const float *g,
          float *f, rt_solve_report *report, void *stream);

/* ---- out-of-core solve --------------------------------------------------
 * The iteration of `solve`, for a volume whose state does not fit on the
 * device.  g and f stay in host memory, and every iteration streams the
 * volume through the device in z-slabs of at most `slab` slices, in
 * increasing z (the slab decomposition of Sec. 7).  Slabs carry one halo
 * slice on either side:
 *   - f~ of the next slab's first slice, not yet updated (z-gradient);
 *   - h2 of the previous slab's last slice, already updated (divergence).
 * Every voxel therefore sees the operands of the in-core iteration, and the
 * iterate is the one `solve` returns, bit for bit.
 * Host g [Ntheta][Nz][Ns] and f [Nz][N][N][K] (in: start, out: result); phi
 * and S as for rt_plan_create.  Plain form (FP32).
 * Memory: pinned host copies of f, g and the state f~, h1, h2, and on the
 * device one slab with its halos plus a plan per slab height.
 * check_every and tol must be 0: there are no per-iteration monitors.  The
 * report's residual and objective are taken at the final f by one more pass.
 * rel_change is 0.  Uses `stream` and blocks until done. */
int rt_solve_ooc(const rt_geom *geom, const double *phi, const double *S,
                 const rt_solve_params *params, const float *g, float *f, int32_t slab,
                 rt_solve_report *report, void *stream);

/* ---- initial guess (Secs. 5-6: the iteration starts from an FBP) ---------
 * q = the projections convolved over the detector with the Shepp-Logan
 * kernel h(n) = -2 / (pi^2 (4 n^2 - 1)) (unit bin spacing; bins outside
 * [0, Ns) count as zero).  Device g, q, both [Ntheta][Nz][Ns]; async on
 * `stream`. */
int rt_fbp_filter(const rt_plan *plan, const float *g, float *q, void *stream);

/* f_out = the FBP initial guess in coefficient form.  Frame m (m < Npi) is
 * the static FBP of half-turn m (Sec. 5): the filtered projections of that
 * half-turn, back-projected with the transpose of the projector and weighted
 * by pi / Ntheta0.  A frame sees the object averaged over its half-turn, so
 * f_out holds the minimum-norm least-squares coefficients of
 *   sum_k B[m][k] f_k = F_m,  B[m][k] = mean of Phi[i][k] over half-turn m,
 * for the plan's basis (FP64 pseudo-inverse on the host; a rank-deficient B
 * is RT_E_ARG).  Device g [Ntheta][Nz][Ns], f_out [Nz][N][N][K].  Needs
 * Npi <= 64.  Allocates (Ntheta Nz Ns + 2 Nz N^2 Npi + Ntheta0 Nz Ns Npi)
 * floats of temporaries for the call and blocks on `stream` before it
 * returns. */
int rt_fbp(const rt_plan *plan, const float *g, float *f_out, void *stream);

/* ---- resumable job/step form of solve, for serving ---------------------
 * A job owns the solver state (f~, h1, h2, work arrays) on the device; the
 * caller still owns g and f.  rt_job_create runs the power iteration (if
 * tau/sigma are not given) on `stream` and blocks for its scalars; it runs
 * on slice 0 alone, since R_T applies the same operator to every slice and
 * its norm is that of the one-slice operator.
 * rt_job_step issues n more iterations on `stream` without blocking (a
 * monitor every check_every iterations blocks for 40 bytes). */
typedef struct rt_job rt_job;

/* Device bytes one job of this geometry needs: plan (tables, scratch, and
 * for RT_FORM_SF the BF16 copy of the volume) + job state.  The caller's g
 * and f are not included. */
int rt_job_bytes(const rt_geom *geom, rt_form form, rt_prec prec, size_t *bytes);
int rt_job_create(const rt_plan *plan, const rt_solve_params *params, const float *g,
                  float *f, void *stream, rt_job **out);
int rt_job_step(rt_job *job, int32_t n, void *stream);
/* 1 when n_iter iterations are done or the tolerance stopped the loop. */
int rt_job_done(const rt_job *job);
int rt_job_iters(const rt_job *job);
/* Fill the report; computes residual and objective at the current f
 * (blocks on `stream`). */
int rt_job_report(rt_job *job, rt_solve_report *report, void *stream);
/* Host checkpoint of the whole iteration state (f, f~, h1, h2, counters,
 * tau, sigma): rt_job_checkpoint_bytes gives the size; both calls block. */
int rt_job_checkpoint_bytes(const rt_job *job, size_t *bytes);
int rt_job_checkpoint(const rt_job *job, void *host_buf, void *stream);
int rt_job_restore(rt_job *job, const void *host_buf, void *stream);
void rt_job_destroy(rt_job *job);

/* ---- FP64 reductions (deterministic order), used by the monitors -------
 * *out = sum_e x[e] * y[e] over n FP32 device values, accumulated in FP64
 * with a fixed tree; blocks on `stream`.  y may equal x. */
int rt_dot(const float *x, const float *y, size_t n, double *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rt_dot with
 * its partial sums in a static device array of the library (2049 doubles per
 * GPU, held until the process ends) instead of a per-call allocation.  Same
 * arguments, result and summation order as rt_dot (bitwise equal).  The
 * array holds the partials of the widest reduction launch (2048 workgroups,
 * whatever n), so no n is too large; a launch that needed more would fail
 * with RT_E_SHAPE.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (different streams or threads) race and must be
 * serialised by the caller.  Blocks on `stream` for the result. */
int rt_dot_noalloc(const float *x, const float *y, size_t n, double *out, void *stream);

/* ---- per-kernel timing --------------------------------------------------
 * When enabled, every kernel launch records a HIP event pair on its stream.
 * rt_timing_read sums the elapsed times of all recorded launches of the
 * named kernel ("k_project", "k_contract", "k_fold", "k_backproject",
 * "k_grad_shrink", "k_div_update", "k_tv_grad", "k_tv_div", "k_shrink", ...)
 * and blocks until they have completed; rt_timing_reset frees the records. */
int rt_timing_enable(int on);
int rt_timing_reset(void);
int rt_timing_read(const char *kernel, double *total_ms, int64_t *launches);

/* ---- measurement aid -----------------------------------------------------
 * The FP32 fused multiply-add issue rate of the device: n_blocks workgroups
 * of 256 threads, each thread 8 independent chains of 16 * n_iter unpacked
 * FMAs, no memory traffic inside the loop.  out: device float[n_blocks * 256]
 * (one value per thread, to keep the chains live).  *ms = elapsed time of the
 * launch between two events on `stream`; *flop = 2 * 8 * 16 * n_iter * 256 *
 * n_blocks.  Blocks until the kernel is done.  Not part of the method. */
int rt_calib_fma(int32_t n_blocks, int32_t n_iter, float *out, double *ms, double *flop,
                 void *stream);

/* Thread-local message of the last error on this thread ("" if none). */
const char *rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RT4D_H */

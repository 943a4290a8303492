// Internal declarations of librt4d: plan and job state, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "rt4d.h"

namespace rt {

// ------------------------------------------------------------------ errors
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
#define RT_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::rt::hip_fail(e_, #call);   \
    } while (0)

// Records HIP events around one kernel launch when timing is enabled
// (rt_timing_enable); construct right before the launch, stop() right after.
class KTimer {
  public:
    KTimer(const char *name, hipStream_t s);
    void stop();
    ~KTimer();

  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_{}, b_{};
    bool live_ = false;
};

// ------------------------------------------------------------- host tables
struct Tables {
    std::vector<double> theta, t;       // [Ntheta]
    std::vector<int32_t> cls, rot, flip;
    std::vector<double> phi;            // [Ntheta][K]
    std::vector<double> S;              // [Nt][K]
    std::vector<double> ccos, csin;     // [Ntheta0] cos/sin of theta0_a
};

// Work layout of the ray-driven projector: classes of one walk direction
// (rows when |cos| >= |sin|, columns otherwise) are grouped A at a time; one
// workgroup owns (group, slice, channel chunk, bin tile).
// Staged lines of the plain projector: KC channels of a position in a row of
// line_stride(KC) floats (an odd number of 16-byte groups, so that 16
// consecutive positions fall in distinct LDS bank groups), LINE_GUARD zero
// positions at each end of a line.
constexpr int LINE_GUARD = 2;
__host__ __device__ constexpr int line_stride(int kc) { return (kc / 4) % 2 ? kc : kc + 4; }

struct FwdCfg {
    int A = 1;            // classes per group
    int ngroups = 0;
    int KC = 4;           // channels per chunk (4, 8, 16)
    int nkc = 1;          // channel chunks
    int BT = 1;           // bins per tile
    int nbt = 1;          // bin tiles
    int stride = 4;       // floats per staged position (KC + padding)
    int nbuf = 2;         // LDS line buffers (1 when two padded lines do not fit)
    bool tl = false;      // two-level ray sums (N > 512)
    int vec = 1;          // 4: float4 staging loads
    int pf = 4;           // float4 per thread that hold one staged line (4 or 8)
    int nth = 512;        // threads per workgroup (1024: 16 waves of 2 rays, KC = 16)
    size_t lds = 0;       // bytes of LDS per workgroup
};

struct AdjCfg {
    int KC = 4, nkc = 1, stride = 4, vec = 1;
    int TQ = 32, TR = 32; // pixel tile
    int CA = 8;           // classes staged per round
    int WMAX = 0;         // bins of the widest staged window
    size_t lds = 0;
};

// Synthesise-first (precision) projector: A classes per group, NPP frame
// columns each (Npi rounded up to 4), A * NPP <= 32 columns in one MFMA tile;
// lines in chunks of PCH positions, CS floats per LDS row; the BF16 shadow of
// f has KP = K rounded up to 16 channels per voxel.
struct SfCfg {
    int A = 1, ngroups = 0, BT = 1, nbt = 1, PCH = 32, CS = 20, NPP = 4, KP = 16;
    int UB = 1;           // bins per thread and class slot (BT = 512 UB covers Ns <= 2048)
    // line parts: with NLP > 1 a workgroup walks N / NLP lines of its slice
    // and stores partial ray sums, which k_sf_finish adds in a fixed order
    // (large slices: the BF16 copy of one part then stays in the last-level
    // cache while every class group of the slice streams it)
    int NLP = 1;
    // B operand staging: 0 = through registers, one step ahead; 3 = global ->
    // LDS copies into a 3-stage ring per wave, two steps ahead (KB = 2)
    int DS = 0;
    size_t lds = 0;
};

struct TvCfg {
    int KT = 8;           // compile-time channel bound (8, 16, 32, 64)
};

struct Plan {
    rt_geom g{};
    rt_form form = RT_FORM_PF;
    rt_prec prec = RT_PREC_FP32;
    int device = 0;
    int n0 = 1;           // Ntheta0 = Ntheta / Npi
    Tables T;
    std::vector<uint8_t> lperm;   // host copy of d_lperm
    FwdCfg fwd;
    AdjCfg adj;
    SfCfg sf;
    TvCfg tv;

    float *d_phi = nullptr;     // [Ntheta][K]
    float *d_S = nullptr;       // [Nt][K]
    double *d_ccos = nullptr;   // [Ntheta0]
    double *d_csin = nullptr;
    int *d_gcls = nullptr;      // [ngroups][A], -1 = empty slot
    int *d_gwalk = nullptr;     // [ngroups]
    uint8_t *d_lperm = nullptr; // [Ntheta0][64] forward lane -> bin offset in its block of 64
    int *d_gcls_sf = nullptr;   // class groups of the synthesise-first projector
    int *d_gwalk_sf = nullptr;
    float *d_scr = nullptr;     // [Ntheta0][Nz][Ns][K]: P (forward), g~ (adjoint)
    float *d_frames = nullptr;  // [Nz][Nt][N][N]: time frames for tv_grad / tv_norm
    double *d_part = nullptr;   // FP64 partial sums
    size_t part_cap = 0;        // doubles in d_part
    double *d_red = nullptr;    // final FP64 sums (16 doubles)
    void *d_f16 = nullptr;      // synthesise-first: BF16 shadow of f, [Nz][N][N][KP]
    float *d_psf = nullptr;     // synthesise-first, NLP > 1: partial ray sums [NLP][Ntheta][Nz][Ns]
    // bumped by every write of d_f16, so that a job knows whether the shadow
    // still holds its own f~
    mutable unsigned long long shadow_gen = 0;
    size_t bytes = 0;
};

struct Job {
    const Plan *plan = nullptr;
    rt_solve_params prm{};
    const float *g = nullptr;
    float *f = nullptr;
    float *ft = nullptr;        // extrapolated primal f~
    float *h1 = nullptr;        // dual of the data term, sinogram shaped
    float *h2 = nullptr;        // dual of the TV term, [Nz][Nt][4][N][N]
    float *Ff = nullptr;        // time frames of f~, [Nz][Nt][N][N]
    float *work = nullptr;      // R_T* h1, coefficient shaped
    float *sino = nullptr;      // R_T f for the report, sinogram shaped
    double tau = 0, sigma = 0, L_R = 0, L_G = 0;
    double tau0 = 0, sigma0 = 0;   // steps of the first iteration (the accelerated form adapts tau, sigma)
    int iters = 0;
    unsigned long long shadow_gen = ~0ull;   // plan shadow_gen when d_f16 last held this f~
    bool stopped = false;
    double residual = 0, objective = 0, rel_change = 0;
    size_t bytes = 0;
};

// ------------------------------------------------------------ sizes/helpers
inline size_t nf_of(const rt_geom &g) { return (size_t)g.Nz * g.N * g.N * g.K; }
inline size_t ng_of(const rt_geom &g) { return (size_t)g.Ntheta * g.Nz * g.Ns; }
inline size_t n4_of(const rt_geom &g) { return (size_t)g.Nz * g.N * g.N * g.Nt; }
size_t job_state_bytes(const rt_geom &g);
size_t plan_scratch_bytes(const rt_geom &g);
size_t shadow_bytes(const rt_geom &g);   // BF16 shadow of f (synthesise-first plans)
int sf_line_parts(const rt_geom &g);     // NLP of a synthesise-first plan
size_t sf_partial_bytes(const rt_geom &g);   // its partial ray sums (0 when NLP = 1)
// FBP initial guess (fbp.hip): the Shepp-Logan filter of the projections, and
// the whole guess (filter, half-turn back-projections, least-squares
// coefficients; blocks on s before it returns)
int launch_fbp_filter(const Plan &p, const float *g, float *q, hipStream_t s);
int fbp_init(const Plan &p, const float *g, float *f, hipStream_t s);

int check_geom(const rt_geom *g);
// checks the form and precision and resolves RT_FORM_AUTO (in place)
int pick_form(const rt_geom *geom, rt_form *form, rt_prec *prec);
int check_plan(const rt_plan *p);

// ---------------------------------------------------------------- launchers
// Projector (proj_pf.hip).  mode of the contraction epilogue:
enum ContractMode { CONTRACT_STORE = 0, CONTRACT_PROX = 1 };
int launch_forward_pf(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                      float *h1, float sigma, double *part, hipStream_t s);
int launch_adjoint_pf(const Plan &p, const float *g, float *out, hipStream_t s);
int forward_partials(const Plan &p);      // workgroups (= FP64 partials) of the h1 prox
int launch_backproject(const Plan &p, float *out, hipStream_t s);   // from g~ in d_scr
// Precision form (proj_sf.hip)
int launch_forward_sf(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                      float *h1, float sigma, double *part, hipStream_t s);   // converts f first
int launch_forward_sf16(const Plan &p, float *g, int mode, const float *gdata, float *h1,
                        float sigma, double *part, hipStream_t s);            // from d_f16
int launch_to_bf16(const Plan &p, const float *f, hipStream_t s);            // f -> d_f16
int launch_fold_mfma(const Plan &p, const float *g, hipStream_t s);
unsigned sf_blocks(const Plan &p);     // projection workgroups (line parts included)
unsigned sf_partials(const Plan &p);   // FP64 partials of the forward's h1 prox
int sf_slots(int npp, int ub, int kb);   // classes per workgroup the kernel is built for
// Dispatch on the plan's form: R_T (with the h1 prox when mode = CONTRACT_PROX) and R_T*
int launch_forward(const Plan &p, const float *f, float *g, int mode, const float *gdata,
                   float *h1, float sigma, double *part, hipStream_t s);
int launch_adjoint(const Plan &p, const float *g, float *out, hipStream_t s);
unsigned voxel_blocks(const rt_geom &g);  // workgroups (= partials) of the voxel kernels

// 4D TV (tv.hip)
int launch_tv_grad(const Plan &p, const float *f, float lambda2, float *pout, hipStream_t s);
int launch_tv_div(const Plan &p, const float *pin, float lambda2, float *out, hipStream_t s);
int launch_shrink(const Plan &p, float *pio, float lambda1, size_t n4, hipStream_t s);
// F = S f (time frames, planar)
int launch_frames(const Plan &p, const float *f, float *F, hipStream_t s);
// The three TV steps below compute slices [zbeg, zend) of the plan's Nz
// (zend < 0: all of them); the other slices only serve as z-neighbours, which
// lets a z-slab with halo slices be processed exactly as inside the volume.
// h2 <- shrink(h2 + sigma grad F), F = S f~; FP64 partial sum of |grad F| per block
int launch_grad_shrink(const Plan &p, const float *Ff, float *h2, float sigma, float lambda1,
                       float lambda2, double *part, hipStream_t s, int zbeg = 0, int zend = -1);
// f+ = (f - tau*adj + tau*S^T div h2) * cinv; f~ = f+ + theta (f+ - f) (the
// plain loop, cinv = theta = 1: f~ = 2 f+ - f); f = f+; Ff = S f~;
// partials |f+ - f|^2, |f+|^2; synthesise-first plans also refresh the BF16
// shadow d_f16 of f~ (and bump shadow_gen)
int launch_div_update(const Plan &p, const float *h2, const float *adj, float *f, float *ft,
                      float *Ff, float tau, float lambda2, double *part, hipStream_t s,
                      int zbeg = 0, int zend = -1, float cinv = 1.f, float theta = 1.f);
// sum over voxels and frames of |grad S f| (FP64 partials)
int launch_tv_norm(const Plan &p, const float *f, float lambda2, double *part, hipStream_t s,
                   int zbeg = 0, int zend = -1);

// Step rule and job buffers of the solver (solve.cpp), shared with the
// out-of-core driver (ooc.cpp)
double plan_s_norm(const Plan &p);
int job_power_iteration(Job &J, hipStream_t s);
int job_alloc(Job &J);
void job_free(Job &J);
int solve_params_check(const rt_solve_params *prm);
// Steps of the accelerated form after an iteration taken with tau, sigma:
// theta = 1 / sqrt(1 + 2 mu tau), tau <- theta tau, sigma <- sigma / theta
// (theta = 1 for the plain loop).  Returns theta; cinv = 1 / (1 + mu tau) of
// that iteration's primal prox.
double cp_steps(const rt_solve_params &P, double *tau, double *sigma, double *cinv);

// Reductions and vector helpers (reduce.hip)
int reduce_blocks(int nblocks_hint, size_t n);
int launch_dot_partials(const float *x, const float *y, size_t n, double *part, int nblocks,
                        hipStream_t s);
int launch_diff_sq_partials(const float *x, const float *y, size_t n, double *part, int nblocks,
                            hipStream_t s);
// out[j] = sum over i < nb of part[i*stride + j], j < width (fixed order)
int launch_finish(const double *part, int nb, int width, double *out, hipStream_t s);
int launch_fill(float *x, float v, size_t n, hipStream_t s);
int launch_scale(float *x, const double *num_den, size_t n, hipStream_t s);
int launch_copy(float *dst, const float *src, size_t n, hipStream_t s);
int launch_seeded_uniform(float *x, size_t n, uint64_t seed, hipStream_t s);

}  // namespace rt

struct rt_plan {
    rt::Plan impl;
};
struct rt_job {
    rt::Job impl;
};

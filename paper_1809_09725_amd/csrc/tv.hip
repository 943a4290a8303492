// 4D total variation of the paper's penalty (Sec. 2, eq. TV1) on Nt time
// frames F_m = sum_k S[m][k] f_k, and the steps of Fig. 2 that use it.
//
//   grad:  p_m = (dx F_m, dy F_m, dz F_m, lambda2 (F_{m+1} - F_m)), forward
//          differences that are zero at the last index of each axis
//   div:   S^T div p, div = -grad^T: backward differences with the boundary
//          rows of the discrete TV literature, lambda2 on the time axis
//   shrink the prox of sigma F2* (Sec. 3): p / max(1, |p|_2 / lambda1)
//
// Layouts: f is [Nz][N][N][K] (basis index innermost, as the projector wants
// it); the frames F [Nz][Nt][N][N] and the dual p [Nz][Nt][4][N][N] are
// component planes, so one thread per voxel reads and writes whole coalesced
// rows.  The K-innermost rows of f go through LDS: a workgroup of 256
// consecutive voxels loads (or stores) its 256*K values as contiguous float4,
// and each thread works on its own voxel from LDS.  All kernels here are
// bound by HBM bandwidth.
#include "common.h"
#include "internal.h"

namespace rt {
namespace {

constexpr int ZC = 4;   // consecutive slices per work item of the gradient and divergence

// LDS row stride (floats) of one voxel's K values: odd, so that 32
// consecutive voxels read with ds_read_b32 hit 32 different banks.
__host__ __device__ constexpr int kstride(int KT) { return KT + 1; }

// The arithmetic of one voxel and frame (explicit fmaf throughout: no
// contraction choice is left to the compiler, so every kernel that takes a
// step rounds it alike).
//
// Dual TV step: a = h + sigma g, h <- a / max(1, |a|_2 / lambda1), as
// a * min(1, lambda1 / |a|_2) with the hardware reciprocal square root
// (about 1 ulp; |a|^2 is held at or above the smallest normal float).
__device__ inline float4 shrink_step(float4 h, float gx, float gy, float gz, float gt, float sigma,
                                     float lambda1)
{
    const float ax = fmaf(sigma, gx, h.x);
    const float ay = fmaf(sigma, gy, h.y);
    const float az = fmaf(sigma, gz, h.z);
    const float at = fmaf(sigma, gt, h.w);
    const float n2 = fmaf(at, at, fmaf(az, az, fmaf(ay, ay, ax * ax)));
    const float sc = lambda1 <= 0.f
                         ? 0.f
                         : fminf(1.f, lambda1 * __builtin_amdgcn_rsqf(fmaxf(n2, 1.17549435e-38f)));
    return make_float4(ax * sc, ay * sc, az * sc, at * sc);
}

// Backward-difference divergence of one voxel and frame from the dual's
// components at the voxel (xc, yc, zc, tc) and at its lower neighbours (xp,
// yp, zp, tp); absent terms are passed as 0 (the boundary rows of div =
// -grad^T); the z pair only counts when the volume has more than one slice.
__device__ inline float div_step(float xc, float xp, float yc, float yp, bool zax, float zc,
                                 float zp, float tc, float tp, float lambda2)
{
    float d = xc - xp;
    d += yc - yp;
    if (zax) d += zc - zp;
    return fmaf(lambda2, tc - tp, d);
}

// Primal step and extrapolation of one coefficient: sdiv = (S^T div h2)_k.
__device__ inline void primal_step(float fo, float adj, float sdiv, float tau, float cinv,
                                   float theta, int accel, float &fnw, float &fx)
{
    fnw = fmaf(tau, sdiv, fmaf(-tau, adj, fo));
    if (accel) {
        fnw *= cinv;
        fx = fmaf(theta, fnw - fo, fnw);
    } else {
        fx = fmaf(2.f, fnw, -fo);
    }
}

// Cooperative copy of voxels [v0, v0 + nv) x K floats from global
// (contiguous) to LDS rows of stride KS.
template <int KT>
__device__ inline void f_to_lds(const float *__restrict__ src, size_t v0, int nv, int K,
                                float *__restrict__ lds)
{
    constexpr int KS = kstride(KT);
    const float *base = src + v0 * K;
    const int n = nv * K;
    if ((K & 3) == 0) {
        for (int e = threadIdx.x * 4; e < n; e += NT * 4) {
            const float4 x = *(const float4 *)(base + e);
            const int v = e / K, k = e % K;
            float *d = lds + v * KS + k;
            d[0] = x.x; d[1] = x.y; d[2] = x.z; d[3] = x.w;
        }
    } else {
        for (int e = threadIdx.x; e < n; e += NT) lds[(e / K) * KS + e % K] = base[e];
    }
}

template <int KT>
__device__ inline void lds_to_f(const float *__restrict__ lds, size_t v0, int nv, int K,
                                float *__restrict__ dst)
{
    constexpr int KS = kstride(KT);
    float *base = dst + v0 * K;
    const int n = nv * K;
    if ((K & 3) == 0) {
        for (int e = threadIdx.x * 4; e < n; e += NT * 4) {
            const int v = e / K, k = e % K;
            const float *s = lds + v * KS + k;
            *(float4 *)(base + e) = make_float4(s[0], s[1], s[2], s[3]);
        }
    } else {
        for (int e = threadIdx.x; e < n; e += NT) base[e] = lds[(e / K) * KS + e % K];
    }
}

// S into LDS as [Nt][KT], zero padded.
template <int KT>
__device__ inline void stage_S(const float *__restrict__ S, int K, int Nt, float *sS)
{
    for (int e = threadIdx.x; e < Nt * KT; e += NT) {
        const int m = e / KT, k = e % KT;
        sS[e] = k < K ? S[m * K + k] : 0.f;
    }
}

// F[z][m][pv] = sum_k S[m][k] f_k(v) from the LDS row of voxel v.
template <int KT>
__device__ inline void write_frames(const float *__restrict__ row, const float *__restrict__ sS,
                                    float *__restrict__ F, size_t v, size_t plane, int Nt, int K)
{
    float c[KT];   // channels K..KT-1 of the LDS row are padding, never written
#pragma unroll
    for (int k = 0; k < KT; ++k) c[k] = k < K ? row[k] : 0.f;
    const size_t z = v / plane, pv = v % plane;
    float *Fz = F + z * Nt * plane + pv;
    for (int m = 0; m < Nt; ++m) {
        const float *Sm = sS + m * KT;
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < KT; ++k) s = fmaf(Sm[k], c[k], s);
        __builtin_nontemporal_store(s, Fz + (size_t)m * plane);   // read next by the gradient
    }
}

// Frames of f: F = S f, planar.
template <int KT>
__global__ __launch_bounds__(NT) void k_frames(const float *__restrict__ f,
                                               const float *__restrict__ S,
                                               float *__restrict__ F, int N, int Nz, int K, int Nt)
{
    extern __shared__ float sm[];
    float *sS = sm;                          // [Nt][KT]
    float *rows = sm + Nt * KT;              // [NT][KS]
    stage_S<KT>(S, K, Nt, sS);
    const size_t plane = (size_t)N * N, nvox = plane * Nz;
    for (size_t v0 = (size_t)blockIdx.x * NT; v0 < nvox; v0 += (size_t)gridDim.x * NT) {
        const int nv = (int)std::min<size_t>(NT, nvox - v0);
        __syncthreads();
        f_to_lds<KT>(f, v0, nv, K, rows);
        __syncthreads();
        if ((int)threadIdx.x < nv)
            write_frames<KT>(rows + threadIdx.x * kstride(KT), sS, F, v0 + threadIdx.x, plane, Nt, K);
    }
}

// MODE 0: p = grad F (store).  MODE 1: h2 <- shrink(h2 + sigma grad F).
// MODE 2: no store.  With part != NULL each workgroup writes the FP64 sum of
// |grad F| over its voxels and frames.  Slices [zbeg, zend) of the Nz present
// are computed (and summed); the others only serve as z-neighbours.
template <int MODE>
__global__ __launch_bounds__(NT) void k_grad(const float *__restrict__ F, float lambda2,
                                             float sigma, float lambda1, float *__restrict__ p,
                                             double *__restrict__ part, int N, int Nz, int Nt,
                                             int zbeg, int zend, int carry)
{
    __shared__ double sh[NT / 64];
    // carry != 0: sFn[m][thread] holds the frames of slice z+1 at the
    // thread's pixel, read as z-neighbours, so the next slice of the work item
    // takes its own frames from LDS instead of reading them again
    extern __shared__ float sFn[];   // [Nt][NT] when carry
    const size_t plane = (size_t)N * N;
    const size_t nitem = plane * ((zend - zbeg + ZC - 1) / ZC);
    double tvs = 0.0;
    float *cf = sFn + threadIdx.x;
    // a work item is one (row, column) over ZC consecutive slices; the
    // workgroups of a plane's rows y and y+1 share an XCD's L2 (xcd_remap)
    const size_t lid = xcd_remap(blockIdx.x, gridDim.x);
    for (size_t it = lid * NT + threadIdx.x; it < nitem; it += (size_t)gridDim.x * NT)
    for (int z0 = zbeg + (int)(it / plane) * ZC, z = z0, ze = min(zend, z + ZC); z < ze; ++z) {
        const size_t pv = it % plane;
        const int q = (int)(pv % N);
        const int r = (int)(pv / N);
        const bool hx = q < N - 1, hy = r < N - 1, hz = z < Nz - 1;
        const bool own = carry && z > z0;   // this slice's frames are in LDS
        const float *Fz = F + (size_t)z * Nt * plane + pv;
        float *pz = (MODE != 2) ? p + (size_t)z * Nt * 4 * plane + pv : nullptr;
        float F0 = own ? cf[0] : Fz[0];
        for (int m = 0; m < Nt; ++m) {
            const float *Fm = Fz + (size_t)m * plane;
            const float gx = hx ? Fm[1] - F0 : 0.f;
            const float gy = hy ? Fm[N] - F0 : 0.f;
            const float Fzn = hz ? Fm[(size_t)Nt * plane] : 0.f;
            const float gz = hz ? Fzn - F0 : 0.f;
            float gt = 0.f, F1 = 0.f;
            if (m < Nt - 1) {
                F1 = own ? cf[(m + 1) * NT] : Fm[plane];
                gt = lambda2 * (F1 - F0);
            }
            if (carry) cf[m * NT] = Fzn;   // frame m of slice z+1 (entry m was last read above)
            if (part) tvs += sqrt((double)gx * gx + (double)gy * gy + (double)gz * gz + (double)gt * gt);
            if (MODE == 0) {
                float *pm = pz + (size_t)m * 4 * plane;
                pm[0] = gx;
                pm[plane] = gy;
                pm[2 * plane] = gz;
                pm[3 * plane] = gt;
            } else if (MODE == 1) {
                float *pm = pz + (size_t)m * 4 * plane;
                // h2 of this voxel is read and written once here and next read
                // after the back-projection has streamed through L2: streaming
                // (non-temporal) accesses leave L2 to the frames' neighbour reads
                const float4 h = make_float4(__builtin_nontemporal_load(pm),
                                             __builtin_nontemporal_load(pm + plane),
                                             __builtin_nontemporal_load(pm + 2 * plane),
                                             __builtin_nontemporal_load(pm + 3 * plane));
                const float4 a = shrink_step(h, gx, gy, gz, gt, sigma, lambda1);
                __builtin_nontemporal_store(a.x, pm);
                __builtin_nontemporal_store(a.y, pm + plane);
                __builtin_nontemporal_store(a.z, pm + 2 * plane);
                __builtin_nontemporal_store(a.w, pm + 3 * plane);
            }
            F0 = F1;
        }
    }
    if (part) {
        const double s = block_sum(tvs, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

// MODE 0: out = S^T div p.  MODE 1 (Fig. 2 steps 5-6):
//   f+ = f - tau adj + tau S^T div h2;  f~ = 2 f+ - f;  f = f+;  Ff = S f~
// with FP64 partials |f+ - f|^2 and |f+|^2 per workgroup when part != NULL.
// With a uniformly convex term mu/2 |f|^2 (accel != 0) the primal step is its
// prox, f+ = (f - tau adj + tau S^T div h2) * cinv, cinv = 1 / (1 + mu tau),
// and the extrapolation takes the step's theta: f~ = f+ + theta (f+ - f).
// Slices [zbeg, zend) of the Nz present are computed; the others only serve
// as z-neighbours.
template <int KT, int MODE>
__global__ __launch_bounds__(NT) void k_div(const float *__restrict__ pin,
                                            const float *__restrict__ S, float lambda2,
                                            float *__restrict__ out, const float *__restrict__ adj,
                                            float *__restrict__ ft, float *__restrict__ Ff,
                                            float tau, float cinv, float theta, int accel,
                                            double *__restrict__ part,
                                            __bf16 *__restrict__ f16, int KP, int N, int Nz,
                                            int K, int Nt, int zbeg, int zend)
{
    constexpr int KS = kstride(KT);
    extern __shared__ float sm[];
    float *sS = sm;                          // [Nt][KT]
    float *rows = sm + Nt * KT;              // [NT][KS]
    __shared__ double sh[NT / 64];
    stage_S<KT>(S, K, Nt, sS);
    const size_t plane = (size_t)N * N;
    const size_t ntile = (plane + NT - 1) / NT;
    const size_t ntask = ntile * ((zend - zbeg + ZC - 1) / ZC);
    double dn2 = 0.0, fn2 = 0.0;
    // a task is NT consecutive voxels of a plane over ZC consecutive slices
    // (the z-neighbour plane of h2 is then still in L2)
    for (size_t task = blockIdx.x; task < ntask; task += gridDim.x)
    for (int zz = zbeg + (int)(task / ntile) * ZC, ze = min(zend, zz + ZC); zz < ze; ++zz) {
        const size_t pv0 = (task % ntile) * NT;
        const size_t v0 = (size_t)zz * plane + pv0;
        const int nv = (int)std::min<size_t>(NT, plane - pv0);
        const size_t v = v0 + threadIdx.x;
        __syncthreads();   // S staged; the previous chunk is done with rows
        if ((int)threadIdx.x < nv) {
            const int q = (int)(v % N);
            const int r = (int)((v / N) % N);
            const size_t z = v / plane, pv = v % plane;
            const float *pz = pin + z * Nt * 4 * plane + pv;
            float acc[KT];
#pragma unroll
            for (int k = 0; k < KT; ++k) acc[k] = 0.f;
            float tprev = 0.f;
            for (int m = 0; m < Nt; ++m) {
                const float *pm = pz + (size_t)m * 4 * plane;
                const float tcur = m < Nt - 1 ? pm[3 * plane] : 0.f;
                const float d = div_step(
                    q < N - 1 ? pm[0] : 0.f, q > 0 ? pm[-1] : 0.f,
                    r < N - 1 ? pm[plane] : 0.f, r > 0 ? pm[plane - N] : 0.f, Nz > 1,
                    (int)z < Nz - 1 ? pm[2 * plane] : 0.f,
                    z > 0 ? *(pm + 2 * plane - (size_t)Nt * 4 * plane) : 0.f, tcur, tprev, lambda2);
                tprev = tcur;
                const float *Sm = sS + m * KT;
#pragma unroll
                for (int k = 0; k < KT; ++k) acc[k] = fmaf(Sm[k], d, acc[k]);
            }
            float *row = rows + threadIdx.x * KS;
#pragma unroll
            for (int k = 0; k < KT; ++k) row[k] = acc[k];
        }
        __syncthreads();
        if (MODE == 0) {
            lds_to_f<KT>(rows, v0, nv, K, out);
        } else {
            // element e of the chunk: voxel e / K, channel e % K, contiguous in f
            float *fb = out + v0 * K;
            const float *ab = adj + v0 * K;
            float *tb = ft + v0 * K;
            const int n = nv * K;
            for (int e = threadIdx.x; e < n; e += NT) {
                float *slot = rows + (e / K) * KS + e % K;
                // f, R*h1 and f~ are touched once per iteration: streaming accesses
                const float fo = __builtin_nontemporal_load(fb + e);
                float fnw, fx;
                primal_step(fo, __builtin_nontemporal_load(ab + e), slot[0], tau, cinv, theta, accel,
                            fnw, fx);
                const float dd = fnw - fo;
                if (part) {
                    dn2 += (double)dd * dd;
                    fn2 += (double)fnw * fnw;
                }
                __builtin_nontemporal_store(fnw, fb + e);
                __builtin_nontemporal_store(fx, tb + e);
                slot[0] = fx;
            }
            __syncthreads();
            if ((int)threadIdx.x < nv)
                write_frames<KT>(rows + threadIdx.x * KS, sS, Ff, v, plane, Nt, K);
            if (f16) {   // BF16 shadow of f~ for the synthesise-first projector
                const int n8 = KP / 8;
                for (int e = threadIdx.x; e < nv * n8; e += NT) {
                    const int vl = e / n8, k0 = (e % n8) * 8;
                    const float *row = rows + vl * KS;
                    typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
                    v8bf o;
#pragma unroll
                    for (int q = 0; q < 8; ++q) o[q] = (__bf16)(k0 + q < K ? row[k0 + q] : 0.f);
                    *(v8bf *)(f16 + (v0 + vl) * KP + k0) = o;
                }
            }
        }
    }
    if (MODE == 1 && part) {
        const double a = block_sum(dn2, sh);
        const double b = block_sum(fn2, sh);
        if (threadIdx.x == 0) {
            part[2 * blockIdx.x] = a;
            part[2 * blockIdx.x + 1] = b;
        }
    }
}

__global__ __launch_bounds__(NT) void k_shrink(float *__restrict__ p, float lambda1, size_t plane,
                                               size_t nzt)
{
    // p is [nzt = Nz*Nt][4][plane]
    const size_t n = nzt * plane;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT) {
        float *b = p + (e / plane) * 4 * plane + e % plane;
        const float x = b[0], y = b[plane], z = b[2 * plane], w = b[3 * plane];
        const float nrm = sqrtf(x * x + y * y + z * z + w * w);
        const float sc = lambda1 <= 0.f ? 0.f : (nrm > lambda1 ? lambda1 / nrm : 1.f);
        b[0] = x * sc;
        b[plane] = y * sc;
        b[2 * plane] = z * sc;
        b[3 * plane] = w * sc;
    }
}

size_t tv_lds(const Plan &p)
{
    return ((size_t)p.g.Nt * p.tv.KT + (size_t)NT * kstride(p.tv.KT)) * sizeof(float);
}

}  // namespace

unsigned voxel_blocks(const rt_geom &g)
{
    const size_t nvox = (size_t)g.Nz * g.N * g.N;
    return (unsigned)std::max<size_t>(1, std::min<size_t>((nvox + NT - 1) / NT, 8192));
}

int launch_frames(const Plan &p, const float *f, float *F, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    const unsigned nb = voxel_blocks(p.g);
    const size_t lds = tv_lds(p);
    const rt_geom &g = p.g;
    KTimer kt("k_frames", s);
    switch (p.tv.KT) {
    case 8: hipLaunchKernelGGL(k_frames<8>, dim3(nb), dim3(NT), lds, s, f, p.d_S, F, g.N, g.Nz, g.K, g.Nt); break;
    case 16: hipLaunchKernelGGL(k_frames<16>, dim3(nb), dim3(NT), lds, s, f, p.d_S, F, g.N, g.Nz, g.K, g.Nt); break;
    case 32: hipLaunchKernelGGL(k_frames<32>, dim3(nb), dim3(NT), lds, s, f, p.d_S, F, g.N, g.Nz, g.K, g.Nt); break;
    default: hipLaunchKernelGGL(k_frames<64>, dim3(nb), dim3(NT), lds, s, f, p.d_S, F, g.N, g.Nz, g.K, g.Nt); break;
    }
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

// LDS of the gradient's slice-to-slice carry: one float per frame and
// thread, when it fits a modest budget (else the kernel reads again)
static size_t carry_lds(const rt_geom &g)
{
    const size_t b = (size_t)g.Nt * NT * sizeof(float);
    return b <= 32 * 1024 ? b : 0;
}

static int launch_grad_mode(const Plan &p, int mode, const char *name, const float *F, float *pout,
                            float sigma, float lambda1, float lambda2, double *part, hipStream_t s,
                            int zbeg = 0, int zend = -1)
{
    if (zend < 0) zend = p.g.Nz;
    if (zend <= zbeg) return RT_OK;
    const unsigned nb = voxel_blocks(p.g);
    const rt_geom &g = p.g;
    const size_t lds = carry_lds(g);
    const int carry = lds > 0;
    KTimer kt(name, s);
    if (mode == 0)
        hipLaunchKernelGGL(k_grad<0>, dim3(nb), dim3(NT), lds, s, F, lambda2, sigma, lambda1, pout, part, g.N, g.Nz, g.Nt, zbeg, zend, carry);
    else if (mode == 1)
        hipLaunchKernelGGL(k_grad<1>, dim3(nb), dim3(NT), lds, s, F, lambda2, sigma, lambda1, pout, part, g.N, g.Nz, g.Nt, zbeg, zend, carry);
    else
        hipLaunchKernelGGL(k_grad<2>, dim3(nb), dim3(NT), lds, s, F, lambda2, sigma, lambda1, pout, part, g.N, g.Nz, g.Nt, zbeg, zend, carry);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_tv_grad(const Plan &p, const float *f, float lambda2, float *pout, hipStream_t s)
{
    int rc = launch_frames(p, f, p.d_frames, s);
    if (rc) return rc;
    return launch_grad_mode(p, 0, "k_tv_grad", p.d_frames, pout, 0.f, 0.f, lambda2, nullptr, s);
}

int launch_grad_shrink(const Plan &p, const float *Ff, float *h2, float sigma, float lambda1,
                       float lambda2, double *part, hipStream_t s, int zbeg, int zend)
{
    return launch_grad_mode(p, 1, "k_grad_shrink", Ff, h2, sigma, lambda1, lambda2, part, s, zbeg,
                            zend);
}

int launch_tv_norm(const Plan &p, const float *f, float lambda2, double *part, hipStream_t s,
                   int zbeg, int zend)
{
    int rc = launch_frames(p, f, p.d_frames, s);
    if (rc) return rc;
    return launch_grad_mode(p, 2, "k_tv_norm", p.d_frames, nullptr, 0.f, 0.f, lambda2, part, s,
                            zbeg, zend);
}

template <int MODE>
static void launch_div_t(const Plan &p, const float *pin, float lambda2, float *out,
                         const float *adj, float *ft, float *Ff, float tau, float cinv,
                         float theta, double *part, __bf16 *f16, hipStream_t s, int zbeg, int zend)
{
    const unsigned nb = voxel_blocks(p.g);
    const size_t lds = tv_lds(p);
    const rt_geom &g = p.g;
    const int KP = p.sf.KP;
    const int accel = cinv != 1.f || theta != 1.f;
#define RT_DIV(KT) hipLaunchKernelGGL((k_div<KT, MODE>), dim3(nb), dim3(NT), lds, s, pin, p.d_S, \
                                      lambda2, out, adj, ft, Ff, tau, cinv, theta, accel, part,   \
                                      f16, KP, g.N, g.Nz, g.K, g.Nt, zbeg, zend)
    switch (p.tv.KT) {
    case 8: RT_DIV(8); break;
    case 16: RT_DIV(16); break;
    case 32: RT_DIV(32); break;
    default: RT_DIV(64); break;
    }
#undef RT_DIV
}

int launch_tv_div(const Plan &p, const float *pin, float lambda2, float *out, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    KTimer kt("k_tv_div", s);
    launch_div_t<0>(p, pin, lambda2, out, nullptr, nullptr, nullptr, 0.f, 1.f, 1.f, nullptr, nullptr,
                    s, 0, p.g.Nz);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_div_update(const Plan &p, const float *h2, const float *adj, float *f, float *ft,
                      float *Ff, float tau, float lambda2, double *part, hipStream_t s, int zbeg,
                      int zend, float cinv, float theta)
{
    if (zend < 0) zend = p.g.Nz;
    if (zend <= zbeg) return RT_OK;
    KTimer kt("k_div_update", s);
    __bf16 *f16 = p.form == RT_FORM_SF ? (__bf16 *)p.d_f16 : nullptr;
    launch_div_t<1>(p, h2, lambda2, f, adj, ft, Ff, tau, cinv, theta, part, f16, s, zbeg, zend);
    kt.stop();
    RT_HIP(hipGetLastError());
    if (f16) ++p.shadow_gen;
    return RT_OK;
}

int launch_shrink(const Plan &p, float *pio, float lambda1, size_t n4, hipStream_t s)
{
    if (n4 == 0) return RT_OK;
    const size_t plane = (size_t)p.g.N * p.g.N;
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((n4 + NT - 1) / NT, 8192));
    KTimer kt("k_shrink", s);
    hipLaunchKernelGGL(k_shrink, dim3(nb), dim3(NT), 0, s, pio, lambda1, plane, n4 / plane);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rt

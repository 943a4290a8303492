// 4D total variation of the paper's penalty (Sec. 2, eq. TV1) on Nt time
// frames F_m = sum_k S[m][k] f_k, and the steps of Fig. 2 that use it.
//
//   grad:  p_m = (dx F_m, dy F_m, dz F_m, lambda2 (F_{m+1} - F_m)), forward
//          differences that are zero at the last index of each axis
//   div:   S^T div p, div = -grad^T: backward differences with the boundary
//          rows of the discrete TV literature, lambda2 on the time axis
//   shrink the prox of sigma F2* (Sec. 3): p / max(1, |p|_2 / lambda1)
//
// One thread per voxel; the K coefficients of a voxel are 4*K contiguous
// bytes, its Nt*4 dual values 16*Nt contiguous bytes, so every access is a
// coalesced row of the volume.  These kernels are bound by HBM bandwidth.
#include "common.h"
#include "internal.h"

namespace rt {
namespace {

template <int KT>
__device__ inline void load_k(const float *__restrict__ src, int K, float (&c)[KT])
{
    if ((K & 3) == 0) {
#pragma unroll
        for (int k = 0; k < KT; k += 4) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (k < K) v = *(const float4 *)(src + k);
            c[k] = v.x; c[k + 1] = v.y; c[k + 2] = v.z; c[k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < KT; ++k) c[k] = k < K ? src[k] : 0.f;
    }
}

template <int KT>
__device__ inline void store_k(float *__restrict__ dst, int K, const float (&c)[KT])
{
    if ((K & 3) == 0) {
#pragma unroll
        for (int k = 0; k < KT; k += 4)
            if (k < K) *(float4 *)(dst + k) = make_float4(c[k], c[k + 1], c[k + 2], c[k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < KT; ++k)
            if (k < K) dst[k] = c[k];
    }
}

template <int KT>
__device__ inline float frame(const float *__restrict__ Srow, const float (&c)[KT])
{
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k) s = fmaf(Srow[k], c[k], s);
    return s;
}

// S into LDS as [Nt][KT], zero padded.
template <int KT>
__device__ inline void stage_S(const float *__restrict__ S, int K, int Nt, float *sS)
{
    for (int e = threadIdx.x; e < Nt * KT; e += NT) {
        const int m = e / KT, k = e % KT;
        sS[e] = k < K ? S[m * K + k] : 0.f;
    }
    __syncthreads();
}

// MODE 0: p = grad f~ (store).  MODE 1: h2 <- shrink(h2 + sigma grad f~).
// MODE 2: only the partial sum of |grad f| (no store).
// With part != NULL each workgroup writes the FP64 sum of |grad f~| over its voxels.
template <int KT, int MODE>
__global__ __launch_bounds__(NT) void k_grad(const float *__restrict__ f,
                                             const float *__restrict__ S, float lambda2,
                                             float sigma, float lambda1, float *__restrict__ p,
                                             double *__restrict__ part, int N, int Nz, int K,
                                             int Nt)
{
    extern __shared__ float sS[];
    __shared__ double sh[NT / 64];
    stage_S<KT>(S, K, Nt, sS);
    const size_t nvox = (size_t)Nz * N * N;
    const size_t plane = (size_t)N * N;
    double tvs = 0.0;
    for (size_t v = (size_t)blockIdx.x * NT + threadIdx.x; v < nvox; v += (size_t)gridDim.x * NT) {
        const int q = (int)(v % N);
        const int r = (int)((v / N) % N);
        const int z = (int)(v / plane);
        float c0[KT], cx[KT], cy[KT], cz[KT];
        load_k<KT>(f + v * K, K, c0);
        const bool hx = q < N - 1, hy = r < N - 1, hz = z < Nz - 1;
        if (hx) load_k<KT>(f + (v + 1) * K, K, cx);
        if (hy) load_k<KT>(f + (v + N) * K, K, cy);
        if (hz) load_k<KT>(f + (v + plane) * K, K, cz);
        float F0 = frame<KT>(sS, c0);
        for (int m = 0; m < Nt; ++m) {
            const float *Sm = sS + m * KT;
            const float px = hx ? frame<KT>(Sm, cx) - F0 : 0.f;
            const float py = hy ? frame<KT>(Sm, cy) - F0 : 0.f;
            const float pz = hz ? frame<KT>(Sm, cz) - F0 : 0.f;
            float pt = 0.f, F1 = 0.f;
            if (m < Nt - 1) {
                F1 = frame<KT>(Sm + KT, c0);
                pt = lambda2 * (F1 - F0);
            }
            if (part) tvs += sqrt((double)px * px + (double)py * py + (double)pz * pz + (double)pt * pt);
            float4 *dst = (float4 *)(p + (v * Nt + m) * 4);
            if (MODE == 0) {
                *dst = make_float4(px, py, pz, pt);
            } else if (MODE == 1) {
                float4 h = *dst;
                h.x = fmaf(sigma, px, h.x);
                h.y = fmaf(sigma, py, h.y);
                h.z = fmaf(sigma, pz, h.z);
                h.w = fmaf(sigma, pt, h.w);
                const float nrm = sqrtf(h.x * h.x + h.y * h.y + h.z * h.z + h.w * h.w);
                const float sc = lambda1 <= 0.f ? 0.f : (nrm > lambda1 ? lambda1 / nrm : 1.f);
                *dst = make_float4(h.x * sc, h.y * sc, h.z * sc, h.w * sc);
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
//   f+ = f - tau adj + tau S^T div h2;  f~ = 2 f+ - f;  f = f+
// with FP64 partials |f+ - f|^2 and |f+|^2 per workgroup (2 per block).
template <int KT, int MODE>
__global__ __launch_bounds__(NT) void k_div(const float *__restrict__ pin,
                                            const float *__restrict__ S, float lambda2,
                                            float *__restrict__ out, const float *__restrict__ adj,
                                            float *__restrict__ ft, float tau,
                                            double *__restrict__ part, int N, int Nz, int K, int Nt)
{
    extern __shared__ float sS[];
    __shared__ double sh[NT / 64];
    stage_S<KT>(S, K, Nt, sS);
    const size_t nvox = (size_t)Nz * N * N;
    const size_t plane = (size_t)N * N;
    double dn2 = 0.0, fn2 = 0.0;
    for (size_t v = (size_t)blockIdx.x * NT + threadIdx.x; v < nvox; v += (size_t)gridDim.x * NT) {
        const int q = (int)(v % N);
        const int r = (int)((v / N) % N);
        const int z = (int)(v / plane);
        float acc[KT];
#pragma unroll
        for (int k = 0; k < KT; ++k) acc[k] = 0.f;
        const float *pv = pin + v * Nt * 4;
        const float *px = pin + (q > 0 ? v - 1 : v) * Nt * 4;       // read only when q > 0
        const float *py = pin + (r > 0 ? v - N : v) * Nt * 4;       // r > 0
        const float *pz = pin + (z > 0 ? v - plane : v) * Nt * 4;   // z > 0
        for (int m = 0; m < Nt; ++m) {
            const float4 c = *(const float4 *)(pv + m * 4);
            float d = (q < N - 1 ? c.x : 0.f) - (q > 0 ? px[m * 4 + 0] : 0.f);
            d += (r < N - 1 ? c.y : 0.f) - (r > 0 ? py[m * 4 + 1] : 0.f);
            d += (z < Nz - 1 ? c.z : 0.f) - (z > 0 ? pz[m * 4 + 2] : 0.f);
            d += lambda2 * ((m < Nt - 1 ? c.w : 0.f) - (m > 0 ? pv[(m - 1) * 4 + 3] : 0.f));
            const float *Sm = sS + m * KT;
#pragma unroll
            for (int k = 0; k < KT; ++k) acc[k] = fmaf(Sm[k], d, acc[k]);
        }
        if (MODE == 0) {
            store_k<KT>(out + v * K, K, acc);
        } else {
            float fo[KT], ad[KT], fnw[KT], fext[KT];
            load_k<KT>(out + v * K, K, fo);
            load_k<KT>(adj + v * K, K, ad);
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                fnw[k] = fo[k] - tau * ad[k] + tau * acc[k];
                const float dd = fnw[k] - fo[k];
                fext[k] = 2.f * fnw[k] - fo[k];
                if (k < K) {
                    dn2 += (double)dd * dd;
                    fn2 += (double)fnw[k] * fnw[k];
                }
            }
            store_k<KT>(out + v * K, K, fnw);
            store_k<KT>(ft + v * K, K, fext);
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

__global__ __launch_bounds__(NT) void k_shrink(float *__restrict__ p, float lambda1, size_t n4)
{
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n4; e += (size_t)gridDim.x * NT) {
        float4 h = *(float4 *)(p + e * 4);
        const float nrm = sqrtf(h.x * h.x + h.y * h.y + h.z * h.z + h.w * h.w);
        const float sc = lambda1 <= 0.f ? 0.f : (nrm > lambda1 ? lambda1 / nrm : 1.f);
        *(float4 *)(p + e * 4) = make_float4(h.x * sc, h.y * sc, h.z * sc, h.w * sc);
    }
}

}  // namespace

unsigned voxel_blocks(const rt_geom &g)
{
    const size_t nvox = (size_t)g.Nz * g.N * g.N;
    return (unsigned)std::max<size_t>(1, std::min<size_t>((nvox + NT - 1) / NT, 8192));
}

#define RT_TV_DISPATCH(NAME, KERNEL, MODE, ...)                                                   \
    do {                                                                                          \
        const unsigned nb_ = voxel_blocks(p.g);                                                   \
        KTimer kt_(NAME, s);                                                                      \
        const size_t sm_ = (size_t)p.g.Nt * p.tv.KT * sizeof(float);                              \
        switch (p.tv.KT) {                                                                        \
        case 8: hipLaunchKernelGGL((KERNEL<8, MODE>), dim3(nb_), dim3(NT), sm_, s, __VA_ARGS__); break;   \
        case 16: hipLaunchKernelGGL((KERNEL<16, MODE>), dim3(nb_), dim3(NT), sm_, s, __VA_ARGS__); break; \
        case 32: hipLaunchKernelGGL((KERNEL<32, MODE>), dim3(nb_), dim3(NT), sm_, s, __VA_ARGS__); break; \
        default: hipLaunchKernelGGL((KERNEL<64, MODE>), dim3(nb_), dim3(NT), sm_, s, __VA_ARGS__); break; \
        }                                                                                         \
        kt_.stop();                                                                               \
        RT_HIP(hipGetLastError());                                                                \
    } while (0)

int launch_tv_grad(const Plan &p, const float *f, float lambda2, float *pout, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    RT_TV_DISPATCH("k_tv_grad", k_grad, 0, f, p.d_S, lambda2, 0.f, 0.f, pout, (double *)nullptr, p.g.N,
                   p.g.Nz, p.g.K, p.g.Nt);
    return RT_OK;
}

int launch_grad_shrink(const Plan &p, const float *ft, float *h2, float sigma, float lambda1,
                       float lambda2, double *part, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    RT_TV_DISPATCH("k_grad_shrink", k_grad, 1, ft, p.d_S, lambda2, sigma, lambda1, h2, part, p.g.N, p.g.Nz,
                   p.g.K, p.g.Nt);
    return RT_OK;
}

int launch_tv_norm(const Plan &p, const float *f, float lambda2, double *part, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    RT_TV_DISPATCH("k_tv_norm", k_grad, 2, f, p.d_S, lambda2, 0.f, 0.f, (float *)nullptr, part, p.g.N,
                   p.g.Nz, p.g.K, p.g.Nt);
    return RT_OK;
}

int launch_tv_div(const Plan &p, const float *pin, float lambda2, float *out, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    RT_TV_DISPATCH("k_tv_div", k_div, 0, pin, p.d_S, lambda2, out, (const float *)nullptr, (float *)nullptr,
                   0.f, (double *)nullptr, p.g.N, p.g.Nz, p.g.K, p.g.Nt);
    return RT_OK;
}

int launch_div_update(const Plan &p, const float *h2, const float *adj, float *f, float *ft,
                      float tau, float lambda2, double *part, hipStream_t s)
{
    if (p.g.Nz == 0) return RT_OK;
    RT_TV_DISPATCH("k_div_update", k_div, 1, h2, p.d_S, lambda2, f, adj, ft, tau, part, p.g.N, p.g.Nz, p.g.K,
                   p.g.Nt);
    return RT_OK;
}

int launch_shrink(const Plan &p, float *pio, float lambda1, size_t n4, hipStream_t s)
{
    (void)p;
    if (n4 == 0) return RT_OK;
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((n4 + NT - 1) / NT, 8192));
    KTimer kt("k_shrink", s);
    hipLaunchKernelGGL(k_shrink, dim3(nb), dim3(NT), 0, s, pio, lambda1, n4);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rt

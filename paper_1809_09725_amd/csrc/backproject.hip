// Pixel-driven back-projection of the folded sinogram g~ (Sec. 4, eq.
// radadjapr): out_k(z,r,q) = sum_a sum_b w(theta0_a, b, q, r) g~(a,z,b,k), the
// exact transpose of the ray-driven forward projection: the weight of bin b
// for pixel p is max(0, 1 - |s_b - s_p| / c) / c with c = max(|cos|, |sin|),
// Joseph's linear interpolation written from the pixel's side.
//
// A 32x32 pixel tile takes the classes in rounds of CA; each round stages in
// LDS the window of detector bins the tile's pixels reach for each class
// (all KC channels of a bin in one row), then every pixel takes the two bins
// around its s_p for each class.  A pixel's position relative to its class's
// window is formed in FP64 once per class and stepped over the thread's rows
// in 32.32 fixed point (the integer part is the window row, the fraction
// gives the weights); weights and sums in FP32.
#include "common.h"
#include "internal.h"

namespace rt {
namespace {

constexpr int BP_VPT = 4;     // pixels per thread (rows 8 apart)
// Thread -> pixel: wave w of the tile takes columns 8w..8w+7 and lane l row
// l / 8 of each 8-row step, so the 64 taps of one read instruction come from
// an 8 x 8 pixel block.  Their detector positions then span few bins per
// 16-lane pass of the LDS, which measured 4.1 cycles per 16-byte read on
// sampled angles, against 7.2 for 2 rows x 32 columns.
__device__ inline int bp_col(int tid) { return 8 * (tid >> 6) + (tid & 7); }
__device__ inline int bp_row(int tid) { return (tid >> 3) & 7; }
constexpr int BP_MAXCA = 16;  // classes staged per round, at most

// Four workgroups per CU: the bound holds the 16-channel kernel to 128
// VGPRs (4 waves per SIMD, no spills) instead of 158 (3 waves), which
// measured 5% faster at 512^2 and 2% at 1024^2
template <int KC, int VEC>
__global__ __launch_bounds__(NT, 4) void k_backproject(
    const float *__restrict__ gt, float *__restrict__ out, const double *__restrict__ ccos,
    const double *__restrict__ csin, int N, int Nz, int Ns, int K, int n0, int nkc, int ntq,
    int ntr, int CA, int WMAX, unsigned nblocks)
{
    constexpr int stride = KC + 4;   // an odd number of 16-byte groups per bin
    extern __shared__ float win[];   // [CA][WMAX][stride]
    __shared__ int s_wb[BP_MAXCA], s_we[BP_MAXCA];   // window rows [wb, we) hold bins 0..Ns-1
    __shared__ long long s_goff[BP_MAXCA];           // element offset of window row 0's bin in gt
    __shared__ float s_inv[BP_MAXCA];                     // 1/c, c = max(|cos|, |sin|)
    __shared__ float s_ic1[BP_MAXCA], s_s1[BP_MAXCA];     // 1 - 1/c and 2^-32 / c
    __shared__ double s_base[BP_MAXCA];                   // hS - (bin of window row 0)
    __shared__ long long s_D[BP_MAXCA];                   // 8 sin in 32.32 fixed point
    unsigned lid = xcd_remap(blockIdx.x, nblocks);
    const int tq = lid % ntq;
    lid /= ntq;
    const int tr = lid % ntr;
    lid /= ntr;
    const int kc = lid % nkc;
    const int z = lid / nkc;
    const int tid = threadIdx.x;
    const int k0 = kc * KC;
    const double hN = 0.5 * (double)(N - 1), hS = 0.5 * (double)(Ns - 1);

    const int q = tq * 32 + bp_col(tid);
    const double x = (double)q - hN;
    const double y0 = (double)(tr * 32 + bp_row(tid)) - hN;   // rows y0 + 8j, j < BP_VPT
    const double xlo = (double)(tq * 32) - hN, xhi = xlo + 31.0;
    const double ylo = (double)(tr * 32) - hN, yhi = ylo + 31.0;

    float acc[BP_VPT][KC];
#pragma unroll
    for (int j = 0; j < BP_VPT; ++j)
#pragma unroll
        for (int k = 0; k < KC; ++k) acc[j][k] = 0.f;

    for (int a0 = 0; a0 < n0; a0 += CA) {
        const int nca = min(CA, n0 - a0);
        __syncthreads();
        if (tid < nca) {
            // detector window of class a over the tile: s_p is affine in
            // (x, y) and each rounding step is monotone, so the extreme
            // positions of the tile's pixels are at its corners
            const double cs = ccos[a0 + tid], sn = csin[a0 + tid];
            const double u00 = fma(xlo, cs, fma(ylo, sn, hS));
            const double u10 = fma(xhi, cs, fma(ylo, sn, hS));
            const double u01 = fma(xlo, cs, fma(yhi, sn, hS));
            const double u11 = fma(xhi, cs, fma(yhi, sn, hS));
            const double umin = fmin(fmin(u00, u10), fmin(u01, u11));
            const double umax = fmax(fmax(u00, u10), fmax(u01, u11));
            // one spare bin on each side: a pixel's s_p, formed incrementally
            // over its rows, may round an ulp outside [umin, umax]
            const int lo = (int)floor(umin) - 1;
            const int wn = (int)floor(umax) + 3 - lo;
            s_wb[tid] = max(0, -lo);
            s_we[tid] = min(wn, Ns - lo);
            s_goff[tid] = (((long long)(a0 + tid) * Nz + z) * Ns + lo) * K + k0;
            const double ic = 1.0 / fmax(fabs(cs), fabs(sn));
            s_inv[tid] = (float)ic;
            s_ic1[tid] = (float)(1.0 - ic);
            s_s1[tid] = (float)ic * 2.3283064365386963e-10f;
            s_base[tid] = hS - (double)lo;
            s_D[tid] = (long long)llrint(sn * 34359738368.0);
        }
        __syncthreads();
        {
            // NT / CA threads per class window (CA divides NT): thread j of
            // class c stages channel group j % NG of window rows j / NG, j / NG
            // + RS, ...; the class's bounds and offsets are read once per
            // round and the products fit 24 bits (w < WMAX, K <= 64).  The
            // window holds g~ / c, so that the weights below are c times the
            // triangle weights, in [0, 1].
            constexpr int NG = VEC == 4 ? KC / 4 : KC;   // channel groups per window row
            const int tpc = NT / CA;
            const int c = tid / tpc, j = tid - c * tpc;
            const int q = j % NG, RS = tpc / NG;
            const int kofs = VEC == 4 ? 4 * q : q;   // first channel of the group
            if (c < nca) {
                const int wb = s_wb[c], we = s_we[c];
                const float sc = s_inv[c];
                const bool kin = k0 + kofs < K;
                const float *src = gt + s_goff[c] + kofs;
                float *dst = win + __mul24(c, WMAX) * stride + kofs;
                for (int w = j / NG; w < WMAX; w += RS) {
                    const bool in = kin && w >= wb && w < we;
                    if constexpr (VEC == 4) {
                        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (in) v = *(const float4 *)(src + __mul24(w, K));
                        v.x *= sc;
                        v.y *= sc;
                        v.z *= sc;
                        v.w *= sc;
                        *(float4 *)(dst + __mul24(w, stride)) = v;
                    } else {
                        dst[__mul24(w, stride)] = in ? src[__mul24(w, K)] * sc : 0.f;
                    }
                }
            }
        }
        __syncthreads();
        for (int c = 0; c < nca; ++c) {
            const double cs = ccos[a0 + c], sn = csin[a0 + c];
            const float ic1 = s_ic1[c], s1 = s_s1[c];
            // s_p minus the bin of the window's row 0, for the thread's first
            // row: at least 1 up to FP64 rounding (the window keeps a spare bin
            // below the tile's lowest position), so truncation is floor
            const double rel = fma(x, cs, fma(y0, sn, s_base[c]));
            const unsigned hi = (unsigned)rel;
            const unsigned lo = (unsigned)((rel - (double)hi) * 4294967296.0);
            // 32.32 fixed point whose integer part is the LDS row (class c's
            // rows start at c WMAX); rows 8 apart add 8 sin, rounded to 2^-32,
            // which moves a position by at most 2^-31 over the thread's rows
            unsigned long long U = ((unsigned long long)(hi + (unsigned)(c * WMAX)) << 32) | lo;
            const unsigned long long D = (unsigned long long)s_D[c];
#pragma unroll
            for (int j = 0; j < BP_VPT; ++j) {
                if (j) {
                    U += D;
                    asm volatile("" : "+v"(U));   // one 64-bit add per row, not j*D
                }
                const unsigned row = (unsigned)(U >> 32);
                const float fq = (float)(unsigned)U;   // the fraction in units of 2^-32
                // triangle weights of the bins floor(u) and floor(u)+1 times c
                // (the window holds g~ / c), max(0, 1 - |s_b - s_p| / c), which
                // is at most 1: one fma with the clamp to [0, 1] each
                const float w0 = fminf(fmaxf(fmaf(-fq, s1, 1.f), 0.f), 1.f);
                const float w1 = fminf(fmaxf(fmaf(fq, s1, ic1), 0.f), 1.f);
                const float *t0 = win + __umul24(row, stride);
#pragma unroll
                for (int k = 0; k < KC; k += 4) {
                    const float4 x0 = *(const float4 *)(t0 + k);
                    const float4 x1 = *(const float4 *)(t0 + stride + k);
                    acc[j][k + 0] = fmaf(w1, x1.x, fmaf(w0, x0.x, acc[j][k + 0]));
                    acc[j][k + 1] = fmaf(w1, x1.y, fmaf(w0, x0.y, acc[j][k + 1]));
                    acc[j][k + 2] = fmaf(w1, x1.z, fmaf(w0, x0.z, acc[j][k + 2]));
                    acc[j][k + 3] = fmaf(w1, x1.w, fmaf(w0, x0.w, acc[j][k + 3]));
                }
            }
        }
    }

    if (q >= N) return;
#pragma unroll
    for (int j = 0; j < BP_VPT; ++j) {
        const int r = tr * 32 + bp_row(tid) + 8 * j;
        if (r >= N) continue;
        float *dst = out + (((size_t)z * N + r) * N + q) * K + k0;
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (k0 + k < K) dst[k] = acc[j][k];
    }
}

template <int KC, int VEC>
static void launch_bp_t(const Plan &p, float *out, hipStream_t s, unsigned nb, int ntq, int ntr)
{
    const rt_geom &G = p.g;
    const AdjCfg &B = p.adj;
    KTimer kt("k_backproject", s);
    hipLaunchKernelGGL((k_backproject<KC, VEC>), dim3(nb), dim3(NT), B.lds, s, p.d_scr, out,
                       p.d_ccos, p.d_csin, G.N, G.Nz, G.Ns, G.K, p.n0, B.nkc, ntq, ntr, B.CA,
                       B.WMAX, nb);
    kt.stop();
}

}  // namespace

int launch_backproject(const Plan &p, float *out, hipStream_t s)
{
    const rt_geom &G = p.g;
    const AdjCfg &B = p.adj;
    if (G.Nz == 0) return RT_OK;
    const int ntq = (G.N + 31) / 32, ntr = (G.N + 31) / 32;
    const unsigned nb = (unsigned)G.Nz * B.nkc * ntr * ntq;
    if (B.vec == 4) {
        switch (B.KC) {
        case 4: launch_bp_t<4, 4>(p, out, s, nb, ntq, ntr); break;
        case 8: launch_bp_t<8, 4>(p, out, s, nb, ntq, ntr); break;
        default: launch_bp_t<16, 4>(p, out, s, nb, ntq, ntr); break;
        }
    } else {
        switch (B.KC) {
        case 4: launch_bp_t<4, 1>(p, out, s, nb, ntq, ntr); break;
        case 8: launch_bp_t<8, 1>(p, out, s, nb, ntq, ntr); break;
        default: launch_bp_t<16, 1>(p, out, s, nb, ntq, ntr); break;
        }
    }
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rt

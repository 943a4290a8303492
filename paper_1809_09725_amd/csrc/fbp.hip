// Initial guess of Secs. 5-6: a static filtered back-projection (FBP, with
// the Shepp-Logan filter) of every half-turn, then the coefficients f_k whose
// half-turn averages reproduce those frames in the least-squares sense.
//
//   q(i,z,b)  = sum_{b'} h(b - b') g(i,z,b'),  h(n) = -2 / (pi^2 (4 n^2 - 1))
//   F_m       = (pi / Ntheta0) sum over the projections i of half-turn m of
//               the transpose of the projector applied to q(i,.,.)
//   B[m][k]   = mean of Phi[i][k] over the projections of half-turn m
//   f_k       = sum_m A[k][m] F_m,   A = B^+ (minimum-norm least squares)
//
// Kernels
//   k_shepp_logan  each projection row convolved with h over the detector
//                  (bins outside [0, Ns) are zero)
//   k_analysis     per voxel, the K x Npi matrix A applied to the Npi frames
// The half-turn back-projection runs the library's own transpose (fold-sum
// and pixel-driven back-projection) through an internal plan whose basis is
// the half-turn indicator scaled by pi / Ntheta0.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "internal.h"

namespace rt {
namespace {

constexpr int SL_T = 256;   // threads of a filter workgroup

// A workgroup filters RPW rows (RPW = 1024 / Nsp, at least 1); each thread
// owns runs of 4 consecutive output bins of one row.  The rows and the kernel
// values are staged in LDS:
//   rows[RPW][Nsp], hs[j] = h(j - (Nsp + 3)) for j = 0 .. 2 Nsp + 7,
// with Nsp = Ns rounded up to 4 (rows padded with zeros).  Per 4 inputs a
// thread reads them once (the same address in every lane of the row) and 8
// kernel values (consecutive lanes 16 bytes apart), and issues 16 FMAs.
__global__ __launch_bounds__(SL_T) void k_shepp_logan(const float *__restrict__ g,
                                                      float *__restrict__ q, long rows, int Ns,
                                                      int Nsp, int RPW)
{
    extern __shared__ float4 sl4[];
    float *srow = (float *)sl4;             // [RPW][Nsp]
    float *hs = srow + (size_t)RPW * Nsp;   // [2 Nsp + 8]
    const long r0 = (long)blockIdx.x * RPW;
    for (int e = threadIdx.x; e < RPW * Nsp; e += SL_T) {
        const long r = r0 + e / Nsp;
        const int b = e % Nsp;
        srow[e] = (r < rows && b < Ns) ? g[r * Ns + b] : 0.f;
    }
    for (int j = threadIdx.x; j < 2 * Nsp + 8; j += SL_T) {
        const double n = (double)(j - (Nsp + 3));
        hs[j] = (float)(-2.0 / (M_PI * M_PI * (4.0 * n * n - 1.0)));
    }
    __syncthreads();
    const int TPR = SL_T / RPW;             // threads per row
    const int rr = threadIdx.x / TPR, lt = threadIdx.x % TPR;
    const long r = r0 + rr;
    if (r >= rows) return;
    const float *row = srow + (size_t)rr * Nsp;
    for (int b0 = 4 * lt; b0 < Ns; b0 += 4 * TPR) {
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int c0 = 0; c0 < Nsp; c0 += 4) {
            const float4 x = *(const float4 *)(row + c0);
            const int base = b0 - c0 + Nsp;   // hs index of h(b0 - c0 - 3)
            const float4 h0 = *(const float4 *)(hs + base);
            const float4 h1 = *(const float4 *)(hs + base + 4);
            const float hw[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
            const float xv[4] = {x.x, x.y, x.z, x.w};
            // output b0 + o, input c0 + i: h(b0 + o - c0 - i) = hw[3 + o - i]
#pragma unroll
            for (int o = 0; o < 4; ++o)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[o] = fmaf(hw[3 + o - i], xv[i], acc[o]);
        }
        float *out = q + r * Ns;
#pragma unroll
        for (int o = 0; o < 4; ++o)
            if (b0 + o < Ns) out[b0 + o] = acc[o];
    }
}

// f[v][k] = sum_m A[k][m] F[v][m] for every voxel v.  A is staged in LDS as
// [Npi][4 * KB4] (zero-padded channels); a thread owns one voxel, reads its
// Npi frame values once and keeps the K sums in float4 registers.
template <int KB4>
__global__ __launch_bounds__(NT) void k_analysis(const float *__restrict__ F,
                                                 const float *__restrict__ A,
                                                 float *__restrict__ f, long nvox, int Npi, int K)
{
    extern __shared__ float4 sa4[];   // [Npi][KB4]
    for (int e = threadIdx.x; e < Npi * KB4 * 4; e += NT) {
        const int m = e / (4 * KB4), k = e % (4 * KB4);
        ((float *)sa4)[e] = k < K ? A[(size_t)k * Npi + m] : 0.f;
    }
    __syncthreads();
    for (long v = (long)blockIdx.x * NT + threadIdx.x; v < nvox; v += (long)gridDim.x * NT) {
        float4 acc[KB4];
#pragma unroll
        for (int j = 0; j < KB4; ++j) acc[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        const float *fr = F + v * Npi;
        for (int m = 0; m < Npi; ++m) {
            const float x = fr[m];
#pragma unroll
            for (int j = 0; j < KB4; ++j) {
                const float4 a = sa4[m * KB4 + j];
                acc[j].x = fmaf(a.x, x, acc[j].x);
                acc[j].y = fmaf(a.y, x, acc[j].y);
                acc[j].z = fmaf(a.z, x, acc[j].z);
                acc[j].w = fmaf(a.w, x, acc[j].w);
            }
        }
        float *o = f + v * K;
        if ((K & 3) == 0) {
#pragma unroll
            for (int j = 0; j < KB4; ++j)
                if (4 * j < K) *(float4 *)(o + 4 * j) = acc[j];
        } else {
#pragma unroll
            for (int j = 0; j < KB4; ++j) {
                const float w[4] = {acc[j].x, acc[j].y, acc[j].z, acc[j].w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * j + i < K) o[4 * j + i] = w[i];
            }
        }
    }
}

// Minimum-norm least-squares inverse of B [Npi][K] in FP64 on the host:
// B^T (B B^T)^-1 when Npi <= K, (B^T B)^-1 B^T otherwise (both equal B^+ for
// a matrix of full rank); returned as A [K][Npi].  Gauss-Jordan elimination
// with partial pivoting; a rank-deficient B is an error.
int pseudo_inverse(const std::vector<double> &B, int Npi, int K, std::vector<double> &A)
{
    const bool wide = Npi <= K;
    const int n = wide ? Npi : K;   // order of the Gram matrix
    std::vector<double> M((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            if (wide)
                for (int k = 0; k < K; ++k) s += B[(size_t)i * K + k] * B[(size_t)j * K + k];
            else
                for (int m = 0; m < Npi; ++m) s += B[(size_t)m * K + i] * B[(size_t)m * K + j];
            M[(size_t)i * n + j] = s;
        }
    // right-hand sides: B (n = Npi rows of K) or B^T (n = K rows of Npi)
    const int w = wide ? K : Npi;
    std::vector<double> R((size_t)n * w);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < w; ++c) R[(size_t)i * w + c] = wide ? B[(size_t)i * K + c] : B[(size_t)c * K + i];
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, std::fabs(M[(size_t)i * n + i]));
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (std::fabs(M[(size_t)i * n + col]) > std::fabs(M[(size_t)piv * n + col])) piv = i;
        if (!(std::fabs(M[(size_t)piv * n + col]) > 1e-12 * dmax))
            return fail(RT_E_ARG, "the half-turn means of the basis are rank deficient");
        if (piv != col) {
            for (int j = 0; j < n; ++j) std::swap(M[(size_t)col * n + j], M[(size_t)piv * n + j]);
            for (int j = 0; j < w; ++j) std::swap(R[(size_t)col * w + j], R[(size_t)piv * w + j]);
        }
        const double d = M[(size_t)col * n + col];
        for (int j = 0; j < n; ++j) M[(size_t)col * n + j] /= d;
        for (int j = 0; j < w; ++j) R[(size_t)col * w + j] /= d;
        for (int i = 0; i < n; ++i) {
            if (i == col) continue;
            const double fct = M[(size_t)i * n + col];
            if (fct == 0.0) continue;
            for (int j = 0; j < n; ++j) M[(size_t)i * n + j] -= fct * M[(size_t)col * n + j];
            for (int j = 0; j < w; ++j) R[(size_t)i * w + j] -= fct * R[(size_t)col * w + j];
        }
    }
    // wide: R = (B B^T)^-1 B  [Npi][K]  -> A = R^T;  tall: R = (B^T B)^-1 B^T  [K][Npi] = A
    A.assign((size_t)K * Npi, 0.0);
    for (int k = 0; k < K; ++k)
        for (int m = 0; m < Npi; ++m)
            A[(size_t)k * Npi + m] = wide ? R[(size_t)m * K + k] : R[(size_t)k * Npi + m];
    return RT_OK;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

int launch_fbp_filter(const Plan &p, const float *g, float *q, hipStream_t s)
{
    const rt_geom &G = p.g;
    const long rows = (long)G.Ntheta * G.Nz;
    if (rows == 0 || G.Ns == 0) return RT_OK;
    const int Nsp = (G.Ns + 3) / 4 * 4;
    const int RPW = std::max(1, std::min(8, 1024 / Nsp));
    const size_t lds = ((size_t)RPW * Nsp + 2 * (size_t)Nsp + 8) * sizeof(float);
    if (lds > 160 * 1024) return fail(RT_E_SHAPE, "the Shepp-Logan filter stages rows of at most 13000 bins");
    if (lds > 64 * 1024)
        RT_HIP(hipFuncSetAttribute((const void *)k_shepp_logan,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const unsigned nb = (unsigned)((rows + RPW - 1) / RPW);
    KTimer kt("k_shepp_logan", s);
    hipLaunchKernelGGL(k_shepp_logan, dim3(nb), dim3(SL_T), lds, s, g, q, rows, G.Ns, Nsp, RPW);
    kt.stop();
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int fbp_init(const Plan &p, const float *g, float *f, hipStream_t s)
{
    const rt_geom &G = p.g;
    if (G.Npi > 64) return fail(RT_E_SHAPE, "the FBP initial guess handles at most 64 half-turns");
    const size_t nvox = (size_t)G.Nz * G.N * G.N;
    if (nvox == 0) return RT_OK;
    // half-turn means of the basis and their pseudo-inverse (FP64, host)
    const int K = G.K, Npi = G.Npi, n0 = p.n0;
    std::vector<double> B((size_t)Npi * K, 0.0), A;
    for (int i = 0; i < G.Ntheta; ++i)
        for (int k = 0; k < K; ++k) B[(size_t)(i / n0) * K + k] += p.T.phi[(size_t)i * K + k];
    for (double &b : B) b /= (double)n0;
    int rc = pseudo_inverse(B, Npi, K, A);
    if (rc) return rc;
    std::vector<float> A32(A.begin(), A.end());
    // internal plan: the same geometry with the half-turn indicator basis
    rt_geom gm = G;
    gm.K = Npi;
    gm.Nt = Npi;
    std::vector<double> ind((size_t)G.Ntheta * Npi, 0.0);
    for (int i = 0; i < G.Ntheta; ++i) ind[(size_t)i * Npi + i / n0] = M_PI / (double)n0;
    rt_plan *ip = nullptr;
    if ((rc = rt_plan_create(&gm, RT_FORM_PF, RT_PREC_FP32, ind.data(), nullptr, &ip))) return rc;
    struct PlanGuard {
        rt_plan *p;
        ~PlanGuard() { rt_plan_destroy(p); }
    } guard{ip};
    DevBuf q, F, dA;
    RT_HIP(hipMalloc(&q.p, std::max<size_t>(ng_of(G), 1) * sizeof(float)));
    RT_HIP(hipMalloc(&F.p, nvox * Npi * sizeof(float)));
    RT_HIP(hipMalloc(&dA.p, A32.size() * sizeof(float)));
    auto run = [&]() -> int {
        RT_HIP(hipMemcpyAsync(dA.p, A32.data(), A32.size() * sizeof(float), hipMemcpyHostToDevice, s));
        int r = launch_fbp_filter(p, g, (float *)q.p, s);
        if (r) return r;
        if ((r = launch_adjoint(ip->impl, (const float *)q.p, (float *)F.p, s))) return r;
        const int kb4 = (K + 3) / 4;
        const int KB4 = kb4 <= 2 ? 2 : kb4 <= 4 ? 4 : kb4 <= 8 ? 8 : 16;
        const size_t lds = (size_t)Npi * KB4 * 4 * sizeof(float);
        const unsigned nb = (unsigned)std::min<size_t>((nvox + NT - 1) / NT, 16384);
        KTimer kt("k_analysis", s);
#define RT_AN(B) hipLaunchKernelGGL(k_analysis<B>, dim3(nb), dim3(NT), lds, s, (const float *)F.p, \
                                    (const float *)dA.p, f, (long)nvox, Npi, K)
        if (KB4 == 2) RT_AN(2);
        else if (KB4 == 4) RT_AN(4);
        else if (KB4 == 8) RT_AN(8);
        else RT_AN(16);
#undef RT_AN
        kt.stop();
        RT_HIP(hipGetLastError());
        return RT_OK;
    };
    rc = run();
    // the temporaries, the host copy of A and the internal plan are released
    // on return: wait for the stream first, on the error path too
    const hipError_t e = hipStreamSynchronize(s);
    if (rc) return rc;
    if (e != hipSuccess) return fail(RT_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return RT_OK;
}

}  // namespace rt

// Measurement aid: the issue rate of plain (unpacked) FP32 fused multiply-add
// on this device, the ceiling of every kernel here whose work is FP32 FMAs
// (the projectors, the Shepp-Logan filter).  Each thread runs eight
// independent FMA chains, so the loop is bound by VALU issue alone: no memory
// traffic, no dependency stalls at two or more waves per SIMD.
#include "common.h"
#include "internal.h"

namespace rt {
namespace {

constexpr int CHAINS = 8;

__global__ __launch_bounds__(NT) void k_calib_fma(float *__restrict__ out, int n_iter, float a, float b)
{
    float x[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = (float)(threadIdx.x + c);
    for (int it = 0; it < n_iter; ++it) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) x[c] = fmaf(x[c], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += x[c];
    // a and b keep |x| bounded; the store keeps the chains live
    out[(size_t)blockIdx.x * NT + threadIdx.x] = s;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" int rt_calib_fma(int32_t n_blocks, int32_t n_iter, float *out, double *ms,
                            double *flop, void *stream)
{
    if (n_blocks < 1 || n_iter < 1 || !out || !ms || !flop)
        return fail(RT_E_ARG, "rt_calib_fma: bad argument");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RT_HIP(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "rt_calib_fma: event");
    }
    int rc = RT_OK;
    float t = 0.f;
    if ((he = hipEventRecord(e0, s)) != hipSuccess) {
        rc = hip_fail(he, "rt_calib_fma: record");
    } else {
        {
            KTimer tm("k_calib_fma", s);
            k_calib_fma<<<n_blocks, NT, 0, s>>>(out, n_iter, 0.999f, 0.001f);
        }
        if ((he = hipGetLastError()) != hipSuccess || (he = hipEventRecord(e1, s)) != hipSuccess ||
            (he = hipEventSynchronize(e1)) != hipSuccess ||
            (he = hipEventElapsedTime(&t, e0, e1)) != hipSuccess)
            rc = hip_fail(he, "rt_calib_fma: launch");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != RT_OK) return rc;
    *ms = t;
    *flop = 2.0 * CHAINS * 16.0 * (double)n_iter * (double)NT * (double)n_blocks;
    return RT_OK;
}

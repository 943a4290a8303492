// FP64 reductions with a fixed summation tree, and small vector kernels.
//
// A reduction runs in two launches: a fixed number of workgroups each sum a
// grid-strided share of the input in FP64 (wave64 butterfly through
// __shfl_xor, then the four wave sums in order) and write one partial; one
// workgroup then sums the partials in a fixed order.  The grid size depends
// only on n, so the result is bitwise reproducible for a given shape.
#include <mutex>
#include <unordered_map>

#include "common.h"
#include "internal.h"

namespace rt {
namespace {

template <int DIFF>
__global__ __launch_bounds__(NT) void k_dot(const float *__restrict__ x, const float *__restrict__ y,
                                            size_t n, double *__restrict__ part)
{
    __shared__ double sh[NT / 64];
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT) {
        if (DIFF) {
            const double d = (double)x[e] - (double)y[e];
            s += d * d;
        } else {
            s += (double)x[e] * (double)y[e];
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[j] = sum_{i < nb} part[i * width + j]: thread t sums i = t, t+NT, ...
// in order, then the NT thread sums are combined by block_sum.
__global__ __launch_bounds__(NT) void k_finish(const double *__restrict__ part, int nb, int width,
                                               double *__restrict__ out)
{
    __shared__ double sh[NT / 64];
    for (int j = 0; j < width; ++j) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nb; i += NT) s += part[(size_t)i * width + j];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[j] = s;
    }
}

__global__ __launch_bounds__(NT) void k_fill(float *__restrict__ x, float v, size_t n)
{
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT)
        x[e] = v;
}

// x <- x / sqrt(nd[0]) in FP64 (normalisation step of the power iteration)
__global__ __launch_bounds__(NT) void k_scale(float *__restrict__ x, const double *__restrict__ nd,
                                              size_t n)
{
    const double inv = 1.0 / sqrt(nd[0]);
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT)
        x[e] = (float)((double)x[e] * inv);
}

__global__ __launch_bounds__(NT) void k_copy(float *__restrict__ d, const float *__restrict__ s,
                                             size_t n)
{
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT)
        d[e] = s[e];
}

// SplitMix64 (Steele, Lea, Flood 2014) used counter-style: value j is the
// output mix of state seed + (j+1)*0x9E3779B97F4A7C15; the top 24 bits give
// u in [0,1) and x = 2u - 1 is exact in FP32.
__global__ __launch_bounds__(NT) void k_seeded(float *__restrict__ x, size_t n, uint64_t seed)
{
    for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT) {
        uint64_t z = seed + ((uint64_t)e + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const int m = (int)(z >> 40);                 // 0 .. 2^24 - 1
        x[e] = (float)(2 * m - (1 << 24)) * (1.0f / 16777216.0f);
    }
}

unsigned grid_for(size_t n, unsigned cap)
{
    return (unsigned)std::max<size_t>(1, std::min<size_t>((n + NT - 1) / NT, cap));
}

}  // namespace

int reduce_blocks(int, size_t n) { return (int)grid_for(n, 2048); }

int launch_dot_partials(const float *x, const float *y, size_t n, double *part, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot<0>, dim3(nb), dim3(NT), 0, s, x, y, n, part);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_diff_sq_partials(const float *x, const float *y, size_t n, double *part, int nb,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_dot<1>, dim3(nb), dim3(NT), 0, s, x, y, n, part);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_finish(const double *part, int nb, int width, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(NT), 0, s, part, nb, width, out);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_fill(float *x, float v, size_t n, hipStream_t s)
{
    if (!n) return RT_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 8192)), dim3(NT), 0, s, x, v, n);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_scale(float *x, const double *nd, size_t n, hipStream_t s)
{
    if (!n) return RT_OK;
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n, 8192)), dim3(NT), 0, s, x, nd, n);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_copy(float *d, const float *src, size_t n, hipStream_t s)
{
    if (!n) return RT_OK;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 8192)), dim3(NT), 0, s, d, src, n);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

int launch_seeded_uniform(float *x, size_t n, uint64_t seed, hipStream_t s)
{
    if (!n) return RT_OK;
    hipLaunchKernelGGL(k_seeded, dim3(grid_for(n, 8192)), dim3(NT), 0, s, x, n, seed);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

}  // namespace rt

// ---- the allocation-free variant of rt_dot -------------------------------
// Its partials live in a file-scope device array instead of a per-call
// allocation.  In host code `scratch` names a host-side stand-in, not device
// memory: the device address comes from hipGetSymbolAddress, once per device
// with that device current, and only that address is passed to kernels.
namespace rt {
namespace {

constexpr int DOT_MAX_PARTIALS = 2048;   // grid_for(n, 2048): the widest reduction launch
__device__ __align__(256) double scratch[DOT_MAX_PARTIALS + 1];   // partials, then the sum

std::mutex g_scratch_mu;
std::unordered_map<int, double *> g_scratch_ptr;   // device -> address of its copy

int scratch_ptr(double **out)
{
    int dev = 0;
    RT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "rt_dot_noalloc: hipGetSymbolAddress(scratch)");
        it = g_scratch_ptr.emplace(dev, (double *)p).first;
    }
    *out = it->second;
    return RT_OK;
}

}  // namespace
}  // namespace rt

extern "C" int rt_dot_noalloc(const float *x, const float *y, size_t n, double *out, void *stream)
{
    using namespace rt;
    if (!out || (n && (!x || !y))) return fail(RT_E_ARG, "rt_dot_noalloc: NULL argument");
    if (n == 0) {
        *out = 0.0;
        return RT_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const int nb = reduce_blocks(0, n);
    if (nb > DOT_MAX_PARTIALS)
        return fail(RT_E_SHAPE, "rt_dot_noalloc: %d partials exceed the static scratch of %d", nb,
                    DOT_MAX_PARTIALS);
    double *part = nullptr;
    int rc = scratch_ptr(&part);
    if (rc) return rc;
    double *res = part + nb;
    // every partial is written before k_finish reads it: nothing to clear
    rc = launch_dot_partials(x, y, n, part, nb, s);
    if (!rc) rc = launch_finish(part, nb, 1, res, s);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "rt_dot_noalloc readback");
    }
    return rc;
}

extern "C" int rt_dot(const float *x, const float *y, size_t n, double *out, void *stream)
{
    using namespace rt;
    if (!out || (n && (!x || !y))) return fail(RT_E_ARG, "rt_dot: NULL argument");
    if (n == 0) {
        *out = 0.0;
        return RT_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const int nb = reduce_blocks(0, n);
    double *part = nullptr, *res = nullptr;
    RT_HIP(hipMallocAsync((void **)&part, (nb + 1) * sizeof(double), s));
    res = part + nb;
    int rc = launch_dot_partials(x, y, n, part, nb, s);
    if (!rc) rc = launch_finish(part, nb, 1, res, s);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "rt_dot readback");
    }
    (void)hipFreeAsync(part, s);
    return rc;
}

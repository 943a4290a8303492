// Device helpers shared by the kernels of librt4d.
#pragma once

#include <hip/hip_runtime.h>

namespace rt {

constexpr int NT = 256;   // threads per workgroup (4 wave64)

// The dispatcher deals consecutive workgroups round-robin to the 8 XCDs of
// MI355X, each with its own L2.  Remap so that XCD x receives a contiguous
// run of logical ids: neighbouring logical ids (which share input slices)
// then run on the same L2.  Bijective on [0, nblocks).
__device__ inline unsigned xcd_remap(unsigned bid, unsigned nblocks)
{
    const unsigned q = nblocks >> 3;
    if (bid < (q << 3)) return (bid & 7u) * q + (bid >> 3);
    return bid;
}

// Sum of one double per thread over the workgroup; the result is valid in
// thread 0.  Wave64 butterfly, then the 4 wave sums in order.
__device__ inline double block_sum(double v, double *sh /* >= NT/64 doubles of LDS */)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    return r;
}

}  // namespace rt

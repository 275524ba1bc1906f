// Fixed-order sums of per-workgroup partials (the reductions' first pass).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace grg {

// acc[k] += partials[(i nrhs + r) K + k] for i = threadIdx.x, + 256, ... < n,
// in that order (a workgroup of 256 threads); the loads of four consecutive i are issued before any of
// them is added (the partials come from another kernel: each load is a
// round trip to L2 or memory).
template <int K>
__device__ __forceinline__ void strided_sum(const double *__restrict__ partials, int n, int nrhs, int r,
                                            double (&acc)[3])
{
    int i = threadIdx.x;
    for (; i + 3 * 256 < n; i += 4 * 256) {
        double v[4][K];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = partials[((size_t)(i + u * 256) * nrhs + r) * K + k];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += v[u][k];
    }
    for (; i < n; i += 256)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += partials[((size_t)i * nrhs + r) * K + k];
}

}  // namespace grg

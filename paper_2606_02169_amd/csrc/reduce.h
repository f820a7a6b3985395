// Deterministic FP64 block reductions for wave64 (no atomics): a fixed shuffle tree inside each
// wave, then the waves' partials summed in wave order by the first wave.
#pragma once

#include <hip/hip_runtime.h>

namespace mrmf {

template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_down(v[k], off, 64);
    }
}

// Sums v over the block; the result is valid in thread 0.  `lds` must hold NV * (blockDim/64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    wave_sum<NV>(v);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wave * NV + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += lds[w * NV + k];
            v[k] = s;
        }
    }
    __syncthreads();
}

}  // namespace mrmf

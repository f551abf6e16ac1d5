// Device-side helpers shared by the gfx950 kernels of the BOSP library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrep {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

// Sum over the 64 lanes of a wavefront; every lane receives the total.
// Butterfly with a fixed order, so the result is bitwise reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    return v;
}

// Block-wide sum for blockDim.x == NT (multiple of 64); `red` is LDS scratch of
// NT/64 doubles.  Deterministic: per-wave butterfly, then a fixed-order sum of
// the wave totals by wave 0.  All threads receive the result.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    constexpr int NW = NT / WAVE;
    const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += red[i];
    __syncthreads();
    return t;
}

// "Last block" completion ticket for two-stage deterministic reductions:
// every block writes its partial, fences, then bumps the counter; the block
// that observes count == nblocks - 1 performs the final fixed-order reduction
// and resets the counter to zero so that the next launch (or graph replay)
// starts clean.
__device__ __forceinline__ bool last_block_arrives(unsigned* counter, unsigned nblocks) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(counter, 1u);
        is_last = (prev == nblocks - 1);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return is_last;
}

}  // namespace lrep

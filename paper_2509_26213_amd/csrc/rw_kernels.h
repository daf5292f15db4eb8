// Host helpers shared by the translation units, and the device-side
// reduction helpers of the CG kernels.
#pragma once

#include "rw_internal.h"

namespace rw {

rw_status invalid(const std::string& msg);
rw_status check_volume(const rw_volume* vol);
Geom make_geom(rw_dims d);
WCoef make_wcoef(const rw_volume* vol, double beta, double w_eps);
rw_status stream_enter(rw_context* ctx, void* user);
rw_status stream_leave(rw_context* ctx, void* user);
rw_status label_counts(rw_context* ctx, const uint8_t* lab, int64_t n, unsigned int* host256);
rw_status ensure_events(rw_context* ctx, size_t n);

// Sum NQ per-thread values over a 256-thread block in a fixed order (wave
// butterfly, then the four wave totals in wave order); thread 0..NQ-1 write
// out[q].  Every thread of the block must call it.
template <int NQ>
__device__ __forceinline__ void block_sum_store(double (&v)[NQ], double* __restrict__ out) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double a = v[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        v[q] = a;
    }
    __shared__ double sh[NT / 64][NQ];
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sh[wid][q] = v[q];
    }
    __syncthreads();
    if (tid < NQ) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += sh[w][tid];
        out[tid] = s;
    }
}

// Fixed-order sum over blocks of the NQ-quantity partials; result in sums[]
// (shared) visible to every thread after return.  One 256-thread block.
template <int NQ>
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int nblocks,
                                             double* sums) {
    __shared__ double sh[256];
    const int tid = threadIdx.x;
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = 0.0;
    for (int b = tid; b < nblocks; b += 256) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) a[q] += part[(int64_t)b * NQ + q];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        sh[tid] = a[q];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) sh[tid] += sh[tid + o];
            __syncthreads();
        }
        if (tid == 0) sums[q] = sh[0];
        __syncthreads();
    }
}

}  // namespace rw

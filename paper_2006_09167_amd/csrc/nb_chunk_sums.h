// Deterministic chunked sums shared by the force and backward reductions (device code).
#pragma once

#include "nb_internal.h"

constexpr int kRedThreads = 256;

// Deterministic two-stage reductions of per-item partial sums (structure of arrays, K
// values, one column per item rank).  Stage 1: one block per chunk of up to kChunkItems
// consecutive ranks of one segment sums each value (fixed butterfly and wave order) into
// the chunk partial.  Stage 2: one block per segment adds its chunks in order.
template <typename T>
__device__ inline void chunk_sums(const T* __restrict__ vals, int stride, int K, int p0, int p1,
                                  double* __restrict__ out) {
    constexpr int kG = 16;                 // values summed per pass (loads issued together)
    __shared__ double s_w[kRedThreads / kWave][kG];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int k0 = 0; k0 < K; k0 += kG) {
        const int g = min(kG, K - k0);
        double acc[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) acc[q] = 0.0;
        // Rows past the last value re-read row g-1 (in bounds, never written out), so
        // every load of a pass is unconditional and all of them are in flight together.
#pragma unroll 2
        for (int i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
            T v[kG];
#pragma unroll
            for (int q = 0; q < kG; ++q) v[q] = vals[(size_t)(k0 + min(q, g - 1)) * stride + i];
#pragma unroll
            for (int q = 0; q < kG; ++q) acc[q] += (double)v[q];
        }
#pragma unroll
        for (int q = 0; q < kG; ++q) {
            for (int off = 1; off < kWave; off <<= 1) acc[q] += __shfl_xor(acc[q], off);
            if (lane == 0) s_w[wv][q] = acc[q];
        }
        __syncthreads();
        if (threadIdx.x < g) {
            double t = 0.0;
            for (int w = 0; w < kRedThreads / kWave; ++w) t += s_w[w][threadIdx.x];
            out[k0 + threadIdx.x] = t;
        }
        __syncthreads();
    }
}

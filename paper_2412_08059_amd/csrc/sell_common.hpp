// Device helpers shared by the SELL-64 kernels: fma in the working
// precision, wave and block sums, the fixed-order reduction of per-block
// partials, and the XCD-aware walk of slice groups.

#pragma once

#include "mpcg_internal.hpp"

#include <cmath>

namespace mpcg {

template <typename T> __device__ inline T fma_t(T a, T b, T c);
template <> __device__ inline float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ inline double fma_t<double>(double a, double b, double c) { return fma(a, b, c); }

__device__ inline double sell_wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double sell_block_sum(double v, double *sm)
{
    v = sell_wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += sm[i];
    __syncthreads();
    return s;
}

__device__ inline double sell_reduce_partials(const double *p, int cnt, double *sm)
{
    // four loads in flight per thread, added in index order (the same bits
    // as one at a time)
    double acc = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kBlock < cnt; i += 4 * kBlock) {
        const double p0 = p[i], p1 = p[i + kBlock], p2 = p[i + 2 * kBlock], p3 = p[i + 3 * kBlock];
        acc += p0;
        acc += p1;
        acc += p2;
        acc += p3;
    }
    for (; i < cnt; i += kBlock) acc += p[i];
    double s = sell_block_sum(acc, sm);
    if (threadIdx.x == 0) sm[kBlock / 64] = s;
    __syncthreads();
    s = sm[kBlock / 64];
    __syncthreads();
    return s;
}

// FP32 accumulation (dot_acc = 1): the same trees in float; partials are
// stored widened to double and narrowed back, both exact.
__device__ inline float sell_wave_sum_f(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline float sell_block_sum_f(float v, double *sm)
{
    v = sell_wave_sum_f(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = (double)v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += (float)sm[i];
    __syncthreads();
    return s;
}

__device__ inline double sell_reduce_partials_f(const double *p, int cnt, double *sm)
{
    float acc = 0.0f;
    for (int i = threadIdx.x; i < cnt; i += kBlock) acc += (float)p[i];
    float s = sell_block_sum_f(acc, sm);
    if (threadIdx.x == 0) sm[kBlock / 64] = (double)s;
    __syncthreads();
    const double r = sm[kBlock / 64];
    __syncthreads();
    return r;
}

// Slice groups (kBlock / 64 slices, one per wave) of an XCD's contiguous
// range are dealt round-robin to that XCD's blocks: at any moment the blocks
// of one XCD work on a narrow window of consecutive rows, so the rows that a
// stencil's neighbour planes gather are still in that XCD's L2.
struct SliceWalk {
    int g, g_end, step;   // group index, end, stride
};

__device__ inline SliceWalk slice_walk(int nslices)
{
    constexpr int per = kBlock / 64;
    const int ngroups = (nslices + per - 1) / per;
    const int nb = gridDim.x, b = blockIdx.x;
    const int nx = nb < kNumXcd ? nb : kNumXcd;           // XCDs that hold blocks
    const int q = nb / nx, rem = nb % nx;
    const int x = b % nx, i = b / nx;
    const int bx = q + (x < rem ? 1 : 0);                 // blocks on this XCD (>= 1)
    const int64_t before = (int64_t)x * q + (x < rem ? x : rem);
    SliceWalk w;                                          // groups in proportion to blocks
    w.g = (int)(before * ngroups / nb) + i;
    w.g_end = (int)((before + bx) * ngroups / nb);
    w.step = bx;
    return w;
}

}  // namespace mpcg

// Exact sums of products on the device: every inner product of the library is the
// double nearest the exact sum (exact products through fma, double-double
// accumulation, one rounding), so any summation order gives the same double.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ftk {

// Exact-sum helpers: a sum of exact products carried as an unevaluated pair
// (hi, lo), rounded once at the end.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    double t = a + b;
    double bb = t - a;
    e = (a - (t - bb)) + (b - bb);
    s = t;
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e)
{
    double t = a + b;
    e = b - (t - a);
    s = t;
}

__device__ __forceinline__ void dd_add(double &hi, double &lo, double x)
{
    double s, e;
    two_sum(hi, x, s, e);
    e = e + lo;
    fast_two_sum(s, e, hi, lo);
}

__device__ __forceinline__ void dd_add_dd(double &hi, double &lo, double bh, double bl)
{
    double s, e, t, f;
    two_sum(hi, bh, s, e);
    two_sum(lo, bl, t, f);
    e = e + t;
    fast_two_sum(s, e, s, e);
    e = e + f;
    fast_two_sum(s, e, hi, lo);
}

// adds a*b exactly: the rounded product goes to (hi, lo), its error to err
__device__ __forceinline__ void acc_prod(double &hi, double &lo, double &err, double a, double b)
{
    double p = a * b;
    err = err + fma(a, b, -p);
    dd_add(hi, lo, p);
}

// Block-wide reduction of (hi, lo) pairs in a fixed order; result in thread 0.
template <int BLOCK>
__device__ __forceinline__ void block_reduce_dd(double &hi, double &lo)
{
    __shared__ double sh[BLOCK / 64][2];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double oh = __shfl_xor(hi, off, 64);
        double ol = __shfl_xor(lo, off, 64);
        dd_add_dd(hi, lo, oh, ol);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        sh[wave][0] = hi;
        sh[wave][1] = lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        hi = sh[0][0];
        lo = sh[0][1];
        for (int w = 1; w < BLOCK / 64; ++w) dd_add_dd(hi, lo, sh[w][0], sh[w][1]);
    }
}

// Sum of nparts (hi, lo) partials, rounded; valid in thread 0 (block of kBlock).
template <int BLOCK = kBlock>
__device__ __forceinline__ double reduce_partials(const double *partials, int nparts)
{
    double hi = 0.0, lo = 0.0;
    for (int i = threadIdx.x; i < nparts; i += BLOCK) dd_add_dd(hi, lo, partials[2 * i], partials[2 * i + 1]);
    block_reduce_dd<BLOCK>(hi, lo);
    return hi + lo;
}

template <int BLOCK>
__device__ __forceinline__ void write_partial(double *partials, double hi, double lo, double err)
{
    dd_add(hi, lo, err);
    block_reduce_dd<BLOCK>(hi, lo);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = hi;
        partials[2 * blockIdx.x + 1] = lo;
    }
}

}  // namespace ftk

// Reductions after the trajectory kernels, shared by the plain and batched paths.
#pragma once

#include "nh_device.h"

namespace nh {

// Momentum-space quadrature at radius k by one 256-thread block
// (Eqs. density_integral and localdensity with the background density that
// follows them): out[k] = sum_jl W_jl f0(y_j ratio_kjl) / sum_jl W_jl f0(y_j),
// W_jl = w_y,j w_mu,l.  Fixed summation order: thread-strided partial sums,
// then a tree in LDS.
__device__ __forceinline__ void reduce_radius(const TrajParams &P, const GridPtrs &g,
                                              const double *__restrict__ ratio, int k,
                                              double *__restrict__ out)
{
    const long long ne = (long long)P.n_y * P.n_mu;
    double num = 0.0, den = 0.0;
    const double *rk = ratio + (size_t)k * ne;
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) {
        const int j = (int)(e / P.n_mu);
        const int l = (int)(e - (long long)j * P.n_mu);
        const double W = g.wy[j] * g.wmu[l];
        const double yj = g.y[j];
        num += W * f0_eval(g.f0, yj * rk[e]);
        den += W * f0_eval(g.f0, yj);
    }
    __shared__ double sn[256], sd[256];
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sn[threadIdx.x] += sn[threadIdx.x + s];
            sd[threadIdx.x] += sd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sn[0] / sd[0];
}

// Integer statistics of trajectories t = first, first + step, ... < n (exact
// under any summation order), added into
// stats = [accepted, rejected, max(acc+rej), failed, fp64 attempts, free exits].
// Called by every thread of a block of at most 1024 threads.
__device__ __forceinline__ void reduce_stats_range(const TrajStat *__restrict__ stat, long long first,
                                                   long long n, long long step, unsigned long long *stats)
{
    unsigned long long acc = 0, rej = 0, mx = 0, fail = 0, f64 = 0, fre = 0;
    for (long long t = first; t < n; t += step) {
        const TrajStat ts = stat[t];
        const unsigned long long a = (unsigned)ts.acc, r = (unsigned)ts.rej;
        acc += a;
        rej += r;
        mx = a + r > mx ? a + r : mx;
        fail += (ts.status & 0xff) != ST_OK;
        fre += (ts.status & ST_FREE_EXIT) != 0;
        f64 += (unsigned)ts.fp64;
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_down(acc, off);
        rej += __shfl_down(rej, off);
        const unsigned long long m2 = __shfl_down(mx, off);
        mx = m2 > mx ? m2 : mx;
        fail += __shfl_down(fail, off);
        f64 += __shfl_down(f64, off);
        fre += __shfl_down(fre, off);
    }
    // then across the block's waves in LDS, so that one set of atomics per
    // block (not per wave) meets the same six counters
    __shared__ unsigned long long part[16][6];
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (__lane_id() == 0) {
        part[w][0] = acc;
        part[w][1] = rej;
        part[w][2] = mx;
        part[w][3] = fail;
        part[w][4] = f64;
        part[w][5] = fre;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int c = threadIdx.x;
        unsigned long long v = part[0][c];
        for (int i = 1; i < nw; ++i) v = (c == 2) ? (part[i][c] > v ? part[i][c] : v) : v + part[i][c];
        if (c == 2) atomicMax(stats + c, v);
        else atomicAdd(stats + c, v);
    }
}

}  // namespace nh

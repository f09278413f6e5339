// The momentum-space quadrature (Eqs. density_integral and localdensity with
// the background density that follows them):
//   n/nbar_k = sum_jl W_jl f0(y_j ratio_kjl) / sum_jl W_jl f0(y_j),
// W_jl = w_y,j w_mu,l, shared by the trajectory kernels' epilogue (fused
// quadrature), the reduction over stored ratios and the batched forms.
//
// The sums are exact.  Every term is scaled by a power of two (so that the
// background sum lies in [1, 2)) and converted to a 128-bit fixed-point number
// with 96 fraction bits; the additions are then integer additions, which are
// associative, so a profile does not depend on the order of its terms: the
// fused epilogue (terms added by atomics as trajectories finish) and the
// reduction over stored ratios give the same bits, for any launch shape or
// queue order.  Terms of at least 2^-44 of the background sum convert exactly,
// smaller ones lose less than 2^-96 of it each; the integer part holds 32 bits
// (n/nbar < 4e9).  The converted sum is rounded to FP64 once.
#pragma once

#include "nh_device.h"

namespace nh {

// 128-bit unsigned fixed point: value = (hi 2^64 + lo) 2^-96.
struct Fix128 {
    unsigned long long lo, hi;
};

__device__ __forceinline__ Fix128 to_fix(double c)
{
    const double t = c * 4294967296.0;                       // c 2^32, exact
    const unsigned long long hi = (unsigned long long)t;     // floor
    const double r = t - (double)hi;                          // exact, in [0, 1)
    return Fix128{(unsigned long long)(r * 18446744073709551616.0), hi};
}

__device__ __forceinline__ void fix_add(Fix128 &a, const Fix128 &b)
{
    const unsigned long long lo = a.lo + b.lo;
    a.hi += b.hi + (lo < a.lo ? 1ull : 0ull);
    a.lo = lo;
}

// Atomic a += b on two consecutive words (lo, hi): the carry out of lo is added
// to hi by the thread that caused it, so the final pair is exact whatever the
// interleaving.
__device__ __forceinline__ void fix_atomic_add(unsigned long long *a, const Fix128 &b)
{
    const unsigned long long old = atomicAdd(a, b.lo);
    const unsigned long long carry = (old + b.lo < old) ? 1ull : 0ull;
    if (b.hi + carry) atomicAdd(a + 1, b.hi + carry);
}

__device__ __forceinline__ double fix_to_double(const Fix128 &a)
{
    return (double)a.hi * 2.3283064365386963e-10 + (double)a.lo * 1.2621774483536189e-29;   // 2^-32, 2^-96
}

// Term (j, l) of the sums for speed ratio P_i/P0: W_jl f0(y_j ratio), scaled.
__device__ __forceinline__ double quad_term(const GridPtrs &g, int j, int l, double ratio, double scale)
{
    const double W = g.wy[j] * g.wmu[l];
    const double f = f0_eval(g.f0, g.y[j] * ratio);
    return (W * f) * scale;
}

// The power of two that brings the background sum into [1, 2), from an FP64
// sum in a fixed order by one 256-thread block (every block and kernel that
// calls it gets the same value).  Called by all threads of the block.
__device__ __forceinline__ double quad_scale(const TrajParams &P, const GridPtrs &g)
{
    const long long ne = (long long)P.n_y * P.n_mu;
    double den = 0.0;
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) {
        const int j = (int)(e / P.n_mu);
        const int l = (int)(e - (long long)j * P.n_mu);
        den += quad_term(g, j, l, 1.0, 1.0);
    }
    __shared__ double sd[256];
    sd[threadIdx.x] = den;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sd[threadIdx.x] += sd[threadIdx.x + s];
        __syncthreads();
    }
    const double d = sd[0];
    __syncthreads();
    return d > 0.0 ? __builtin_amdgcn_ldexp(1.0, -__builtin_amdgcn_frexp_exp(d) + 1) : 1.0;
}

// Exact sum over the block's threads (256) of per-thread fixed-point values;
// the result is valid in thread 0.
__device__ __forceinline__ Fix128 block_fix_sum(Fix128 v)
{
    __shared__ unsigned long long slo[256], shi[256];
    slo[threadIdx.x] = v.lo;
    shi[threadIdx.x] = v.hi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            Fix128 a{slo[threadIdx.x], shi[threadIdx.x]};
            fix_add(a, Fix128{slo[threadIdx.x + s], shi[threadIdx.x + s]});
            slo[threadIdx.x] = a.lo;
            shi[threadIdx.x] = a.hi;
        }
        __syncthreads();
    }
    const Fix128 r{slo[0], shi[0]};
    __syncthreads();
    return r;
}

// The background sum, exactly, by one 256-thread block (valid in thread 0).
__device__ __forceinline__ Fix128 quad_den(const TrajParams &P, const GridPtrs &g, double scale)
{
    const long long ne = (long long)P.n_y * P.n_mu;
    Fix128 den{0ull, 0ull};
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) {
        const int j = (int)(e / P.n_mu);
        const int l = (int)(e - (long long)j * P.n_mu);
        fix_add(den, to_fix(quad_term(g, j, l, 1.0, scale)));
    }
    return block_fix_sum(den);
}

// n/nbar at radius k from the stored ratios, by one 256-thread block.
__device__ __forceinline__ void reduce_radius(const TrajParams &P, const GridPtrs &g,
                                              const double *__restrict__ ratio, int k,
                                              double *__restrict__ out)
{
    const double scale = quad_scale(P, g);
    const long long ne = (long long)P.n_y * P.n_mu;
    const double *rk = ratio + (size_t)k * ne;
    Fix128 num{0ull, 0ull};
    for (long long e = threadIdx.x; e < ne; e += blockDim.x) {
        const int j = (int)(e / P.n_mu);
        const int l = (int)(e - (long long)j * P.n_mu);
        fix_add(num, to_fix(quad_term(g, j, l, rk[e], scale)));
    }
    const Fix128 n = block_fix_sum(num);
    const Fix128 d = quad_den(P, g, scale);
    if (threadIdx.x == 0) out[k] = fix_to_double(n) / fix_to_double(d);
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

// ---------------------------------------------------------------------------
// fused quadrature: the trajectory kernels add each finished trajectory's term
// and statistics directly, with no per-trajectory output
// ---------------------------------------------------------------------------

// Workgroup statistics in LDS, flushed to the global counters once at the end.
struct BlockStats {
    unsigned long long acc, rej, mx, fail, f64, fre;
};

__device__ __forceinline__ void block_stats_init(BlockStats &b)
{
    if (threadIdx.x == 0) b = BlockStats{0, 0, 0, 0, 0, 0};
}

// The fused kernels' LDS partial sums start at this byte offset after a table
// of the given size; a launch holds at most QUAD_LDS_LIMIT bytes of dynamic LDS
// (160 KiB per workgroup on gfx950, less room for the kernels' static LDS).
constexpr size_t QUAD_LDS_LIMIT = 160 * 1024 - 1024;
__host__ __device__ constexpr size_t quad_lds_offset(size_t table_bytes)
{
    return (table_bytes + 15) & ~(size_t)15;
}

// The same on a workgroup's LDS copy (no other workgroup touches it).
__device__ __forceinline__ void fix_lds_add(unsigned long long *a, const Fix128 &b)
{
    const unsigned long long old = __hip_atomic_fetch_add(a, b.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const unsigned long long c = b.hi + ((old + b.lo < old) ? 1ull : 0ull);
    if (c) __hip_atomic_fetch_add(a + 1, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Workgroup partial sums of radii 0 .. q.lds_n-1: (lo, hi) pairs in LDS,
// cleared before the workgroup's first trajectory (then a barrier) and added
// to the global sums once after its last (after a barrier).  An LDS atomic
// returns in far fewer cycles than a device-scope one, and the lane that
// finishes a trajectory waits for it (the carry).
__device__ __forceinline__ void quad_lds_init(unsigned long long *lacc, int n)
{
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) lacc[i] = 0ull;
}

__device__ __forceinline__ void quad_lds_flush(const QuadAcc &q, const unsigned long long *lacc)
{
    for (int k = threadIdx.x; k < q.lds_n; k += blockDim.x) {
        const Fix128 v{lacc[2 * k], lacc[2 * k + 1]};
        if (v.lo | v.hi) fix_atomic_add(q.num + 2 * (size_t)k, v);
    }
}

// A finished trajectory (radius k, momentum j, angle l): its quadrature term
// into radius k's sum (the workgroup's LDS partial when there is one), its
// statistics into the workgroup's.
__device__ __forceinline__ void fused_finish_ix(const GridPtrs &g, const QuadAcc &q, unsigned long long *lacc,
                                                BlockStats &b, const TrajIdx &ix, double ratio, const TrajStat &ts)
{
    const int l = ix.l, j = ix.j, k = ix.k;
    const Fix128 v = to_fix(quad_term(g, j, l, ratio, *q.scale));
    if (k < q.lds_n) fix_lds_add(lacc + 2 * k, v);
    else fix_atomic_add(q.num + 2 * (size_t)k, v);
    const unsigned long long a = (unsigned)ts.acc, r = (unsigned)ts.rej;
    __hip_atomic_fetch_add(&b.acc, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(&b.rej, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_max(&b.mx, a + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if ((ts.status & 0xff) != ST_OK) __hip_atomic_fetch_add(&b.fail, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (ts.fp64) __hip_atomic_fetch_add(&b.f64, (unsigned long long)(unsigned)ts.fp64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (ts.status & ST_FREE_EXIT) __hip_atomic_fetch_add(&b.fre, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The same for trajectory t = (k n_y + j) n_mu + l.
__device__ __forceinline__ void fused_finish(const TrajParams &P, const GridPtrs &g, const QuadAcc &q,
                                             unsigned long long *lacc, BlockStats &b, long long t, double ratio,
                                             const TrajStat &ts)
{
    fused_finish_ix(g, q, lacc, b, traj_idx(t, P), ratio, ts);
}

// Finished trajectories of a fused launch wait in their wavefront's ring in
// LDS: 64 records in parallel arrays, the final speed squared, the trajectory
// index with the status word from bit 48, the accepted and rejected step
// counts and (N64, the FP32C form) the FP64 attempt count.  When the next
// finishers would overflow it, the whole wavefront sums the ring at once, one
// record a lane (the speed ratio, the quadrature term, the fixed-point add and
// the statistics), instead of running that code with the one or two lanes
// that finish in a pass.  The sums are exact, so the order changes no result.
// A launch of 2^48 or more trajectories sums each finisher at once.
template <bool N64>
struct FinishRing {
    static constexpr int SLOTS = 64;
    static constexpr int ENTRY = N64 ? 28 : 24;   // bytes a record
    double *n2;
    long long *tw;
    uint2 *st;
    unsigned *n64;

    __device__ __forceinline__ static FinishRing of(char *base)
    {
        char *b = base + (threadIdx.x >> 6) * (SLOTS * ENTRY);
        return FinishRing{(double *)b, (long long *)(b + SLOTS * 8), (uint2 *)(b + SLOTS * 16),
                          (unsigned *)(b + SLOTS * 24)};
    }

    // Records i < n, record i by lane i.  The speed ratio repeats the
    // arithmetic of the trajectory's start (the initial speed from the grid)
    // and of its end, so it is the value an immediate finish would compute.
    __device__ __forceinline__ void flush(unsigned n, const TrajParams &P, const GridPtrs &g, const QuadAcc &qa,
                                          unsigned long long *lacc, BlockStats &bst) const
    {
        const unsigned i = __lane_id();
        if (i < n) {
            const long long w = tw[i];
            const uint2 c = st[i];
            const TrajIdx ix = traj_idx(w & ((1ll << 48) - 1), P);
            const double V = g.y[ix.j] * P.vfac;
            const double v0n = sqrt(norm2(V * g.mu[ix.l], V * g.smu[ix.l]));
            const double ratio = sqrt(n2[i]) / v0n;
            fused_finish_ix(g, qa, lacc, bst, ix, ratio,
                            TrajStat{(int)c.x, (int)c.y, (int)(w >> 48), N64 ? (int)n64[i] : 0});
        }
    }

    // Called by every lane of the wavefront: the lanes with `fin` set put
    // their trajectory t in the ring (after a flush if it would overflow);
    // nfin, the ring's fill, is wave-uniform.  Returns whether this lane's
    // trajectory went in.
    __device__ __forceinline__ bool put(bool fin, unsigned &nfin, long long t, int status, int acc, int rej, int f64,
                                        double speed2, const TrajParams &P, const GridPtrs &g, const QuadAcc &qa,
                                        unsigned long long *lacc, BlockStats &bst) const
    {
        const unsigned long long fm = __ballot(fin);
        if (fm == 0ull) return false;
        const unsigned nf = (unsigned)__popcll(fm);
        if (nfin + nf > (unsigned)SLOTS) {
            flush(nfin, P, g, qa, lacc, bst);
            nfin = 0;
        }
        if (fin) {
            const unsigned slot =
                nfin + __builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
            n2[slot] = speed2;
            tw[slot] = t | ((long long)status << 48);
            st[slot] = make_uint2((unsigned)acc, (unsigned)rej);
            if constexpr (N64) n64[slot] = (unsigned)f64;
        }
        nfin += nf;
        return fin;
    }
};

// After the workgroup's last trajectory (all threads, after a barrier).
__device__ __forceinline__ void block_stats_flush(const BlockStats &b, unsigned long long *stats)
{
    if (threadIdx.x == 0) {
        atomicAdd(stats + 0, b.acc);
        atomicAdd(stats + 1, b.rej);
        atomicMax(stats + 2, b.mx);
        atomicAdd(stats + 3, b.fail);
        atomicAdd(stats + 4, b.f64);
        atomicAdd(stats + 5, b.fre);
    }
}

}  // namespace nh

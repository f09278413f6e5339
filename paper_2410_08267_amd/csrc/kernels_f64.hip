// FP64 trajectory kernels and the profile reduction.
//
// One wavefront lane integrates one relic trajectory backward in u = ln a
// (Sec. II.C) through the halo's force (Sec. II.B, App. A).  Nothing here is a
// dense contraction, so there is no MFMA: the work is FP64 VALU arithmetic on
// register-resident state, with the u-dependent coefficients either read as
// wave-uniform scalars (RK4: every lane sits at the same u) or interpolated
// from an LDS copy of the FP64 table (Dormand-Prince: every lane has its own u).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "nh_dp5.h"
#include "nh_reduce.h"

namespace nh {

// (Dormand-Prince tableau and step: nh_dp5.h)

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------

__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// No halo: the force vanishes everywhere, so every velocity is unchanged.
// Grid-stride: the grid is capped, n may exceed 2^32.
__global__ void k_free_all(long long n, TrajOut o)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        o.ratio[t] = 1.0;
        o.stat[t] = TrajStat{0, 0, ST_OK | ST_FREE_EXIT, 0};
    }
}

// Capped grids for the one-thread-per-item kernels (the dispatch size is 32-bit).
constexpr long long MAX_BLOCKS = 1ll << 20;
static unsigned capped_blocks(long long n, int block)
{
    long long b = (n + block - 1) / block;
    if (b > MAX_BLOCKS) b = MAX_BLOCKS;
    return (unsigned)(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------------------
// classical RK4, n_steps equal steps; all lanes share u
// ---------------------------------------------------------------------------

// One trajectory t (a lane past the end, t >= n_traj, only keeps its wave company).
template <bool FUSED>
__device__ __forceinline__ void rk4_one(const TrajParams &P, const GridPtrs &g, const TrajOut &o, long long t,
                                        const QuadAcc &qa, BlockStats &bst)
{
    const bool valid = t < P.n_traj;
    double x = 0.0, y = 0.0, vx = 0.0, vy = 0.0, v0n = 1.0;
    if (valid) {
        const TrajIdx ix = traj_idx(t, P);
        const int l = ix.l, j = ix.j, k = ix.k;
        const double V = g.y[j] * P.vfac;
        x = g.r[k];
        vx = V * g.mu[l];
        vy = V * g.smu[l];
        v0n = sqrt(norm2(vx, vy));
    }
    const double r_exit2 = P.r_exit * P.r_exit;
    // App. B cull: a path that never reaches R needs no steps
    const bool culled = valid && P.cull_D > 0.0 && never_enters(x, vx, vy, P.cull_D, cull_radius2(P.r_exit));
    bool active = valid && !culled;
    bool freed = culled;
    int steps = 0;
    const double h = P.rk_h;
    const double hh = 0.5 * h;
    for (int n = 0; n < P.n_steps; ++n) {
        if (__ballot(active) == 0ull) break;
        const double *c0 = g.tab + (size_t)(2 * n) * NCOL;    // wave-uniform rows
        double ca[NCOL], cb[NCOL], cc[NCOL];
#pragma unroll
        for (int q = 0; q < NCOL; ++q) {
            ca[q] = c0[q];
            cb[q] = c0[NCOL + q];
            cc[q] = c0[2 * NCOL + q];
        }
        double k1x, k1y, k1u, k1v, k2x, k2y, k2u, k2v, k3x, k3y, k3u, k3v, k4x, k4y, k4u, k4v;
        rhs(ca, ca[COL_R], x, y, vx, vy, k1x, k1y, k1u, k1v);
        rhs(cb, cb[COL_R], x + hh * k1x, y + hh * k1y, vx + hh * k1u, vy + hh * k1v, k2x, k2y, k2u, k2v);
        rhs(cb, cb[COL_R], x + hh * k2x, y + hh * k2y, vx + hh * k2u, vy + hh * k2v, k3x, k3y, k3u, k3v);
        rhs(cc, cc[COL_R], x + h * k3x, y + h * k3y, vx + h * k3u, vy + h * k3v, k4x, k4y, k4u, k4v);
        const double h6 = h / 6.0;
        if (active) {
            x = x + h6 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
            y = y + h6 * (k1y + 2.0 * k2y + 2.0 * k3y + k4y);
            vx = vx + h6 * (k1u + 2.0 * k2u + 2.0 * k3u + k4u);
            vy = vy + h6 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
            ++steps;
            if (P.r_exit > 0.0 && x * x + y * y >= r_exit2 && x * vx + y * vy <= 0.0) {
                active = false;
                freed = true;
            }
        }
    }
    if (valid) {
        const double ratio = sqrt(norm2(vx, vy)) / v0n;
        int st = ST_OK;
        if (!(isfinite(x) && isfinite(y) && isfinite(vx) && isfinite(vy))) st = ST_NONFINITE;
        const TrajStat ts{steps, 0, st | (freed ? ST_FREE_EXIT : 0), 0};
        if constexpr (FUSED) {
            fused_finish(P, g, qa, nullptr, bst, t, ratio, ts);
        } else {
            o.ratio[t] = ratio;
            o.stat[t] = ts;
        }
    }
}

template <bool FUSED>
__global__ __launch_bounds__(256) void k_rk4_f64(TrajParams P, GridPtrs g, TrajOut o, QuadAcc qa)
{
    __shared__ BlockStats bst;
    if constexpr (FUSED) {
        block_stats_init(bst);
        __syncthreads();
    }
    // grid-stride over wave-aligned chunks (the grid is capped)
    for (long long base = (long long)blockIdx.x * blockDim.x; base < P.n_traj;
         base += (long long)gridDim.x * blockDim.x)
        rk4_one<FUSED>(P, g, o, base + threadIdx.x, qa, bst);
    if constexpr (FUSED) {
        __syncthreads();
        block_stats_flush(bst, qa.stats);
    }
}


// ---------------------------------------------------------------------------
// Dormand-Prince 5(4), adaptive; persistent waves refill lanes from a queue
// ---------------------------------------------------------------------------

// One block per CU: the table takes most of the LDS.  The kernel fits 128
// VGPRs, so blocks of up to 1024 threads (four waves per SIMD) are possible;
// 768 (three waves per SIMD) is the default: a single profile has ~1e6
// trajectories, and more lanes per profile lengthen the tail where the last
// long trajectories run alone.  The autotuner picks per workload.
constexpr int DP5_MAX_BLOCK = 1024;
constexpr int DP5_DEFAULT_BLOCK = 768;
constexpr int START_RADII = 256;   // radii whose start force a workgroup keeps in LDS

// CULL: some start radius lies beyond R_exit.  Without one no relic can be
// culled, and the kernel leaves the test out: its branch alone costs the
// trajectory loop a few percent in register moves.
// FUSED: each finished trajectory adds its quadrature term and statistics
// directly (QuadAcc); nothing is written per trajectory.
// The table: K, Kc, 1/s and c in LDS (TabCoefSplit), the drift column A from
// g.tabA; R, constant or not, is not needed by the right-hand side.
template <bool CULL, bool HIST, bool FUSED>
__global__ __launch_bounds__(DP5_MAX_BLOCK) void k_dp5_f64(TrajParams P, GridPtrs g, TrajOut o,
                                                           unsigned long long *counter, QuadAcc qa)
{
    extern __shared__ double lds_tab[];
    __shared__ BlockStats bst;
    // the wavefronts' rings (when on) and the workgroup's partial sums follow the table
    char *const ring_base = (char *)lds_tab + quad_lds_offset((size_t)P.n_tab * SPLIT_ROW * sizeof(double));
    unsigned long long *const lacc =
        (unsigned long long *)(ring_base + (FUSED && qa.ring ? blockDim.x * FinishRing<false>::ENTRY : 0));
    const FinishRing<false> R = FinishRing<false>::of(ring_base);
    const bool ring = FUSED && qa.ring;
    if constexpr (FUSED) {
        block_stats_init(bst);
        quad_lds_init(lacc, qa.lds_n);
    }
    // stage K, Kc, 1/s and c of every node into rows of SPLIT_ROW doubles
    for (int i = threadIdx.x; i < P.n_tab * 4; i += blockDim.x) {
        const int node = i >> 2, col = i & 3;
        lds_tab[node * SPLIT_ROW + col] = g.tab[node * NCOL + COL_K + col];
    }
    __syncthreads();

    const TabCoefSplit<HIST> cf{lds_tab, g.tabA, P.n_tab, P.tab_u0, P.tab_inv_du, P.R_const, P.pw, P.kn};
    __shared__ StartCache sc;
    start_cache_fill(sc, cf, P.h0, P.u_start, P.u_end);
    __syncthreads();
    // the first stage's force at the common start depends on the radius
    // alone: once per radius here (the first START_RADII radii), instead of a
    // right-hand side with one or two lanes active at every trajectory start
    __shared__ double g0s[START_RADII];
    const int n_g0 = min(P.n_r, START_RADII);
    for (int k = threadIdx.x; k < n_g0; k += blockDim.x) g0s[k] = start_g(sc, g.r[k]);
    __syncthreads();
    DpCtl ctl;
    ctl.u_end = P.u_end;
    ctl.rtol = P.rtol;
    ctl.atol_x = P.atol_x;
    ctl.atol_v = P.atol_v;
    ctl.r_exit2 = P.r_exit2;
    ctl.max_steps = (int)P.max_steps;

    long long t = -1;          // -1: wants work, -2: queue drained, >= 0: trajectory
    double v0n = 1.0;
    Lane64 L{};
    WaveQueue wq{0ull, 0ull};
    unsigned nfin = 0;         // records in the wavefront's ring
    for (;;) {
        const bool need = (t == -1);
        const long long p = wave_claim(need, counter, wq);
        if (need) {
            if (p < P.n_traj) {
                t = traj_of(p, P);
                const TrajIdx ix = traj_idx(t, P);
                const int l = ix.l, j = ix.j, k = ix.k;
                const double V = g.y[j] * P.vfac;
                const double vx0 = V * g.mu[l], vy0 = V * g.smu[l];
                if (!ring) v0n = sqrt(norm2(vx0, vy0));
                if (CULL && never_enters(g.r[k], vx0, vy0, P.cull_D, cull_radius2(P.r_exit))) {
                    // App. B cull: the path never reaches R, the momentum is final
                    const TrajStat ts{0, 0, ST_OK | ST_FREE_EXIT, 0};
                    if constexpr (FUSED) {
                        fused_finish_ix(g, qa, lacc, bst, ix, 1.0, ts);
                    } else {
                        o.ratio[t] = 1.0;
                        o.stat[t] = ts;
                    }
                    t = -1;
                } else {
                    if (k < START_RADII) dp5_start_g(L, sc, g0s[k], g.r[k], vx0, vy0, P.u_start);
                    else dp5_start_cached(L, sc, g.r[k], vx0, vy0, P.u_start);
                }
            } else {
                t = -2;
            }
        }
        // leave once every lane found the queue drained; lanes whose new
        // trajectory was culled (t == -1) claim again on the next pass
        if (__ballot(t != -2) == 0ull) break;
        int st = -1;
        if (t >= 0) {
            st = dp5_attempt(L, cf, ctl);
            if (st >= 0 && !ring) {
                const double ratio = sqrt(norm2(L.vx, L.vy)) / v0n;
                const TrajStat ts{L.nacc, L.nrej, st, 0};
                if constexpr (FUSED) {
                    fused_finish(P, g, qa, lacc, bst, t, ratio, ts);
                } else {
                    o.ratio[t] = ratio;
                    o.stat[t] = ts;
                }
                t = -1;
            }
        }
        if (ring && R.put(t >= 0 && st >= 0, nfin, t, st, L.nacc, L.nrej, 0, norm2(L.vx, L.vy), P, g, qa, lacc, bst))
            t = -1;
    }
    if constexpr (FUSED) {
        if (ring && nfin) R.flush(nfin, P, g, qa, lacc, bst);
        __syncthreads();
        block_stats_flush(bst, qa.stats);
        quad_lds_flush(qa, lacc);
    }
}

// Fused quadrature, before the trajectories: the power-of-two scale of the
// sums, the exact background sum, and cleared radius sums and statistics
// (one 256-thread block; a kernel rather than memsets, so that a captured
// sequence replays correctly).
__global__ __launch_bounds__(256) void k_quad_setup(TrajParams P, GridPtrs g, QuadAcc qa)
{
    for (long long i = threadIdx.x; i < 2 * (long long)P.n_r; i += blockDim.x) qa.num[i] = 0ull;
    if (threadIdx.x < 6) qa.stats[threadIdx.x] = 0ull;
    const double scale = quad_scale(P, g);
    const Fix128 den = quad_den(P, g, scale);
    if (threadIdx.x == 0) {
        *qa.scale = scale;
        qa.den[0] = den.lo;
        qa.den[1] = den.hi;
    }
}

// Fused quadrature, after the trajectories: n/nbar_k = num_k / den.  With no
// halo every term equals its background term, so num_k = den: exactly 1.
__global__ __launch_bounds__(256) void k_quad_finish(int n_r, QuadAcc qa, int free_all, double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_r) return;
    const Fix128 den{qa.den[0], qa.den[1]};
    const Fix128 num = free_all ? den : Fix128{qa.num[2 * (size_t)k], qa.num[2 * (size_t)k + 1]};
    out[k] = fix_to_double(num) / fix_to_double(den);
}

// ---------------------------------------------------------------------------
// momentum-space quadrature: n/nbar_k = sum W f(y_j ratio) / sum W f(y_j)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_reduce_profile(TrajParams P, GridPtrs g,
                                                        const double *__restrict__ ratio,
                                                        double *__restrict__ out)
{
    reduce_radius(P, g, ratio, blockIdx.x, out);
}

// Angle-integrated distribution at every radius and momentum node (the
// integrand of Eq. localdensity before the momentum sum):
//   out[k n_y + j] = sum_l w_mu,l f0(y_j ratio_kjl), l in index order.
__global__ __launch_bounds__(256) void k_reduce_integrand(TrajParams P, GridPtrs g,
                                                          const double *__restrict__ ratio,
                                                          double *__restrict__ out)
{
    const long long n = (long long)P.n_r * P.n_y;
    for (long long kj = (long long)blockIdx.x * blockDim.x + threadIdx.x; kj < n;
         kj += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(kj % P.n_y);
        const double yj = g.y[j];
        const double *rk = ratio + kj * P.n_mu;
        double acc = 0.0;
        for (int l = 0; l < P.n_mu; ++l) acc += g.wmu[l] * f0_eval(g.f0, yj * rk[l]);
        out[kj] = acc;
    }
}

// Several masses from the same ratios: block (mass, radius) uses that mass's
// momentum grid and weights.
__global__ __launch_bounds__(256) void k_reduce_masses(TrajParams P, GridPtrs g,
                                                       const double *__restrict__ ratio,
                                                       const double *__restrict__ ym,
                                                       const double *__restrict__ wm,
                                                       double *__restrict__ out)
{
    const int im = blockIdx.y, k = blockIdx.x;
    GridPtrs gm = g;
    gm.y = ym + (size_t)im * P.n_y;
    gm.wy = wm + (size_t)im * P.n_y;
    reduce_radius(P, gm, ratio, k, out + (size_t)im * P.n_r);
}

// Integer statistics (exact under any summation order).
// stats: [accepted, rejected, max(acc+rej), failed, fp64 steps, free exits]
__global__ __launch_bounds__(256) void k_reduce_stats(long long n, TrajOut o,
                                                      unsigned long long *stats)
{
    reduce_stats_range(o.stat, (long long)blockIdx.x * blockDim.x + threadIdx.x, n,
                       (long long)gridDim.x * blockDim.x, stats);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

const void *fill_u64_kernel() { return (const void *)k_fill_u64; }

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_free_all(long long n, const TrajOut &o, hipStream_t s)
{
    hipLaunchKernelGGL(k_free_all, dim3(capped_blocks(n, 256)), dim3(256), 0, s, n, o);
    return hipGetLastError();
}

hipError_t launch_rk4_f64(const TrajParams &P, const GridPtrs &g, const TrajOut &o, const QuadAcc *qa, hipStream_t s)
{
    if (qa)
        hipLaunchKernelGGL(k_rk4_f64<true>, dim3(capped_blocks(P.n_traj, 256)), dim3(256), 0, s, P, g, o, *qa);
    else
        hipLaunchKernelGGL(k_rk4_f64<false>, dim3(capped_blocks(P.n_traj, 256)), dim3(256), 0, s, P, g, o,
                           QuadAcc{});
    return hipGetLastError();
}

// The LDS attribute and the occupancy query cost host time at every launch;
// their answer depends only on the kernel, the block size and the LDS bytes,
// so it is kept per (kernel, block, bytes) in a fixed table (no heap memory:
// the allocation-free entry point launches through here too).
hipError_t occupancy_cached(const void *fn, int block, size_t lds, int *per_cu)
{
    struct Entry {
        const void *fn;
        int block;
        size_t lds;
        int per_cu;
    };
    constexpr int CAP = 256;
    static std::mutex mu;
    static Entry cache[CAP];
    static int n = 0;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < n; ++i)
        if (cache[i].fn == fn && cache[i].block == block && cache[i].lds == lds) {
            *per_cu = cache[i].per_cu;
            return hipSuccess;
        }
    // the attribute is a per-kernel upper bound: never lower it below a size
    // an earlier launch of the same kernel relies on (a kernel seen more often
    // than the table holds keeps the largest size it has been given)
    static struct {
        const void *fn;
        size_t lds;
    } attr_max[CAP];
    static int n_attr = 0;
    size_t attr = lds;
    int slot = -1;
    for (int i = 0; i < n_attr; ++i)
        if (attr_max[i].fn == fn) {
            slot = i;
            attr = std::max(attr, attr_max[i].lds);
        }
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)attr);
    if (e != hipSuccess) return e;
    if (slot < 0 && n_attr < CAP) slot = n_attr++, attr_max[slot].fn = fn;
    if (slot >= 0) attr_max[slot].lds = attr;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, fn, block, lds);
    if (e != hipSuccess) return e;
    if (n < CAP) cache[n++] = Entry{fn, block, lds, *per_cu};
    return hipSuccess;
}

// The fused kernels' per-workgroup partial sums (16 bytes a radius after the
// table) are used when they fit in LDS and keep the occupancy; otherwise the
// terms go straight to the global sums.
hipError_t quad_lds_plan(const void *fn, int block, int per_cu, int n_r, size_t &lds, QuadAcc &q)
{
    q.lds_n = 0;
    const size_t base = quad_lds_offset(lds);
    const size_t with = base + (size_t)n_r * 2 * sizeof(unsigned long long);
    if (n_r < 1 || with > QUAD_LDS_LIMIT) return hipSuccess;
    int per_cu2 = 0;
    const hipError_t e = occupancy_cached(fn, block, with, &per_cu2);
    if (e != hipSuccess) return e;
    if (per_cu2 == per_cu) {
        q.lds_n = n_r;
        lds = with;
    }
    return hipSuccess;
}

template <bool CULL, bool HIST, bool FUSED>
static hipError_t launch_dp5_k(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                               unsigned long long *counter, const QuadAcc &qa, int n_cu, hipStream_t s)
{
    const int B = P.block > 0 ? P.block : DP5_DEFAULT_BLOCK;
    size_t lds = (size_t)P.n_tab * SPLIT_ROW * sizeof(double);
    int per_cu = 0;
    hipError_t e = occupancy_cached((const void *)k_dp5_f64<CULL, HIST, FUSED>, B, lds, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    QuadAcc q = qa;
    q.ring = 0;
    if (FUSED) {
        // the wavefronts' rings of finished trajectories, when they keep the occupancy
        // (trajectory indices below 2^48: the status word shares their record)
        const size_t with = quad_lds_offset(lds) + (size_t)B * FinishRing<false>::ENTRY;
        int per_cu2 = 0;
        if (with <= QUAD_LDS_LIMIT && P.n_traj < (1ll << 48)) {
            e = occupancy_cached((const void *)k_dp5_f64<CULL, HIST, FUSED>, B, with, &per_cu2);
            if (e != hipSuccess) return e;
            if (per_cu2 == per_cu) {
                q.ring = 1;
                lds = with;
            }
        }
        e = quad_lds_plan((const void *)k_dp5_f64<CULL, HIST, FUSED>, B, per_cu, P.n_r, lds, q);
        if (e != hipSuccess) return e;
    }
    long long grid = (long long)n_cu * per_cu;
    if (P.max_wg > 0 && grid > P.max_wg) grid = P.max_wg;
    const long long need = (P.n_traj + B - 1) / B;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    TrajParams Pk = P;
    Pk.r_exit2 = exit_radius2(P);
    auto *kern = k_dp5_f64<CULL, HIST, FUSED>;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(B), lds, s, Pk, g, o, counter, q);
    return hipGetLastError();
}

template <bool HIST, bool FUSED>
static hipError_t launch_dp5_hist(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                                  unsigned long long *counter, const QuadAcc &qa, int n_cu, hipStream_t s)
{
    return P.cull_D > 0.0 ? launch_dp5_k<true, HIST, FUSED>(P, g, o, counter, qa, n_cu, s)
                          : launch_dp5_k<false, HIST, FUSED>(P, g, o, counter, qa, n_cu, s);
}

hipError_t launch_dp5_f64(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                          unsigned long long *counter, const QuadAcc *qa, int n_cu, hipStream_t s)
{
    const QuadAcc q = qa ? *qa : QuadAcc{};
    if (qa)
        return P.hist ? launch_dp5_hist<true, true>(P, g, o, counter, q, n_cu, s)
                      : launch_dp5_hist<false, true>(P, g, o, counter, q, n_cu, s);
    return P.hist ? launch_dp5_hist<true, false>(P, g, o, counter, q, n_cu, s)
                  : launch_dp5_hist<false, false>(P, g, o, counter, q, n_cu, s);
}

hipError_t launch_quad_setup(const TrajParams &P, const GridPtrs &g, const QuadAcc &qa, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_setup, dim3(1), dim3(256), 0, s, P, g, qa);
    return hipGetLastError();
}

hipError_t launch_quad_finish(int n_r, const QuadAcc &qa, bool free_all, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_quad_finish, dim3((unsigned)((n_r + 255) / 256)), dim3(256), 0, s, n_r, qa,
                       free_all ? 1 : 0, out);
    return hipGetLastError();
}

hipError_t launch_reduce_profile(const TrajParams &P, const GridPtrs &g, const double *ratio,
                                 double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_profile, dim3(P.n_r), dim3(256), 0, s, P, g, ratio, out);
    return hipGetLastError();
}

hipError_t launch_reduce_integrand(const TrajParams &P, const GridPtrs &g, const double *ratio, double *out,
                                   hipStream_t s)
{
    const long long n = (long long)P.n_r * P.n_y;
    hipLaunchKernelGGL(k_reduce_integrand, dim3(capped_blocks(n, 256)), dim3(256), 0, s, P, g, ratio, out);
    return hipGetLastError();
}

hipError_t launch_reduce_masses(const TrajParams &P, const GridPtrs &g, const double *ratio, const double *ym,
                                const double *wm, int n_mass, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_masses, dim3((unsigned)P.n_r, (unsigned)n_mass), dim3(256), 0, s, P, g, ratio, ym,
                       wm, out);
    return hipGetLastError();
}

hipError_t launch_reduce_stats(long long n, const TrajOut &o, unsigned long long *stats,
                               hipStream_t s)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_reduce_stats, dim3((unsigned)blocks), dim3(256), 0, s, n, o, stats);
    return hipGetLastError();
}

}  // namespace nh

namespace nh {

// ---------------------------------------------------------------------------
// FP64 FMA throughput probe: 8 independent chains per lane, no memory traffic
// in the loop; the sum is stored so nothing is dead code.
// ---------------------------------------------------------------------------

constexpr int FMA_PROBE_ITERS = 4096;
constexpr int FMA_PROBE_CHAINS = 8;

__global__ __launch_bounds__(1024) void k_fma_probe(double *out, double seed)
{
    double a[FMA_PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < FMA_PROBE_CHAINS; ++c) a[c] = seed + threadIdx.x * 1e-9 + c;
    const double m = 0.999999999, k = 1e-9;
    for (int it = 0; it < FMA_PROBE_ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < FMA_PROBE_CHAINS; ++c) a[c] = fma(a[c], m, k);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < FMA_PROBE_CHAINS; ++c) s += a[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_fma_probe(double *out, int blocks, hipStream_t s, double *flop)
{
    hipLaunchKernelGGL(k_fma_probe, dim3(blocks), dim3(1024), 0, s, out, 1.0);
    *flop = 2.0 * FMA_PROBE_ITERS * FMA_PROBE_CHAINS * 1024.0 * blocks;
    return hipGetLastError();
}

}  // namespace nh

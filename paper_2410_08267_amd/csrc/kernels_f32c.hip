// FP32-compensated Dormand-Prince kernel (the precision form).
//
// State: positions in FP32 with a Kahan compensation term each (the carried
// rounding error of the accumulated position), velocities in FP32, time u and
// step h in FP64 (u also indexes the coefficient table).  Right-hand sides,
// stage sums, error norm and step control run in FP32.  The coefficient table
// stays FP64 for the H(z)-derived drift and kick columns (interpolated in FP64,
// rounded to FP32 afterwards); the halo's radii and concentration are an FP32
// copy; both sit in LDS.  An attempt whose |h| is below a threshold (the short
// steps the controller takes near pericentre) runs the FP64 step instead, on
// the FP64 table, after re-evaluating the first stage in FP64.  The speed ratio
// and the quadrature downstream stay FP64.  The choice is per lane, so a
// trajectory's result does not depend on which trajectories share its
// wavefront.
#include <hip/hip_runtime.h>

#include "nh_dp5_f32.h"
#include "nh_launch.h"
#include "nh_reduce.h"

namespace nh {

// CULL: some start radius lies beyond R_exit (otherwise no relic can be culled
// and the test is left out of the trajectory loop)
// FUSED: each finished trajectory adds its quadrature term and statistics
// directly (QuadAcc); nothing is written per trajectory.
// WIDE: up to 1024 threads (four waves per SIMD) instead of 768.
template <int NC, bool CULL, bool HIST, bool FUSED, bool WIDE>
__global__ __launch_bounds__(WIDE ? 1024 : 768) void k_dp5_f32c(TrajParams P, GridPtrs g, TrajOut o,
                                                                unsigned long long *counter, QuadAcc qa)
{
    extern __shared__ double lds_mix[];
    __shared__ BlockStats bst;
    // the wavefronts' rings of finished trajectories (when on) and the
    // workgroup's partial sums follow the table
    char *const ring_base = (char *)lds_mix + quad_lds_offset(f32c_table_bytes<NC, true>(P.n_tab));
    unsigned long long *const lacc =
        (unsigned long long *)(ring_base + (FUSED && qa.ring ? blockDim.x * FinishRing<true>::ENTRY : 0));
    const FinishRing<true> R = FinishRing<true>::of(ring_base);
    const bool ring = FUSED && qa.ring;
    if constexpr (FUSED) {
        block_stats_init(bst);
        quad_lds_init(lacc, qa.lds_n);
    }
    stage_f32c_table<NC, true>(lds_mix, g.tab, P.n_tab, threadIdx.x, blockDim.x);
    __syncthreads();

    // The request's coefficient sources and step controls.  WIDE: re-read
    // from the kernel arguments where they are used (scalar loads, kept in
    // place by an index the compiler cannot see through), since held for the
    // whole launch they overflow the scalar registers at four waves per SIMD;
    // otherwise read once (the index is a constant zero and the compiler
    // hoists the reads).
    struct Src {
        TabCoef32<NC, HIST, true> cf;    // K, Kc (FP64) and 1/s, c (FP32) from LDS, A from device memory
        TabCoef<NC, NCOL, HIST> cf64;    // the promoted FP64 steps: the FP64 table in device memory
        DpCtl32 ctl;
        DpCtl ctl64;
        double h_fp64;
    };
    const auto opaque_zero = [&]() {
        int z = 0;
        if constexpr (WIDE) asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        return z;
    };
    const auto src = [&]() {
        const int z = opaque_zero();
        const TrajParams &Pa = (&P)[z];
        const GridPtrs &ga = (&g)[z];
        Src r{{lds_mix, (const float *)(lds_mix + (size_t)Pa.n_tab * f32c_t64<true>), NC, Pa.n_tab, Pa.tab_u0,
               Pa.tab_inv_du, (float)fmin(Pa.R_const, 1.0e30), Pa.pw, Pa.kn, ga.tabA},
              {ga.tab, Pa.n_tab, Pa.tab_u0, Pa.tab_inv_du, Pa.R_const, Pa.pw, Pa.kn}, {}, {}, Pa.h_fp64};
        f32c_controls(Pa, r.ctl, r.ctl64);
        return r;
    };

    long long t = -1;
    double v0n = 1.0;
    Lane32 L{};
    WaveQueue wq{0ull, 0ull};
    unsigned nfin = 0;   // records in the wavefront's ring
    for (;;) {
        const bool need = (t == -1);
        const long long p = wave_claim(need, counter, wq);
        if (need) {
            // WIDE: the claim reads the arguments in place too (see src)
            const int zc = opaque_zero();
            const TrajParams &Pc = (&P)[zc];
            const GridPtrs &gc = (&g)[zc];
            if (p < Pc.n_traj) {
                t = traj_of(p, Pc);
                const TrajIdx ix = traj_idx(t, Pc);
                const int l = ix.l, j = ix.j, k = ix.k;
                const double V = gc.y[j] * Pc.vfac;
                const double vx0 = V * gc.mu[l], vy0 = V * gc.smu[l];
                if (!ring) v0n = sqrt(norm2(vx0, vy0));
                if (CULL && never_enters(gc.r[k], vx0, vy0, Pc.cull_D, cull_radius2(Pc.r_exit))) {
                    // App. B cull: the path never reaches R, the momentum is final
                    const TrajStat ts{0, 0, ST_OK | ST_FREE_EXIT, 0};
                    if constexpr (FUSED) {
                        fused_finish(Pc, gc, qa, lacc, bst, t, 1.0, ts);
                    } else {
                        o.ratio[t] = 1.0;
                        o.stat[t] = ts;
                    }
                    t = -1;
                } else {
                    f32c_start(L, src().cf, gc.r[k], vx0, vy0, Pc.h0, Pc.u_start, Pc.u_end);
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
            const Src a = src();
            st = f32c_attempt(L, a.cf, a.cf64, a.ctl, a.ctl64, a.h_fp64);
            if (st >= 0 && !ring) {
                const double fx = L.vx, fy = L.vy;
                const double ratio = sqrt(norm2(fx, fy)) / v0n;
                const TrajStat ts{L.nacc, L.nrej, st, L.n64};
                if constexpr (FUSED) {
                    const int zf = opaque_zero();
                    fused_finish((&P)[zf], (&g)[zf], qa, lacc, bst, t, ratio, ts);
                } else {
                    o.ratio[t] = ratio;
                    o.stat[t] = ts;
                }
                t = -1;
            }
        }
        if (ring) {
            const int zf = opaque_zero();
            if (R.put(t >= 0 && st >= 0, nfin, t, st, L.nacc, L.nrej, L.n64, norm2((double)L.vx, (double)L.vy),
                      (&P)[zf], (&g)[zf], qa, lacc, bst))
                t = -1;
        }
    }
    if constexpr (FUSED) {
        if (ring && nfin) R.flush(nfin, P, g, qa, lacc, bst);
        __syncthreads();
        block_stats_flush(bst, qa.stats);
        quad_lds_flush(qa, lacc);
    }
}

template <int NC, bool CULL, bool HIST, bool FUSED, bool WIDE>
static hipError_t launch_f32c_w(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                                unsigned long long *counter, const QuadAcc &qa, int n_cu, int B, hipStream_t s)
{
    size_t lds = f32c_table_bytes<NC, true>(P.n_tab);
    int per_cu = 0;
    hipError_t e = occupancy_cached((const void *)k_dp5_f32c<NC, CULL, HIST, FUSED, WIDE>, B, lds, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    QuadAcc q = qa;
    q.ring = 0;
    if (FUSED) {
        // the wavefronts' rings of finished trajectories, when they keep the occupancy
        const size_t with = quad_lds_offset(lds) + (size_t)B * FinishRing<true>::ENTRY;
        int per_cu2 = 0;
        if (with <= QUAD_LDS_LIMIT && P.n_traj < (1ll << 48)) {
            e = occupancy_cached((const void *)k_dp5_f32c<NC, CULL, HIST, FUSED, WIDE>, B, with, &per_cu2);
            if (e != hipSuccess) return e;
            if (per_cu2 == per_cu) {
                q.ring = 1;
                lds = with;
            }
        }
        e = quad_lds_plan((const void *)k_dp5_f32c<NC, CULL, HIST, FUSED, WIDE>, B, per_cu, P.n_r, lds, q);
        if (e != hipSuccess) return e;
    }
    long long grid = (long long)n_cu * per_cu;
    if (P.max_wg > 0 && grid > P.max_wg) grid = P.max_wg;
    const long long need = (P.n_traj + B - 1) / B;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    TrajParams Pk = P;
    Pk.r_exit2 = exit_radius2(P);
    auto *kern = k_dp5_f32c<NC, CULL, HIST, FUSED, WIDE>;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(B), lds, s, Pk, g, o, counter, q);
    return hipGetLastError();
}

template <int NC, bool CULL, bool HIST, bool FUSED>
static hipError_t launch_f32c_nc(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                                 unsigned long long *counter, const QuadAcc &qa, int n_cu, hipStream_t s)
{
    // default 512 (a single profile's tail grows with more lanes), at most 1024;
    // above 768 the kernel built for four waves per SIMD, which re-reads the
    // request's parameters at each use (a few values spill at that bound, so
    // it is slower at 768 and below than the one that holds them)
    const int B = P.block > 0 ? (P.block < 1024 ? P.block : 1024) : 512;
    return B > 768 ? launch_f32c_w<NC, CULL, HIST, FUSED, true>(P, g, o, counter, qa, n_cu, B, s)
                   : launch_f32c_w<NC, CULL, HIST, FUSED, false>(P, g, o, counter, qa, n_cu, B, s);
}

template <bool HIST, bool FUSED>
static hipError_t launch_f32c_hist(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                                   unsigned long long *counter, const QuadAcc &qa, int n_cu, hipStream_t s)
{
    const bool cull = P.cull_D > 0.0;
    if (P.R_const > 0.0)
        return cull ? launch_f32c_nc<NCOL - 1, true, HIST, FUSED>(P, g, o, counter, qa, n_cu, s)
                    : launch_f32c_nc<NCOL - 1, false, HIST, FUSED>(P, g, o, counter, qa, n_cu, s);
    return cull ? launch_f32c_nc<NCOL, true, HIST, FUSED>(P, g, o, counter, qa, n_cu, s)
                : launch_f32c_nc<NCOL, false, HIST, FUSED>(P, g, o, counter, qa, n_cu, s);
}

hipError_t launch_dp5_f32c(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                           unsigned long long *counter, const QuadAcc *qa, int n_cu, hipStream_t s)
{
    const QuadAcc q = qa ? *qa : QuadAcc{};
    if (qa)
        return P.hist ? launch_f32c_hist<true, true>(P, g, o, counter, q, n_cu, s)
                      : launch_f32c_hist<false, true>(P, g, o, counter, q, n_cu, s);
    return P.hist ? launch_f32c_hist<true, false>(P, g, o, counter, q, n_cu, s)
                  : launch_f32c_hist<false, false>(P, g, o, counter, q, n_cu, s);
}

}  // namespace nh

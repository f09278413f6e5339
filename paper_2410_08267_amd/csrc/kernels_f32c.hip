// FP32-compensated Dormand-Prince kernel (the precision form).
//
// State: positions in FP32 with a Kahan compensation term each (the carried
// rounding error of the accumulated position), velocities in FP32, time u and
// step h in FP64 (u also indexes the coefficient table).  Right-hand sides,
// stage sums, error norm and step control run in FP32 on an FP32 copy of the
// FP64 coefficient table held in LDS.  An attempt whose |h| is below a
// threshold (the short steps the controller takes near pericentre) runs the
// FP64 step instead, on the FP64 table, after re-evaluating the first stage in
// FP64.  The speed ratio and the quadrature downstream stay FP64.  The choice
// is per lane, so a trajectory's result does not depend on which trajectories
// share its wavefront.
#include <hip/hip_runtime.h>

#include "nh_dp5_f32.h"

namespace nh {

template <int NC>
__global__ __launch_bounds__(512) void k_dp5_f32c(TrajParams P, GridPtrs g, TrajOut o,
                                                   unsigned long long *counter)
{
    extern __shared__ float lds32[];
    for (int i = threadIdx.x; i < P.n_tab * NC; i += blockDim.x) {
        const int node = i / NC, col = i - node * NC;
        lds32[i] = (float)g.tab[node * NCOL + col];
    }
    __syncthreads();

    const TabCoef32<NC> cf{lds32, P.n_tab, P.tab_u0, P.tab_inv_du, (float)fmin(P.R_const, 1.0e30)};
    // the promoted FP64 steps read the FP64 table from global memory (rows of NCOL)
    const TabCoef<NC, NCOL> cf64{g.tab, P.n_tab, P.tab_u0, P.tab_inv_du, P.R_const};
    // FP32 cannot resolve the FP64 tolerance; it integrates at max(rtol, 1e-6)
    const double rtol32 = fmax(P.rtol, 1.0e-6);
    DpCtl32 ctl;
    ctl.u_end = P.u_end;
    ctl.rtol = (float)rtol32;
    ctl.atol_x = (float)fmax(P.atol_x, rtol32);
    ctl.atol_v = (float)fmax(P.atol_v, rtol32);
    ctl.r_exit2 = P.r_exit > 0.0 ? (float)(P.r_exit * P.r_exit) : -1.0f;
    ctl.max_steps = (int)P.max_steps;
    DpCtl ctl64;
    ctl64.u_end = P.u_end;
    ctl64.rtol = rtol32;
    ctl64.atol_x = fmax(P.atol_x, rtol32);
    ctl64.atol_v = fmax(P.atol_v, rtol32);
    ctl64.r_exit2 = P.r_exit > 0.0 ? P.r_exit * P.r_exit : -1.0;
    ctl64.max_steps = (int)P.max_steps;

    long long t = -1;
    double v0n = 1.0;
    Lane32 L{};
    for (;;) {
        const bool need = (t == -1);
        const long long p = wave_claim(need, counter);
        if (need) {
            if (p < P.n_traj) {
                t = traj_of(p, P);
                const int l = (int)(t % P.n_mu);
                const long long kj = t / P.n_mu;
                const int j = (int)(kj % P.n_y);
                const int k = (int)(kj / P.n_y);
                const double V = g.y[j] * P.vfac;
                const double vx0 = V * g.mu[l], vy0 = V * g.smu[l];
                v0n = sqrt(norm2(vx0, vy0));
                L.x = (float)g.r[k];
                L.xc = (float)(g.r[k] - (double)L.x);
                L.y = 0.0f;
                L.yc = 0.0f;
                L.vx = (float)vx0;
                L.vy = (float)vy0;
                L.u = 0.0;
                L.h = -fabs(P.h0);
                if (fabs(L.h) > fabs(P.u_end)) L.h = P.u_end;
                L.nacc = L.nrej = L.natt = L.n64 = 0;
                L.rej_prev = false;
                float c[NCOL], R;
                cf.at(0.0, c, R);
                rhs32(c, R, L.x, L.y, L.vx, L.vy, L.k1x, L.k1y, L.k1u, L.k1v);
            } else {
                t = -2;
            }
        }
        if (__ballot(t >= 0) == 0ull) break;
        if (t >= 0) {
            int st;
            if (fabs(L.h) < P.h_fp64) {
                // promoted attempt in FP64
                Lane64 D;
                D.x = (double)L.x + (double)L.xc;
                D.y = (double)L.y + (double)L.yc;
                D.vx = L.vx;
                D.vy = L.vy;
                D.u = L.u;
                D.h = L.h;
                D.nacc = L.nacc;
                D.nrej = L.nrej;
                D.natt = L.natt;
                D.rej_prev = L.rej_prev;
                double c[NCOL], R;
                cf64.at(D.u, c, R);
                rhs(c, R, D.x, D.y, D.vx, D.vy, D.k1x, D.k1y, D.k1u, D.k1v);
                st = dp5_attempt(D, cf64, ctl64);
                L.x = (float)D.x;
                L.xc = (float)(D.x - (double)L.x);
                L.y = (float)D.y;
                L.yc = (float)(D.y - (double)L.y);
                L.vx = (float)D.vx;
                L.vy = (float)D.vy;
                L.u = D.u;
                L.h = D.h;
                L.k1x = (float)D.k1x;
                L.k1y = (float)D.k1y;
                L.k1u = (float)D.k1u;
                L.k1v = (float)D.k1v;
                L.nacc = D.nacc;
                L.nrej = D.nrej;
                L.natt = D.natt;
                L.rej_prev = D.rej_prev;
                ++L.n64;
            } else {
                st = dp5_attempt32(L, cf, ctl);
            }
            if (st >= 0) {
                const double fx = L.vx, fy = L.vy;
                o.ratio[t] = sqrt(norm2(fx, fy)) / v0n;
                o.stat[t] = TrajStat{L.nacc, L.nrej, st, L.n64};
                t = -1;
            }
        }
    }
}

template <int NC>
static hipError_t launch_f32c_nc(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                                 unsigned long long *counter, int n_cu, hipStream_t s)
{
    const int B = P.block > 0 ? P.block : 512;
    const size_t lds = (size_t)P.n_tab * NC * sizeof(float);
    hipError_t e = hipFuncSetAttribute((const void *)k_dp5_f32c<NC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dp5_f32c<NC>, B, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    long long grid = (long long)n_cu * per_cu;
    const long long need = (P.n_traj + B - 1) / B;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_dp5_f32c<NC>, dim3((unsigned)grid), dim3(B), lds, s, P, g, o, counter);
    return hipGetLastError();
}

hipError_t launch_dp5_f32c(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                           unsigned long long *counter, int n_cu, hipStream_t s)
{
    if (P.R_const > 0.0) return launch_f32c_nc<NCOL - 1>(P, g, o, counter, n_cu, s);
    return launch_f32c_nc<NCOL>(P, g, o, counter, n_cu, s);
}

}  // namespace nh

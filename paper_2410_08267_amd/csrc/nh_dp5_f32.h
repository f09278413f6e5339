// The FP32-compensated Dormand-Prince step of one trajectory, shared by the
// plain and batched kernels.
//
// State: positions in FP32 with a Kahan compensation term each (the carried
// rounding error of the accumulated position), velocities in FP32, time u and
// step h in FP64 (u also indexes the coefficient table).  Right-hand sides,
// stage sums, error norm and step control run in FP32; the drift and kick
// coefficients are interpolated in FP64 and rounded afterwards (TabCoef32).
#pragma once

#include "nh_dp5.h"

namespace nh {

namespace dp32 {
constexpr float c2 = 1.0f / 5.0f, c3 = 3.0f / 10.0f, c4 = 4.0f / 5.0f, c5 = 8.0f / 9.0f;
constexpr float a21 = 1.0f / 5.0f;
constexpr float a31 = 3.0f / 40.0f, a32 = 9.0f / 40.0f;
constexpr float a41 = 44.0f / 45.0f, a42 = -56.0f / 15.0f, a43 = 32.0f / 9.0f;
constexpr float a51 = 19372.0f / 6561.0f, a52 = -25360.0f / 2187.0f, a53 = 64448.0f / 6561.0f,
                a54 = -212.0f / 729.0f;
constexpr float a61 = 9017.0f / 3168.0f, a62 = -355.0f / 33.0f, a63 = 46732.0f / 5247.0f,
                a64 = 49.0f / 176.0f, a65 = -5103.0f / 18656.0f;
constexpr float b1 = 35.0f / 384.0f, b3 = 500.0f / 1113.0f, b4 = 125.0f / 192.0f,
                b5 = -2187.0f / 6784.0f, b6 = 11.0f / 84.0f;
constexpr float e1 = (float)(35.0 / 384.0 - 5179.0 / 57600.0);
constexpr float e3 = (float)(500.0 / 1113.0 - 7571.0 / 16695.0);
constexpr float e4 = (float)(125.0 / 192.0 - 393.0 / 640.0);
constexpr float e5 = (float)(-2187.0 / 6784.0 + 92097.0 / 339200.0);
constexpr float e6 = (float)(11.0 / 84.0 - 187.0 / 2100.0);
constexpr float e7 = (float)(-1.0 / 40.0);
}  // namespace dp32

// I(q) in FP32, branch-free, in the FP64 kernels' form (nfw_I): 1+q = m 2^e
// with e the exponent of (1+q) sqrt(2), s = (m-1)/(m+1) from q - (2^e - 1)
// and (1+q) + 2^e, and
//   I = e ln2 + (1 - 2^e)/(1+q) + s^2 (1 + 1/m) + 2 (s^3/3 + ... + s^9/9),
// one reciprocal for both divisions.  At e = 0 the first two terms vanish
// (a few ulp of I for any small q); just above q = sqrt(2) - 1 e ln2 and
// (1 - 2^e)/(1+q) cancel to a twenty-fifth of their size (~1e-6 of I).
__device__ __forceinline__ float nfw_I32(float q)
{
    const float w0 = 1.0f + q;
    const int e = __builtin_amdgcn_frexp_expf(w0 * 1.41421356f) - 1;
    const float p2 = __builtin_amdgcn_ldexpf(1.0f, e);
    const float N = q - (p2 - 1.0f), D = w0 + p2;
    const float rp = __builtin_amdgcn_rcpf(D * w0);
    const float s = N * (w0 * rp);
    const float iw = D * rp;
    const float s2 = s * s;
    float p = fmaf(s2, 2.0f / 9.0f, 2.0f / 7.0f);
    p = fmaf(s2, p, 2.0f / 5.0f);
    p = fmaf(s2, p, 2.0f / 3.0f);
    const float small = fmaf(s2, fmaf(p2, iw, 1.0f), s * s2 * p);
    return fmaf((float)e, 0.693147182f, fmaf(-p2, iw, iw)) + small;
}

__device__ __forceinline__ void rhs32(const float c[NCOL], float R, float x, float y, float vx,
                                      float vy, float &dx, float &dy, float &dvx, float &dvy)
{
    const float r2 = fmaf(x, x, y * y);
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float q = fminf(r * c[COL_INVS], c[COL_C]);
    const float I = nfw_I32(q);
    // max(., 0) as in rhs(): the bracket is >= 0 inside R and <= 0 beyond it
    (void)R;
    const float g = fmaxf(fmaf(c[COL_K] * I, ri * ri * ri, -c[COL_KC]), 0.0f);
    dx = c[COL_A] * vx;
    dy = c[COL_A] * vy;
    dvx = -g * x;
    dvy = -g * y;
}

// Coefficients of the FP32 attempts.  The H(z)-derived columns A, K and Kc
// (drift and kick, Sec. II.A) are interpolated from an FP64 table (rows of 3
// doubles) with the FP64 stencil of the FP64 kernels and rounded to FP32 only
// afterwards (K and Kc after their power-law factor when HIST, which also keeps
// the stencils inside spline pieces); 1/s, c and a moving R come from an FP32
// table (rows of NC - 3 floats) with the same weights rounded to FP32.
// SPLIT: as in the plain FP64 kernel, A comes from its node-by-node copy in
// device memory and the LDS rows hold only K and Kc (a quarter of the table's
// LDS bytes per stage less; the same FMA chain, so the same bits).
constexpr int F32C_T64 = 3;   // FP64 columns: A, K, Kc
template <bool SPLIT>
constexpr int f32c_t64 = SPLIT ? F32C_T64 - 1 : F32C_T64;   // FP64 columns in LDS
template <int NC, bool SPLIT = false>
__host__ __device__ constexpr size_t f32c_table_bytes(int n_tab)
{
    return (size_t)n_tab * (f32c_t64<SPLIT> * sizeof(double) + (NC - F32C_T64) * sizeof(float));
}

template <int NC, bool HIST = false, bool SPLIT = false>
struct TabCoef32 {
    const double *t64;      // n_tab rows of A, K, Kc (SPLIT: K, Kc)
    const float *t32;       // n_tab rows of 1/s, c (, R)
    int nc, n_tab;          // nc: NCOL when this request's R moves (possible only when NC == NCOL)
    double u0, inv_du;
    float R_const;
    PowFactor pw;
    Knots kn;
    const double *a = nullptr;   // SPLIT: n_tab values of A
    __device__ __forceinline__ void at(double u, float c[NCOL], float &R) const
    {
        constexpr int N32 = NC - F32C_T64;
        constexpr int T64 = f32c_t64<SPLIT>;
        const Stencil4 w = table_stencil<HIST>(n_tab, u0, inv_du, kn, u);
        const double *r64 = stencil_rows(t64, w, T64);
        double A, K, Kc;
        if constexpr (SPLIT) {
            A = stencil_a(w, (a - 1) + (unsigned)w.i1);
            K = stencil_col(w, r64, T64, 0);
            Kc = stencil_col(w, r64, T64, 1);
        } else {
            A = stencil_col(w, r64, T64, 0);
            K = stencil_col(w, r64, T64, 1);
            Kc = stencil_col(w, r64, T64, 2);
        }
        if constexpr (HIST) {
            const double f = pow_factor(pw, u);
            K *= f;
            Kc *= f;
        }
        c[COL_A] = (float)A;
        c[COL_K] = (float)K;
        c[COL_KC] = (float)Kc;
        const float wa = (float)w.wa, wb = (float)w.wb, wc = (float)w.wc, wd = (float)w.wd;
        const float *r32 = (t32 - N32) + __umul24((unsigned)w.i1, (unsigned)N32);
#pragma unroll
        for (int k = 0; k < N32; ++k)
            c[F32C_T64 + k] = fmaf(wd, r32[3 * N32 + k], fmaf(wc, r32[2 * N32 + k], fmaf(wb, r32[N32 + k], wa * r32[k])));
        R = (NC == NCOL && nc == NCOL) ? c[COL_R] : R_const;
    }
    // SPLIT tables: the coefficients at uP and at uQ <= uP, a fraction of a
    // step apart, from one five-row window where their stencils start on the
    // same or adjacent nodes, P's weights shifted onto Q's rows (a zero weight
    // on the unused end row); lanes whose stencils lie further apart read P's
    // own rows.  Either way the values equal those of two at() calls bit for
    // bit: an FMA with a zero weight adds an exact zero.
    static constexpr bool paired = SPLIT;
    __device__ __forceinline__ void at2(double uP, double uQ, float cP[NCOL], float &RP, float cQ[NCOL],
                                        float &RQ) const
    {
        static_assert(SPLIT, "the paired window reads the split layout");
        constexpr int N32 = NC - F32C_T64;
        constexpr int T64 = f32c_t64<SPLIT>;
        const Stencil4 wQ = table_stencil<HIST>(n_tab, u0, inv_du, kn, uQ);
        const Stencil4 wP = table_stencil<HIST>(n_tab, u0, inv_du, kn, uP);
        const int d = wP.i1 - wQ.i1;
        const bool sh = d == 1;
        const double v0 = sh ? 0.0 : wP.wa, v1 = sh ? wP.wa : wP.wb, v2 = sh ? wP.wb : wP.wc;
        const double v3 = sh ? wP.wc : wP.wd, v4 = sh ? wP.wd : 0.0;
        const int row4i = min(wQ.i1 + 3, n_tab - 1);
        double q64[F32C_T64], p64[F32C_T64];   // A, K, Kc
        {
            const double *aq = (a - 1) + (unsigned)wQ.i1;
            const double r0 = aq[0], r1 = aq[1], r2 = aq[2], r3 = aq[3];
            q64[0] = fma(wQ.wd, r3, fma(wQ.wc, r2, fma(wQ.wb, r1, wQ.wa * r0)));
            p64[0] = fma(v4, a[(unsigned)row4i], fma(v3, r3, fma(v2, r2, fma(v1, r1, v0 * r0))));
        }
        const double *row = stencil_rows(t64, wQ, T64);
        const double *row4 = tab_row(t64, row4i, T64);
#pragma unroll
        for (int k = 0; k < T64; ++k) {
            const double r0 = row[k], r1 = row[T64 + k], r2 = row[2 * T64 + k], r3 = row[3 * T64 + k];
            q64[1 + k] = fma(wQ.wd, r3, fma(wQ.wc, r2, fma(wQ.wb, r1, wQ.wa * r0)));
            p64[1 + k] = fma(v4, row4[k], fma(v3, r3, fma(v2, r2, fma(v1, r1, v0 * r0))));
        }
        const float qa = (float)wQ.wa, qb = (float)wQ.wb, qc = (float)wQ.wc, qd = (float)wQ.wd;
        const float f0 = (float)v0, f1 = (float)v1, f2 = (float)v2, f3 = (float)v3, f4 = (float)v4;
        const float *r32 = (t32 - N32) + __umul24((unsigned)wQ.i1, (unsigned)N32);
        const float *r32e = t32 + __umul24((unsigned)row4i, (unsigned)N32);
#pragma unroll
        for (int k = 0; k < N32; ++k) {
            const float r0 = r32[k], r1 = r32[N32 + k], r2 = r32[2 * N32 + k], r3 = r32[3 * N32 + k];
            cQ[F32C_T64 + k] = fmaf(qd, r3, fmaf(qc, r2, fmaf(qb, r1, qa * r0)));
            cP[F32C_T64 + k] = fmaf(f4, r32e[k], fmaf(f3, r3, fmaf(f2, r2, fmaf(f1, r1, f0 * r0))));
        }
        if ((unsigned)d > 1u) {
            p64[0] = stencil_a(wP, (a - 1) + (unsigned)wP.i1);
            const double *rp = stencil_rows(t64, wP, T64);
#pragma unroll
            for (int k = 0; k < T64; ++k) p64[1 + k] = stencil_col(wP, rp, T64, k);
            const float pa = (float)wP.wa, pb = (float)wP.wb, pc = (float)wP.wc, pd = (float)wP.wd;
            const float *rp32 = (t32 - N32) + __umul24((unsigned)wP.i1, (unsigned)N32);
#pragma unroll
            for (int k = 0; k < N32; ++k)
                cP[F32C_T64 + k] =
                    fmaf(pd, rp32[3 * N32 + k], fmaf(pc, rp32[2 * N32 + k], fmaf(pb, rp32[N32 + k], pa * rp32[k])));
        }
        if constexpr (HIST) {
            const double fP = pow_factor(pw, uP), fQ = pow_factor(pw, uQ);
            p64[1] *= fP;
            p64[2] *= fP;
            q64[1] *= fQ;
            q64[2] *= fQ;
        }
#pragma unroll
        for (int k = 0; k < F32C_T64; ++k) {
            cP[k] = (float)p64[k];
            cQ[k] = (float)q64[k];
        }
        RP = (NC == NCOL && nc == NCOL) ? cP[COL_R] : R_const;
        RQ = (NC == NCOL && nc == NCOL) ? cQ[COL_R] : R_const;
    }
};

// Copy the first NC columns of FP64 table rows (stride NCOL) into the FP32C
// layout at dst: n_tab rows of A, K, Kc (FP64; SPLIT: K, Kc), then n_tab rows
// of the other NC - 3 columns (FP32); by the threads first, first + step, ...
template <int NC, bool SPLIT = false>
__device__ __forceinline__ void stage_f32c_table(void *dst, const double *src, int n_tab, int first, int step)
{
    constexpr int N32 = NC - F32C_T64;
    constexpr int T64 = f32c_t64<SPLIT>;
    constexpr int C0 = F32C_T64 - T64;   // first FP64 column held in LDS
    double *t64 = (double *)dst;
    float *t32 = (float *)(t64 + (size_t)n_tab * T64);
    for (int i = first; i < n_tab * T64; i += step) {
        const int node = i / T64, col = i - node * T64;
        t64[i] = src[node * NCOL + C0 + col];
    }
    for (int i = first; i < n_tab * N32; i += step) {
        const int node = i / N32, col = i - node * N32;
        t32[i] = (float)src[node * NCOL + F32C_T64 + col];
    }
}

struct Lane32 {
    float x, y, xc, yc, vx, vy;   // xc, yc: Kahan compensation of the positions
    double u, h;
    float k1x, k1y, k1u, k1v;
    int nacc, nrej, natt, n64;
    bool rej_prev;
};

// Compensated sum: s + c accumulates d with the rounding error carried in c.
__device__ __forceinline__ void kahan_add(float &s, float &c, float d)
{
    const float y = __fadd_rn(d, c);
    const float t = __fadd_rn(s, y);
    c = __fsub_rn(y, __fsub_rn(t, s));
    s = t;
}

struct DpCtl32 {
    double u_end;
    float rtol, atol_x, atol_v;
    float r_exit2;
    int max_steps;
};

// One FP32 attempt.  Returns -1 while the trajectory continues, else its status.
template <class CF>
__device__ __forceinline__ int dp5_attempt32(Lane32 &L, const CF &cf, const DpCtl32 &ctl)
{
    using namespace dp32;
    if (L.natt >= ctl.max_steps) return ST_MAXSTEPS;
    ++L.natt;
    bool last = false;
    double hd = L.h;
    if (L.u + hd - ctl.u_end <= 0.0) {
        hd = ctl.u_end - L.u;
        last = true;
    }
    const float h = (float)hd;
    const double u = L.u;
    const float x = L.x + L.xc, y = L.y + L.yc, vx = L.vx, vy = L.vy;
    const float k1x = L.k1x, k1y = L.k1y, k1u = L.k1u, k1v = L.k1v;
    float c[NCOL], R, cb[NCOL], Rb;
    float k2x, k2y, k2u, k2v, k3x, k3y, k3u, k3v, k4x, k4y, k4u, k4v;
    float k5x, k5y, k5u, k5v, k6x, k6y, k6u, k6v, k7x, k7y, k7u, k7v;

    // stages 2 and 3 lie a tenth of a step apart: one table window for both
    // where the source has one
    if constexpr (CF::paired) {
        cf.at2(u + (double)c2 * hd, u + (double)c3 * hd, c, R, cb, Rb);
    } else {
        cf.at(u + (double)c2 * hd, c, R);
    }
    rhs32(c, R, x + h * (a21 * k1x), y + h * (a21 * k1y), vx + h * (a21 * k1u), vy + h * (a21 * k1v),
          k2x, k2y, k2u, k2v);
    if constexpr (!CF::paired) cf.at(u + (double)c3 * hd, cb, Rb);
    rhs32(cb, Rb, x + h * (a31 * k1x + a32 * k2x), y + h * (a31 * k1y + a32 * k2y),
          vx + h * (a31 * k1u + a32 * k2u), vy + h * (a31 * k1v + a32 * k2v), k3x, k3y, k3u, k3v);
    cf.at(u + (double)c4 * hd, c, R);
    rhs32(c, R, x + h * (a41 * k1x + a42 * k2x + a43 * k3x), y + h * (a41 * k1y + a42 * k2y + a43 * k3y),
          vx + h * (a41 * k1u + a42 * k2u + a43 * k3u), vy + h * (a41 * k1v + a42 * k2v + a43 * k3v),
          k4x, k4y, k4u, k4v);
    cf.at(u + (double)c5 * hd, c, R);
    rhs32(c, R, x + h * (a51 * k1x + a52 * k2x + a53 * k3x + a54 * k4x),
          y + h * (a51 * k1y + a52 * k2y + a53 * k3y + a54 * k4y),
          vx + h * (a51 * k1u + a52 * k2u + a53 * k3u + a54 * k4u),
          vy + h * (a51 * k1v + a52 * k2v + a53 * k3v + a54 * k4v), k5x, k5y, k5u, k5v);
    cf.at(u + hd, c, R);
    rhs32(c, R, x + h * (a61 * k1x + a62 * k2x + a63 * k3x + a64 * k4x + a65 * k5x),
          y + h * (a61 * k1y + a62 * k2y + a63 * k3y + a64 * k4y + a65 * k5y),
          vx + h * (a61 * k1u + a62 * k2u + a63 * k3u + a64 * k4u + a65 * k5u),
          vy + h * (a61 * k1v + a62 * k2v + a63 * k3v + a64 * k4v + a65 * k5v), k6x, k6y, k6u, k6v);
    const float dxs = h * (b1 * k1x + b3 * k3x + b4 * k4x + b5 * k5x + b6 * k6x);
    const float dys = h * (b1 * k1y + b3 * k3y + b4 * k4y + b5 * k5y + b6 * k6y);
    const float x5 = x + dxs, y5 = y + dys;
    const float vx5 = vx + h * (b1 * k1u + b3 * k3u + b4 * k4u + b5 * k5u + b6 * k6u);
    const float vy5 = vy + h * (b1 * k1v + b3 * k3v + b4 * k4v + b5 * k5v + b6 * k6v);
    rhs32(c, R, x5, y5, vx5, vy5, k7x, k7y, k7u, k7v);

    const float ex = h * (e1 * k1x + e3 * k3x + e4 * k4x + e5 * k5x + e6 * k6x + e7 * k7x);
    const float ey = h * (e1 * k1y + e3 * k3y + e4 * k4y + e5 * k5y + e6 * k6y + e7 * k7y);
    const float eu = h * (e1 * k1u + e3 * k3u + e4 * k4u + e5 * k5u + e6 * k6u + e7 * k7u);
    const float ev = h * (e1 * k1v + e3 * k3v + e4 * k4v + e5 * k5v + e6 * k6v + e7 * k7v);
    const float sx = ctl.atol_x + ctl.rtol * sqrtf(fmaxf(fmaf(x, x, y * y), fmaf(x5, x5, y5 * y5)));
    const float sv = ctl.atol_v + ctl.rtol * sqrtf(fmaxf(fmaf(vx, vx, vy * vy), fmaf(vx5, vx5, vy5 * vy5)));
    const float isx = __builtin_amdgcn_rcpf(sx), isv = __builtin_amdgcn_rcpf(sv);
    const float qx = ex * isx, qy = ey * isx, qu = eu * isv, qv = ev * isv;
    const float err2 = 0.25f * (qx * qx + qy * qy + qu * qu + qv * qv);
    if (!(err2 <= 1.0e30f)) return ST_NONFINITE;
    if (err2 <= 1.0f) {
        ++L.nacc;
        L.u = last ? ctl.u_end : u + hd;
        kahan_add(L.x, L.xc, dxs);
        kahan_add(L.y, L.yc, dys);
        L.vx = vx5;
        L.vy = vy5;
        L.k1x = k7x;
        L.k1y = k7y;
        L.k1u = k7u;
        L.k1v = k7v;
        if (last) return ST_OK;
        if (ctl.r_exit2 >= 0.0f && fmaf(x5, x5, y5 * y5) >= ctl.r_exit2 && fmaf(x5, vx5, y5 * vy5) <= 0.0f)
            return ST_OK | ST_FREE_EXIT;
        float f = err2 == 0.0f ? 5.0f
                               : 0.9f * __builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf(err2));
        f = fminf(L.rej_prev ? 1.0f : 5.0f, fmaxf(0.2f, f));
        L.h = hd * (double)f;
        L.rej_prev = false;
    } else {
        ++L.nrej;
        const float f = 0.9f * __builtin_amdgcn_exp2f(-0.1f * __builtin_amdgcn_logf(err2));
        L.h = hd * (double)fminf(5.0f, fmaxf(0.2f, f));
        L.rej_prev = true;
    }
    if (fabs(L.h) <= 8.881784197001252e-16 * fmax(1.0, fabs(L.u))) return ST_UNDERFLOW;
    return -1;
}

// Start a trajectory at u = u_start: FP32 state from the FP64 initial conditions,
// first stage evaluated in FP32.
template <class CF>
__device__ __forceinline__ void f32c_start(Lane32 &L, const CF &cf, double x0, double vx0, double vy0,
                                           double h0, double u_start, double u_end)
{
    L.x = (float)x0;
    L.xc = (float)(x0 - (double)L.x);
    L.y = 0.0f;
    L.yc = 0.0f;
    L.vx = (float)vx0;
    L.vy = (float)vy0;
    L.u = u_start;
    L.h = -fabs(h0);
    if (fabs(L.h) > fabs(u_end - u_start)) L.h = u_end - u_start;
    L.nacc = L.nrej = L.natt = L.n64 = 0;
    L.rej_prev = false;
    float c[NCOL], R;
    cf.at(u_start, c, R);
    rhs32(c, R, L.x, L.y, L.vx, L.vy, L.k1x, L.k1y, L.k1u, L.k1v);
}

// One attempt of the FP32-compensated form: in FP64 (state widened, first
// stage re-evaluated on the FP64 table cf64) when |h| < h_fp64, else in FP32.
// Returns -1 while the trajectory continues, else its status.
template <class CF32, class CF64>
__device__ __forceinline__ int f32c_attempt(Lane32 &L, const CF32 &cf, const CF64 &cf64, const DpCtl32 &ctl,
                                            const DpCtl &ctl64, double h_fp64)
{
    if (!(fabs(L.h) < h_fp64)) return dp5_attempt32(L, cf, ctl);
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
    const int st = dp5_attempt(D, cf64, ctl64);
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
    return st;
}

// Step control of the FP32-compensated form: it integrates at
// max(rtol, P.rtol32), 1e-7 by default (the FP32 state's own rounding, ~1e-7
// relative per step in the velocities, bounds what a tighter tolerance could
// buy); the promoted FP64 attempts use the same tolerances.
__device__ __forceinline__ void f32c_controls(const TrajParams &P, DpCtl32 &ctl, DpCtl &ctl64)
{
    const double rtol32 = fmax(P.rtol, P.rtol32);
    ctl.u_end = P.u_end;
    ctl.rtol = (float)rtol32;
    ctl.atol_x = (float)fmax(P.atol_x, rtol32);
    ctl.atol_v = (float)fmax(P.atol_v, rtol32);
    ctl.r_exit2 = P.r_exit > 0.0 ? (float)(P.r_exit * P.r_exit) : -1.0f;
    ctl.max_steps = (int)P.max_steps;
    ctl64.u_end = P.u_end;
    ctl64.rtol = rtol32;
    ctl64.atol_x = fmax(P.atol_x, rtol32);
    ctl64.atol_v = fmax(P.atol_v, rtol32);
    ctl64.r_exit2 = P.r_exit2;
    ctl64.max_steps = (int)P.max_steps;
}

}  // namespace nh

// The Dormand-Prince 5(4) step of one trajectory in FP64, shared by the plain
// and batched kernels.  Tableau: Dormand & Prince (1980); step control: Hairer,
// Norsett & Wanner, Solving ODEs I, Sec. II.4 (see nh_dopri5 in nuhalo.h).
#pragma once

#include "nh_device.h"

namespace nh {

namespace dp {
constexpr double c2 = 1.0 / 5.0, c3 = 3.0 / 10.0, c4 = 4.0 / 5.0, c5 = 8.0 / 9.0;
constexpr double a21 = 1.0 / 5.0;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0,
                 a54 = -212.0 / 729.0;
constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0,
                 a64 = 49.0 / 176.0, a65 = -5103.0 / 18656.0;
// fifth-order weights (= seventh stage row, FSAL)
constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0,
                 b5 = -2187.0 / 6784.0, b6 = 11.0 / 84.0;
// e = b - b* (fourth-order embedded weights b*)
constexpr double e1 = 35.0 / 384.0 - 5179.0 / 57600.0;
constexpr double e3 = 500.0 / 1113.0 - 7571.0 / 16695.0;
constexpr double e4 = 125.0 / 192.0 - 393.0 / 640.0;
constexpr double e5 = -2187.0 / 6784.0 - (-92097.0 / 339200.0);
constexpr double e6 = 11.0 / 84.0 - 187.0 / 2100.0;
constexpr double e7 = 0.0 - 1.0 / 40.0;
}  // namespace dp

// Coefficient source: an FP64 table (LDS rows of NC doubles, or the staged
// global copy with rows of NCOL).  NC = 5 when R is constant.  HIST: the
// request's history is not smooth: stencils stay inside spline pieces (Knots)
// and K and Kc take their power-law factor (PowFactor) here.
template <int NC, int STRIDE = NC, bool HIST = false>
struct TabCoef {
    const double *tab;
    int n_tab;
    double u0, inv_du, R_const;
    PowFactor pw;
    Knots kn;
    __device__ __forceinline__ void at(double u, double c[NCOL], double &R) const
    {
        coef_interp<NC, STRIDE, HIST>(tab, n_tab, u0, inv_du, kn, u, c);
        R = (NC == NCOL) ? c[COL_R] : R_const;
        if constexpr (HIST) {
            const double f = pow_factor(pw, u);
            c[COL_K] *= f;
            c[COL_KC] *= f;
        }
    }
    // coefficients at uP and at uQ <= uP, a fraction of a step apart, from one
    // five-row window where they share it
    static constexpr bool paired = true;
    __device__ __forceinline__ void at2(double uP, double uQ, double cP[NCOL], double &RP, double cQ[NCOL],
                                        double &RQ) const
    {
        coef_interp2<NC, STRIDE, HIST>(tab, n_tab, u0, inv_du, kn, uP, uQ, cP, cQ);
        RP = (NC == NCOL) ? cP[COL_R] : R_const;
        RQ = (NC == NCOL) ? cQ[COL_R] : R_const;
        if constexpr (HIST) {
            const double fP = pow_factor(pw, uP), fQ = pow_factor(pw, uQ);
            cP[COL_K] *= fP;
            cP[COL_KC] *= fP;
            cQ[COL_K] *= fQ;
            cQ[COL_KC] *= fQ;
        }
    }
};

// The plain FP64 kernel's coefficient source: the drift column A from its
// node-by-node copy in device memory (GridPtrs::tabA, read through the vector
// cache) and K, Kc, 1/s and c from LDS rows of SPLIT_ROW doubles.  The LDS is
// the kernel's busiest unit beside the FP64 VALU (random table rows: most of
// its cycles are bank conflicts); taking a fifth of the table reads off it
// pays for the extra vector-memory loads.  A row stride of five doubles (ten
// banks; one unused) spreads random rows over the banks as the five-column
// rows did.  Values equal TabCoef's bit for bit; R (no longer read by the
// right-hand side) is the request's constant.
constexpr int SPLIT_ROW = 5;
template <bool HIST = false>
struct TabCoefSplit {
    const double *lds;     // n_tab rows of K, Kc, 1/s, c (and one unused double)
    const double *a;       // n_tab values of A
    int n_tab;
    double u0, inv_du, R_const;
    PowFactor pw;
    Knots kn;
    __device__ __forceinline__ void at(double u, double c[NCOL], double &R) const
    {
        coef_interp_split<SPLIT_ROW, HIST>(lds, a, n_tab, u0, inv_du, kn, u, c);
        R = R_const;
        if constexpr (HIST) {
            const double f = pow_factor(pw, u);
            c[COL_K] *= f;
            c[COL_KC] *= f;
        }
    }
    static constexpr bool paired = true;
    __device__ __forceinline__ void at2(double uP, double uQ, double cP[NCOL], double &RP, double cQ[NCOL],
                                        double &RQ) const
    {
        coef_interp2_split<SPLIT_ROW, HIST>(lds, a, n_tab, u0, inv_du, kn, uP, uQ, cP, cQ);
        RP = RQ = R_const;
        if constexpr (HIST) {
            const double fP = pow_factor(pw, uP), fQ = pow_factor(pw, uQ);
            cP[COL_K] *= fP;
            cP[COL_KC] *= fP;
            cQ[COL_K] *= fQ;
            cQ[COL_KC] *= fQ;
        }
    }
};

struct DpCtl {
    double u_end;      // integration ends here (below the start)
    double rtol, atol_x, atol_v;
    double r_exit2;    // squared free-streaming exit radius; +inf disables
    int max_steps;
};

struct Lane64 {
    double x, y, vx, vy, u, h;
    double k1x, k1y, k1u, k1v;   // FSAL stage
    int nacc, nrej, natt;
    bool rej_prev;
};

// The first step: -|h0|, clipped to the whole interval.
__host__ __device__ __forceinline__ double dp5_first_step(double h0, double u_start, double u_end)
{
    const double h = -fabs(h0);
    return fabs(h) > fabs(u_end - u_start) ? u_end - u_start : h;
}

// Start a trajectory at u = u_start from the coefficients there (c, R) and
// the first step h: the state and the first stage.
__device__ __forceinline__ void dp5_start_at(Lane64 &L, const double c[NCOL], double R, double x0, double vx0,
                                             double vy0, double h, double u_start)
{
    L.x = x0;
    L.y = 0.0;
    L.vx = vx0;
    L.vy = vy0;
    L.u = u_start;
    L.h = h;
    L.nacc = L.nrej = L.natt = 0;
    L.rej_prev = false;
    rhs(c, R, L.x, L.y, L.vx, L.vy, L.k1x, L.k1y, L.k1u, L.k1v);
}

// Start a trajectory at u = u_start (first stage evaluated here).
template <class CF>
__device__ __forceinline__ void dp5_start(Lane64 &L, const CF &cf, double x0, double vx0, double vy0,
                                          double h0, double u_start, double u_end)
{
    double c[NCOL], R;
    cf.at(u_start, c, R);
    dp5_start_at(L, c, R, x0, vx0, vy0, dp5_first_step(h0, u_start, u_end), u_start);
}

// Every lane of a launch starts at the same u: the coefficients there and the
// first step are computed once per workgroup into LDS (after the table is
// staged; a barrier follows) and read back at each start.  The reads are
// indexed by a zero the compiler cannot see through, so that they stay at the
// start and are not hoisted out of the trajectory loop, where they would hold
// registers for its whole length.  (A volatile read would do the same but
// loses the LDS address space: serialized flat loads, each waited for.)
struct StartCache {
    double v[NCOL + 2];   // c[0..NCOL), then R, then the first step h
};

template <class CF>
__device__ __forceinline__ void start_cache_fill(StartCache &sc, const CF &cf, double h0, double u_start,
                                                 double u_end)
{
    if (threadIdx.x == 0) {
        double c[NCOL], R;
        cf.at(u_start, c, R);
        for (int i = 0; i < NCOL; ++i) sc.v[i] = c[i];
        sc.v[NCOL] = R;
        sc.v[NCOL + 1] = dp5_first_step(h0, u_start, u_end);
    }
}

// The force term g of the first stage at the common start, x0 = (r, 0): it
// depends on the radius alone (the same arithmetic as rhs).
__device__ __forceinline__ double start_g(const StartCache &sc, double r)
{
    double c[NCOL];
    for (int i = 0; i < NCOL; ++i) c[i] = sc.v[i];
    return rhs_g(c, r, 0.0);
}

// Start a trajectory at x0 = (r, 0) from its radius's start force g0
// (start_g): the first stage without evaluating the right-hand side, the
// same bits as dp5_start_cached.
__device__ __forceinline__ void dp5_start_g(Lane64 &L, const StartCache &sc, double g0, double x0, double vx0,
                                            double vy0, double u_start)
{
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    const double *v = sc.v + z;
    L.x = x0;
    L.y = 0.0;
    L.vx = vx0;
    L.vy = vy0;
    L.u = u_start;
    L.h = v[NCOL + 1];
    L.nacc = L.nrej = L.natt = 0;
    L.rej_prev = false;
    L.k1x = v[COL_A] * vx0;
    L.k1y = v[COL_A] * vy0;
    L.k1u = -g0 * L.x;
    L.k1v = -g0 * L.y;
}

__device__ __forceinline__ void dp5_start_cached(Lane64 &L, const StartCache &sc, double x0, double vx0,
                                                 double vy0, double u_start)
{
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    const double *v = sc.v + z;
    double c[NCOL];
    for (int i = 0; i < NCOL; ++i) c[i] = v[i];
    dp5_start_at(L, c, v[NCOL], x0, vx0, vy0, v[NCOL + 1], u_start);
}

// One attempted step.  Returns -1 while the trajectory continues, else its
// final status word (ST_*).
template <class CF>
__device__ __forceinline__ int dp5_attempt(Lane64 &L, const CF &cf, const DpCtl &ctl)
{
    using namespace dp;
    if (L.natt >= ctl.max_steps) return ST_MAXSTEPS;
    ++L.natt;
    bool last = false;
    double h = L.h;
    if (L.u + h - ctl.u_end <= 0.0) {
        h = ctl.u_end - L.u;
        last = true;
    }
    const double x = L.x, y = L.y, vx = L.vx, vy = L.vy, u = L.u;
    const double k1x = L.k1x, k1y = L.k1y, k1u = L.k1u, k1v = L.k1v;
    double c[NCOL], R, cb[NCOL], Rb;
    double k2x, k2y, k2u, k2v, k3x, k3y, k3u, k3v, k4x, k4y, k4u, k4v;
    double k5x, k5y, k5u, k5v, k6x, k6y, k6u, k6v, k7x, k7y, k7u, k7v;

    // stages 2 and 3 lie a tenth of a step apart: one table window for both
    // where the source has one (h < 0, so stage 3 sits at or below stage 2)
    if constexpr (CF::paired) {
        cf.at2(u + c2 * h, u + c3 * h, c, R, cb, Rb);
    } else {
        cf.at(u + c2 * h, c, R);
    }
    rhs(c, R, x + h * (a21 * k1x), y + h * (a21 * k1y), vx + h * (a21 * k1u), vy + h * (a21 * k1v),
        k2x, k2y, k2u, k2v);
    if constexpr (!CF::paired) cf.at(u + c3 * h, cb, Rb);
    rhs(cb, Rb, x + h * (a31 * k1x + a32 * k2x), y + h * (a31 * k1y + a32 * k2y),
        vx + h * (a31 * k1u + a32 * k2u), vy + h * (a31 * k1v + a32 * k2v), k3x, k3y, k3u, k3v);
    cf.at(u + c4 * h, c, R);
    rhs(c, R, x + h * (a41 * k1x + a42 * k2x + a43 * k3x), y + h * (a41 * k1y + a42 * k2y + a43 * k3y),
        vx + h * (a41 * k1u + a42 * k2u + a43 * k3u), vy + h * (a41 * k1v + a42 * k2v + a43 * k3v),
        k4x, k4y, k4u, k4v);
    cf.at(u + c5 * h, c, R);
    rhs(c, R, x + h * (a51 * k1x + a52 * k2x + a53 * k3x + a54 * k4x),
        y + h * (a51 * k1y + a52 * k2y + a53 * k3y + a54 * k4y),
        vx + h * (a51 * k1u + a52 * k2u + a53 * k3u + a54 * k4u),
        vy + h * (a51 * k1v + a52 * k2v + a53 * k3v + a54 * k4v), k5x, k5y, k5u, k5v);
    cf.at(u + h, c, R);
    const double x6 = x + h * (a61 * k1x + a62 * k2x + a63 * k3x + a64 * k4x + a65 * k5x);
    const double y6 = y + h * (a61 * k1y + a62 * k2y + a63 * k3y + a64 * k4y + a65 * k5y);
    const double vx6 = vx + h * (a61 * k1u + a62 * k2u + a63 * k3u + a64 * k4u + a65 * k5u);
    const double vy6 = vy + h * (a61 * k1v + a62 * k2v + a63 * k3v + a64 * k4v + a65 * k5v);
    // the solution and error sums over stages 1-5, formed here so that k2-k5
    // are dead during the last two right-hand sides (the same operations in
    // the same order as the whole sums: b1 k1 + b3 k3 + ... + b6 k6)
    const double sx = b1 * k1x + b3 * k3x + b4 * k4x + b5 * k5x;
    const double sy = b1 * k1y + b3 * k3y + b4 * k4y + b5 * k5y;
    const double su = b1 * k1u + b3 * k3u + b4 * k4u + b5 * k5u;
    const double sv = b1 * k1v + b3 * k3v + b4 * k4v + b5 * k5v;
    const double tx = e1 * k1x + e3 * k3x + e4 * k4x + e5 * k5x;
    const double ty = e1 * k1y + e3 * k3y + e4 * k4y + e5 * k5y;
    const double tu = e1 * k1u + e3 * k3u + e4 * k4u + e5 * k5u;
    const double tv = e1 * k1v + e3 * k3v + e4 * k4v + e5 * k5v;
    rhs(c, R, x6, y6, vx6, vy6, k6x, k6y, k6u, k6v);
    const double x5 = x + h * (sx + b6 * k6x);
    const double y5 = y + h * (sy + b6 * k6y);
    const double vx5 = vx + h * (su + b6 * k6u);
    const double vy5 = vy + h * (sv + b6 * k6v);
    const double wx = tx + e6 * k6x, wy = ty + e6 * k6y, wu = tu + e6 * k6u, wv = tv + e6 * k6v;
    rhs(c, R, x5, y5, vx5, vy5, k7x, k7y, k7u, k7v);   // c7 = c6 = 1: same coefficients

    const double ex = h * (wx + e7 * k7x);
    const double ey = h * (wy + e7 * k7y);
    const double eu = h * (wu + e7 * k7u);
    const double ev = h * (wv + e7 * k7v);
    // sc = atol + rtol max(|.|_n, |.|_{n+1}); max of the norms = sqrt of the max of the squares
    const double scx = ctl.atol_x + ctl.rtol * sqrt_pos(fmax(x * x + y * y, x5 * x5 + y5 * y5));
    const double scv = ctl.atol_v + ctl.rtol * sqrt_pos(fmax(vx * vx + vy * vy, vx5 * vx5 + vy5 * vy5));
    const double rp = rcp64(scx * scv);                 // one reciprocal for both scales
    const double isx = scv * rp, isv = scx * rp;
    const double qx = ex * isx, qy = ey * isx, qu = eu * isv, qv = ev * isv;
    const double err2 = 0.25 * (qx * qx + qy * qy + qu * qu + qv * qv);   // err^2
    if (!(err2 <= 1.0e300)) return ST_NONFINITE;
    const bool accept = err2 <= 1.0;
    // the next trial step's factor, growth capped at 1 right after a rejection
    // (one evaluation for both outcomes: a wavefront holds lanes of each)
    const double fac = step_factor(err2, (accept && L.rej_prev) ? 1.0 : 5.0);
    if (accept) {
        ++L.nacc;
        L.u = last ? ctl.u_end : u + h;
        L.x = x5;
        L.y = y5;
        L.vx = vx5;
        L.vy = vy5;
        L.k1x = k7x;
        L.k1y = k7y;
        L.k1u = k7u;
        L.k1v = k7v;
        if (last) return ST_OK;
        if (x5 * x5 + y5 * y5 >= ctl.r_exit2 && x5 * vx5 + y5 * vy5 <= 0.0) return ST_OK | ST_FREE_EXIT;
        L.h = h * fac;
        L.rej_prev = false;
    } else {
        ++L.nrej;
        L.h = h * fac;
        L.rej_prev = true;
    }
    if (fabs(L.h) <= 8.881784197001252e-16 * fmax(1.0, fabs(L.u))) return ST_UNDERFLOW;
    return -1;
}

}  // namespace nh

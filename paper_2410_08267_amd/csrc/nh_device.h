// Device helpers shared by the trajectory kernels: FP64 elementary functions
// sized for this problem, coefficient interpolation, the right-hand side of the
// equations of motion, the relic distributions and the wavefront work queue.
#pragma once

#include <hip/hip_runtime.h>

#include "nh_internal.h"

namespace nh {

// ---------------------------------------------------------------------------
// FP64 elementary functions.  The hardware rcp/rsq give a first guess good to
// ~2^-26; one third-order correction (the series of (1 - e)^-1 or
// (1 - e)^-1/2 to e^2, error O(e^3) ~ 1e-23) brings it to within an ulp or so
// with a dependency chain of three operations.  No special-case handling:
// callers only pass positive finite arguments (r = 0 is masked by the caller).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double rcp64(double a)
{
    const double r = __builtin_amdgcn_rcp(a);
    const double e = fma(-a, r, 1.0);             // 1/a = r / (1 - e)
    return fma(r, fma(e, e, e), r);               // r (1 + e + e^2)
}

__device__ __forceinline__ double rsq64(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    const double e = fma(-a * y, y, 1.0);         // a^-1/2 = y (1 - e)^-1/2
    const double c = e * fma(e, 0.375, 0.5);      // e/2 + 3 e^2/8
    return fma(y, c, y);
}

// sqrt(a) for positive finite a from the refined reciprocal square root, to
// an ulp or two (the step controller's error scales need no more).
__device__ __forceinline__ double sqrt_pos(double a) { return a * rsq64(a); }

// NFW mass integral I(q) = ln(1+q) - q/(1+q) (Eq. nfw), branch-free for q >= 0.
// 1+q = m 2^e with e = round(log2(1+q)) (the exponent of (1+q) sqrt(2), so m
// lies in [sqrt(1/2), sqrt(2)) up to rounding), ln(1+q) = e ln2 + 2 atanh(s),
// s = (m-1)/(m+1) = N/D with N = q - (2^e - 1) (2^e - 1 is an exact integer,
// so N is the correctly rounded value of 1 + q - 2^e, and s = q/(2+q) when
// e = 0) and D = (1+q) + 2^e.  With 1/m = 2^e/(1+q), the identity
//   2s - q/(1+q) = s^2 (1 + 1/m) + (1 - 2^e)/(1+q)
// gives one form for every e:
//   I = e ln2 + (1 - 2^e)/(1+q) + s^2 (1 + 1/m) + 2 (atanh(s) - s),
// with atanh(s) - s = s^3/3 + s^5/5 + ... + s^19/19 (|s| <= 0.1716).  At e = 0
// the first two terms are exactly zero and the others positive (relative error
// a few ulp for any q); above, the error is a few ulp of the largest term (up
// to ~30 ulp of I just above q = sqrt(2) - 1, where e ln2 and (1 - 2^e)/(1+q)
// cancel to a twenty-fifth of their size).  One reciprocal serves both
// divisions: 1/(D (1+q)).
__device__ __forceinline__ double nfw_I(double q)
{
    const double w0 = 1.0 + q;
    const int e = __builtin_amdgcn_frexp_exp(w0 * 1.4142135623730951) - 1;
    const double p2 = __builtin_amdgcn_ldexp(1.0, e);        // 2^e
    const double N = q - (p2 - 1.0), D = w0 + p2;
    const double rp = rcp64(D * w0);
    const double s = N * (w0 * rp);                          // (m-1)/(m+1)
    const double iw = D * rp;                                // 1/(1+q)
    const double s2 = s * s;
    // 2 s^-3 (atanh(s) - s) = sum_{k=0..8} 2 s2^k / (2k+3) (the next term adds
    // less than 1e-17 to I for |s| <= 0.1716), one Horner chain in s2: the
    // kernels are bound by instruction issue, not by this chain's latency
    double p = fma(s2, 2.0 / 19.0, 2.0 / 17.0);
    p = fma(s2, p, 2.0 / 15.0);
    p = fma(s2, p, 2.0 / 13.0);
    p = fma(s2, p, 2.0 / 11.0);
    p = fma(s2, p, 2.0 / 9.0);
    p = fma(s2, p, 2.0 / 7.0);
    p = fma(s2, p, 2.0 / 5.0);
    p = fma(s2, p, 2.0 / 3.0);
    const double t3 = s * s2 * p;                            // 2 (atanh(s) - s)
    const double small = fma(s2, fma(p2, iw, 1.0), t3);      // s^2 (1 + 1/m) + t3
    // ln 2 as the Cody-Waite pair of fdlibm's log: a high part whose products
    // with small integers are exact, and the remainder
    const double de = (double)e;
    return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, fma(-p2, iw, iw))) + small;
}

// |v|^2 with a fixed operation order (the final and initial speeds must round
// identically so that an untouched velocity gives a ratio of exactly 1).
__device__ __forceinline__ double norm2(double a, double b) { return fma(a, a, b * b); }

// ---------------------------------------------------------------------------
// coefficients and right-hand side
// ---------------------------------------------------------------------------

// 4-point Lagrange (cubic) interpolation on a uniform grid: interval i
// (nodes i..i+1) uses nodes i-1..i+2, the stencil shifted inward in the first
// and last interval.
struct Stencil4 {
    int i1;   // the node at the interval's start: the rows are i1-1 .. i1+2
    double wa, wb, wc, wd;
};

// Weights of nodes i-1..i+2 at fractional position p = s - i.
// With a = p (p-1) and b = (p+1)(p-2) = a - 2:
//   wa = -a (p-2)/6, wb = b (p-1)/2, wc = -b p/2, wd = a (p+1)/6.
__device__ __forceinline__ void stencil_weights(double p, Stencil4 &w)
{
    const double a = fma(p, p, -p);
    const double a6 = a * (1.0 / 6.0);
    const double b2 = fma(a, 0.5, -1.0);     // (a - 2)/2, the same rounding
    w.wa = a6 * (2.0 - p);
    w.wb = fma(b2, p, -b2);
    w.wc = -(b2 * p);
    w.wd = fma(a6, p, a6);
}

// Interval of grid coordinate s on n nodes, clamped to [1, n-3].
__device__ __forceinline__ int stencil_interval(int n, double s)
{
    const int i = (int)s;
    return i < 1 ? 1 : (i > n - 3 ? n - 3 : i);
}

// The same for the coefficient tables, as one three-operand integer median
// (for a bound that is not a constant the compiler emits a compare and a
// select or a min and a max).  The bound is a scalar register where n is
// wave-uniform and a vector register otherwise; either form of the
// instruction computes the lane's own clamp.
__device__ __forceinline__ int table_interval(int n, double s)
{
    int i;
    asm("v_med3_i32 %0, %1, 1, %2" : "=v"(i) : "v"((int)s), "s"(n - 3));
    return i;
}

// Stencil of the coefficient table (nodes u_i = u0 + i du) at u.
__device__ __forceinline__ Stencil4 stencil_at(int n_tab, double u0, double inv_du, double u)
{
    const double s = fma(u, inv_du, -(u0 * inv_du));
    const int i = table_interval(n_tab, s);
    Stencil4 w;
    w.i1 = i;
    stencil_weights(s - (double)i, w);
    return w;
}

// The same restricted to the piece of a sampled history that holds u (Knots):
// the stencil's first node is kept within [k m, (k+1) m - 3] for the piece
// [k m, (k+1) m] of table nodes.  With one piece (m = n_tab - 1) this is
// stencil_at, bit for bit.
__device__ __forceinline__ Stencil4 stencil_at_knots(int n_tab, double u0, double inv_du, const Knots &kn, double u)
{
    const double s = fma(u, inv_du, -(u0 * inv_du));
    const int i = (int)s;
    const int lo = (int)(s * kn.inv_m) * kn.m;
    const int hi = min(lo + kn.m - 3, n_tab - 4);
    const int row = min(max(i - 1, lo), hi);
    Stencil4 w;
    w.i1 = row + 1;
    stencil_weights(s - (double)(row + 1), w);
    return w;
}

template <bool HIST>
__device__ __forceinline__ Stencil4 table_stencil(int n_tab, double u0, double inv_du, const Knots &kn, double u)
{
    if constexpr (HIST) return stencil_at_knots(n_tab, u0, inv_du, kn, u);
    else return stencil_at(n_tab, u0, inv_du, u);
}

// Row `row` of a table of rows of `stride` doubles.  The byte offset is a
// 24-bit multiply (full rate; a 32-bit one is quarter rate): tables have far
// fewer than 2^24 / (8 stride) rows.
__device__ __forceinline__ const double *tab_row(const double *tab, int row, int stride)
{
    return (const double *)((const char *)tab + __umul24((unsigned)row, (unsigned)stride * 8u));
}

// The first row of a stencil, addressed from its interval's node i1 and the
// table base moved back one row (a constant offset), so that no i1 - 1 is
// formed per lookup.
__device__ __forceinline__ const double *stencil_rows(const double *tab, const Stencil4 &w, int stride)
{
    return tab_row(tab - stride, w.i1, stride);
}

// Column k of the interpolated coefficients from rows of `stride` doubles.
// The sum runs node by node as one FMA chain, so that the five-node form
// below reproduces it bit for bit.
__device__ __forceinline__ double stencil_col(const Stencil4 &w, const double *row, int stride, int k)
{
    return fma(w.wd, row[3 * stride + k], fma(w.wc, row[2 * stride + k], fma(w.wb, row[stride + k], w.wa * row[k])));
}

// Coefficients at u from the uniform table, rows of STRIDE doubles of which
// the first NC columns are used (NC = NCOL - 1 when the compensation radius R
// is constant and passed separately).
template <int NC, int STRIDE = NC, bool HIST = false>
__device__ __forceinline__ void coef_interp(const double *__restrict__ tab, int n_tab, double u0,
                                            double inv_du, const Knots &kn, double u, double c[NCOL])
{
    const Stencil4 w = table_stencil<HIST>(n_tab, u0, inv_du, kn, u);
    const double *row = stencil_rows(tab, w, STRIDE);
#pragma unroll
    for (int k = 0; k < NC; ++k) c[k] = stencil_col(w, row, STRIDE, k);
}

// Coefficients at two abscissae a fraction of a step apart (uQ at or below
// uP).  When their stencils start on the same or adjacent nodes, the five
// rows from Q's first node serve both, P's weights shifted by the difference
// (a zero weight on the unused end row); lanes whose stencils lie further
// apart read P's own four rows.  Either way the values equal those of two
// coef_interp calls bit for bit: an FMA with a zero weight adds an exact zero.
// The fifth row index is clamped to the table, where its weight is always zero.
template <int NC, int STRIDE = NC, bool HIST = false>
__device__ __forceinline__ void coef_interp2(const double *__restrict__ tab, int n_tab, double u0,
                                             double inv_du, const Knots &kn, double uP, double uQ,
                                             double cP[NCOL], double cQ[NCOL])
{
    const Stencil4 wQ = table_stencil<HIST>(n_tab, u0, inv_du, kn, uQ);
    const Stencil4 wP = table_stencil<HIST>(n_tab, u0, inv_du, kn, uP);
    const double *row = stencil_rows(tab, wQ, STRIDE);
    const double *row4 = tab_row(tab, min(wQ.i1 + 3, n_tab - 1), STRIDE);
    const int d = wP.i1 - wQ.i1;
    const bool s = d == 1;
    const double v0 = s ? 0.0 : wP.wa, v1 = s ? wP.wa : wP.wb, v2 = s ? wP.wb : wP.wc;
    const double v3 = s ? wP.wc : wP.wd, v4 = s ? wP.wd : 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const double r0 = row[k], r1 = row[STRIDE + k], r2 = row[2 * STRIDE + k], r3 = row[3 * STRIDE + k];
        cQ[k] = fma(wQ.wd, r3, fma(wQ.wc, r2, fma(wQ.wb, r1, wQ.wa * r0)));
        cP[k] = fma(v4, row4[k], fma(v3, r3, fma(v2, r2, fma(v1, r1, v0 * r0))));
    }
    if ((unsigned)d > 1u) {
        const double *rp = stencil_rows(tab, wP, STRIDE);
#pragma unroll
        for (int k = 0; k < NC; ++k) cP[k] = stencil_col(wP, rp, STRIDE, k);
    }
}

// The same from a split table: the drift column A from `a`, one value per node
// (device memory, read through the vector cache), the other four columns
// (K, Kc, 1/s, c) from LDS rows of `stride` doubles.  The values equal those
// of coef_interp / coef_interp2 on the whole table bit for bit: each column
// is the same FMA chain over the same four (or five) node values.
__device__ __forceinline__ double stencil_a(const Stencil4 &w, const double *a)
{
    return fma(w.wd, a[3], fma(w.wc, a[2], fma(w.wb, a[1], w.wa * a[0])));
}

template <int STRIDE, bool HIST = false>
__device__ __forceinline__ void coef_interp_split(const double *__restrict__ lds, const double *__restrict__ a,
                                                  int n_tab, double u0, double inv_du, const Knots &kn, double u,
                                                  double c[NCOL])
{
    const Stencil4 w = table_stencil<HIST>(n_tab, u0, inv_du, kn, u);
    c[COL_A] = stencil_a(w, (a - 1) + (unsigned)w.i1);
    const double *row = stencil_rows(lds, w, STRIDE);
#pragma unroll
    for (int k = 0; k < 4; ++k) c[COL_K + k] = stencil_col(w, row, STRIDE, k);
}

template <int STRIDE, bool HIST = false>
__device__ __forceinline__ void coef_interp2_split(const double *__restrict__ lds, const double *__restrict__ a,
                                                   int n_tab, double u0, double inv_du, const Knots &kn, double uP,
                                                   double uQ, double cP[NCOL], double cQ[NCOL])
{
    const Stencil4 wQ = table_stencil<HIST>(n_tab, u0, inv_du, kn, uQ);
    const Stencil4 wP = table_stencil<HIST>(n_tab, u0, inv_du, kn, uP);
    const int row4i = min(wQ.i1 + 3, n_tab - 1);
    const double *row = stencil_rows(lds, wQ, STRIDE);
    const double *row4 = tab_row(lds, row4i, STRIDE);
    const double *aq = (a - 1) + (unsigned)wQ.i1;
    const int d = wP.i1 - wQ.i1;
    const bool s = d == 1;
    const double v0 = s ? 0.0 : wP.wa, v1 = s ? wP.wa : wP.wb, v2 = s ? wP.wb : wP.wc;
    const double v3 = s ? wP.wc : wP.wd, v4 = s ? wP.wd : 0.0;
    {
        const double r0 = aq[0], r1 = aq[1], r2 = aq[2], r3 = aq[3];
        cQ[COL_A] = fma(wQ.wd, r3, fma(wQ.wc, r2, fma(wQ.wb, r1, wQ.wa * r0)));
        cP[COL_A] = fma(v4, a[(unsigned)row4i], fma(v3, r3, fma(v2, r2, fma(v1, r1, v0 * r0))));
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double r0 = row[k], r1 = row[STRIDE + k], r2 = row[2 * STRIDE + k], r3 = row[3 * STRIDE + k];
        cQ[COL_K + k] = fma(wQ.wd, r3, fma(wQ.wc, r2, fma(wQ.wb, r1, wQ.wa * r0)));
        cP[COL_K + k] = fma(v4, row4[k], fma(v3, r3, fma(v2, r2, fma(v1, r1, v0 * r0))));
    }
    if ((unsigned)d > 1u) {
        cP[COL_A] = stencil_a(wP, (a - 1) + (unsigned)wP.i1);
        const double *rp = stencil_rows(lds, wP, STRIDE);
#pragma unroll
        for (int k = 0; k < 4; ++k) cP[COL_K + k] = stencil_col(wP, rp, STRIDE, k);
    }
}

// Elementary functions of the power-law factors below, written for the
// bounded arguments they take there (|x| of a few units).
//
// ln 2 as the Cody-Waite pair of fdlibm (high part exact in products with
// small integers, and the remainder).
constexpr double LN2_HI = 6.93147180369123816490e-01, LN2_LO = 1.90821492927058770002e-10;

// x = k ln2 + r with k = rint(x / ln2), |r| <= ln2/2 (Cody-Waite reduction).
__device__ __forceinline__ double reduce_ln2(double x, double &k)
{
    k = __builtin_rint(x * 1.4426950408889634);
    return fma(-k, LN2_LO, fma(-k, LN2_HI, x));
}

// (e^r - 1)/r for |r| <= ln2/2 by its Taylor series to r^12 (the first
// omitted term is below 2^-58 of the sum there), Horner in r.
__device__ __forceinline__ double expm1_over_r(double r)
{
    double p = 1.0 / 6227020800.0;                                   // 1/13!
    p = fma(p, r, 1.0 / 479001600.0);
    p = fma(p, r, 1.0 / 39916800.0);
    p = fma(p, r, 1.0 / 3628800.0);
    p = fma(p, r, 1.0 / 362880.0);
    p = fma(p, r, 1.0 / 40320.0);
    p = fma(p, r, 1.0 / 5040.0);
    p = fma(p, r, 1.0 / 720.0);
    p = fma(p, r, 1.0 / 120.0);
    p = fma(p, r, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    return fma(p, r, 1.0);
}

// e^x = 2^k e^r, an ulp or two.
__device__ __forceinline__ double exp_small(double x)
{
    double k;
    const double r = reduce_ln2(x, k);
    return __builtin_amdgcn_ldexp(fma(r, expm1_over_r(r), 1.0), (int)k);
}

// e^x - 1 = 2^k (e^r - 1) + (2^k - 1): with k = 0 (|x| <= ln2/2) the series
// value itself, so small results keep their relative accuracy.
__device__ __forceinline__ double expm1_small(double x)
{
    double k;
    const double r = reduce_ln2(x, k);
    const double t = __builtin_amdgcn_ldexp(1.0, (int)k);
    return fma(t, r * expm1_over_r(r), t - 1.0);
}

// ln x for x > 0: x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln x = e ln2 +
// 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716, the atanh series to s^21 (as two
// interleaved Horner chains).  An ulp or two.
__device__ __forceinline__ double log_pos(double x)
{
    const int e = __builtin_amdgcn_frexp_exp(x * 1.4142135623730951) - 1;
    const double m = __builtin_amdgcn_ldexp(x, -e);
    const double s = (m - 1.0) * rcp64(m + 1.0);
    const double s2 = s * s, z2 = s2 * s2;
    double pe = fma(z2, 2.0 / 19.0, 2.0 / 15.0), po = fma(z2, 2.0 / 21.0, 2.0 / 17.0);
    pe = fma(z2, pe, 2.0 / 11.0);
    po = fma(z2, po, 2.0 / 13.0);
    pe = fma(z2, pe, 2.0 / 7.0);
    po = fma(z2, po, 2.0 / 9.0);
    pe = fma(z2, pe, 2.0 / 3.0);
    po = fma(z2, po, 2.0 / 5.0);
    const double t3 = s * s2 * fma(s2, po, pe);                        // 2 (atanh(s) - s)
    const double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, fma(s, 2.0, t3)));
}

// The power-law factor of K and Kc at u (PowFactor): xi^alpha of the paper's
// growth model and kappa = 1 + a [z/(1+z)]^b (Sec. IV.A, IV.B), from the
// functions above (an ulp or two each; fewer instructions than the
// library's routines); 0^alpha = 0 (alpha > 0 wherever it applies).  Not
// inlined: in the trajectory loops its temporaries would spill.
__device__ __noinline__ double pow_factor(const PowFactor &f, double u)
{
    double s = 1.0;
    if (f.on_mass) {
        const double xi = fmin(fmax((f.zf1 - exp_small(-u)) * f.inv_dz, 0.0), 1.0);
        s = xi > 0.0 ? exp_small(f.alpha * log_pos(xi)) : 0.0;
    }
    if (f.on_kappa) {
        const double zr = -expm1_small(u);   // z / (1+z)
        s *= 1.0 + (zr > 0.0 ? f.ka * exp_small(f.kb * log_pos(zr)) : 0.0);
    }
    return s;
}

// dY/du for Y = (x, y, vx, vy): dx/du = A v, dv/du = -g x with
// g = K I(min(r/s, c)) / r^3 - Kc inside R and 0 outside (and at r = 0).
//
// Kc = K I(c) / R^3, and the NFW truncation radius c s never exceeds R on the
// integration interval (validation keeps the paper geometry at z <= z_i; the
// Delta-200 one has c s = R / 200^(1/3)).  Inside R the bracket is therefore
// >= 0: the NFW fraction of the mass within r, I(q)/I(c), is at least the
// uniform sphere's (r/R)^3.  At and beyond R it is <= 0, since I(q) <= I(c)
// and r^3 >= R^3, where the enclosed perturbation is zero.  max(g, 0) thus
// gives both cases without a compare (R is not needed).  At r = 0 the
// reciprocal square root makes g NaN, and max(NaN, 0) = 0: no force there.
__device__ __forceinline__ double rhs_g(const double c[NCOL], double x, double y)
{
    const double r2 = x * x + y * y;
    const double ri = rsq64(r2);
    const double r = r2 * ri;
    const double q = fmin(r * c[COL_INVS], c[COL_C]);
    const double I = nfw_I(q);
    return fmax(fma(c[COL_K] * I, ri * ri * ri, -c[COL_KC]), 0.0);
}

__device__ __forceinline__ void rhs(const double c[NCOL], double R, double x, double y, double vx,
                                    double vy, double &dx, double &dy, double &dvx, double &dvy)
{
    (void)R;
    const double g = rhs_g(c, x, y);
    dx = c[COL_A] * vx;
    dy = c[COL_A] * vy;
    dvx = -g * x;
    dvy = -g * y;
}

// App. B: a relic whose straight backward path x0 - v0 s, 0 <= s <= D, stays
// at or beyond R_exit (the largest compensation radius) never feels the halo,
// so its momentum is final.  x0 = (r0, 0); R2 = R_exit^2 with a 1e-9 margin.
__device__ __forceinline__ bool never_enters(double r0, double vx0, double vy0, double D, double R2)
{
    double s = r0 * vx0 / norm2(vx0, vy0);
    s = s < 0.0 ? 0.0 : (s > D ? D : s);
    const double px = r0 - vx0 * s, py = -(vy0 * s);
    return norm2(px, py) >= R2;
}

__device__ __forceinline__ double cull_radius2(double r_exit) { return r_exit * r_exit * (1.0 + 1.0e-9); }

// Relic distribution before the halo formed, y = P / (k_B T).
__device__ __forceinline__ double f0_eval(const F0Desc &f, double y)
{
    if (f.kind == NH_F0_FREEZE_IN) return exp(-y) / sqrt(y);
    if (f.kind == NH_F0_TABLE) {
        // ln f0 from its samples in ln y: the cubic through the four samples
        // around ln y inside the range, the end interval's line outside it
        const double s = (log(y) - f.x0) * f.inv_dx;
        const double *v = f.ln_f;
        const int n = f.n;
        double lf;
        if (s < 0.0) {
            lf = v[0] + (v[1] - v[0]) * s;
        } else if (s > (double)(n - 1)) {
            lf = v[n - 1] + (v[n - 1] - v[n - 2]) * (s - (double)(n - 1));
        } else {
            const int i = stencil_interval(n, s);
            Stencil4 w;
            stencil_weights(s - (double)i, w);
            lf = w.wa * v[i - 1] + w.wb * v[i] + w.wc * v[i + 1] + w.wd * v[i + 2];
        }
        return exp(lf);
    }
    return 1.0 / (1.0 + exp(y));
}

// Index arithmetic below runs in 32 bits whenever the launch has fewer than
// 2^32 trajectories (a wave-uniform test): a 64-bit integer division is a
// long software sequence on the vector unit, a 32-bit one a few instructions,
// and a lane pays for them each time it starts or finishes a trajectory.
__device__ __forceinline__ bool idx32(const TrajParams &P) { return P.n_traj <= 0xffffffffLL; }

// Trajectory t = (k n_y + j) n_mu + l -> radius k, momentum j, angle l.
struct TrajIdx {
    int k, j, l;
};

__device__ __forceinline__ TrajIdx traj_idx(long long t, const TrajParams &P)
{
    if (idx32(P)) {
        const unsigned u = (unsigned)t, nm = (unsigned)P.n_mu, ny = (unsigned)P.n_y;
        const unsigned kj = u / nm, k = kj / ny;
        return TrajIdx{(int)k, (int)(kj - k * ny), (int)(u - kj * nm)};
    }
    const long long kj = t / P.n_mu, k = kj / P.n_y;
    return TrajIdx{(int)k, (int)(kj - k * P.n_y), (int)(t - kj * P.n_mu)};
}

template <class I>
__device__ __forceinline__ I traj_of_w(I p, const TrajParams &P)
{
    const I n_mu = (I)P.n_mu, n_y = (I)P.n_y, n_r = (I)P.n_r;
    if (P.order == ORDER_SLOW_FIRST) {
        const I q = p / n_mu, l = p - q * n_mu;
        const I j = q / n_r, k = q - j * n_r;
        return (k * n_y + j) * n_mu + l;
    }
    if (P.order == ORDER_SPREAD) {
        // full 64-trajectory blocks, in rounds of one block per wave of the
        // grid; a round is a (waves per workgroup) x (workgroups) matrix read
        // column-wise, so consecutive blocks - neighbouring radii and momenta,
        // similar in cost - are claimed by different workgroups
        const I P_ = (I)(blockDim.x >> 6), Q_ = (I)gridDim.x, W_ = P_ * Q_;
        const I nbf = (I)(P.n_traj >> 6), b = p >> 6;
        const I full_rounds = nbf / W_;
        if (b < full_rounds * W_) {
            const I r = b / W_, i = b - r * W_;
            const I i_p = i / P_;
            return ((r * W_ + (i - i_p * P_) * Q_ + i_p) << 6) + (p & 63);
        }
        return p;
    }
    if (P.order == ORDER_Y_FASTEST) {
        const I q = p / n_y, j = p - q * n_y;
        const I k = q / n_mu, l = q - k * n_mu;
        return (k * n_y + j) * n_mu + l;
    }
    return p;
}

// Queue position -> trajectory index.
__device__ __forceinline__ long long traj_of(long long p, const TrajParams &P)
{
    if (idx32(P)) return (long long)traj_of_w<unsigned>((unsigned)p, P);
    return traj_of_w<long long>(p, P);
}

// A wavefront's share of the work queue: positions [next, end) it has taken
// from the global counter but not yet handed to its lanes.  A wavefront takes
// QUEUE_BLOCK positions at a time, so the counter (a device-scope atomic,
// performed at the memory side and waited for by the whole wavefront) is
// touched once per QUEUE_BLOCK trajectories instead of once per pass in which
// some lane finished.  Which lane runs which trajectory does not change any
// result.  Positions past the end of the queue mean it is drained.
constexpr unsigned QUEUE_BLOCK = 64;
struct WaveQueue {
    unsigned long long next, end;
};

// Hands the lanes that ask for work (`need`) the wavefront's next positions,
// in lane order, taking a new block when the wavefront's share runs out;
// returns this lane's position (meaningful if `need`).  Called by every lane
// of the wavefront (the new block is taken by lane 0); q stays wave-uniform.
__device__ __forceinline__ long long wave_claim(bool need, unsigned long long *counter, WaveQueue &q)
{
    const unsigned long long mask = __ballot(need);
    if (mask == 0ull) return -1;
    const unsigned n = (unsigned)__popcll(mask);
    const int lane = __lane_id();
    const unsigned rank = (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
    const unsigned long long have = q.end - q.next;
    long long pos;
    if (have >= n) {
        pos = (long long)(q.next + rank);
        q.next += n;
    } else {
        // the rest of this share, then a fresh block (n <= 64 = QUEUE_BLOCK)
        unsigned long long nb = 0;
        if (lane == 0) nb = atomicAdd(counter, (unsigned long long)QUEUE_BLOCK);
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)nb);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(nb >> 32));
        nb = ((unsigned long long)hi << 32) | lo;
        pos = (long long)(rank < have ? q.next + rank : nb + (rank - have));
        q.next = nb + (n - have);
        q.end = nb + QUEUE_BLOCK;
    }
    return pos;
}

// Step-size factor of the controller, min(fmax, max(0.2, 0.9 err^(-1/5))),
// from err^2, as exact as the rest of the FP64 step: adaptive step sequences
// are discontinuous in the accept/reject decisions.  y = err2^(-1/10) starts
// from the FP32 hardware log2/exp2 (relative error ~1e-6) and takes two Newton
// steps y <- y + y (1 - err2 y^10) / 10 (each squares the error, times 5.5).
// Outside [1e-8, 1e7] the clamps decide: 0.9 y > 5.6 below, < 0.18 above.
// Branch-free (the iteration runs on err2 clamped to that range and selects
// pick the clamps' values), so that the lanes of a wavefront that accept and
// those that reject share one instruction stream.  err2 must be finite.
__device__ __forceinline__ double step_factor(double err2, double fcap)
{
    const double e = fmin(fmax(err2, 1.0e-8), 1.0e7);
    const float l2 = __builtin_amdgcn_logf((float)e);
    double y = (double)__builtin_amdgcn_exp2f(-0.1f * l2);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double y2 = y * y, y4 = y2 * y2, y10 = y4 * y4 * y2;
        y = fma(0.1 * y, fma(-e, y10, 1.0), y);
    }
    const double f = fmin(fcap, fmax(0.2, 0.9 * y));
    return err2 < 1.0e-8 ? fcap : (err2 > 1.0e7 ? 0.2 : f);
}

}  // namespace nh

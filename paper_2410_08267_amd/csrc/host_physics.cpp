// Host-side FP64 physics of a request: validation, the coefficient tables the
// kernels interpolate, and the quadrature rules.
//
// Halo model: Sec. II.B (Eqs. rhototal, nfw) with the enclosed mass of App. A
// (attractive sign); background and EOM: Sec. II.A, Eq. (eoms), written in
// u = ln a; growth variants and G(z): Sec. IV.A, IV.B.
#include <algorithm>
#include <cmath>
#include <thread>
#include <cstdio>
#include <cstring>

#include "nh_internal.h"

namespace nh {

namespace {
constexpr double kCbrt200 = 5.8480354764257312;   // 200^(1/3)
}

double nfw_I_host(double q)
{
    // I(q) = ln(1+q) - q/(1+q); below q = 0.01 the Taylor series
    // sum_{k=2..13} (-1)^k (k-1)/k q^k avoids the cancellation.
    if (q < 1.0e-2) {
        double acc = 0.0;
        for (int k = 13; k >= 2; --k) {
            double ck = (double)(k - 1) / (double)k;
            acc = acc * q + ((k & 1) ? -ck : ck);
        }
        return acc * q * q;
    }
    return std::log1p(q) - q / (1.0 + q);
}

void spline_second_derivatives(const double *v, int n, double dx, double *m2)
{
    // Continuity of the first derivative at the interior nodes gives
    // m[i-1] + 4 m[i] + m[i+1] = 6 (v[i-1] - 2 v[i] + v[i+1]) / dx^2, i = 1..n-2.
    // Not-a-knot (third derivative continuous at nodes 1 and n-2) gives
    // m0 = 2 m1 - m2 and m[n-1] = 2 m[n-2] - m[n-3]; substituted, the first and
    // last equations become 6 m1 = r1 and 6 m[n-2] = r[n-2].  Thomas algorithm.
    const int k = n - 2;                       // unknowns m[1..n-2]
    std::vector<double> a(k), b(k), c(k), r(k);
    for (int j = 0; j < k; ++j) {
        const int i = j + 1;
        a[j] = 1.0;
        b[j] = 4.0;
        c[j] = 1.0;
        r[j] = 6.0 * (v[i - 1] - 2.0 * v[i] + v[i + 1]) / (dx * dx);
    }
    b[0] = 6.0;
    c[0] = 0.0;
    b[k - 1] = 6.0;
    a[k - 1] = 0.0;
    for (int j = 1; j < k; ++j) {
        const double w = a[j] / b[j - 1];
        b[j] -= w * c[j - 1];
        r[j] -= w * r[j - 1];
    }
    m2[k] = r[k - 1] / b[k - 1];
    for (int j = k - 2; j >= 0; --j) m2[j + 1] = (r[j] - c[j] * m2[j + 2]) / b[j];
    m2[0] = 2.0 * m2[1] - m2[2];
    m2[n - 1] = 2.0 * m2[n - 2] - m2[n - 3];
}

double spline_eval(const double *v, const double *m2, int n, double x0, double dx, double x)
{
    const double s = (x - x0) / dx;
    int i = (int)std::floor(s);
    i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
    const double t = s - (double)i, w = 1.0 - t;
    return w * v[i] + t * v[i + 1] + dx * dx / 6.0 * ((w * w * w - w) * m2[i] + (t * t * t - t) * m2[i + 1]);
}

double Physics::history(const double *v, const std::vector<double> &v2, double z) const
{
    const double u = -std::log1p(z);
    return spline_eval(v, v2.data(), hist_n, hist_u_min, (0.0 - hist_u_min) / (double)(hist_n - 1), u);
}

Physics::Physics(const nh_request &q)
{
    G = GM_SUN_SI / (KPC_IN_M * 1.0e6);
    H0k = q.cosmo.H0_km_s_Mpc / 1000.0;
    Om = q.cosmo.Omega_m;
    OL = q.cosmo.Omega_L;
    mass_kind = q.halo.mass_kind;
    M0 = q.halo.M0_Msun;
    alpha = q.halo.mass_alpha;
    z_form = q.halo.z_form;
    beta = q.halo.mass_beta;
    conc_kind = q.halo.conc_kind;
    c0 = q.halo.c0;
    gamma = q.halo.conc_gamma;
    kappa_kind = q.halo.kappa_kind;
    ka = q.halo.kappa_a;
    kb = q.halo.kappa_b;
    geometry = q.halo.geometry;
    compensated = q.halo.compensated;
    z_obs = q.integ.z_obs;
    u_start = -std::log1p(z_obs);
    const nh_history &hs = q.halo.history;
    if (mass_kind == NH_MASS_TABLE || conc_kind == NH_CONC_TABLE || kappa_kind == NH_KAPPA_TABLE) {
        hist_n = hs.n;
        hist_u_min = -std::log1p(hs.z_max);
        hist_M = hs.M_Msun;
        hist_c = hs.c;
        hist_kappa = hs.kappa;
        const double du = (0.0 - hist_u_min) / (double)(hist_n - 1);
        if (mass_kind == NH_MASS_TABLE) {
            hist_M2.resize(hist_n);
            spline_second_derivatives(hist_M, hist_n, du, hist_M2.data());
        }
        if (conc_kind == NH_CONC_TABLE) {
            hist_c2.resize(hist_n);
            spline_second_derivatives(hist_c, hist_n, du, hist_c2.data());
        }
        if (kappa_kind == NH_KAPPA_TABLE) {
            hist_kappa2.resize(hist_n);
            spline_second_derivatives(hist_kappa, hist_n, du, hist_kappa2.data());
        }
    }
    // M(z_obs) = (4 pi/3) R^3 rhobar_m0, rhobar_m0 = 3 Om H0^2 / (8 pi G)  =>  R^3 = 2 G M / (Om H0^2)
    R_fixed = std::cbrt(2.0 * G * mass(z_obs) / (Om * H0k * H0k));
    // power-law factors the tables leave out (see PowFactor): xi^alpha unless it
    // is linear in e^{-u} over the whole interval (alpha = 1 with xi > 0 up to
    // z_end) or constant (alpha = 0); kappa = 1 + a [z/(1+z)]^b always
    const double z_end = q.integ.z_end;
    pw.on_mass = mass_kind == NH_MASS_PAPER && alpha > 0.0 && (alpha != 1.0 || z_form < z_end);
    pw.on_kappa = kappa_kind == NH_KAPPA_PAPER;
    pw.zf1 = 1.0 + z_form;
    pw.inv_dz = 1.0 / (z_form - z_obs);
    pw.alpha = alpha;
    pw.ka = ka;
    pw.kb = kb;
}

double Physics::pow_factor(double u) const
{
    double f = 1.0;
    if (pw.on_mass) {
        double xi = (pw.zf1 - std::exp(-u)) * pw.inv_dz;
        xi = xi < 0.0 ? 0.0 : (xi > 1.0 ? 1.0 : xi);
        f = std::pow(xi, pw.alpha);
    }
    if (pw.on_kappa) f *= 1.0 + pw.ka * std::pow(-std::expm1(u), pw.kb);
    return f;
}

double Physics::mass(double z) const
{
    switch (mass_kind) {
    case NH_MASS_PAPER: {
        double xi = (z_form - z) / (z_form - z_obs);
        xi = xi < 0.0 ? 0.0 : (xi > 1.0 ? 1.0 : xi);
        return M0 * std::pow(xi, alpha);
    }
    case NH_MASS_EXPONENTIAL:
        return M0 * std::exp(-beta * z);
    case NH_MASS_TABLE:
        return history(hist_M, hist_M2, z);
    default:
        return 0.0;
    }
}

double Physics::conc(double z) const
{
    if (conc_kind == NH_CONC_TABLE) return history(hist_c, hist_c2, z);
    return conc_kind == NH_CONC_POWER ? c0 * std::pow(1.0 + z, -gamma) : c0;
}

double Physics::kappa(double z) const
{
    switch (kappa_kind) {
    case NH_KAPPA_LOG: return 1.0 + ka * std::log1p(z);
    case NH_KAPPA_PAPER: return 1.0 + ka * std::pow(z / (1.0 + z), kb);
    case NH_KAPPA_CONSTANT: return ka;
    case NH_KAPPA_TABLE: return history(hist_kappa, hist_kappa2, z);
    default: return 1.0;
    }
}

double Physics::hubble(double z) const
{
    double opz = 1.0 + z;
    return H0k * std::sqrt(Om * opz * opz * opz + OL);
}

void Physics::coef(double u, double out[NCOL], bool factored) const
{
    const double opz = std::exp(-u);
    const double z = std::expm1(-u);
    const double H = H0k * std::sqrt(Om * opz * opz * opz + OL);
    out[COL_A] = opz * opz / H;
    const double M = mass(z);
    // the mass and G(z) that K and Kc carry: without the power-law factors
    // when the kernels apply those (M = M0 xi^alpha, kappa = 1 + a s^b)
    const double MK = (factored && pw.on_mass) ? M0 : M;
    const double kK = (factored && pw.on_kappa) ? 1.0 : kappa(z);
    const double c = conc(z);
    out[COL_C] = c;
    if (M == 0.0 && geometry == NH_GEOM_DELTA200) {
        // no halo and no radius at this epoch (validation keeps such epochs
        // off the tabulated interval when they would be interpolated)
        out[COL_K] = 0.0;
        out[COL_KC] = 0.0;
        out[COL_INVS] = 0.0;
        out[COL_R] = 0.0;
        return;
    }
    double R, rv;
    if (geometry == NH_GEOM_DELTA200) {
        R = std::cbrt(2.0 * G * M / (Om * H0k * H0k));
        rv = R / kCbrt200;
    } else {
        R = R_fixed;
        rv = (R_fixed / kCbrt200) * (opz / (1.0 + z_obs));   // fixed physical r200, comoving image
    }
    const double B = kK * G * opz / H;
    out[COL_K] = B * MK / nfw_I_host(c);
    out[COL_KC] = compensated ? B * MK / (R * R * R) : 0.0;
    out[COL_INVS] = c / rv;
    out[COL_R] = compensated ? R : 1.0e300;
}

double Physics::r_exit(double u_end) const
{
    // Beyond the largest compensation radius over [u_end, u_start] the force is
    // exactly zero; an outward-moving relic there never returns (backward
    // motion is along -v, and x.v <= 0 makes |x - s v| grow with s).
    if (!compensated || mass_kind == NH_MASS_ZERO) return compensated ? 0.0 : -1.0;
    if (geometry == NH_GEOM_PAPER) return R_fixed;
    double Rmax = 0.0;
    const int n = 4097;
    for (int i = 0; i < n; ++i) {
        double u = u_start + (u_end - u_start) * (double)i / (double)(n - 1);
        double M = mass(std::expm1(-u));
        double R = std::cbrt(2.0 * G * M / (Om * H0k * H0k));
        Rmax = R > Rmax ? R : Rmax;
    }
    // a sampled M(z) may peak between the scan points: keep a margin so the
    // exit stays exact
    return mass_kind == NH_MASS_TABLE ? Rmax * 1.001 : Rmax;
}

double Physics::drift(double u_end) const
{
    // composite Simpson over 2048 intervals of A(u) = e^{-2u} / H(u) (smooth, so
    // the error is ~1e-13 relative; the cull that uses it keeps a 1e-9 margin)
    const int n = 2048;
    const double h = (u_start - u_end) / n;
    auto A = [&](double u) {
        const double opz = std::exp(-u);
        return opz * opz / (H0k * std::sqrt(Om * opz * opz * opz + OL));
    };
    double s = A(u_end) + A(u_start);
    for (int i = 1; i < n; ++i) s += (i & 1 ? 4.0 : 2.0) * A(u_end + i * h);
    return s * h / 3.0;
}

// FP64: 3073 nodes over u in [-ln 5, 0], cubic interpolation error below
// ~2e-13 relative for the columns of the benchmark halos (checked on the host).
// FP32C: 2049 nodes (~1e-12, far below FP32 rounding), so that two tables of
// the precision form's layout fit one workgroup's LDS in the batched form.
int default_table_nodes(bool f32c) { return f32c ? 2049 : 3073; }

TableGrid table_grid(const Physics &ph, double u_end, int n_max)
{
    TableGrid g;
    if (!ph.sampled()) {
        g.n = n_max;
        g.u0 = u_end;
        g.du = (ph.u_start - u_end) / (double)(n_max - 1);
        g.m = n_max - 1;
        return g;
    }
    const double dh = (0.0 - ph.hist_u_min) / (double)(ph.hist_n - 1);
    int k0 = (int)std::floor((u_end - ph.hist_u_min) / dh);
    int k1 = (int)std::ceil((ph.u_start - ph.hist_u_min) / dh);
    k0 = std::max(0, std::min(k0, ph.hist_n - 2));
    k1 = std::max(k0 + 1, std::min(k1, ph.hist_n - 1));
    const int pieces = k1 - k0;
    g.m = (n_max - 1) / pieces;
    g.n = pieces * g.m + 1;
    g.u0 = ph.hist_u_min + (double)k0 * dh;
    g.du = dh / (double)g.m;
    return g;
}

bool sampled_table_fits(const nh_request *q, int n_max)
{
    const nh_history &h = q->halo.history;
    const bool sampled = q->halo.mass_kind == NH_MASS_TABLE || q->halo.conc_kind == NH_CONC_TABLE ||
                         q->halo.kappa_kind == NH_KAPPA_TABLE;
    if (!sampled || q->integ.method == NH_RK4) return true;
    // at most every sample interval can hold a piece of [u_end, u_start]
    return (n_max - 1) / (h.n - 1) >= 3;
}

void build_interp_table(const Physics &ph, const TableGrid &tg, double *out, int threads)
{
    const int n_tab = tg.n;
    auto rows = [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i) {
            // smooth histories end exactly on u_start; sampled ones on a knot
            double u = (i == n_tab - 1 && !ph.sampled()) ? ph.u_start : tg.u0 + (double)i * tg.du;
            ph.coef(u, out + (size_t)i * NCOL, true);
        }
    };
    // rows are independent: a few host threads may share a large table (the
    // plain solve builds one per request while the device waits; batches
    // already build their requests' tables in parallel)
    const int nt = n_tab >= 1024 ? std::min(threads, (int)std::max(1u, std::thread::hardware_concurrency())) : 1;
    if (nt <= 1) {
        rows(0, n_tab);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    const int chunk = (n_tab + nt - 1) / nt;
    for (int w = 1; w < nt; ++w) th.emplace_back(rows, std::min(n_tab, w * chunk), std::min(n_tab, (w + 1) * chunk));
    rows(0, std::min(n_tab, chunk));
    for (auto &t : th) t.join();
}

void build_rk4_table(const Physics &ph, double u_end, int n_steps, double *out)
{
    // Stage abscissae u_m = u_start + m (u_end - u_start) / (2N), m = 0..2N.
    const double hh = (u_end - ph.u_start) / (double)(2 * n_steps);
    for (int m = 0; m <= 2 * n_steps; ++m) ph.coef(ph.u_start + (double)m * hh, out + (size_t)m * NCOL);
}

void gauss_legendre(int n, double *x, double *w)
{
    // Newton iteration on P_n from Tricomi's initial guesses; nodes ascending.
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double t = std::cos(pi * ((double)i + 0.75) / ((double)n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / (double)k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        // final derivative at the converged node
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / (double)k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = t; p0 = 1.0; }
        dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
        double wi = 2.0 / ((1.0 - t * t) * dp * dp);
        x[i] = -t;
        x[n - 1 - i] = t;
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n & 1) x[n / 2] = 0.0;
}

void y_weights(int n, const double *y, double *w)
{
    // trapezoid in ln y of int dy y^2 f(y) = int dlny y^3 f(y); half weights at the ends
    for (int j = 0; j < n; ++j) {
        double d;
        if (j == 0) d = 0.5 * (std::log(y[1]) - std::log(y[0]));
        else if (j == n - 1) d = 0.5 * (std::log(y[n - 1]) - std::log(y[n - 2]));
        else d = 0.5 * (std::log(y[j + 1]) - std::log(y[j - 1]));
        w[j] = y[j] * y[j] * y[j] * d;
    }
}

long long n_traj_of(const nh_request *q)
{
    return (long long)q->grid.n_r * (long long)q->grid.n_y * (long long)q->grid.n_mu;
}

#define NH_BAD(...)                                   \
    do {                                              \
        if (msg) std::snprintf(msg, msg_len, __VA_ARGS__); \
        return NH_EINVAL;                             \
    } while (0)

int validate(const nh_request *q, char *msg, size_t msg_len)
{
    if (!q) NH_BAD("request is NULL");
    const nh_cosmology &c = q->cosmo;
    if (!std::isfinite(c.H0_km_s_Mpc) || c.H0_km_s_Mpc <= 0) NH_BAD("H0 must be finite and > 0");
    if (!std::isfinite(c.Omega_m) || c.Omega_m <= 0) NH_BAD("Omega_m must be finite and > 0");
    if (!std::isfinite(c.Omega_L) || c.Omega_L < 0) NH_BAD("Omega_L must be finite and >= 0");
    if (std::fabs(c.Omega_m + c.Omega_L - 1.0) > 1e-12) NH_BAD("background must be flat: |Om + OL - 1| <= 1e-12");
    const nh_halo &h = q->halo;
    if (h.mass_kind < NH_MASS_ZERO || h.mass_kind > NH_MASS_TABLE) NH_BAD("unknown mass_kind %d", h.mass_kind);
    if (h.mass_kind != NH_MASS_ZERO && h.mass_kind != NH_MASS_TABLE && (!std::isfinite(h.M0_Msun) || h.M0_Msun <= 0))
        NH_BAD("M0 must be finite and > 0");
    if (h.mass_kind == NH_MASS_PAPER) {
        if (!std::isfinite(h.z_form) || h.z_form <= 0) NH_BAD("z_form must be finite and > 0");
        if (!std::isfinite(h.mass_alpha) || h.mass_alpha < 0) NH_BAD("mass_alpha must be finite and >= 0");
    }
    if (h.mass_kind == NH_MASS_EXPONENTIAL && !std::isfinite(h.mass_beta)) NH_BAD("mass_beta must be finite");
    if (h.conc_kind < NH_CONC_CONSTANT || h.conc_kind > NH_CONC_TABLE) NH_BAD("unknown conc_kind %d", h.conc_kind);
    if (h.conc_kind != NH_CONC_TABLE && (!std::isfinite(h.c0) || h.c0 <= 0)) NH_BAD("c0 must be finite and > 0");
    if (!std::isfinite(h.conc_gamma)) NH_BAD("conc_gamma must be finite");
    if (h.kappa_kind < NH_KAPPA_NONE || h.kappa_kind > NH_KAPPA_TABLE) NH_BAD("unknown kappa_kind %d", h.kappa_kind);
    const bool tabulated = h.mass_kind == NH_MASS_TABLE || h.conc_kind == NH_CONC_TABLE || h.kappa_kind == NH_KAPPA_TABLE;
    if (tabulated) {
        const nh_history &hs = h.history;
        if (hs.n < 4 || hs.n > (1 << 24)) NH_BAD("history needs n in [4, 2^24] samples");
        if (!std::isfinite(hs.z_max) || hs.z_max <= 0) NH_BAD("history z_max must be finite and > 0");
        if (!(hs.z_max >= q->integ.z_end)) NH_BAD("history must cover z_end: z_max >= z_end");
        const double *arrs[3] = {h.mass_kind == NH_MASS_TABLE ? hs.M_Msun : nullptr,
                                 h.conc_kind == NH_CONC_TABLE ? hs.c : nullptr,
                                 h.kappa_kind == NH_KAPPA_TABLE ? hs.kappa : nullptr};
        const bool need[3] = {h.mass_kind == NH_MASS_TABLE, h.conc_kind == NH_CONC_TABLE,
                              h.kappa_kind == NH_KAPPA_TABLE};
        const char *names[3] = {"M_Msun", "c", "kappa"};
        for (int a = 0; a < 3; ++a) {
            if (!need[a]) continue;
            if (!arrs[a]) NH_BAD("history.%s is required", names[a]);
            for (int i = 0; i < hs.n; ++i)
                if (!std::isfinite(arrs[a][i])) NH_BAD("history.%s[%d] must be finite", names[a], i);
        }
        if (need[0]) {
            for (int i = 0; i < hs.n; ++i) {
                if (hs.M_Msun[i] < 0) NH_BAD("history.M_Msun[%d] must be >= 0", i);
                if (h.geometry == NH_GEOM_DELTA200 && !(hs.M_Msun[i] > 0))
                    NH_BAD("delta200 geometry needs M > 0 at every sample (index %d)", i);
            }
            if (!(hs.M_Msun[hs.n - 1] > 0)) NH_BAD("history.M_Msun at z = 0 (the last sample) must be > 0");
        }
        if (need[1]) {
            // the spline must stay positive: check the samples and 8 points per interval
            const double dx = 1.0 / (double)(hs.n - 1);
            for (int i = 0; i < hs.n; ++i)
                if (!(hs.c[i] > 0)) NH_BAD("history.c[%d] must be > 0", i);
            std::vector<double> m2(hs.n);
            spline_second_derivatives(hs.c, hs.n, dx, m2.data());
            for (int i = 0; i + 1 < hs.n; ++i)
                for (int k = 1; k < 8; ++k)
                    if (!(spline_eval(hs.c, m2.data(), hs.n, 0.0, dx, (i + k / 8.0) * dx) > 0))
                        NH_BAD("the interpolated concentration is not positive near sample %d", i);
        }
    }
    if (!std::isfinite(h.kappa_a) || !std::isfinite(h.kappa_b)) NH_BAD("kappa parameters must be finite");
    if (h.geometry != NH_GEOM_PAPER && h.geometry != NH_GEOM_DELTA200) NH_BAD("unknown geometry %d", h.geometry);
    if (h.compensated != 0 && h.compensated != 1) NH_BAD("compensated must be 0 or 1");
    if (!std::isfinite(q->m_eV) || q->m_eV <= 0) NH_BAD("m_eV must be finite and > 0");
    if (q->f0.kind != NH_F0_FERMI_DIRAC && q->f0.kind != NH_F0_FREEZE_IN && q->f0.kind != NH_F0_TABLE)
        NH_BAD("unknown f0 kind %d", q->f0.kind);
    if (q->f0.kind == NH_F0_TABLE) {
        const nh_f0 &f = q->f0;
        if (f.n < 4 || f.n > (1 << 20)) NH_BAD("f0 table needs n in [4, 2^20] samples");
        if (!std::isfinite(f.ln_y0) || !std::isfinite(f.d_ln_y) || !(f.d_ln_y > 0))
            NH_BAD("f0 table needs finite ln_y0 and d_ln_y > 0");
        if (!f.ln_f) NH_BAD("f0 table values are required");
        for (int i = 0; i < f.n; ++i)
            if (!std::isfinite(f.ln_f[i])) NH_BAD("f0 ln_f[%d] must be finite", i);
    }
    if (!std::isfinite(q->f0.T_K) || q->f0.T_K <= 0) NH_BAD("T_K must be finite and > 0");
    const nh_grid &g = q->grid;
    if (g.n_r < 1 || !g.r_kpc) NH_BAD("need n_r >= 1 radii");
    for (int k = 0; k < g.n_r; ++k)
        if (!std::isfinite(g.r_kpc[k]) || g.r_kpc[k] <= 0) NH_BAD("radius %d must be finite and > 0", k);
    if (g.n_y < 2 || !g.y) NH_BAD("need n_y >= 2 momenta");
    for (int j = 0; j < g.n_y; ++j) {
        if (!std::isfinite(g.y[j]) || g.y[j] <= 0) NH_BAD("y[%d] must be finite and > 0", j);
        if (j > 0 && !(g.y[j] > g.y[j - 1])) NH_BAD("y must be strictly ascending (index %d)", j);
    }
    if (g.n_mu < 1 || g.n_mu > 4096) NH_BAD("n_mu must be in [1, 4096]");
    if (g.mu) {
        if (!g.w_mu) NH_BAD("w_mu is required when mu is given");
        for (int l = 0; l < g.n_mu; ++l) {
            if (!std::isfinite(g.mu[l]) || std::fabs(g.mu[l]) >= 1.0) NH_BAD("mu[%d] must satisfy |mu| < 1", l);
            if (!std::isfinite(g.w_mu[l])) NH_BAD("w_mu[%d] must be finite", l);
        }
    }
    const nh_integrator &it = q->integ;
    if (!std::isfinite(it.z_end) || it.z_end <= 0) NH_BAD("z_end must be finite and > 0");
    if (!std::isfinite(it.z_obs) || it.z_obs < 0) NH_BAD("z_obs must be finite and >= 0");
    if (!(it.z_end > it.z_obs)) NH_BAD("z_end must exceed z_obs");
    if (h.geometry == NH_GEOM_PAPER && h.mass_kind != NH_MASS_ZERO &&
        it.z_end > (1.0 + it.z_obs) * kCbrt200 - 1.0 + 1e-12)
        NH_BAD("paper geometry is defined up to z_i = (1 + z_obs) 200^(1/3) - 1");
    if (h.mass_kind == NH_MASS_PAPER && !(h.z_form > it.z_obs)) NH_BAD("z_form must exceed z_obs");
    if (h.geometry == NH_GEOM_DELTA200 && h.mass_kind == NH_MASS_PAPER && !(it.z_end < h.z_form))
        NH_BAD("delta200 geometry needs M(z_end) > 0: z_end < z_form");
    if (it.method == NH_RK4) {
        if (it.n_steps < 1 || it.n_steps > 1000000) NH_BAD("n_steps must be in [1, 1e6]");
        if (it.precision != NH_FP64) NH_BAD("RK4 runs in FP64 only");
    } else if (it.method == NH_DOPRI5) {
        if (!std::isfinite(it.rtol) || it.rtol < 1e-15 || it.rtol >= 1.0) NH_BAD("rtol must be in [1e-15, 1)");
        if (!std::isfinite(it.atol_x) || !std::isfinite(it.atol_v) || !std::isfinite(it.h0)) NH_BAD("atol/h0 must be finite");
    } else {
        NH_BAD("unknown method %d", it.method);
    }
    if (it.precision != NH_FP64 && it.precision != NH_FP32C) NH_BAD("unknown precision %d", it.precision);
    long long nt = n_traj_of(q);
    if (nt > (1LL << 40)) NH_BAD("too many trajectories");
    return NH_OK;
}

}  // namespace nh

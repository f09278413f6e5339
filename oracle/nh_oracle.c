/*
 * nh_oracle.c -- plain FP64 CPU oracle for the backward N-1-body relic
 * trajectories of Worku, Sabti & Kamionkowski (arXiv:2410.08267).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * It is deliberately slow and literal: one trajectory at a time, the halo
 * enclosed mass evaluated from its closed form at every right-hand-side call,
 * no tables, no blocking, no fused arithmetic (built with -ffp-contract=off).
 *
 * What it computes (paper references by section / equation):
 *   background   flat FRW, H(z) = H0 [Om (1+z)^3 + OL]^(1/2)           Sec. II.A
 *   halo         rho_tot of Eq. (rhototal) with the NFW profile of
 *                Eq. (nfw); enclosed perturbation deltaM(r,z) obtained by
 *                integrating rho_tot - rhobar (App. A gives the same
 *                magnitude); mass scaling xi(z) or a chosen M(z), c(z)   Sec. II.B, App. A
 *   force        dPhi/dr = G (1+z) deltaM / r^2 (attractive; the printed
 *                minus sign in Eqs. (Poisson_equation), (potential_derivative)
 *                and App. A is read as a typo because Phi ~ -1/r there)   Sec. II.A, App. A
 *   EOM          Eq. (eoms) re-parametrised from z to u = ln a = -ln(1+z):
 *                  dx/du =  (1+z)^2 / H * v
 *                  dv/du = -kappa G (1+z) / H * deltaM * x / r^3          Sec. II.A, IV.B
 *   integration  backward in time from u = 0 (z0 = 0) to u_end < 0        Sec. II.C
 *                classical RK4 with N equal steps, or Dormand-Prince 5(4)
 *                (Dormand & Prince 1980) with the step control of Hairer,
 *                Norsett & Wanner, Solving ODEs I, Sec. II.4.
 *
 * Units: length kpc (comoving), velocity km/s (comoving v = a u_pec),
 * mass Msun, H in km/s/kpc, G in kpc (km/s)^2 / Msun.
 */
#include <math.h>
#include <stddef.h>
#include <float.h>

/* ---- physical constants (the paper states none; these are IAU/CODATA) ---- */
#define NHO_GM_SUN_SI 1.32712440018e20        /* m^3 s^-2, IAU 2015 nominal GM_sun */
#define NHO_KPC_M     3.0856775814913673e19   /* m per kpc (IAU 2012 au, 648000/pi au per pc) */
/* G in kpc (km/s)^2 / Msun: GM_sun / (1 kpc * (1000 m/km)^2) */
static double nho_G(void) { return NHO_GM_SUN_SI / (NHO_KPC_M * 1.0e6); }

typedef struct {
    /* flat FRW background (Sec. II.A) */
    double H0_km_s_Mpc;
    double Omega_m;
    double Omega_L;
    int    static_background;  /* test only: a == 1, u is plain time, no Hubble drag */
    /* halo (Sec. II.B) */
    int    mass_kind;          /* 0 none, 1 paper xi(z)^alpha * M_h, 2 M0 exp(-beta z), 3 point mass (test),
                                  4 sampled (hist_M) */
    double M0_Msun;
    double mass_alpha;         /* exponent of xi (Sec. IV.A); 1 is the base model */
    double z_form;             /* z_i of xi; 200^(1/3) - 1 in the base model */
    double mass_beta;          /* rate of the exponential M(z) */
    int    conc_kind;          /* 0 constant c0, 1 c0 (1+z)^(-gamma), 2 sampled (hist_c) */
    double c0;
    double conc_gamma;
    int    kappa_kind;         /* 0 none, 1 1 + a ln(1+z), 2 1 + a [z/(1+z)]^b, 3 constant a, 4 sampled
                                  (hist_kappa) (Sec. IV.B) */
    double kappa_a;
    double kappa_b;
    int    geometry;           /* 0 paper: fixed physical r200 = R / 200^(1/3); 1: 200 x mean density at each z */
    int    compensated;        /* 1 paper: underdense shell out to comoving R; 0 plain NFW + point mass */
    double z_obs;              /* observation redshift z0 (Sec. II.B): the halo's reference epoch */
    /* sampled histories: samples at u_i = hist_u_min + i (0 - hist_u_min) / (hist_n - 1), u = ln a,
       given as the pieces of their cubic spline: on [u_i, u_{i+1}] the value is
       p[4i] t^3 + p[4i+1] t^2 + p[4i+2] t + p[4i+3] with t = u - u_i */
    int           hist_n;
    double        hist_u_min;
    const double *hist_M;
    const double *hist_c;
    const double *hist_kappa;
    /* test only: a sampled factor multiplying H(z) in the equations of motion
       (pieces as above, NULL for none): a ripple of the expansion rate, which
       scales both the drift and the kick, probes how the step control responds
       to perturbations the size of a tabulated coefficient's error */
    const double *hist_hmod;
} nho_model;

typedef struct {
    int       method;          /* 0 classical RK4, fixed steps; 1 Dormand-Prince 5(4) adaptive;
                                  2 Dormand-Prince fifth-order solution with n_steps equal steps
                                  (test only: isolates the tableau from the step control) */
    int       n_steps;         /* RK4 step count */
    double    u_start;         /* -ln(1 + z_obs); 0 for observation today */
    double    u_end;           /* -ln(1 + z_end); below u_start for backward integration */
    double    rtol;
    double    atol_x;          /* kpc */
    double    atol_v;          /* km/s */
    double    h0;              /* first trial step in u (negative) */
    long long max_steps;       /* attempted-step budget per trajectory */
    /* Step-control settings for the tests (0 = the defaults of the reading the
       library implements): the largest step growth after an accepted step
       (default 5), and per-component error scales atol + rtol max(|y_i|,
       |y_i'|) instead of the position / velocity pair norms (a library
       integrator's convention, so the controller can be checked against it). */
    double    fmax;
    int       component_scales;
} nho_integ;

enum { NHO_OK = 0, NHO_MAXSTEPS = 1, NHO_UNDERFLOW = 2, NHO_NONFINITE = 3 };

/* ---------------------------------------------------------------------- */
/* background                                                             */
/* ---------------------------------------------------------------------- */

/* H(z) in km/s/kpc (Sec. II.A) */
double nho_hubble(const nho_model *m, double z)
{
    double H0k = m->H0_km_s_Mpc / 1000.0;
    double opz = 1.0 + z;
    return H0k * sqrt(m->Omega_m * opz * opz * opz + m->Omega_L);
}

double nho_G_value(void) { return nho_G(); }

/* ---------------------------------------------------------------------- */
/* halo model (Sec. II.B, App. A)                                          */
/* ---------------------------------------------------------------------- */

/* I(q) = ln(1+q) - q/(1+q), the NFW mass integral of Eq. (nfw).  Below
 * q = 0.01 the two terms cancel; there the Taylor series
 * sum_{k>=2} (-1)^k (k-1)/k q^k (twelve terms) replaces the difference. */
double nho_nfw_I(double q)
{
    if (q < 1.0e-2) {
        double sum = 0.0;
        double qk = q * q;
        for (int k = 2; k <= 13; ++k) {
            double term = ((double)(k - 1) / (double)k) * qk;
            sum += (k % 2 == 0) ? term : -term;
            qk *= q;
        }
        return sum;
    }
    return log1p(q) - q / (1.0 + q);
}

/* M(z): the perturbation's mass scale.  Paper: xi(z) M_h with
 * xi = [(z_i - z)/(z_i - z0)]^alpha clamped to [0,1], z0 = 0 (Sec. II.B, IV.A). */
/* A sampled history at redshift z: the spline piece of the interval that
 * holds u = ln a (the end pieces continue beyond the sampled range). */
static double nho_sampled(const nho_model *m, const double *p, double z)
{
    double u = -log1p(z);
    double du = (0.0 - m->hist_u_min) / (double)(m->hist_n - 1);
    int i = (int)floor((u - m->hist_u_min) / du);
    if (i < 0) i = 0;
    if (i > m->hist_n - 2) i = m->hist_n - 2;
    double t = u - (m->hist_u_min + (double)i * du);
    const double *c = p + 4 * i;
    return ((c[0] * t + c[1]) * t + c[2]) * t + c[3];
}

double nho_mass(const nho_model *m, double z)
{
    switch (m->mass_kind) {
    case 1: {
        double xi = (m->z_form - z) / (m->z_form - m->z_obs);
        if (xi < 0.0) xi = 0.0;
        if (xi > 1.0) xi = 1.0;
        return m->M0_Msun * pow(xi, m->mass_alpha);
    }
    case 2:
        return m->M0_Msun * exp(-m->mass_beta * z);
    case 3:
        return m->M0_Msun;
    case 4:
        return nho_sampled(m, m->hist_M, z);
    default:
        return 0.0;
    }
}

double nho_conc(const nho_model *m, double z)
{
    if (m->conc_kind == 1) return m->c0 * pow(1.0 + z, -m->conc_gamma);
    if (m->conc_kind == 2) return nho_sampled(m, m->hist_c, z);
    return m->c0;
}

/* kappa(z): multiplies G (Sec. IV.B) */
double nho_kappa(const nho_model *m, double z)
{
    switch (m->kappa_kind) {
    case 1: return 1.0 + m->kappa_a * log1p(z);
    case 2: return 1.0 + m->kappa_a * pow(z / (1.0 + z), m->kappa_b);
    case 3: return m->kappa_a;
    case 4: return nho_sampled(m, m->hist_kappa, z);
    default: return 1.0;
    }
}

/* Comoving radii of the halo at redshift z.
 * R: comoving Lagrangian radius, M = (4 pi/3) R^3 rhobar_m0 with
 *    rhobar_m0 = 3 Om H0^2 / (8 pi G), i.e. R^3 = 2 G M / (Om H0^2).
 * rv: comoving image of the NFW truncation radius.  Paper geometry: the
 *    physical r200 = R/(1+z_i) with (1+z_i)/(1+z0) = 200^(1/3) is fixed, so
 *    the comoving radius is r200 (1+z) and R uses M(z0), z0 the observation
 *    redshift.  Geometry 1: R and r200 = R / 200^(1/3) follow M(z). */
void nho_radii(const nho_model *m, double z, double *R, double *rv)
{
    double H0k = m->H0_km_s_Mpc / 1000.0;
    double fac = 2.0 * nho_G() / (m->Omega_m * H0k * H0k);
    double c200 = cbrt(200.0);
    if (m->geometry == 1) {
        *R = cbrt(fac * nho_mass(m, z));
        *rv = *R / c200;
    } else {
        *R = cbrt(fac * nho_mass(m, m->z_obs));
        *rv = (*R / c200) * ((1.0 + z) / (1.0 + m->z_obs));
    }
}

/* Enclosed mass perturbation inside comoving radius r at redshift z:
 * deltaM = int_0^{r/(1+z)} 4 pi r_p^2 [rho_tot - rhobar] dr_p with rho_tot of
 * Eq. (rhototal):
 *   r <  rv      : M(z) [ I(r/s)/I(c) - (r/R)^3 ]
 *   rv <= r < R  : M(z) [ 1 - (r/R)^3 ]
 *   r >= R       : 0
 * where s = rv/c is the comoving scale radius.  (r/R)^3 M is the mean mass
 * that the compensating underdensity removes. */
double nho_deltaM(const nho_model *m, double r, double z)
{
    double Mz = nho_mass(m, z);
    if (Mz == 0.0) return 0.0;
    if (m->mass_kind == 3) return Mz;
    double R, rv;
    nho_radii(m, z, &R, &rv);
    double c = nho_conc(m, z);
    double s = rv / c;
    if (m->compensated) {
        if (r >= R) return 0.0;
        double x = r / R;
        double comp = x * x * x;
        if (r < rv) return Mz * (nho_nfw_I(r / s) / nho_nfw_I(c) - comp);
        return Mz * (1.0 - comp);
    }
    if (r < rv) return Mz * nho_nfw_I(r / s) / nho_nfw_I(c);
    return Mz;
}

/* ---------------------------------------------------------------------- */
/* equations of motion in u = ln a                                         */
/* ---------------------------------------------------------------------- */

/* Y = (x, y, vx, vy).  From Eq. (eoms) with dz = -(1+z) du:
 *   dx/du = A v,             A = (1+z)^2 / H
 *   dv/du = -B deltaM x/r^3, B = kappa G (1+z) / H
 * At r == 0 the force direction is undefined and the acceleration is 0. */
void nho_rhs(const nho_model *m, double u, const double *Y, double *dY)
{
    double A, B, z;
    if (m->static_background) {
        z = 0.0;
        A = 1.0;
        B = nho_kappa(m, 0.0) * nho_G();
    } else {
        double opz = exp(-u);
        z = expm1(-u);
        double H = nho_hubble(m, z);
        if (m->hist_hmod) H *= nho_sampled(m, m->hist_hmod, z);
        A = opz * opz / H;
        B = nho_kappa(m, z) * nho_G() * opz / H;
    }
    double x = Y[0], y = Y[1];
    double r = sqrt(x * x + y * y);
    dY[0] = A * Y[2];
    dY[1] = A * Y[3];
    double dM = nho_deltaM(m, r, z);
    if (r > 0.0 && dM != 0.0) {
        double g = B * dM / (r * r * r);
        dY[2] = -g * x;
        dY[3] = -g * y;
    } else {
        dY[2] = 0.0;
        dY[3] = 0.0;
    }
}

/* ---------------------------------------------------------------------- */
/* classical RK4, N equal steps in u                                       */
/* ---------------------------------------------------------------------- */

/* Stage abscissae are u_m = u_start + m * ((u_end - u_start) / (2N)),
 * m = 0..2N, so that step n evaluates at u_{2n}, u_{2n+1} (twice) and u_{2n+2}. */
static int integrate_rk4(const nho_model *m, const nho_integ *it, double *Y,
                         long long *acc)
{
    int N = it->n_steps;
    double span = it->u_end - it->u_start;
    double h = span / (double)N;
    double hh = span / (double)(2 * N);
    double k1[4], k2[4], k3[4], k4[4], T[4];
    for (int n = 0; n < N; ++n) {
        double u0 = it->u_start + (double)(2 * n) * hh;
        double u1 = it->u_start + (double)(2 * n + 1) * hh;
        double u2 = it->u_start + (double)(2 * n + 2) * hh;
        nho_rhs(m, u0, Y, k1);
        for (int i = 0; i < 4; ++i) T[i] = Y[i] + 0.5 * h * k1[i];
        nho_rhs(m, u1, T, k2);
        for (int i = 0; i < 4; ++i) T[i] = Y[i] + 0.5 * h * k2[i];
        nho_rhs(m, u1, T, k3);
        for (int i = 0; i < 4; ++i) T[i] = Y[i] + h * k3[i];
        nho_rhs(m, u2, T, k4);
        for (int i = 0; i < 4; ++i)
            Y[i] = Y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        for (int i = 0; i < 4; ++i)
            if (!isfinite(Y[i])) { *acc = n + 1; return NHO_NONFINITE; }
    }
    *acc = N;
    return NHO_OK;
}

/* ---------------------------------------------------------------------- */
/* Dormand-Prince 5(4)                                                     */
/* ---------------------------------------------------------------------- */

/* Butcher tableau of Dormand & Prince (1980), fifth-order solution with the
 * embedded fourth-order solution for the error estimate; FSAL. */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0},
};
/* fifth-order weights b (= last row of A, b7 = 0) and fourth-order b* */
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_BS[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

/* Error control (Hairer, Norsett & Wanner I, Sec. II.4):
 *   err = sqrt( mean_i (E_i / sc_i)^2 ),  E = h sum_j (b_j - b*_j) k_j
 *   sc  = atol + rtol * max(|.|_n, |.|_{n+1}), with |.| the Euclidean norm of
 *         the position pair for the x, y components and of the velocity pair
 *         for the vx, vy components (it->component_scales: |y_i| itself);
 *   accept when err <= 1;
 *   h_new = h * min(fmax, max(0.2, 0.9 err^(-1/5))), fmax = 5 (it->fmax when
 *         set), and fmax = 1 for the step right after a rejection;
 *   the last step is cut to land on u_end. */
static int integrate_dp5(const nho_model *m, const nho_integ *it, double *Y,
                         long long *acc_out, long long *rej_out)
{
    const double u_end = it->u_end;
    const double dir = (u_end >= it->u_start) ? 1.0 : -1.0;
    const double fmax = it->fmax > 0.0 ? it->fmax : 5.0;
    double u = it->u_start;
    double h = dir * fabs(it->h0);
    if (fabs(h) > fabs(u_end - u)) h = u_end - u;
    double K[7][4], T[4], Y5[4];
    nho_rhs(m, u, Y, K[0]);
    long long acc = 0, rej = 0, attempts = 0;
    int rejected_prev = 0;
    int status = NHO_OK;
    for (;;) {
        if (attempts >= it->max_steps) { status = NHO_MAXSTEPS; break; }
        ++attempts;
        int last = 0;
        if (dir * (u + h - u_end) >= 0.0) { h = u_end - u; last = 1; }
        for (int s = 1; s < 7; ++s) {
            for (int i = 0; i < 4; ++i) {
                double sum = 0.0;
                for (int j = 0; j < s; ++j) sum += DP_A[s][j] * K[j][i];
                T[i] = Y[i] + h * sum;
            }
            if (s == 6)
                for (int i = 0; i < 4; ++i) Y5[i] = T[i];
            nho_rhs(m, u + DP_C[s] * h, T, K[s]);
        }
        double E[4];
        for (int i = 0; i < 4; ++i) {
            double sum = 0.0;
            for (int j = 0; j < 7; ++j) sum += (DP_B[j] - DP_BS[j]) * K[j][i];
            E[i] = h * sum;
        }
        double sc[4];
        if (it->component_scales) {
            for (int i = 0; i < 4; ++i) {
                double a0 = fabs(Y[i]), a1 = fabs(Y5[i]);
                sc[i] = (i < 2 ? it->atol_x : it->atol_v) + it->rtol * (a0 > a1 ? a0 : a1);
            }
        } else {
            double rx0 = sqrt(Y[0] * Y[0] + Y[1] * Y[1]);
            double rx1 = sqrt(Y5[0] * Y5[0] + Y5[1] * Y5[1]);
            double rv0 = sqrt(Y[2] * Y[2] + Y[3] * Y[3]);
            double rv1 = sqrt(Y5[2] * Y5[2] + Y5[3] * Y5[3]);
            sc[0] = sc[1] = it->atol_x + it->rtol * (rx0 > rx1 ? rx0 : rx1);
            sc[2] = sc[3] = it->atol_v + it->rtol * (rv0 > rv1 ? rv0 : rv1);
        }
        double sum = 0.0;
        for (int i = 0; i < 4; ++i) { double e = E[i] / sc[i]; sum += e * e; }
        double err = sqrt(sum / 4.0);
        if (!isfinite(err)) { status = NHO_NONFINITE; break; }
        if (err <= 1.0) {
            ++acc;
            u = last ? u_end : u + h;
            for (int i = 0; i < 4; ++i) { Y[i] = Y5[i]; K[0][i] = K[6][i]; }
            if (last) break;
            double fac = (err == 0.0) ? fmax : 0.9 * pow(err, -0.2);
            if (fac < 0.2) fac = 0.2;
            if (fac > fmax) fac = fmax;
            if (rejected_prev && fac > 1.0) fac = 1.0;
            h *= fac;
            rejected_prev = 0;
        } else {
            ++rej;
            double fac = 0.9 * pow(err, -0.2);
            if (fac < 0.2) fac = 0.2;
            h *= fac;
            rejected_prev = 1;
        }
        double umag = fabs(u) > 1.0 ? fabs(u) : 1.0;
        if (fabs(h) <= 4.0 * DBL_EPSILON * umag) { status = NHO_UNDERFLOW; break; }
    }
    *acc_out = acc;
    *rej_out = rej;
    return status;
}

/* Fixed-step use of the same tableau (method 2): every step accepted. */
static int integrate_dp5_fixed(const nho_model *m, const nho_integ *it, double *Y,
                               long long *acc)
{
    int N = it->n_steps;
    double h = (it->u_end - it->u_start) / (double)N;
    double K[7][4], T[4];
    for (int n = 0; n < N; ++n) {
        double u = it->u_start + (double)n * h;
        nho_rhs(m, u, Y, K[0]);
        for (int s = 1; s < 7; ++s) {
            for (int i = 0; i < 4; ++i) {
                double sum = 0.0;
                for (int j = 0; j < s; ++j) sum += DP_A[s][j] * K[j][i];
                T[i] = Y[i] + h * sum;
            }
            nho_rhs(m, u + DP_C[s] * h, T, K[s]);
        }
        for (int i = 0; i < 4; ++i) {
            double sum = 0.0;
            for (int j = 0; j < 7; ++j) sum += DP_B[j] * K[j][i];
            Y[i] = Y[i] + h * sum;
        }
    }
    *acc = N;
    return NHO_OK;
}

/* ---------------------------------------------------------------------- */
/* batch entry point                                                       */
/* ---------------------------------------------------------------------- */

/* Integrate n independent trajectories from it->u_start to it->u_end.
 * state: n x 4 array (x, y, vx, vy), overwritten with the final state.
 * acc, rej, status: n entries each (accepted / rejected steps, status code). */
void nho_integrate(const nho_model *m, const nho_integ *it, long n,
                   double *state, long long *acc, long long *rej, int *status)
{
    for (long t = 0; t < n; ++t) {
        double *Y = state + 4 * t;
        long long a = 0, r = 0;
        int st;
        if (it->method == 0)
            st = integrate_rk4(m, it, Y, &a);
        else if (it->method == 2)
            st = integrate_dp5_fixed(m, it, Y, &a);
        else
            st = integrate_dp5(m, it, Y, &a, &r);
        acc[t] = a;
        rej[t] = r;
        status[t] = st;
    }
}

/* Vectorised helpers for the tests: deltaM and the RHS on arrays. */
void nho_deltaM_many(const nho_model *m, long n, const double *r, const double *z, double *out)
{
    for (long i = 0; i < n; ++i) out[i] = nho_deltaM(m, r[i], z[i]);
}

void nho_rhs_many(const nho_model *m, long n, const double *u, const double *Y, double *dY)
{
    for (long i = 0; i < n; ++i) nho_rhs(m, u[i], Y + 4 * i, dY + 4 * i);
}

// Internal declarations shared by the host side of libnuhalo and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "nuhalo.h"

namespace nh {

// Coefficient columns of the equations of motion in u = ln a (Sec. II.A, Eq. eoms
// with dz = -(1+z) du; enclosed mass from Sec. II.B / App. A):
//   dx/du = A(u) v
//   dv/du = -[ K(u) I(min(r s^-1(u), c(u))) / r^3 - Kc(u) ] x   for r < R(u), else 0
// A = (1+z)^2/H, B = kappa G (1+z)/H, K = B M / I(c), Kc = B M / R^3.
enum Col : int { COL_A = 0, COL_K = 1, COL_KC = 2, COL_INVS = 3, COL_C = 4, COL_R = 5, NCOL = 6 };

// Trajectory status word: low byte is the outcome, bit 8 marks the exact free-streaming exit.
enum : int {
    ST_OK = 0,
    ST_MAXSTEPS = 1,
    ST_UNDERFLOW = 2,
    ST_NONFINITE = 3,
    ST_FREE_EXIT = 256,
};

// Queue position -> trajectory index orders for the persistent kernels.
enum : int {
    ORDER_NATURAL = 0,     // t = p
    ORDER_SLOW_FIRST = 1,  // p runs over (j, k, l) with l fastest: low-momentum relics first
    ORDER_Y_FASTEST = 2,   // p runs over (k, l, j) with j fastest: a wave shares radius and direction
    ORDER_SPREAD = 3,      // index order in blocks of 64, the blocks of each round of claims
                           // transposed so that neighbouring (costly) blocks go to different workgroups
};

// Power-law factors of the coefficients K and Kc (Sec. IV.A, IV.B).  The
// growth xi(z)^alpha of the paper's halo model and the paper's G modulation
// kappa = 1 + a [z/(1+z)]^b have an unbounded derivative where xi or z/(1+z)
// reaches 0 (alpha or b below 1), and xi has a kink where it is clamped; a
// cubic table through such a function is wrong near those points by far more
// than rounding.  Requests with either factor tabulate K and Kc without it, and
// the kernels multiply it back, evaluated exactly, at every stage.
struct PowFactor {
    int on_mass;            // M = M0 xi^alpha, xi = clamp((zf1 - e^{-u}) inv_dz, 0, 1)
    int on_kappa;           // kappa = 1 + ka s^kb, s = z/(1+z) = -expm1(u)
    double zf1;             // 1 + z_form
    double inv_dz;          // 1 / (z_form - z_obs)
    double alpha;
    double ka, kb;
};

// Sampled histories (the spline pieces between uniform knots in u, R22): the
// table nodes are placed so that every knot is a node and every piece spans
// m >= 3 table intervals, and the kernels keep each interpolation stencil
// inside one piece, where the history is an exact cubic (a stencil across a
// knot would see the jump of the spline's third derivative).  For smooth
// histories m = n_tab - 1: one piece spans the table, the usual stencil.
struct Knots {
    int m;                  // table intervals per piece
    double inv_m;           // 1 / m
};

// Everything a trajectory kernel needs about one request, passed by value.
struct TrajParams {
    // grid
    int n_r, n_y, n_mu;
    long long n_traj;
    double vfac;            // k_B T c / m: km/s per unit y
    // integration interval (u = ln a, backward from u_start = -ln(1 + z_obs))
    double u_start;
    double u_end;
    // interpolation table: n_tab nodes u_i = u_end + i * du, i = 0..n_tab-1 (DP5)
    int n_tab;
    double tab_u0;
    double tab_inv_du;
    // RK4: n_steps equal steps, stage abscissae m * hh
    int n_steps;
    double rk_h;
    // Dormand-Prince control
    double rtol, atol_x, atol_v, h0;
    long long max_steps;
    // exact free-streaming exit: beyond r_exit moving outward the force is zero forever
    double r_exit;          // <= 0 disables (and disables the cull below)
    double r_exit2;         // r_exit^2, +inf when disabled: set on the host (exit_radius2) so that
                            // the Dormand-Prince kernels hold it as a uniform scalar
    double cull_D;          // int_{u_end}^{u_start} A du: the straight backward path is x0 - v0 s, s <= cull_D;
                            // 0 where no start radius reaches R_exit (no relic can be culled)
    double R_const;         // > 0: the compensation radius is this constant (no R column)
    int order;              // ORDER_*
    int block;              // workgroup size of the persistent kernels
    int max_wg;             // > 0: at most this many workgroups (plain Dormand-Prince launches)
    // FP32-compensated form: steps with |h| below this run in FP64; the FP32
    // attempts integrate at max(rtol, rtol32)
    double h_fp64;
    double rtol32;
    // Dormand-Prince tables of non-smooth histories: power-law factors of K and
    // Kc applied at every stage, stencils kept inside spline pieces; hist = 1
    // when either is needed (the kernels' HIST variant)
    PowFactor pw;
    Knots kn;
    int hist;
};

// The squared free-streaming exit radius the Dormand-Prince kernels test
// against: +inf when the exit is off, so that the test needs no guard.
inline double exit_radius2(const TrajParams &P)
{
    return P.r_exit > 0.0 ? P.r_exit * P.r_exit : __builtin_inf();
}

// The relic's initial distribution as the reduction evaluates it.
struct F0Desc {
    int kind;               // NH_F0_*
    int n;                  // NH_F0_TABLE: samples of ln f0 at ln y = x0 + i dx
    double x0, inv_dx;
    const double *ln_f;     // device, n
};

// Device pointers of one request's staged inputs (one contiguous blob).
struct GridPtrs {
    const double *tab;      // n_tab * NCOL (DP5) or (2 n_steps + 1) * NCOL (RK4)
    const double *tabA;     // DP5: column COL_A of tab, n_tab values (the plain FP64 kernel's drift)
    const double *r;        // n_r
    const double *y;        // n_y
    const double *wy;       // n_y
    const double *mu;       // n_mu
    const double *smu;      // n_mu: sqrt(1 - mu^2)
    const double *wmu;      // n_mu
    F0Desc f0;
};

// Per-trajectory counters, written with one 16-byte store.
struct alignas(16) TrajStat {
    int acc;                // accepted steps
    int rej;                // rejected steps
    int status;             // ST_* word
    int fp64;               // attempts run in FP64 (FP32C form)
};

struct TrajOut {
    double *ratio;          // n_traj: |v_end| / |v0|
    TrajStat *stat;         // n_traj
};

// Device buffers of a fused quadrature (the trajectory kernels add each
// finished trajectory's term, nothing is stored per trajectory): num holds the
// 128-bit fixed-point sum of radius k in words 2k (low) and 2k+1 (high), den
// the background sum likewise, scale the power of two applied to every term,
// stats the six counters of the statistics.
struct QuadAcc {
    unsigned long long *num;
    unsigned long long *den;
    double *scale;
    unsigned long long *stats;
    int lds_n;    // radii 0 .. lds_n-1 summed per workgroup in LDS first (0: straight to num)
    int ring;     // FP64 trajectory kernel: finished trajectories wait in per-wavefront LDS
                  // rings and are summed 64 at a time (0: each when it finishes)
};

// ---- batched and serving forms (scheduling: nh_batch.h) ----

enum : int {
    POLICY_OPEN_FIRST = 0,      // open requests in order (a shared cursor: one workgroup each),
                                // then help the one with the most work left
    POLICY_UNOPENED_FIRST = 1,  // the oldest request nobody has drawn from yet, else help the
                                // one with the most work left (no cursor: the request list
                                // changes between slices)
    POLICY_SHARE = 2,           // the oldest request whose unclaimed work still gives every
                                // workgroup drawing from it, one more included, `share`
                                // trajectories (one nobody draws from: any work), else help
                                // the one with the most work left
};

// One request as the slice kernels see it (device array).
struct BatchReq {
    TrajParams P;
    GridPtrs g;               // staged inputs; g.tab rows of NCOL doubles
    TrajOut o;                // per-trajectory outputs of this request
    double *out;              // n_r profile
    int nc;                   // table columns used: NCOL, or NCOL - 1 when R is constant
    int free_all;             // no halo: every trajectory streams freely (ratio 1)
    int retired;              // cancelled: not claimed, saved lanes drop it
};

struct alignas(16) WgSave {
    int slot_req[2];
    int cur;
    int pad;
};

// Saved state of one lane between slices (FP64 or FP32C lane, raw words).
struct alignas(16) LaneSave {
    long long t;              // trajectory index, < 0: none
    int req, slot;
    unsigned long long w[14];
};

struct SliceArgs {
    const BatchReq *reqs;     // by request id
    unsigned long long *next; // per request id: queue position of the next unclaimed trajectory
    unsigned int *inflight;   // per request id: lanes saved with its trajectories at this slice's end
    const int *order;         // request ids of this launch, oldest first
    int n_order;
    int policy;               // POLICY_*
    unsigned long long *cursor;   // POLICY_OPEN_FIRST: next position of `order` to open
    int *helpers;             // POLICY_SHARE: per request id, workgroups drawing from it (a hint)
    long long share;          // POLICY_SHARE: unclaimed trajectories per workgroup to join
    int n_tab;                // table nodes of every request (slot capacity)
    long long budget_ticks;   // wall-clock ticks (100 MHz) until lanes save and exit; < 0: none
    LaneSave *lane_save;      // per thread of the grid, or null
    WgSave *wg_save;          // per workgroup, or null
    int resume;               // restore lanes and slots saved by the previous slice
};


// Host-side physics of one request, evaluated in FP64 (tables, validation).
struct Physics {
    double G, H0k, Om, OL;
    int mass_kind;
    double M0, alpha, z_form, beta;
    int conc_kind;
    double c0, gamma;
    int kappa_kind;
    double ka, kb;
    int geometry, compensated;
    double z_obs, u_start;  // observation epoch (the halo's reference epoch) and u = -ln(1+z_obs)
    double R_fixed;         // NH_GEOM_PAPER: comoving Lagrangian radius from M(z_obs)
    bool sampled() const { return hist_n > 0; }
    // sampled histories (the *_TABLE kinds): samples at u_i = hist_u_min + i du and
    // the second derivatives of their not-a-knot cubic splines
    int hist_n = 0;
    double hist_u_min = 0.0;
    const double *hist_M = nullptr, *hist_c = nullptr, *hist_kappa = nullptr;
    std::vector<double> hist_M2, hist_c2, hist_kappa2;

    explicit Physics(const nh_request &q);
    double history(const double *v, const std::vector<double> &v2, double z) const;
    double mass(double z) const;
    double conc(double z) const;
    double kappa(double z) const;
    double hubble(double z) const;
    // coefficients at u; factored = true leaves out the power-law factors of
    // K and Kc (pow_factor) that the kernels apply at every stage
    void coef(double u, double out[NCOL], bool factored = false) const;
    double pow_factor(double u) const;   // host value of the factor at u
    PowFactor pw{};                      // which factors this request's tables leave out
    double r_exit(double u_end) const;   // radius beyond which the force is zero at every u
    double drift(double u_end) const;    // int_{u_end}^{u_start} (1+z)^2 / H du
};

// Physical constants (the paper states only T_nu0 = 1.95 K).
constexpr double GM_SUN_SI = 1.32712440018e20;        // m^3 s^-2, IAU 2015 nominal
constexpr double KPC_IN_M = 3.0856775814913673e19;    // m
constexpr double KB_EV_PER_K = 1.380649e-23 / 1.602176634e-19;   // eV / K: k_B / e, exact in SI
constexpr double C_KM_S = 299792.458;                 // km / s

double nfw_I_host(double q);
// Not-a-knot cubic spline through samples v[0..n-1] on a uniform grid (n >= 4):
// spline_second_derivatives fills m2 with its second derivatives at the nodes,
// spline_eval evaluates it at x (the end pieces continue outside the grid).
void spline_second_derivatives(const double *v, int n, double dx, double *m2);
double spline_eval(const double *v, const double *m2, int n, double x0, double dx, double x);
void gauss_legendre(int n, double *x, double *w);
void y_weights(int n, const double *y, double *w);
int validate(const nh_request *q, char *msg, size_t msg_len);
long long n_traj_of(const nh_request *q);

// Table builders (host, FP64).
int default_table_nodes(bool f32c);
// The Dormand-Prince table's grid: n nodes u0 + i du.  Smooth histories: n_max
// nodes on [u_end, u_start].  Sampled histories: the knots at or around
// [u_end, u_start] with m = floor((n_max - 1) / pieces) table intervals per
// piece (m < 3 does not fit: sampled_table_fits).
struct TableGrid {
    int n;
    double u0, du;
    int m;
};
TableGrid table_grid(const Physics &ph, double u_end, int n_max);
bool sampled_table_fits(const nh_request *q, int n_max);
// K and Kc without the request's power-law factors (Physics::pw)
void build_interp_table(const Physics &ph, const TableGrid &tg, double *out, int threads = 1);
void build_rk4_table(const Physics &ph, double u_end, int n_steps, double *out);

}  // namespace nh

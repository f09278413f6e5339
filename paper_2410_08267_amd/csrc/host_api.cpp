// C ABI of libnuhalo: context, plain solve, statistics, diagnostics.
//
// Host work per request (all FP64): validation, the coefficient table of the
// equations of motion, the quadrature weights and Gauss-Legendre nodes.  They
// are packed into one pinned staging buffer and copied to the device in one
// transfer; everything after that runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "nh_context.h"
#include "nh_launch.h"

namespace nh {

thread_local char g_err[512] = "";

int set_err(nh_context *ctx, int code, const char *fmt, ...)
{
    char *dst = ctx ? ctx->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

int ensure_dev(nh_context *ctx, DevBuf &b, size_t bytes)
{
    if (bytes <= b.cap) return NH_OK;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return set_err(ctx, NH_EDEVICE, "hipFree: %s", hipGetErrorString(e));
    }
    size_t cap = std::max(bytes, (size_t)4096);
    hipError_t e = hipMalloc(&b.p, cap);
    if (e != hipSuccess) {
        b.p = nullptr;
        return set_err(ctx, NH_ENOMEM, "hipMalloc(%zu): %s", cap, hipGetErrorString(e));
    }
    b.cap = cap;
    return NH_OK;
}

int ensure_pinned(nh_context *ctx, size_t bytes)
{
    if (bytes <= ctx->h_stage_cap) return NH_OK;
    if (ctx->h_stage) {
        (void)hipHostFree(ctx->h_stage);
        ctx->h_stage = nullptr;
        ctx->h_stage_cap = 0;
    }
    size_t cap = std::max(bytes, (size_t)65536);
    hipError_t e = hipHostMalloc(&ctx->h_stage, cap, hipHostMallocDefault);
    if (e != hipSuccess) {
        ctx->h_stage = nullptr;
        return set_err(ctx, NH_ENOMEM, "hipHostMalloc(%zu): %s", cap, hipGetErrorString(e));
    }
    ctx->h_stage_cap = cap;
    return NH_OK;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Staged inputs of one request: layout and host construction.
Staged stage_layout(const nh_request *q, int table_nodes, int n_mass)
{
    Staged s{};
    const bool rk4 = q->integ.method == NH_RK4;
    s.n_tab = rk4 ? 2 * q->integ.n_steps + 1
                  : (table_nodes > 0 ? table_nodes : default_table_nodes(q->integ.precision == NH_FP32C));
    size_t off = 0;
    s.off_tab = off;  off = align_up(off + (size_t)s.n_tab * NCOL * sizeof(double));
    // Dormand-Prince: the drift column A once more, node by node (the plain
    // FP64 kernel reads it from here and the other columns from LDS)
    s.off_tabA = off; off = align_up(off + (rk4 ? 0 : (size_t)s.n_tab * sizeof(double)));
    s.off_r = off;    off = align_up(off + (size_t)q->grid.n_r * sizeof(double));
    s.off_y = off;    off = align_up(off + (size_t)q->grid.n_y * sizeof(double));
    s.off_wy = off;   off = align_up(off + (size_t)q->grid.n_y * sizeof(double));
    s.off_mu = off;   off = align_up(off + (size_t)q->grid.n_mu * sizeof(double));
    s.off_smu = off;  off = align_up(off + (size_t)q->grid.n_mu * sizeof(double));
    s.off_wmu = off;  off = align_up(off + (size_t)q->grid.n_mu * sizeof(double));
    s.f0_kind = q->f0.kind;
    s.f0_n = q->f0.kind == NH_F0_TABLE ? q->f0.n : 0;
    s.f0_x0 = q->f0.kind == NH_F0_TABLE ? q->f0.ln_y0 : 0.0;
    s.f0_inv_dx = q->f0.kind == NH_F0_TABLE ? 1.0 / q->f0.d_ln_y : 0.0;
    s.off_f0 = off;   off = align_up(off + (size_t)s.f0_n * sizeof(double));
    s.n_mass = n_mass;
    s.off_ym = off;   off = align_up(off + (size_t)n_mass * q->grid.n_y * sizeof(double));
    s.off_wm = off;   off = align_up(off + (size_t)n_mass * q->grid.n_y * sizeof(double));
    s.bytes = off;
    return s;
}

void stage_fill(const nh_request *q, const Staged &s, char *base, TrajParams &P, int table_threads,
                const double *m_eV)
{
    Physics ph(*q);
    const double u_end = -std::log1p(q->integ.z_end);
    const double u_start = -std::log1p(q->integ.z_obs);
    double *tab = (double *)(base + s.off_tab);
    std::memset(&P, 0, sizeof(P));
    P.n_r = q->grid.n_r;
    P.n_y = q->grid.n_y;
    P.n_mu = q->grid.n_mu;
    P.n_traj = n_traj_of(q);
    // km/s per unit y: v = P/m = y k_B T c / m (non-relativistic, Sec. II.D)
    P.vfac = KB_EV_PER_K * q->f0.T_K * C_KM_S / q->m_eV;
    P.u_start = u_start;
    P.u_end = u_end;
    if (q->integ.method == NH_RK4) {
        build_rk4_table(ph, u_end, q->integ.n_steps, tab);
        P.n_steps = q->integ.n_steps;
        P.rk_h = (u_end - u_start) / (double)q->integ.n_steps;
    } else {
        const TableGrid tg = table_grid(ph, u_end, s.n_tab);
        build_interp_table(ph, tg, tab, table_threads);
        double *tabA = (double *)(base + s.off_tabA);
        for (int i = 0; i < tg.n; ++i) tabA[i] = tab[(size_t)i * NCOL + COL_A];
        P.n_tab = tg.n;
        P.tab_u0 = tg.u0;
        P.tab_inv_du = ph.sampled() ? 1.0 / tg.du : (double)(tg.n - 1) / (u_start - u_end);
        P.kn.m = tg.m;
        P.kn.inv_m = 1.0 / (double)tg.m;
    }
    const double rt = q->integ.rtol;
    P.rtol = rt;
    P.atol_x = q->integ.atol_x > 0 ? q->integ.atol_x : rt * 1.0;
    P.atol_v = q->integ.atol_v > 0 ? q->integ.atol_v : rt * 1.0;
    P.h0 = q->integ.h0 != 0.0 ? q->integ.h0 : -1.0e-3;
    P.max_steps = q->integ.max_steps > 0 ? q->integ.max_steps : 1000000;
    if (P.max_steps > 2000000000LL) P.max_steps = 2000000000LL;
    P.r_exit = ph.r_exit(u_end);
    // App. B cull, enabled only where it can act: a relic that starts inside
    // R_exit is never farther than its start radius from the halo, so only
    // start radii at or beyond R_exit (with a margin) can hold culled relics
    P.cull_D = 0.0;
    if (P.r_exit > 0.0) {
        double rmax = 0.0;
        for (int k = 0; k < q->grid.n_r; ++k) rmax = std::max(rmax, q->grid.r_kpc[k]);
        if (rmax * rmax >= 0.999 * P.r_exit * P.r_exit) P.cull_D = ph.drift(u_end);
    }
    // paper geometry (or no compensation): R does not depend on u
    if (q->halo.geometry == NH_GEOM_PAPER || !q->halo.compensated)
        P.R_const = q->halo.compensated ? ph.R_fixed : 1.0e300;
    P.order = ORDER_SLOW_FIRST;
    P.h_fp64 = 0.0;
    // Dormand-Prince tables leave the power-law factors of K and Kc to the
    // kernels and keep stencils inside spline pieces; RK4 rows are exact
    // coefficients at the stage abscissae
    if (q->integ.method != NH_RK4) {
        P.pw = ph.pw;
        P.hist = (ph.pw.on_mass || ph.pw.on_kappa || ph.sampled()) ? 1 : 0;
    }

    std::memcpy(base + s.off_r, q->grid.r_kpc, sizeof(double) * q->grid.n_r);
    std::memcpy(base + s.off_y, q->grid.y, sizeof(double) * q->grid.n_y);
    y_weights(q->grid.n_y, q->grid.y, (double *)(base + s.off_wy));
    double *mu = (double *)(base + s.off_mu);
    double *smu = (double *)(base + s.off_smu);
    double *wmu = (double *)(base + s.off_wmu);
    if (q->grid.mu) {
        std::memcpy(mu, q->grid.mu, sizeof(double) * q->grid.n_mu);
        std::memcpy(wmu, q->grid.w_mu, sizeof(double) * q->grid.n_mu);
    } else {
        gauss_legendre(q->grid.n_mu, mu, wmu);
    }
    for (int l = 0; l < q->grid.n_mu; ++l) smu[l] = std::sqrt(1.0 - mu[l] * mu[l]);
    if (s.f0_n > 0) std::memcpy(base + s.off_f0, q->f0.ln_f, sizeof(double) * s.f0_n);
    // other masses: the same velocities are momenta y m_k / m, weights of that grid
    for (int k = 0; k < s.n_mass; ++k) {
        double *ym = (double *)(base + s.off_ym) + (size_t)k * q->grid.n_y;
        double *wm = (double *)(base + s.off_wm) + (size_t)k * q->grid.n_y;
        const double f = m_eV[k] / q->m_eV;
        for (int j = 0; j < q->grid.n_y; ++j) ym[j] = q->grid.y[j] * f;
        y_weights(q->grid.n_y, ym, wm);
    }
}

GridPtrs grid_ptrs(const Staged &s, const char *dev)
{
    GridPtrs g;
    g.tab = (const double *)(dev + s.off_tab);
    g.tabA = (const double *)(dev + s.off_tabA);
    g.r = (const double *)(dev + s.off_r);
    g.y = (const double *)(dev + s.off_y);
    g.wy = (const double *)(dev + s.off_wy);
    g.mu = (const double *)(dev + s.off_mu);
    g.smu = (const double *)(dev + s.off_smu);
    g.wmu = (const double *)(dev + s.off_wmu);
    g.f0.kind = s.f0_kind;
    g.f0.n = s.f0_n;
    g.f0.x0 = s.f0_x0;
    g.f0.inv_dx = s.f0_inv_dx;
    g.f0.ln_f = s.f0_n > 0 ? (const double *)(dev + s.off_f0) : nullptr;
    return g;
}

size_t per_traj_bytes(const nh_request *q)
{
    (void)q;
    return sizeof(double) + sizeof(TrajStat);
}

int wait_pending(nh_context *ctx)
{
    if (!ctx->pending) return NH_OK;
    HIPCHK(hipEventSynchronize(ctx->ev_done));
    return NH_OK;
}

int solve_launch(nh_context *ctx, const nh_request *q, const Staged &s, TrajParams P, const SolveBufs &b,
                 double *d_out, hipStream_t stream, int n_mass, double *d_integrand)
{
    const GridPtrs g = grid_ptrs(s, b.blob);
    const long long n = P.n_traj;
    const bool fused = b.qa.num != nullptr;
    const bool free_all = q->halo.mass_kind == NH_MASS_ZERO;
    unsigned long long *counter = b.small;
    unsigned long long *stats = counter + 8;
    HIPCHK(launch_fill_u64(counter, 16, 0ull, stream));
    if (fused) HIPCHK(launch_quad_setup(P, g, b.qa, stream));

    TrajOut o;
    o.ratio = b.ratio;
    o.stat = b.stat;
    const QuadAcc *qa = fused ? &b.qa : nullptr;

    HIPCHK(hipEventRecord(ctx->ev_t0, stream));
    if (free_all) {
        if (fused) HIPCHK(launch_fill_u64(stats + 5, 1, (unsigned long long)n, stream));   // all free exits
        else HIPCHK(launch_free_all(n, o, stream));
    } else if (q->integ.method == NH_RK4) {
        HIPCHK(launch_rk4_f64(P, g, o, qa, stream));
    } else {
        const bool f32 = q->integ.precision == NH_FP32C;
        if (f32) {
            P.h_fp64 = ctx->h_fp64;
            P.rtol32 = ctx->rtol32;
        }
        P.order = ctx->queue_order;
        P.block = ctx->block_threads > 0 ? ctx->block_threads : ctx->tuned_plain_block[f32];
        P.max_wg = ctx->max_workgroups;
        if (f32) HIPCHK(launch_dp5_f32c(P, g, o, counter, qa, ctx->n_cu, stream));
        else HIPCHK(launch_dp5_f64(P, g, o, counter, qa, ctx->n_cu, stream));
    }
    HIPCHK(hipEventRecord(ctx->ev_t1, stream));
    if (fused) {
        HIPCHK(launch_quad_finish(P.n_r, b.qa, free_all, d_out, stream));
    } else {
        if (n_mass > 0)
            HIPCHK(launch_reduce_masses(P, g, b.ratio, (const double *)(b.blob + s.off_ym),
                                        (const double *)(b.blob + s.off_wm), n_mass, d_out, stream));
        else
            HIPCHK(launch_reduce_profile(P, g, b.ratio, d_out, stream));
        if (d_integrand) HIPCHK(launch_reduce_integrand(P, g, b.ratio, d_integrand, stream));
        HIPCHK(launch_reduce_stats(n, o, stats, stream));
    }
    // the statistics come back with the solve itself, so reading them later
    // does not wait for whatever the caller enqueued on the stream since
    HIPCHK(hipMemcpyAsync(ctx->h_stats, stats, 8 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipEventRecord(ctx->ev_done, stream));
    ctx->pending = true;
    ctx->last_n_traj = n;
    ctx->last_traj_kept = !fused;
    return NH_OK;
}

int solve_enqueue(nh_context *ctx, const nh_request *q, double *d_out, double *d_ratio,
                  hipStream_t stream, int n_mass, const double *m_eV, double *d_integrand)
{
    int rc = validate(q, ctx->err, sizeof(ctx->err));
    if (rc != NH_OK) return rc;
    if (n_mass < 0 || n_mass > 4096) return set_err(ctx, NH_EINVAL, "n_mass must be in [1, 4096]");
    for (int k = 0; k < n_mass; ++k)
        if (!m_eV || !std::isfinite(m_eV[k]) || !(m_eV[k] > 0))
            return set_err(ctx, NH_EINVAL, "mass %d must be finite and > 0", k);
    HIPCHK(hipSetDevice(ctx->device));
    if ((rc = wait_pending(ctx)) != NH_OK) return rc;
    ctx->pending = false;

    const Staged s = stage_layout(q, ctx->table_nodes, n_mass);
    if (!sampled_table_fits(q, s.n_tab))
        return set_err(ctx, NH_EINVAL, "%d history samples need at least 3 of the %d table nodes per sample interval",
                       q->halo.history.n, s.n_tab);
    if ((rc = ensure_pinned(ctx, s.bytes)) != NH_OK) return rc;
    TrajParams P;
    stage_fill(q, s, (char *)ctx->h_stage, P, 4, m_eV);
    if (!ctx->free_exit && P.r_exit > 0.0) {
        P.r_exit = -1.0;
        P.cull_D = 0.0;
    }
    if ((rc = ensure_dev(ctx, ctx->blob, s.bytes)) != NH_OK) return rc;
    HIPCHK(hipMemcpyAsync(ctx->blob.p, ctx->h_stage, s.bytes, hipMemcpyHostToDevice, stream));
    if ((rc = ensure_dev(ctx, ctx->small, 64 * sizeof(unsigned long long))) != NH_OK) return rc;

    SolveBufs b{};
    b.blob = (char *)ctx->blob.p;
    b.small = (unsigned long long *)ctx->small.p;
    // the quadrature runs in the trajectory kernels' epilogue unless something
    // per trajectory is wanted: speed ratios, other masses, the distribution
    // per momentum node, or per-trajectory statistics
    const bool fused = !d_ratio && n_mass == 0 && !d_integrand && !ctx->keep_traj;
    const long long n = P.n_traj;
    if (fused) {
        if ((rc = ensure_dev(ctx, ctx->quad, quad_bytes(q->grid.n_r))) != NH_OK) return rc;
        b.qa = quad_acc(ctx->quad.p, q->grid.n_r, b.small + 8);
    } else {
        if (!d_ratio) {
            if ((rc = ensure_dev(ctx, ctx->ratio, (size_t)n * sizeof(double))) != NH_OK) return rc;
            d_ratio = (double *)ctx->ratio.p;
        }
        if ((rc = ensure_dev(ctx, ctx->stat, (size_t)n * sizeof(TrajStat))) != NH_OK) return rc;
        b.ratio = d_ratio;
        b.stat = (TrajStat *)ctx->stat.p;
    }
    return solve_launch(ctx, q, s, P, b, d_out, stream, n_mass, d_integrand);
}

size_t quad_bytes(int n_r) { return ((size_t)2 * n_r + 4) * sizeof(unsigned long long); }

QuadAcc quad_acc(void *base, int n_r, unsigned long long *stats)
{
    QuadAcc qa;
    qa.num = (unsigned long long *)base;
    qa.den = qa.num + 2 * (size_t)n_r;
    qa.scale = (double *)(qa.den + 2);
    qa.stats = stats;
    qa.lds_n = 0;   // set per launch by the trajectory kernels' launchers
    qa.ring = 0;    // likewise
    return qa;
}

int collect_stats(nh_context *ctx, nh_stats *out)
{
    HIPCHK(hipSetDevice(ctx->device));
    if (!ctx->pending && ctx->last_n_traj < 0) return set_err(ctx, NH_EINVAL, "no solve to report");
    HIPCHK(hipEventSynchronize(ctx->ev_done));
    unsigned long long h[8] = {0};
    std::memcpy(h, ctx->h_stats, sizeof(h));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
    nh_stats st{};
    st.n_traj = ctx->last_n_traj;
    st.accepted_steps = (long long)h[0];
    st.rejected_steps = (long long)h[1];
    st.max_steps_one_traj = (long long)h[2];
    st.n_failed = (long long)h[3];
    st.fp64_steps = (long long)h[4];
    st.free_exits = (long long)h[5];
    st.kernel_ms = ms;
    if (out) *out = st;
    ctx->pending = false;
    if (st.n_failed > 0) {
        set_err(ctx, NH_ESTEPS, "%lld trajectories did not finish cleanly", st.n_failed);
        return NH_ESTEPS;
    }
    return NH_OK;
}

}  // namespace nh

using namespace nh;

extern "C" {

const char *nh_version(void) { return "nuhalo 0.1 (gfx950)"; }

int nh_fp64_fma_peak(nh_context *ctx, double *tflops)
{
    if (!ctx || !tflops) return set_err(ctx, NH_EINVAL, "context and tflops are required");
    HIPCHK(hipSetDevice(ctx->device));
    int rc;
    if ((rc = wait_pending(ctx)) != NH_OK) return rc;
    const int blocks = ctx->n_cu * 8;
    if ((rc = ensure_dev(ctx, ctx->out, (size_t)blocks * 1024 * sizeof(double))) != NH_OK) return rc;
    double best = 0.0, flop = 0.0;
    for (int rep = 0; rep < 4; ++rep) {
        HIPCHK(hipEventRecord(ctx->ev_t0, ctx->stream));
        HIPCHK(launch_fma_probe((double *)ctx->out.p, blocks, ctx->stream, &flop));
        HIPCHK(hipEventRecord(ctx->ev_t1, ctx->stream));
        HIPCHK(hipEventSynchronize(ctx->ev_t1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
        if (rep > 0 && ms > 0.f) best = std::max(best, flop / (ms * 1e-3) / 1e12);   // first launch warms up
    }
    *tflops = best;
    return NH_OK;
}

int nh_device_function(nh_context *ctx, int fn, const nh_request *req, long long n, const double *x, double *y)
{
    if (!ctx) return set_err(ctx, NH_EINVAL, "context is required");
    if (fn != NH_FN_NFW_I && fn != NH_FN_POW_FACTOR) return set_err(ctx, NH_EINVAL, "unknown function %d", fn);
    if (n < 0 || n > (1ll << 26) || (n > 0 && (!x || !y))) return set_err(ctx, NH_EINVAL, "bad n/x/y");
    PowFactor pw{};
    if (fn == NH_FN_POW_FACTOR) {
        if (!req) return set_err(ctx, NH_EINVAL, "req is required for NH_FN_POW_FACTOR");
        int rc = validate(req, ctx->err, sizeof(ctx->err));
        if (rc != NH_OK) return rc;
        pw = Physics(*req).pw;
    }
    if (n == 0) return NH_OK;
    HIPCHK(hipSetDevice(ctx->device));
    int rc;
    if ((rc = wait_pending(ctx)) != NH_OK) return rc;
    const size_t bytes = (size_t)n * sizeof(double);
    if ((rc = ensure_dev(ctx, ctx->out, 2 * bytes)) != NH_OK) return rc;
    double *dx = (double *)ctx->out.p, *dy = dx + n;
    HIPCHK(hipMemcpyAsync(dx, x, bytes, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(launch_device_fn(fn == NH_FN_NFW_I ? FN_NFW_I : FN_POW_FACTOR, pw, n, dx, dy, ctx->stream));
    HIPCHK(hipMemcpyAsync(y, dy, bytes, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return NH_OK;
}

const char *nh_strerror(int code)
{
    switch (code) {
    case NH_OK: return "ok";
    case NH_EINVAL: return "invalid argument";
    case NH_ENOMEM: return "out of memory";
    case NH_EDEVICE: return "device error";
    case NH_ESTEPS: return "some trajectories did not finish (max_steps or step underflow)";
    case NH_ENONFINITE: return "non-finite trajectory state";
    case NH_EBUSY: return "request does not fit the free budget";
    case NH_ENOTREADY: return "ticket not finished";
    case NH_ENOTFOUND: return "unknown ticket";
    case NH_ECANCELED: return "ticket cancelled";
    default: return "unknown error";
    }
}

const char *nh_last_error(const nh_context *ctx) { return ctx ? ctx->err : g_err; }

int nh_footprint_bytes(const nh_request *req, size_t *bytes)
{
    if (!bytes) return set_err(nullptr, NH_EINVAL, "bytes is NULL");
    int rc = validate(req, g_err, sizeof(g_err));
    if (rc != NH_OK) return rc;
    const Staged s = stage_layout(req, 0);
    *bytes = s.bytes + (size_t)n_traj_of(req) * per_traj_bytes(req) + (size_t)req->grid.n_r * sizeof(double);
    return NH_OK;
}

int nh_set_option(nh_context *ctx, int option, double value)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!std::isfinite(value)) return set_err(ctx, NH_EINVAL, "option value must be finite");
    switch (option) {
    case NH_OPT_QUEUE_ORDER:
        if (value != 0.0 && value != 1.0 && value != 2.0 && value != 3.0)
            return set_err(ctx, NH_EINVAL, "queue order is 0, 1, 2 or 3");
        ctx->queue_order = (int)value;
        return NH_OK;
    case NH_OPT_FREE_EXIT:
        if (value != 0.0 && value != 1.0) return set_err(ctx, NH_EINVAL, "free exit is 0 or 1");
        ctx->free_exit = value != 0.0;
        return NH_OK;
    case NH_OPT_FP64_BELOW_H:
        if (value < 0.0) return set_err(ctx, NH_EINVAL, "threshold must be >= 0");
        ctx->h_fp64 = value;
        return NH_OK;
    case NH_OPT_TRAJECTORY_STATS:
        if (value != 0.0 && value != 1.0) return set_err(ctx, NH_EINVAL, "trajectory statistics is 0 or 1");
        ctx->keep_traj = value != 0.0;
        return NH_OK;
    case NH_OPT_FP32C_RTOL:
        if (value < 1.0e-9 || value > 1.0e-3)
            return set_err(ctx, NH_EINVAL, "FP32C tolerance floor must be in [1e-9, 1e-3]");
        ctx->rtol32 = value;
        return NH_OK;
    case NH_OPT_BLOCK_THREADS:
        if (value != 0.0 && (value < 64 || value > 1024 || value != (double)(64 * (int)(value / 64))))
            return set_err(ctx, NH_EINVAL, "block threads must be 0 (default) or a multiple of 64 in [64, 1024]");
        ctx->block_threads = (int)value;
        return NH_OK;
    case NH_OPT_TABLE_NODES:
        if (value != 0.0 && (value < 64 || value > 3073 || value != (double)(int)value))
            return set_err(ctx, NH_EINVAL, "table nodes must be 0 (default) or an integer in [64, 3073]");
        ctx->table_nodes = (int)value;
        return NH_OK;
    case NH_OPT_SLICE_US:
        if (value < 200.0 || value > 1.0e6) return set_err(ctx, NH_EINVAL, "slice length must be in [200, 1e6] us");
        ctx->slice_us = value;
        return NH_OK;
    case NH_OPT_BATCH_SLOTS:
        if (value != 0.0 && value != 1.0 && value != 2.0)
            return set_err(ctx, NH_EINVAL, "batch slots is 0 (default), 1 or 2");
        ctx->batch_slots = (int)value;
        return NH_OK;
    case NH_OPT_SERVE_GRAPH:
        if (value != 0.0 && value != 1.0) return set_err(ctx, NH_EINVAL, "serve graph is 0 or 1");
        ctx->serve_graph = value != 0.0;
        return NH_OK;
    case NH_OPT_WORKGROUPS:
        if (value != 0.0 && (value < 1 || value > 65536 || value != (double)(int)value))
            return set_err(ctx, NH_EINVAL, "workgroups must be 0 (default) or an integer in [1, 65536]");
        ctx->max_workgroups = (int)value;
        return NH_OK;
    default:
        return set_err(ctx, NH_EINVAL, "unknown option %d", option);
    }
}

int nh_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > 4096 || !x || !w) return set_err(nullptr, NH_EINVAL, "need 1 <= n <= 4096 and x, w");
    gauss_legendre(n, x, w);
    return NH_OK;
}

int nh_coefficients(const nh_request *req, int n, const double *u, double *out)
{
    int rc = validate(req, g_err, sizeof(g_err));
    if (rc != NH_OK) return rc;
    if (n < 0 || (n > 0 && (!u || !out))) return set_err(nullptr, NH_EINVAL, "bad n/u/out");
    Physics ph(*req);
    for (int i = 0; i < n; ++i) ph.coef(u[i], out + (size_t)i * NCOL);
    return NH_OK;
}

int nh_context_create(int device, nh_context **out)
{
    if (!out) return set_err(nullptr, NH_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0)
        return set_err(nullptr, NH_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
    if (device < 0 || device >= ndev) return set_err(nullptr, NH_EINVAL, "device %d out of range", device);
    nh_context *ctx = new (std::nothrow) nh_context();
    if (!ctx) return set_err(nullptr, NH_ENOMEM, "context allocation");
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&ctx->ev_done) != hipSuccess || hipEventCreate(&ctx->ev_t0) != hipSuccess ||
        hipEventCreate(&ctx->ev_t1) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_stats, 8 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        set_err(nullptr, NH_EDEVICE, "stream/event creation failed");
        nh_context_destroy(ctx);
        return NH_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->n_cu = prop.multiProcessorCount;
    if (ctx->n_cu <= 0) ctx->n_cu = 256;
    *out = ctx;
    return NH_OK;
}

int nh_context_destroy(nh_context *ctx)
{
    if (!ctx) return NH_OK;
    (void)hipSetDevice(ctx->device);
    serve_shutdown(ctx);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    (void)hipDeviceSynchronize();
    for (DevBuf *b : {&ctx->blob, &ctx->ratio, &ctx->stat, &ctx->small, &ctx->out, &ctx->bctr, &ctx->quad})
        if (b->p) (void)hipFree(b->p);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    if (ctx->h_stats) (void)hipHostFree(ctx->h_stats);
    if (ctx->ev_done) (void)hipEventDestroy(ctx->ev_done);
    if (ctx->ev_t0) (void)hipEventDestroy(ctx->ev_t0);
    if (ctx->ev_t1) (void)hipEventDestroy(ctx->ev_t1);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return NH_OK;
}

int nh_solve_async(nh_context *ctx, const nh_request *req, double *d_out, double *d_ratio,
                   void *stream)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!d_out) return set_err(ctx, NH_EINVAL, "d_out is NULL");
    return solve_enqueue(ctx, req, d_out, d_ratio, (hipStream_t)stream, 0, nullptr);
}

int nh_solve_integrand(nh_context *ctx, const nh_request *req, double *d_out, double *d_integrand, double *d_ratio,
                       void *stream)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!d_out || !d_integrand) return set_err(ctx, NH_EINVAL, "d_out and d_integrand are required");
    return solve_enqueue(ctx, req, d_out, d_ratio, (hipStream_t)stream, 0, nullptr, d_integrand);
}

int nh_solve_masses(nh_context *ctx, const nh_request *req, int n_mass, const double *m_eV, double *d_out,
                    double *d_ratio, void *stream)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!d_out || !m_eV) return set_err(ctx, NH_EINVAL, "d_out and m_eV are required");
    if (n_mass < 1) return set_err(ctx, NH_EINVAL, "n_mass must be in [1, 4096]");
    return solve_enqueue(ctx, req, d_out, d_ratio, (hipStream_t)stream, n_mass, m_eV);
}

int nh_last_stats(nh_context *ctx, nh_stats *stats)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    return collect_stats(ctx, stats);
}

int nh_last_trajectory_stats(nh_context *ctx, size_t capacity, int *accepted, int *rejected, int *status)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (ctx->last_n_traj < 0) return set_err(ctx, NH_EINVAL, "no solve to report");
    if (!ctx->last_traj_kept)
        return set_err(ctx, NH_EINVAL, "the last solve kept no per-trajectory results (pass a ratio buffer or set "
                                       "NH_OPT_TRAJECTORY_STATS)");
    if (capacity < (size_t)ctx->last_n_traj)
        return set_err(ctx, NH_EINVAL, "arrays of %zu entries for %lld trajectories", capacity, ctx->last_n_traj);
    HIPCHK(hipSetDevice(ctx->device));
    if (ctx->pending) HIPCHK(hipEventSynchronize(ctx->ev_done));
    const size_t n = (size_t)ctx->last_n_traj;
    std::vector<TrajStat> h(n);
    HIPCHK(hipMemcpy(h.data(), ctx->stat.p, n * sizeof(TrajStat), hipMemcpyDeviceToHost));
    for (size_t t = 0; t < n; ++t) {
        if (accepted) accepted[t] = h[t].acc;
        if (rejected) rejected[t] = h[t].rej;
        if (status) status[t] = h[t].status;
    }
    return NH_OK;
}

int nh_solve(nh_context *ctx, const nh_request *req, double *n_over_nbar, nh_stats *stats)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!n_over_nbar) return set_err(ctx, NH_EINVAL, "output is NULL");
    int rc = validate(req, ctx->err, sizeof(ctx->err));
    if (rc != NH_OK) return rc;
    if ((rc = ensure_dev(ctx, ctx->out, (size_t)req->grid.n_r * sizeof(double))) != NH_OK) return rc;
    rc = solve_enqueue(ctx, req, (double *)ctx->out.p, nullptr, ctx->stream, 0, nullptr);
    if (rc != NH_OK) return rc;
    rc = collect_stats(ctx, stats);
    if (rc != NH_OK && rc != NH_ESTEPS) return rc;
    hipError_t e = hipMemcpy(n_over_nbar, ctx->out.p, (size_t)req->grid.n_r * sizeof(double),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_err(ctx, NH_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    return rc;
}

}  // extern "C"

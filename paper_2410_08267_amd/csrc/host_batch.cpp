// Batched solve: many heterogeneous requests in one persistent slice launch.
//
// Host work: validation, per-request tables and grids (built on a few host
// threads), descriptors; one transfer to the device; then the slice kernel,
// the profile reductions of every request and their statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "nh_batch_host.h"
#include "nh_launch.h"

namespace nh {

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int request_columns(const nh_request *q)
{
    return (q->halo.compensated && q->halo.geometry == NH_GEOM_DELTA200) ? NCOL : NCOL - 1;
}

int batch_block(const nh_context *ctx, bool f32c, int slots)
{
    // FP64 slices fit four waves per SIMD (1024 threads, 128 VGPRs); FP32C
    // slices with two table slots three (768 threads, 170 VGPRs), with one
    // slot four (the request parameters sit in scalar registers)
    const int cap = (!f32c || slots == 1) ? 1024 : 768;
    if (ctx->block_threads > 0) return std::min(ctx->block_threads, cap);
    return ctx->tuned_batch_block[f32c] > 0 ? std::min(ctx->tuned_batch_block[f32c], cap) : cap;
}

int batch_slots(const nh_context *ctx, bool f32c)
{
    if (ctx->batch_slots > 0) return ctx->batch_slots;
    return ctx->tuned_batch_slots[f32c] > 0 ? ctx->tuned_batch_slots[f32c] : 1;
}

int batch_table_nodes(nh_context *ctx, bool f32c, int nc, int slots, int *n_tab)
{
    const int cap = std::min(slice_max_table_nodes(f32c, nc, slots), default_table_nodes(f32c));
    if (ctx->table_nodes > 0) {
        if (ctx->table_nodes > cap)
            return set_err(ctx, NH_EINVAL,
                           "%d table(s) per workgroup of %d columns fit at most %d nodes in LDS (%s)", slots, nc,
                           cap, f32c ? "FP32C" : "FP64");
        *n_tab = ctx->table_nodes;
    } else {
        *n_tab = cap;
    }
    return NH_OK;
}

void describe(const nh_context *ctx, const nh_request *q, const Staged &s, char *host_base, const char *dev_base,
              double *ratio, TrajStat *stat, double *out, BatchReq &d)
{
    std::memset(&d, 0, sizeof(d));
    stage_fill(q, s, host_base, d.P, 1);
    if (!ctx->free_exit && d.P.r_exit > 0.0) {
        d.P.r_exit = -1.0;
        d.P.cull_D = 0.0;
    }
    d.P.r_exit2 = exit_radius2(d.P);
    d.P.order = ctx->queue_order;
    d.P.h_fp64 = q->integ.precision == NH_FP32C ? ctx->h_fp64 : 0.0;
    d.P.rtol32 = ctx->rtol32;
    d.g = grid_ptrs(s, dev_base);
    d.o.ratio = ratio;
    d.o.stat = stat;
    d.out = out;
    d.nc = d.P.R_const > 0.0 ? NCOL - 1 : NCOL;
    d.free_all = q->halo.mass_kind == NH_MASS_ZERO;
    d.retired = 0;
}

int check_batchable(nh_context *ctx, const nh_request *q, int index, int precision)
{
    char msg[400];
    int rc = validate(q, msg, sizeof(msg));
    if (rc != NH_OK) return set_err(ctx, rc, "request %d: %s", index, msg);
    if (q->integ.method != NH_DOPRI5)
        return set_err(ctx, NH_EINVAL, "request %d: the batched and serving forms integrate with NH_DOPRI5", index);
    if (precision >= 0 && q->integ.precision != precision)
        return set_err(ctx, NH_EINVAL, "request %d: all requests of a batch share one precision", index);
    return NH_OK;
}

void stats_from_words(const unsigned long long *w, long long n_traj, double kernel_ms, nh_stats &st)
{
    st.n_traj = n_traj;
    st.accepted_steps = (long long)w[0];
    st.rejected_steps = (long long)w[1];
    st.max_steps_one_traj = (long long)w[2];
    st.n_failed = (long long)w[3];
    st.fp64_steps = (long long)w[4];
    st.free_exits = (long long)w[5];
    st.kernel_ms = kernel_ms;
}

void parallel_for(int n, const std::function<void(int)> &fn)
{
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::min({n, hw, 16});
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int w = 0; w < nt; ++w)
        th.emplace_back([&, w] {
            for (int i = w; i < n; i += nt) fn(i);
        });
    for (auto &t : th) t.join();
}

}  // namespace nh

using namespace nh;

extern "C" {

int nh_solve_batch(nh_context *ctx, int n_req, const nh_request *reqs, double *d_out, nh_stats *stats,
                   void *stream)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (n_req < 1 || n_req > 65535) return set_err(ctx, NH_EINVAL, "n_req must be in [1, 65535]");
    if (!reqs || !d_out) return set_err(ctx, NH_EINVAL, "reqs and d_out are required");
    int rc;
    for (int i = 0; i < n_req; ++i)
        if ((rc = check_batchable(ctx, &reqs[i], i, reqs[0].integ.precision)) != NH_OK) return rc;
    const bool f32c = reqs[0].integ.precision == NH_FP32C;
    int nc = NCOL - 1;
    for (int i = 0; i < n_req; ++i) nc = std::max(nc, request_columns(&reqs[i]));
    const int slots = batch_slots(ctx, f32c);
    int n_tab = 0;
    if ((rc = batch_table_nodes(ctx, f32c, nc, slots, &n_tab)) != NH_OK) return rc;
    hipStream_t s = (hipStream_t)stream;

    HIPCHK(hipSetDevice(ctx->device));
    if ((rc = wait_pending(ctx)) != NH_OK) return rc;
    ctx->pending = false;

    // layout: per-request blobs, then descriptors, order and radius offsets
    std::vector<Staged> st(n_req);
    std::vector<size_t> off(n_req);
    std::vector<long long> toff(n_req);
    std::vector<int> roff(n_req + 1);
    size_t bytes = 0;
    long long ntot = 0, nmax = 0;
    long long rtot = 0;
    for (int i = 0; i < n_req; ++i) {
        st[i] = stage_layout(&reqs[i], n_tab);
        if (!sampled_table_fits(&reqs[i], n_tab))
            return set_err(ctx, NH_EINVAL, "request %d: %d history samples need at least 3 of the %d table nodes "
                           "per sample interval", i, reqs[i].halo.history.n, n_tab);
        off[i] = bytes;
        bytes += align_up(st[i].bytes);
        const long long n = n_traj_of(&reqs[i]);
        toff[i] = ntot;
        ntot += n;
        nmax = std::max(nmax, n);
        roff[i] = (int)rtot;
        rtot += reqs[i].grid.n_r;
    }
    if (rtot > (1ll << 31) - 1) return set_err(ctx, NH_EINVAL, "too many radii in one batch");
    roff[n_req] = (int)rtot;
    const size_t off_desc = bytes;
    bytes += align_up((size_t)n_req * sizeof(BatchReq));
    const size_t off_order = bytes;
    bytes += align_up((size_t)n_req * sizeof(int));
    const size_t off_rstart = bytes;
    bytes += align_up((size_t)(n_req + 1) * sizeof(int));

    if ((rc = ensure_pinned(ctx, bytes)) != NH_OK) return rc;
    if ((rc = ensure_dev(ctx, ctx->blob, bytes)) != NH_OK) return rc;
    if ((rc = ensure_dev(ctx, ctx->ratio, (size_t)ntot * sizeof(double))) != NH_OK) return rc;
    if ((rc = ensure_dev(ctx, ctx->stat, (size_t)ntot * sizeof(TrajStat))) != NH_OK) return rc;
    // counters: next[n_req], cursor, statistics 8 words per request
    const size_t n_words = (size_t)n_req + 1 + 8 * (size_t)n_req;
    if ((rc = ensure_dev(ctx, ctx->bctr, n_words * sizeof(unsigned long long))) != NH_OK) return rc;
    unsigned long long *d_next = (unsigned long long *)ctx->bctr.p;
    unsigned long long *d_cursor = d_next + n_req;
    unsigned long long *d_stats = d_cursor + 1;

    char *h = (char *)ctx->h_stage;
    const char *dev = (const char *)ctx->blob.p;
    BatchReq *hdesc = (BatchReq *)(h + off_desc);
    double *ratio = (double *)ctx->ratio.p;
    TrajStat *tstat = (TrajStat *)ctx->stat.p;
    parallel_for(n_req, [&](int i) {
        describe(ctx, &reqs[i], st[i], h + off[i], dev + off[i], ratio + toff[i], tstat + toff[i], d_out + roff[i],
                 hdesc[i]);
    });
    int *horder = (int *)(h + off_order);
    int *hrstart = (int *)(h + off_rstart);
    for (int i = 0; i < n_req; ++i) horder[i] = i;
    for (int i = 0; i <= n_req; ++i) hrstart[i] = roff[i];

    HIPCHK(hipMemcpyAsync(ctx->blob.p, h, bytes, hipMemcpyHostToDevice, s));
    HIPCHK(launch_fill_u64(d_next, (int)n_words, 0ull, s));

    SliceArgs A{};
    A.reqs = (const BatchReq *)(dev + off_desc);
    A.next = d_next;
    A.inflight = nullptr;
    A.order = (const int *)(dev + off_order);
    A.n_order = n_req;
    A.policy = POLICY_OPEN_FIRST;
    A.cursor = d_cursor;
    A.n_tab = n_tab;
    A.budget_ticks = -1;
    A.lane_save = nullptr;
    A.wg_save = nullptr;
    A.resume = 0;
    bool pow = false;
    for (int i = 0; i < n_req; ++i) pow = pow || hdesc[i].P.hist;
    const int block = batch_block(ctx, f32c, slots);
    int grid = 0;
    HIPCHK(slice_capacity(f32c, nc, slots, pow, n_tab, block, ctx->n_cu, &grid));
    const long long need = (ntot + block - 1) / block;
    if (grid > need) grid = (int)std::max(1ll, need);

    HIPCHK(hipEventRecord(ctx->ev_t0, s));
    HIPCHK(launch_slice(A, f32c, nc, slots, pow, grid, block, s));
    HIPCHK(hipEventRecord(ctx->ev_t1, s));
    const int chunks = (int)std::min(256ll, std::max(1ll, (nmax + 256 * 64 - 1) / (256 * 64)));
    HIPCHK(launch_reduce_batch(A.reqs, A.order, (const int *)(dev + off_rstart), n_req, (int)rtot, d_stats,
                               chunks, s));
    std::vector<unsigned long long> hs(8 * (size_t)n_req);
    HIPCHK(hipMemcpyAsync(hs.data(), d_stats, hs.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(ctx->ev_done, s));
    HIPCHK(hipEventSynchronize(ctx->ev_done));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->ev_t0, ctx->ev_t1));
    ctx->last_n_traj = ntot;

    long long failed = 0;
    for (int i = 0; i < n_req; ++i) {
        nh_stats one{};
        stats_from_words(&hs[8 * (size_t)i], n_traj_of(&reqs[i]), ms, one);
        failed += one.n_failed;
        if (stats) stats[i] = one;
    }
    if (failed > 0) return set_err(ctx, NH_ESTEPS, "%lld trajectories did not finish cleanly", failed);
    return NH_OK;
}

}  // extern "C"

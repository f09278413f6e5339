// Autotuner for the Dormand-Prince launches: the workgroup size of the plain
// kernels, and the workgroup size and tables per workgroup of the batched
// slice kernels, chosen by timing candidates on a sample of requests.
//
// What the candidates trade: more waves per SIMD hide more of the FP64
// dependency latency (VALU issue rises from ~68 % at two waves to ~90 % at
// four) but run every wave, and so the longest trajectories of a profile,
// more slowly; where a profile's longest trajectories approach a lane's share
// of the work, its tail grows.  Which wins depends on the halo, the grid and
// the precision, so it is measured rather than fixed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "nh_context.h"

namespace nh {

namespace {

struct Cand {
    int block, slots;
};

std::vector<Cand> candidates(int form, bool f32c)
{
    std::vector<Cand> c;
    if (form == NH_FORM_PLAIN) {
        const int fp64[] = {256, 384, 512, 640, 768, 1024}, fp32[] = {256, 384, 512, 640, 768, 1024};
        if (f32c)
            for (int b : fp32) c.push_back({b, 0});
        else
            for (int b : fp64) c.push_back({b, 0});
    } else if (f32c) {
        // two FP32 tables of 3073 nodes fit one workgroup's LDS, and one slot
        // allows 1024 threads; the results do not depend on either
        for (int s : {1, 2})
            for (int b : {256, 384, 512, 768, 1024})
                if (s == 1 || b <= 768) c.push_back({b, s});
    } else {
        // FP64 batches keep one 3073-node table per workgroup: the plain
        // form's table, so that a batched profile equals the plain one
        for (int b : {512, 768, 1024}) c.push_back({b, 1});
    }
    return c;
}

// Total trajectory-kernel time of the sample under the context's current options.
int time_sample(nh_context *ctx, int form, int n_req, const nh_request *reqs, double *d_out,
                std::vector<nh_stats> &st, double &ms)
{
    ms = 0.0;
    if (form == NH_FORM_BATCH) {
        const int rc = nh_solve_batch(ctx, n_req, reqs, d_out, st.data(), ctx->stream);
        if (rc != NH_OK && rc != NH_ESTEPS && rc != NH_ENONFINITE) return rc;
        ms = st[0].kernel_ms;     // one launch for the whole batch
        return NH_OK;
    }
    for (int i = 0; i < n_req; ++i) {
        int rc = solve_enqueue(ctx, &reqs[i], d_out, nullptr, ctx->stream, 0, nullptr);
        if (rc != NH_OK) return rc;
        nh_stats s{};
        rc = collect_stats(ctx, &s);
        if (rc != NH_OK && rc != NH_ESTEPS) return rc;
        ms += s.kernel_ms;
    }
    return NH_OK;
}

}  // namespace

}  // namespace nh

using namespace nh;

extern "C" int nh_autotune(nh_context *ctx, int form, int n_req, const nh_request *reqs, nh_tune_result *result)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (form != NH_FORM_PLAIN && form != NH_FORM_BATCH) return set_err(ctx, NH_EINVAL, "unknown form %d", form);
    if (n_req < 1 || n_req > 65535 || !reqs) return set_err(ctx, NH_EINVAL, "n_req must be in [1, 65535]");
    const int prec = reqs[0].integ.precision;
    if (prec != NH_FP64 && prec != NH_FP32C) return set_err(ctx, NH_EINVAL, "unknown precision");
    long long max_r = 0, sum_r = 0;
    for (int i = 0; i < n_req; ++i) {
        if (reqs[i].integ.method != NH_DOPRI5)
            return set_err(ctx, NH_EINVAL, "request %d: only Dormand-Prince launches are tuned", i);
        if (reqs[i].integ.precision != prec)
            return set_err(ctx, NH_EINVAL, "request %d: the sample must share one precision", i);
        if (reqs[i].grid.n_r < 1 || reqs[i].grid.n_r > (1 << 24))
            return set_err(ctx, NH_EINVAL, "request %d: n_r out of range", i);
        max_r = std::max<long long>(max_r, reqs[i].grid.n_r);
        sum_r += reqs[i].grid.n_r;
    }
    if (!serve_idle(ctx)) return set_err(ctx, NH_EBUSY, "the serving loop is busy");
    const bool f32c = prec == NH_FP32C;
    const std::vector<Cand> cand = candidates(form, f32c);

    HIPCHK(hipSetDevice(ctx->device));
    int rc = wait_pending(ctx);
    if (rc != NH_OK) return rc;
    double *d_out = nullptr;
    const size_t out_bytes = (size_t)(form == NH_FORM_BATCH ? sum_r : max_r) * sizeof(double);
    if (hipMalloc((void **)&d_out, out_bytes) != hipSuccess)
        return set_err(ctx, NH_ENOMEM, "autotune output buffer of %zu bytes", out_bytes);

    const int saved_block = ctx->block_threads, saved_slots = ctx->batch_slots;
    int &tuned_block = form == NH_FORM_PLAIN ? ctx->tuned_plain_block[f32c] : ctx->tuned_batch_block[f32c];
    std::vector<nh_stats> st((size_t)n_req);
    double default_ms = 0.0, best_ms = 1e300;
    Cand best = cand[0];
    // the built-in default first: it is also the warm-up
    ctx->block_threads = 0;
    ctx->batch_slots = 0;
    const int saved_tuned_block = tuned_block, saved_tuned_slots = ctx->tuned_batch_slots[f32c];
    tuned_block = 0;
    if (form == NH_FORM_BATCH) ctx->tuned_batch_slots[f32c] = 0;
    rc = time_sample(ctx, form, n_req, reqs, d_out, st, default_ms);
    if (rc == NH_OK) rc = time_sample(ctx, form, n_req, reqs, d_out, st, default_ms);
    for (size_t k = 0; rc == NH_OK && k < cand.size(); ++k) {
        ctx->block_threads = cand[k].block;
        ctx->batch_slots = cand[k].slots;
        double t = 1e300;
        for (int pass = 0; rc == NH_OK && pass < 2; ++pass) {
            double ms = 0.0;
            rc = time_sample(ctx, form, n_req, reqs, d_out, st, ms);
            t = std::min(t, ms);
        }
        if (rc == NH_OK && t < best_ms) {
            best_ms = t;
            best = cand[k];
        }
    }
    ctx->block_threads = saved_block;
    ctx->batch_slots = saved_slots;
    (void)hipFree(d_out);
    if (rc != NH_OK) {
        tuned_block = saved_tuned_block;
        ctx->tuned_batch_slots[f32c] = saved_tuned_slots;
        return rc;
    }
    tuned_block = best.block;
    if (form == NH_FORM_BATCH) ctx->tuned_batch_slots[f32c] = best.slots;
    if (result) {
        result->form = form;
        result->precision = prec;
        result->block_threads = best.block;
        result->batch_slots = form == NH_FORM_BATCH ? best.slots : 0;
        result->n_tried = (int)cand.size();
        result->best_ms = best_ms;
        result->default_ms = default_ms;
    }
    return NH_OK;
}

// Continuous-batching server of one context.
//
// Admission: a request's device footprint (tables, grids, per-trajectory
// results, profile) is carved out of one budgeted device region by a
// first-fit allocator; a request that does not fit is refused (NH_EBUSY).
// Inputs are staged on the host at admission.  A worker thread runs the slice
// kernel in time slices over the admitted requests: between slices it uploads
// newly admitted requests, retires cancelled ones, finds the requests whose
// trajectories have all finished (queue exhausted and none saved in flight),
// reduces their profiles and statistics on the device and hands the results
// to nh_poll.  Trajectories cut by a slice boundary are saved and resumed bit
// for bit, so a served profile equals the plain path's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nh_batch_host.h"
#include "nh_launch.h"

namespace nh {

namespace {

constexpr int SERVE_CAP = 1024;   // requests admitted at once (descriptor slots)
constexpr int SERVE_SHARE_TPL = 16;   // POLICY_SHARE: trajectories per lane to justify one more workgroup
constexpr size_t GRANULE = 256;

size_t round_up(size_t x) { return (x + GRANULE - 1) & ~(GRANULE - 1); }

// First-fit allocator over one device region; frees coalesce with neighbours.
class Arena {
  public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = round_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0;
};

enum class St { Queued, Active, Done, Cancelled };

using Clock = std::chrono::steady_clock;

struct Ticket {
    uint64_t id = 0;
    St st = St::Queued;
    bool cancel = false;          // cancellation asked while on the device
    bool retired = false;         // cancellation applied on the device
    int slot = -1;
    size_t off = 0, bytes = 0;    // region inside the arena
    int n_r = 0;
    long long n_traj = 0;
    std::vector<char> blob;       // staged inputs
    size_t blob_bytes = 0;
    BatchReq desc{};
    std::vector<double> result;
    nh_stats stats{};
    int rc = NH_OK;
    double kernel_ms = 0.0;
    Clock::time_point t_submit;
};

}  // namespace

struct ServeState {
    std::mutex mu;
    std::thread worker;
    std::condition_variable cv;
    bool stop = false;
    bool running = false;
    size_t budget = 0;
    // session parameters, fixed while anything is admitted
    int precision = -1;
    int n_tab = 0, slots = 1, block = 512, grid = 0;
    long long slice_ticks = 0;        // NH_OPT_SLICE_US in device clock ticks
    double ticks_per_ms = 100000.0;
    double claim_rate = 0.0;          // trajectories claimed per ms of slice (running estimate)
    char *arena_base = nullptr;
    size_t arena_bytes = 0;
    Arena arena;
    uint64_t next_id = 1;
    std::unordered_map<uint64_t, Ticket *> tickets;
    std::deque<Ticket *> queued;
    std::vector<Ticket *> active;     // admission order
    std::vector<int> free_slots;
    char failure[256] = "";
    // device state
    BatchReq *d_desc = nullptr;
    unsigned long long *d_next = nullptr;
    unsigned int *d_inflight = nullptr;
    int *d_helpers = nullptr;           // per request id: workgroups drawing from it (POLICY_SHARE)
    unsigned long long *d_stats = nullptr;
    int *d_order = nullptr, *d_list = nullptr, *d_rstart = nullptr;
    LaneSave *d_lanes = nullptr;
    WgSave *d_wg = nullptr;
    size_t lanes_cap = 0, wg_cap = 0;
    bool resume = false;
    bool use_graph = true;            // slices as replays of a HIP graph (per table layout)
    SliceGraph graph[4];              // [five | six columns] + 2 [with power-law factors]
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // pinned host mirrors; h_desc changes under `mu`, h_desc_up is the snapshot
    // the worker uploads at a slice boundary
    BatchReq *h_desc = nullptr, *h_desc_up = nullptr;
    int *h_order = nullptr, *h_list = nullptr, *h_rstart = nullptr;
    unsigned long long *h_next = nullptr, *h_stats = nullptr;
    unsigned int *h_inflight = nullptr;
    int *h_zero = nullptr;              // SERVE_CAP zeros: the source that resets d_helpers
};

namespace {

size_t ticket_bytes(const Staged &s, long long n_traj, int n_r)
{
    return round_up(s.bytes) + round_up((size_t)n_traj * sizeof(double)) +
           round_up((size_t)n_traj * sizeof(TrajStat)) + round_up((size_t)n_r * sizeof(double));
}

int alloc_device_state(nh_context *ctx, ServeState &S)
{
    if (S.d_desc) return NH_OK;
    HIPCHK(hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&S.ev0));
    HIPCHK(hipEventCreate(&S.ev1));
    HIPCHK(hipMalloc((void **)&S.d_desc, SERVE_CAP * sizeof(BatchReq)));
    HIPCHK(hipMalloc((void **)&S.d_next, SERVE_CAP * sizeof(unsigned long long)));
    HIPCHK(hipMalloc((void **)&S.d_inflight, SERVE_CAP * sizeof(unsigned int)));
    HIPCHK(hipMalloc((void **)&S.d_helpers, SERVE_CAP * sizeof(int)));
    HIPCHK(hipMalloc((void **)&S.d_stats, 8 * SERVE_CAP * sizeof(unsigned long long)));
    HIPCHK(hipMalloc((void **)&S.d_order, SERVE_CAP * sizeof(int)));
    HIPCHK(hipMalloc((void **)&S.d_list, SERVE_CAP * sizeof(int)));
    HIPCHK(hipMalloc((void **)&S.d_rstart, (SERVE_CAP + 1) * sizeof(int)));
    HIPCHK(hipHostMalloc((void **)&S.h_desc, SERVE_CAP * sizeof(BatchReq), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_desc_up, SERVE_CAP * sizeof(BatchReq), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_order, SERVE_CAP * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_list, SERVE_CAP * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_rstart, (SERVE_CAP + 1) * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_next, SERVE_CAP * sizeof(unsigned long long), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_inflight, SERVE_CAP * sizeof(unsigned int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_zero, SERVE_CAP * sizeof(int), hipHostMallocDefault));
    std::memset(S.h_zero, 0, SERVE_CAP * sizeof(int));
    HIPCHK(hipMemcpy(S.d_helpers, S.h_zero, SERVE_CAP * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipHostMalloc((void **)&S.h_stats, 8 * SERVE_CAP * sizeof(unsigned long long), hipHostMallocDefault));
    std::memset(S.h_desc, 0, SERVE_CAP * sizeof(BatchReq));
    for (int i = 0; i < SERVE_CAP; ++i) S.h_desc[i].retired = 1;   // unused slots are never claimed
    S.free_slots.clear();
    for (int i = SERVE_CAP - 1; i >= 0; --i) S.free_slots.push_back(i);
    return NH_OK;
}

// Session parameters for the first request admitted into an empty server.
int start_session(nh_context *ctx, ServeState &S, bool f32c)
{
    S.slots = batch_slots(ctx, f32c);
    S.block = batch_block(ctx, f32c, S.slots);
    int rc = batch_table_nodes(ctx, f32c, NCOL, S.slots, &S.n_tab);
    if (rc != NH_OK) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    // one grid for every slice (saved lanes are indexed by it): what fits for both layouts
    S.grid = 1 << 30;
    for (int nc : {(int)NCOL - 1, (int)NCOL})
        for (bool pow : {false, true}) {
            int g = 0;
            HIPCHK(slice_capacity(f32c, nc, S.slots, pow, S.n_tab, S.block, ctx->n_cu, &g));
            S.grid = std::min(S.grid, g);
        }
    const size_t lanes = (size_t)S.grid * S.block;
    if (lanes > S.lanes_cap) {
        if (S.d_lanes) HIPCHK(hipFree(S.d_lanes));
        S.d_lanes = nullptr;
        HIPCHK(hipMalloc((void **)&S.d_lanes, lanes * sizeof(LaneSave)));
        S.lanes_cap = lanes;
    }
    if ((size_t)S.grid > S.wg_cap) {
        if (S.d_wg) HIPCHK(hipFree(S.d_wg));
        S.d_wg = nullptr;
        HIPCHK(hipMalloc((void **)&S.d_wg, (size_t)S.grid * sizeof(WgSave)));
        S.wg_cap = S.grid;
    }
    int rate_khz = 0;
    HIPCHK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (rate_khz <= 0) rate_khz = 100000;
    S.slice_ticks = (long long)((double)ctx->slice_us * rate_khz / 1000.0);
    S.ticks_per_ms = (double)rate_khz;
    S.resume = false;
    S.precision = f32c ? NH_FP32C : NH_FP64;
    S.use_graph = ctx->serve_graph;
    for (SliceGraph &G : S.graph) slice_graph_destroy(G);   // launch shape may have changed
    return NH_OK;
}

int ensure_arena(nh_context *ctx, ServeState &S)
{
    if (S.arena_base) return NH_OK;
    size_t want = S.budget;
    if (want == 0) {
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        want = std::min((size_t)(0.8 * (double)fr), (size_t)32 << 30);
    }
    want &= ~(GRANULE - 1);
    if (want < GRANULE) return set_err(ctx, NH_EINVAL, "serving budget too small");
    if (hipMalloc((void **)&S.arena_base, want) != hipSuccess) {
        S.arena_base = nullptr;
        return set_err(ctx, NH_ENOMEM, "could not allocate the serving budget (%zu bytes)", want);
    }
    S.arena_bytes = want;
    S.arena.reset(want);
    return NH_OK;
}

void release_ticket_memory(ServeState &S, Ticket *t)
{
    if (t->bytes) S.arena.release(t->off, t->bytes);
    t->bytes = 0;
    if (t->slot >= 0) {
        S.h_desc[t->slot].retired = 1;
        S.free_slots.push_back(t->slot);
        t->slot = -1;
    }
    t->blob.clear();
    t->blob.shrink_to_fit();
}

#define WCHK(call)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) {                                                                      \
            std::snprintf(fail, sizeof(fail), "%s: %s", #call, hipGetErrorString(e_));               \
            return false;                                                                            \
        }                                                                                            \
    } while (0)

// One slice and everything between it and the next.  Called without the lock.
bool run_slice(nh_context *ctx, ServeState &S, char (&fail)[256])
{
    std::vector<Ticket *> upload, run, retiring;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        while (!S.queued.empty()) {
            Ticket *t = S.queued.front();
            S.queued.pop_front();
            t->st = St::Active;
            S.active.push_back(t);
            upload.push_back(t);
        }
        for (Ticket *t : S.active) {
            if (t->cancel && !t->retired) {
                t->retired = true;
                S.h_desc[t->slot].retired = 1;
            }
            if (t->retired) retiring.push_back(t);
            else run.push_back(t);
        }
        std::memcpy(S.h_desc_up, S.h_desc, SERVE_CAP * sizeof(BatchReq));
    }
    hipStream_t s = S.stream;
    for (Ticket *t : upload) {
        WCHK(hipMemcpyAsync(S.arena_base + t->off, t->blob.data(), t->blob_bytes, hipMemcpyHostToDevice, s));
        S.h_next[t->slot] = 0;
        WCHK(hipMemcpyAsync(S.d_next + t->slot, S.h_next + t->slot, sizeof(unsigned long long),
                            hipMemcpyHostToDevice, s));
        WCHK(hipMemcpyAsync(S.d_helpers + t->slot, S.h_zero + t->slot, sizeof(int), hipMemcpyHostToDevice, s));
    }
    int nc = NCOL - 1;
    bool pow = false;
    for (size_t i = 0; i < run.size(); ++i) {
        S.h_order[i] = run[i]->slot;
        nc = std::max(nc, run[i]->desc.nc);
        pow = pow || run[i]->desc.P.hist;
    }
    SliceArgs A{};
    A.reqs = S.d_desc;
    A.next = S.d_next;
    A.inflight = S.d_inflight;
    A.order = S.d_order;
    A.n_order = (int)run.size();
    // Oldest first, each request spread over as many workgroups as its
    // unclaimed work keeps busy for SERVE_SHARE_TPL trajectories per lane
    // (a workgroup drains before it changes request, so fewer would be
    // idle): under load a request no longer runs on the one workgroup that
    // opened it while fresh requests keep arriving.
    A.policy = POLICY_SHARE;
    A.cursor = nullptr;
    A.helpers = S.d_helpers;
    A.share = (long long)S.block * SERVE_SHARE_TPL;
    A.n_tab = S.n_tab;
    // Slice length: NH_OPT_SLICE_US, stretched up to 8x while the admitted
    // backlog would take more than four such slices to claim.  Every slice
    // boundary costs ~0.6 ms of drain and restart plus a host round trip, so
    // a loaded server runs longer slices (throughput), a light one short ones
    // (latency); the backlog is re-read at every boundary.
    long long unclaimed = 0;
    for (Ticket *t : run) {
        const long long left = t->n_traj - (long long)S.h_next[t->slot];
        unclaimed += left > 0 ? left : 0;
    }
    long long ticks = S.slice_ticks;
    if (S.claim_rate > 0.0) {
        const double backlog_ms = (double)unclaimed / S.claim_rate;
        const double want = 0.25 * backlog_ms * S.ticks_per_ms;
        if (want > (double)ticks) ticks = (long long)std::min(want, 8.0 * (double)S.slice_ticks);
    }
    unsigned long long claimed_before = 0;
    for (Ticket *t : run)
        claimed_before += std::min<unsigned long long>(S.h_next[t->slot], (unsigned long long)t->n_traj);
    A.budget_ticks = ticks;
    A.lane_save = S.d_lanes;
    A.wg_save = S.d_wg;
    A.resume = S.resume ? 1 : 0;
    const bool f32c = S.precision == NH_FP32C;
    if (S.use_graph) {
        // uploads, in-flight clear, slice kernel and read-backs as one graph launch
        SliceGraph &G = S.graph[(nc == NCOL ? 1 : 0) + (pow ? 2 : 0)];
        if (!G.exec) {
            SliceGraphBufs b{};
            b.d_desc = S.d_desc;
            b.d_order = S.d_order;
            b.d_next = S.d_next;
            b.d_inflight = S.d_inflight;
            b.h_desc = S.h_desc_up;
            b.h_order = S.h_order;
            b.h_next = S.h_next;
            b.h_inflight = S.h_inflight;
            b.desc_bytes = SERVE_CAP * sizeof(BatchReq);
            b.order_bytes = SERVE_CAP * sizeof(int);
            b.next_bytes = SERVE_CAP * sizeof(unsigned long long);
            b.inflight_bytes = SERVE_CAP * sizeof(unsigned int);
            WCHK(slice_graph_build(G, b, A, f32c, nc, S.slots, pow, S.grid, S.block));
        }
        WCHK(hipEventRecord(S.ev0, s));
        WCHK(slice_graph_launch(G, A, s));
        WCHK(hipEventRecord(S.ev1, s));
    } else {
        WCHK(hipMemcpyAsync(S.d_desc, S.h_desc_up, SERVE_CAP * sizeof(BatchReq), hipMemcpyHostToDevice, s));
        if (!run.empty())
            WCHK(hipMemcpyAsync(S.d_order, S.h_order, run.size() * sizeof(int), hipMemcpyHostToDevice, s));
        WCHK(launch_fill_u64((unsigned long long *)S.d_inflight, SERVE_CAP / 2, 0ull, s));
        WCHK(hipEventRecord(S.ev0, s));
        WCHK(launch_slice(A, f32c, nc, S.slots, pow, S.grid, S.block, s));
        WCHK(hipEventRecord(S.ev1, s));
        WCHK(hipMemcpyAsync(S.h_next, S.d_next, SERVE_CAP * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        WCHK(hipMemcpyAsync(S.h_inflight, S.d_inflight, SERVE_CAP * sizeof(unsigned int), hipMemcpyDeviceToHost,
                            s));
    }
    S.resume = true;
    WCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    WCHK(hipEventElapsedTime(&ms, S.ev0, S.ev1));
    {
        unsigned long long claimed_after = 0;
        for (Ticket *t : run)
            claimed_after += std::min<unsigned long long>(S.h_next[t->slot], (unsigned long long)t->n_traj);
        const double got = (double)(claimed_after > claimed_before ? claimed_after - claimed_before : 0);
        if (ms > 0.f && got > 0.0) {
            const double r = got / ms;
            S.claim_rate = S.claim_rate > 0.0 ? 0.7 * S.claim_rate + 0.3 * r : r;
        }
    }

    // finished requests: queue exhausted and nothing saved in flight
    std::vector<Ticket *> done;
    for (Ticket *t : run) {
        t->kernel_ms += ms;
        if (S.h_next[t->slot] >= (unsigned long long)t->n_traj && S.h_inflight[t->slot] == 0) done.push_back(t);
    }
    if (!done.empty()) {
        int rt = 0;
        long long nmax = 1;
        for (size_t i = 0; i < done.size(); ++i) {
            S.h_list[i] = done[i]->slot;
            S.h_rstart[i] = rt;
            rt += done[i]->n_r;
            nmax = std::max(nmax, done[i]->n_traj);
        }
        S.h_rstart[done.size()] = rt;
        const int nd = (int)done.size();
        WCHK(hipMemcpyAsync(S.d_list, S.h_list, nd * sizeof(int), hipMemcpyHostToDevice, s));
        WCHK(hipMemcpyAsync(S.d_rstart, S.h_rstart, (nd + 1) * sizeof(int), hipMemcpyHostToDevice, s));
        WCHK(launch_fill_u64(S.d_stats, 8 * nd, 0ull, s));
        const int chunks = (int)std::min(256ll, (nmax + 256 * 64 - 1) / (256 * 64));
        WCHK(launch_reduce_batch(S.d_desc, S.d_list, S.d_rstart, nd, rt, S.d_stats, chunks, s));
        WCHK(hipMemcpyAsync(S.h_stats, S.d_stats, 8 * nd * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        for (Ticket *t : done) {
            t->result.resize(t->n_r);
            WCHK(hipMemcpyAsync(t->result.data(), t->desc.out, t->n_r * sizeof(double), hipMemcpyDeviceToHost, s));
        }
        WCHK(hipStreamSynchronize(s));
    }
    const Clock::time_point now = Clock::now();
    {
        std::lock_guard<std::mutex> lk(S.mu);
        for (size_t i = 0; i < done.size(); ++i) {
            Ticket *t = done[i];
            stats_from_words(&S.h_stats[8 * i], t->n_traj, t->kernel_ms, t->stats);
            t->stats.latency_ms = std::chrono::duration<double, std::milli>(now - t->t_submit).count();
            t->rc = t->stats.n_failed > 0 ? NH_ESTEPS : NH_OK;
            release_ticket_memory(S, t);
            if (t->cancel) {
                t->st = St::Cancelled;
                t->result.clear();
            } else {
                t->st = St::Done;
            }
        }
        // a retired request was dropped by the slice that just ran: its memory is free now
        for (Ticket *t : retiring) {
            release_ticket_memory(S, t);
            t->st = St::Cancelled;
        }
        std::vector<Ticket *> keep;
        for (Ticket *t : S.active)
            if (t->st == St::Active) keep.push_back(t);
        S.active.swap(keep);
        if (S.active.empty() && S.queued.empty()) S.precision = -1;   // the next request starts a session
    }
    return true;
}

void worker_main(nh_context *ctx, ServeState *S)
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop || !S->queued.empty() || !S->active.empty(); });
            if (S->stop) return;
        }
        char fail[256] = "";
        if (!run_slice(ctx, *S, fail)) {
            // a device failure ends every admitted request
            std::lock_guard<std::mutex> lk(S->mu);
            std::snprintf(S->failure, sizeof(S->failure), "%s", fail);
            for (Ticket *t : S->active) {
                t->st = St::Done;
                t->rc = NH_EDEVICE;
                release_ticket_memory(*S, t);
            }
            for (Ticket *t : S->queued) {
                t->st = St::Done;
                t->rc = NH_EDEVICE;
                release_ticket_memory(*S, t);
            }
            S->active.clear();
            S->queued.clear();
            S->precision = -1;
            S->resume = false;
        }
    }
}

ServeState *state_of(nh_context *ctx)
{
    if (!ctx->serve) ctx->serve = new (std::nothrow) ServeState();
    return ctx->serve;
}

}  // namespace

bool serve_idle(nh_context *ctx)
{
    ServeState *S = ctx->serve;
    if (!S) return true;
    std::lock_guard<std::mutex> lk(S->mu);
    return S->active.empty() && S->queued.empty();
}

void serve_shutdown(nh_context *ctx)
{
    ServeState *S = ctx->serve;
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    for (SliceGraph &G : S->graph) slice_graph_destroy(G);
    for (void *p : {(void *)S->d_desc, (void *)S->d_next, (void *)S->d_inflight, (void *)S->d_helpers, (void *)S->d_stats,
                    (void *)S->d_order, (void *)S->d_list, (void *)S->d_rstart, (void *)S->d_lanes,
                    (void *)S->d_wg, (void *)S->arena_base})
        if (p) (void)hipFree(p);
    for (void *p : {(void *)S->h_desc, (void *)S->h_desc_up, (void *)S->h_order, (void *)S->h_list, (void *)S->h_rstart,
                    (void *)S->h_next, (void *)S->h_inflight, (void *)S->h_zero, (void *)S->h_stats})
        if (p) (void)hipHostFree(p);
    if (S->ev0) (void)hipEventDestroy(S->ev0);
    if (S->ev1) (void)hipEventDestroy(S->ev1);
    if (S->stream) (void)hipStreamDestroy(S->stream);
    for (auto &kv : S->tickets) delete kv.second;
    delete S;
    ctx->serve = nullptr;
}

}  // namespace nh

using namespace nh;

extern "C" {

int nh_serve_set_budget(nh_context *ctx, size_t bytes)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    ServeState *S = state_of(ctx);
    if (!S) return set_err(ctx, NH_ENOMEM, "serving state");
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->active.empty() || !S->queued.empty())
        return set_err(ctx, NH_EBUSY, "the serving budget can change only while nothing is admitted");
    if (S->arena_base) {
        if (hipSetDevice(ctx->device) != hipSuccess || hipFree(S->arena_base) != hipSuccess)
            return set_err(ctx, NH_EDEVICE, "could not release the previous serving budget");
        S->arena_base = nullptr;
        S->arena.reset(0);
    }
    S->budget = bytes;
    return NH_OK;
}

int nh_submit(nh_context *ctx, const nh_request *req, uint64_t *ticket)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    if (!req || !ticket) return set_err(ctx, NH_EINVAL, "req and ticket are required");
    int rc = check_batchable(ctx, req, 0, -1);
    if (rc != NH_OK) return rc;
    ServeState *S = state_of(ctx);
    if (!S) return set_err(ctx, NH_ENOMEM, "serving state");
    const Clock::time_point t0 = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return set_err(ctx, NH_EINVAL, "the server is shutting down");
    if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, NH_EDEVICE, "hipSetDevice failed");
    if ((rc = alloc_device_state(ctx, *S)) != NH_OK) return rc;
    if ((rc = ensure_arena(ctx, *S)) != NH_OK) return rc;
    const bool f32c = req->integ.precision == NH_FP32C;
    if (S->precision < 0) {
        if ((rc = start_session(ctx, *S, f32c)) != NH_OK) return rc;
    } else if (S->precision != req->integ.precision) {
        return set_err(ctx, NH_EINVAL, "this server is serving %s requests", S->precision == NH_FP32C ? "FP32C" : "FP64");
    }
    if (S->free_slots.empty()) return set_err(ctx, NH_EBUSY, "%d requests are admitted already", SERVE_CAP);
    const Staged lay = stage_layout(req, S->n_tab);
    if (!sampled_table_fits(req, S->n_tab)) {
        if (S->active.empty() && S->queued.empty()) S->precision = -1;
        return set_err(ctx, NH_EINVAL, "%d history samples need at least 3 of the %d table nodes per sample interval",
                       req->halo.history.n, S->n_tab);
    }
    const long long n_traj = n_traj_of(req);
    const size_t bytes = ticket_bytes(lay, n_traj, req->grid.n_r);
    size_t off = 0;
    if (!S->arena.alloc(bytes, off)) {
        const bool empty = S->active.empty() && S->queued.empty();
        if (empty) S->precision = -1;
        return set_err(ctx, NH_EBUSY, "request needs %zu bytes; %zu of %zu in use", bytes, S->arena.used(),
                       S->arena.size());
    }
    Ticket *t = new (std::nothrow) Ticket();
    if (!t) {
        S->arena.release(off, bytes);
        return set_err(ctx, NH_ENOMEM, "ticket");
    }
    t->id = S->next_id++;
    t->slot = S->free_slots.back();
    S->free_slots.pop_back();
    t->off = off;
    t->bytes = bytes;
    t->n_r = req->grid.n_r;
    t->n_traj = n_traj;
    t->blob_bytes = lay.bytes;
    t->blob.resize(lay.bytes);
    char *dev = S->arena_base + off;
    double *ratio = (double *)(dev + round_up(lay.bytes));
    TrajStat *stat = (TrajStat *)((char *)ratio + round_up((size_t)n_traj * sizeof(double)));
    double *out = (double *)((char *)stat + round_up((size_t)n_traj * sizeof(TrajStat)));
    describe(ctx, req, lay, t->blob.data(), dev, ratio, stat, out, t->desc);
    S->h_desc[t->slot] = t->desc;
    t->t_submit = t0;
    S->tickets[t->id] = t;
    S->queued.push_back(t);
    if (!S->running) {
        S->running = true;
        S->worker = std::thread(worker_main, ctx, S);
    }
    S->cv.notify_all();
    *ticket = t->id;
    return NH_OK;
}

int nh_poll(nh_context *ctx, uint64_t ticket, double *out, nh_stats *stats)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    ServeState *S = ctx->serve;
    if (!S) return set_err(ctx, NH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return set_err(ctx, NH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Ticket *t = it->second;
    if (t->st == St::Queued || t->st == St::Active) return NH_ENOTREADY;
    int rc;
    if (t->st == St::Cancelled) {
        rc = set_err(ctx, NH_ECANCELED, "ticket %llu was cancelled", (unsigned long long)ticket);
    } else {
        rc = t->rc;
        if (rc == NH_EDEVICE) {
            set_err(ctx, rc, "serving failed: %s", S->failure);
        } else {
            if (!out) return set_err(ctx, NH_EINVAL, "out is NULL");
            std::memcpy(out, t->result.data(), t->result.size() * sizeof(double));
            if (stats) *stats = t->stats;
            if (rc == NH_ESTEPS)
                set_err(ctx, rc, "%lld trajectories did not finish cleanly", t->stats.n_failed);
        }
    }
    S->tickets.erase(it);
    delete t;
    return rc;
}

int nh_cancel(nh_context *ctx, uint64_t ticket)
{
    if (!ctx) return set_err(nullptr, NH_EINVAL, "context is NULL");
    ServeState *S = ctx->serve;
    if (!S) return set_err(ctx, NH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return set_err(ctx, NH_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Ticket *t = it->second;
    switch (t->st) {
    case St::Queued: {
        auto q = std::find(S->queued.begin(), S->queued.end(), t);
        if (q != S->queued.end()) S->queued.erase(q);
        release_ticket_memory(*S, t);
        t->st = St::Cancelled;
        if (S->active.empty() && S->queued.empty()) S->precision = -1;
        break;
    }
    case St::Active:
        t->cancel = true;     // applied at the next slice boundary
        break;
    case St::Done:
        t->st = St::Cancelled;
        t->result.clear();
        break;
    case St::Cancelled:
        break;
    }
    return NH_OK;
}

}  // extern "C"
